"""GPU proposer kernels against the fp64 reference (oracle.mlp): every
gradient element within 1e-4 of the largest (fp32 sums over at most 4096
rows), the forward within 1e-5, one Adam step element by element, bf16
inference close to fp32, and Adam training that lowers the loss."""
import numpy as np
import pytest
import torch

import paper_2412_18629_amd as rs
from oracle import mlp

pytestmark = pytest.mark.gpu


def _data(n, seed):
    rng = np.random.default_rng(seed)
    p = (mlp.init(seed) + rng.normal(0, 0.02, mlp.NPARAM)).astype(np.float32)
    X = rng.normal(0, 1, (n, mlp.NIN)).astype(np.float32)
    t = rng.normal(0, 1, n).astype(np.float32)
    return p, X, t


@pytest.mark.parametrize("n,seed", [(1, 0), (37, 1), (512, 2), (4096, 3)])
def test_gradient_matches_oracle(n, seed):
    p, X, t = _data(n, seed)
    g, loss = rs.rs_mlp_grad(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda(),
                             torch.from_numpy(t).cuda())
    g_ref = mlp.grad(p.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    # element by element: the fp32 accumulation over n rows bounds each
    # element's error by a small multiple of the largest element
    tol = 1e-4 * np.max(np.abs(g_ref)) + 1e-7
    diff = np.abs(g.cpu().numpy() - g_ref)
    assert diff.max() <= tol, (diff.max(), tol, int(diff.argmax()))
    assert abs(loss.item() - mlp.loss(p, X, t)) <= 1e-4 * max(1.0, mlp.loss(p, X, t))


def test_forward_matches_oracle():
    p, X, t = _data(1000, 4)
    y = rs.rs_mlp_forward(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda()).cpu().numpy()
    y_ref, _ = mlp.forward(p, X)
    assert np.max(np.abs(y - y_ref)) <= 1e-5 * max(1.0, np.max(np.abs(y_ref)))


def test_bf16_inference_close_to_fp32():
    p, X, t = _data(2000, 5)
    rng = np.random.default_rng(5)
    mean = rng.normal(0, 2, mlp.NIN).astype(np.float32)
    std = rng.uniform(0.5, 3, mlp.NIN).astype(np.float32)
    raw = X * std + mean
    model = torch.from_numpy(np.concatenate([mean, std, p])).cuda()
    y = rs.rs_mlp_infer(model, torch.from_numpy(raw).cuda()).cpu().numpy()
    y_ref, _ = mlp.forward(p, (raw - mean) / std)
    scale = np.max(np.abs(y_ref))
    assert np.max(np.abs(y - y_ref)) <= 0.03 * scale


def test_standardize_and_training_lower_loss():
    rng = np.random.default_rng(6)
    teacher = mlp.init(7)
    Xr = rng.normal(3, 2, (8192, mlp.NIN)).astype(np.float32)
    X = torch.from_numpy(Xr).cuda()
    mean = torch.empty(mlp.NIN, device="cuda"); std = torch.empty(mlp.NIN, device="cuda")
    rs.rs_mlp_standardize(X, mean, std, compute=True)
    assert np.allclose(mean.cpu().numpy(), Xr.mean(0), atol=1e-3)
    assert np.allclose(std.cpu().numpy(), Xr.std(0), rtol=1e-3)
    t = torch.from_numpy(mlp.forward(teacher, X.cpu().numpy())[0].astype(np.float32)).cuda()
    params = torch.from_numpy(mlp.init(8).astype(np.float32)).cuda()
    m = torch.zeros_like(params); v = torch.zeros_like(params)
    loss = torch.zeros(1, device="cuda")
    first = None
    for step in range(1, 301):
        idx = torch.arange((step * 1024) % 8192, (step * 1024) % 8192 + 1024, device="cuda")
        rs.rs_mlp_train_step(params, m, v, step, X[idx].contiguous(), t[idx].contiguous(), 3e-3,
                             loss)
        if first is None:
            first = loss.item()
    _, final = rs.rs_mlp_grad(params, X, t)
    assert final.item() < 0.2 * first


@pytest.mark.parametrize("step,seed", [(1, 11), (7, 12)])
def test_adam_step_matches_oracle(step, seed):
    # one rs_mlp_train_step from given parameters and moments against the
    # fp64 Adam step: moments element by element within the gradient's
    # tolerance, parameters wherever the gradient is well above it (where
    # the update's direction is not decided by rounding)
    rng = np.random.default_rng(seed)
    p, X, t = _data(2048, seed)
    m0 = (rng.normal(0, 1e-3, mlp.NPARAM)).astype(np.float32)
    v0 = (rng.uniform(0, 1e-6, mlp.NPARAM)).astype(np.float32)
    lr = 1e-3
    P, M, V = (torch.from_numpy(a.copy()).cuda() for a in (p, m0, v0))
    loss = torch.zeros(1, device="cuda")
    rs.rs_mlp_train_step(P, M, V, step, torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda(),
                         lr, loss)
    pr, mr, vr, lr_loss = mlp.adam_step(p, m0, v0, step, X, t, lr)
    g_ref = mlp.grad(p.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    tol_g = 1e-4 * np.max(np.abs(g_ref)) + 1e-7
    assert abs(loss.item() - lr_loss) <= 1e-4 * max(1.0, lr_loss)
    assert np.max(np.abs(M.cpu().numpy() - mr)) <= 0.1 * tol_g + 1e-9
    dv = np.abs(V.cpu().numpy() - vr)
    assert np.all(dv <= 1e-3 * (2 * np.abs(g_ref) * tol_g + tol_g ** 2) + 1e-6 * vr + 1e-12)
    sure = np.abs(g_ref) > 100 * tol_g
    assert sure.sum() > mlp.NPARAM // 4
    dp = np.abs(P.cpu().numpy() - pr)[sure]
    assert dp.max() <= 0.05 * lr + 1e-6, dp.max()
