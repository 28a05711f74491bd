"""GPU proposer kernels against the fp64 reference (oracle.mlp): gradients
within 1e-4 relative, forward within 1e-5, bf16 inference close to fp32,
and Adam training that lowers the loss."""
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
    err = np.linalg.norm(g.cpu().numpy() - g_ref) / np.linalg.norm(g_ref)
    assert err <= 1e-4, err
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
