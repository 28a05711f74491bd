"""Training of the linking-length proposer on the GPU with the library's kernels.

Training pairs come from the exact method itself: for every node of the
hierarchy on seeded 256^3 workloads (seeds 100-199 for the shipped model), (features, ln l) where l^2 is the exact
linking length the batched form chose.  The network is trained with the
library's own forward / backward / Adam kernels (rs_mlp_train_step); this
module only shuffles minibatch indices and moves tensors.

    python -m paper_2412_18629_amd.learn --seeds 100-199 --out paper_2412_18629_amd/mlp_c256.bin
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np
import torch

import paper_2412_18629_amd as rs
from paper_2412_18629_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(HERE, "mlp_c256.bin")


def collect(seeds, config="c256", device="cuda", verbose=True, min_size=0):
    """(features [n, 24], ln l [n]) device tensors from the exact batched form,
    for nodes with more than min_size members."""
    cfg = synth.CONFIGS[config] if isinstance(config, str) else config
    xs, ys = [], []
    for seed in seeds:
        t0 = time.time()
        arrs = synth.generate(cfg, seed, device=device)
        lab, _ = rs.rs_fof3d(*arrs[:3], cfg.box, cfg.link_len)
        tree = rs.rs_phase_fof_batch(*arrs, cfg.box, lab, cfg.min_group, cfg.min_sub, cfg.f,
                                     flags=rs.RS_BATCHED | rs.RS_FEATURES)
        keep = (tree["l2"] > 0) & (tree["size"] > min_size)
        xs.append(tree["features"][keep].contiguous())
        ys.append((0.5 * torch.log(tree["l2"][keep].double())).float())
        if verbose:
            print(f"seed {seed}: {int(keep.sum())} nodes in {time.time() - t0:.1f} s", flush=True)
        del arrs, lab, tree
    return torch.cat(xs).contiguous(), torch.cat(ys).contiguous()


def init_params(seed=0):
    """He-normal weights, zero biases, in the library's flat layout."""
    rng = np.random.default_rng(seed)
    w1 = rng.normal(0.0, np.sqrt(2.0 / 24), (64, 24))
    w2 = rng.normal(0.0, np.sqrt(2.0 / 64), (64, 64))
    w3 = rng.normal(0.0, np.sqrt(2.0 / 64), 64)
    return np.concatenate([w1.ravel(), np.zeros(64), w2.ravel(), np.zeros(64), w3.ravel(),
                           np.zeros(1)]).astype(np.float32)


def train(X, y, epochs=20, batch=4096, lr=1e-3, seed=0, verbose=True):
    """Standardise features, then Adam on mean squared error of ln l.
    Returns (mean, std, params) as numpy arrays and the per-epoch losses."""
    dev = X.device
    X = X.clone()
    mean = torch.empty(rs.RS_NFEAT, dtype=torch.float32, device=dev)
    std = torch.empty(rs.RS_NFEAT, dtype=torch.float32, device=dev)
    rs.rs_mlp_standardize(X, mean, std, compute=True)
    params = torch.from_numpy(init_params(seed)).to(dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    n = X.shape[0]
    step = 0
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g, device=dev)
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            xb = X[idx].contiguous()
            yb = y[idx].contiguous()
            step += 1
            rs.rs_mlp_train_step(params, m, v, step, xb, yb, lr, loss)
            if b0 % (16 * batch) == 0:
                tot += float(loss.item())
                cnt += 1
        losses.append(tot / max(cnt, 1))
        if verbose:
            print(f"epoch {ep}: loss {losses[-1]:.4f}", flush=True)
    return mean.cpu().numpy(), std.cpu().numpy(), params.cpu().numpy(), losses


def save(path, mean, std, params):
    with open(path, "wb") as f:
        f.write(rs.pack_model(mean, std, params))


def load_model(path=DEFAULT_MODEL) -> bytes:
    with open(path, "rb") as f:
        return f.read()


def _seeds(spec):
    a, _, b = spec.partition("-")
    return list(range(int(a), int(b or a) + 1))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", default="100-199")
    ap.add_argument("--config", default="c256")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--min-size", type=int, default=0,
                    help="train only on nodes with more members (the proposer is applied to "
                         "nodes of more than 2048)")
    ap.add_argument("--out", default=DEFAULT_MODEL)
    args = ap.parse_args(argv)
    X, y = collect(_seeds(args.seeds), args.config, min_size=args.min_size)
    print(f"training on {X.shape[0]} (node, level) pairs", flush=True)
    mean, std, params, _ = train(X, y, epochs=args.epochs)
    save(args.out, mean, std, params)
    print(f"wrote {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
