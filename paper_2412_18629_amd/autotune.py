"""Autotuner for the launch shapes of the batched level pipeline.

For every knob of the library's tuning table (rs_tune_*: threads per
workgroup of the size-bucketed small-node kernels, the XCD chunk of the
large-node search kernels) it times each allowed value on the benchmark
workload with the other knobs at their best so far, keeps the fastest, and
checks that every candidate produced exactly the same tree.  The table is
written as JSON next to the package; bench.py and the tests apply it with
paper_2412_18629_amd.load_tuning().

    python -m paper_2412_18629_amd.autotune [--config c512] [--reps 2]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import torch

import paper_2412_18629_amd as rs
from paper_2412_18629_amd import learn, synth

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuning_gfx950.json")

# the instrumented kernels each knob moves (rs_profile names), reported beside
# the wall time of the whole 6D call, which decides (the level-0 small
# subtrees overlap the large-node levels, so their own span is not exclusive)
KNOB_KERNELS = {
    "small_threads_256": ("phase_small", "phase_small_level0", "phase_small_children"),
    "small_threads_1024": ("phase_small", "phase_small_level0", "phase_small_children"),
    "small_threads_2048": ("phase_small", "phase_small_level0", "phase_small_children"),
    "xcd_chunk": ("phase_large_nn", "phase_large_nn_fallback", "phase_large_link"),
}
FIELDS = ("level", "min_index", "parent", "size", "l2", "a", "c", "sx2", "sv2", "deepest")


def _digest(tree):
    h = hashlib.sha256()
    for k in FIELDS:
        h.update(tree[k].cpu().numpy().tobytes())
    return h.hexdigest()


def _measure(run, kernels, reps):
    run()                                            # warm-up at this setting
    rs.rs_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        tree = run()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1000.0 / reps
    kern = sum(rs.rs_profile_get(k)[0] for k in kernels) / reps
    rs.rs_profile_enable(False)
    return wall, kern, _digest(tree)


def tune(config="c512", reps=2, verbose=True):
    cfg = synth.CONFIGS[config]
    dev = torch.device("cuda:0")
    arrs = synth.generate(cfg, 0, device=dev)
    torch.cuda.empty_cache()
    labels = torch.empty(cfg.n, dtype=torch.int32, device=dev)
    rs.rs_fof3d(*arrs[:3], cfg.box, cfg.link_len, labels=labels)
    model = learn.load_model()

    def run():
        return rs.rs_phase_fof_batch(*arrs, cfg.box, labels, cfg.min_group, cfg.min_sub, cfg.f,
                                     flags=rs.RS_LEARNED, model=model)

    knobs = rs.tune_knobs()
    choice = {k: v[0] for k, v in knobs.items()}
    timings, kernel_ms, ref = {}, {}, None
    for knob, (_, allowed) in knobs.items():
        timings[knob] = {}
        for value in allowed:
            rs.tune_set(knob, value)
            ms, kern_ms, dig = _measure(run, KNOB_KERNELS[knob], reps)
            if ref is None:
                ref = dig
            if dig != ref:
                raise RuntimeError(f"{knob}={value} changed the result")
            timings[knob][str(value)] = ms
            kernel_ms.setdefault(knob, {})[str(value)] = kern_ms
            if verbose:
                print(f"{knob} = {value}: {ms:.2f} ms per 6D call ({kern_ms:.2f} ms in "
                      f"{', '.join(KNOB_KERNELS[knob])})", flush=True)
        best = min(allowed, key=lambda v: timings[knob][str(v)])
        choice[knob] = best
        rs.tune_set(knob, best)
    return {"workload": config, "form": "learned", "reps": reps, "choice": choice,
            "timings_ms": timings, "kernel_ms": kernel_ms, "result_sha256": ref,
            "device": torch.cuda.get_device_name(0), "time": time.strftime("%Y-%m-%d")}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c512")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--out", default=DEFAULT_TABLE)
    args = ap.parse_args(argv)
    table = tune(args.config, args.reps)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps(table["choice"]), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
