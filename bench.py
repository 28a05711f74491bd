"""Benchmark: particles/s through the 3D + hierarchical 6D FoF hot path.

One step = rs_fof3d over the whole box, then rs_phase_fof_batch over every
3D group, on the 512^3 synthetic workload (inputs resident in HBM before the
timed region).  Prints one JSON line with the throughput, the roofline of the
dominant kernel (HIP events recorded by the library on its launch stream)
and the CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--form learned|batched|plain]

The timed form is the learned one (the committed proposer); the line also
reports the learned form's speed-up over the batched form and over the plain
form (one group per launch sequence) on the same data, the small-node
kernels' figures, and the halo-property and seed-assignment calls over the
last step's hierarchy.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

import paper_2412_18629_amd as rs  # noqa: E402
from paper_2412_18629_amd import learn, synth  # noqa: E402

METRIC = "particles/s through 3D+6D FoF at 512³ (labels == oracle); learned vs plain speedup"
HBM_PEAK_GBS = 8000.0

# algorithmic bytes per work unit of each instrumented kernel
KERNEL_BYTES = {
    "fof3d_link": 16.0,        # 12 B sorted position in, 4 B parent out, per particle
    "phase_large_nn": 28.0,    # 24 B position+velocity in, 4 B d^2 out, per member
    "phase_large_link": 32.0,  # 24 B pos+vel + 4 B d^2 in, 4 B parent out, per member
    "phase_large_nn_fallback": 28.0,
}
# the small-node subtree kernels (side streams): 28 B member record in and
# 4 B deepest node out per member of a subtree root (deeper levels stay in LDS)
SMALL_BYTES = 32.0
SMALL_MAX = 2048
# halo properties: one 24-byte record read per member of every node
PROPS_BYTES = 24.0
# seed assignment: one (particle, seed) test is d^2 = fl(fl(a Dx) + fl(c Dv)),
# 19 fp32 adds, subtracts and multiplies (3 + 3 differences, 3 + 3 squares,
# 2 + 2 sums, 2 scalings, 1 sum); no FMA by definition and no packed
# arithmetic, so the bound is the plain vector ALU rate: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz = 39.3 T operations/s (the 157.3 TFLOP/s fp32 figure
# counts a packed FMA as four)
SEED_FLOPS = 19.0
ALU_PEAK_TFLOPS = 256 * 64 * 2.4e9 / 1e12
FLAGS = {"learned": rs.RS_LEARNED, "batched": rs.RS_BATCHED, "plain": rs.RS_PLAIN}

# device symbol and source files of each instrumented kernel (the PMC summary
# is only used while these sources are unchanged)
KERNEL_SYMBOL = {
    # the timed instantiations (32-bit member offsets, no pair counters)
    "fof3d_link": ("void rs::k_link<true, true, false>(", ["fof3d.hip", "common.h"]),
    "phase_large_nn": ("void rs::k_tree_nn<true, false>(",
                       ["phase_tree.hip", "phase_common.h", "common.h"]),
    "phase_large_link": ("void rs::k_tile_link<true, false>(",
                         ["phase_tile.hip", "phase_common.h", "common.h"]),
    "phase_small": ("void rs::k_small_subtree<",
                    ["phase_small.hip", "phase_common.h", "common.h"]),
    "halo_props": ("rs::k_pr_large(", ["props.hip", "common.h"]),
}
CSRC = os.path.join(HERE, "paper_2412_18629_amd", "csrc")
PMC_SUMMARY = os.path.join(HERE, "profiles", "pmc_traffic_c512.json")


def source_digest(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SYMBOL[kernel][1]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _pmc_rows(path, counter):
    """{dispatch id: (kernel name, summed counter value in KiB)}"""
    out = {}
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            d = int(r["Dispatch_Id"])
            name, v = out.get(d, (r["Kernel_Name"], 0.0))
            out[d] = (name, v + float(r["Counter_Value"]))
    return out


def _kernel_values(rows, kernel):
    """Counter values of one timed kernel's dispatches, in dispatch order.  A
    `k_tree_nn` dispatch that follows the acceptance of the learned brackets
    (`k_laccept`) is the refinement pass, timed as phase_large_nn_fallback and
    left out of phase_large_nn."""
    sym = KERNEL_SYMBOL[kernel][0]
    out, prev = [], ""
    for d in sorted(rows):
        name, v = rows[d]
        if name.startswith(sym):
            if not (kernel == "phase_large_nn" and "k_laccept" in prev):
                out.append(v)
        elif "rs::" in name:
            prev = name
    return out


# vector ALU: 256 CUs x 4 SIMDs of 16 lanes, so a full wave64 VALU
# instruction occupies its SIMD for 4 cycles.  SQ_INSTS_VALU counts the VALU
# instructions the wavefronts issued; GRBM_GUI_ACTIVE is the busy cycles,
# summed over the 8 XCDs (per XCD it matches the kernel's duration at the
# shader clock).  Charging every counted instruction 4 cycles gives the
# issue density: 1.0 means one VALU instruction per SIMD every 4 cycles.
# It is not a strict utilisation: instructions that read one lane into a
# scalar register, or run with few lanes enabled, are counted but take
# fewer cycles, so a saturated kernel can read slightly above 1.
N_SIMD = 1024
N_XCD = 8
VALU_CYCLES = 4


def valu_busy(insts, gui_active):
    """VALU issue density (4 cycles charged per counted instruction, over
    every SIMD's cycles) from SQ_INSTS_VALU and GRBM_GUI_ACTIVE summed over a
    kernel's dispatches."""
    if insts <= 0 or gui_active <= 0:
        return None
    return insts * VALU_CYCLES / (gui_active / N_XCD * N_SIMD)


def pmc_summary(fetch_csv, write_csv, copy_bytes, command, out_path, valu_csv=None):
    """Per-launch HBM traffic of the instrumented kernels from a FETCH_SIZE run
    and a WRITE_SIZE run of this script (with --probe-copy), each counter
    scaled by what it reads for the plain device copy of known size; with a
    third run of SQ_INSTS_VALU and GRBM_GUI_ACTIVE, the fraction of the
    vector ALU issue cycles each kernel used."""
    fe, wr = _pmc_rows(fetch_csv, "FETCH_SIZE"), _pmc_rows(write_csv, "WRITE_SIZE")
    va = _pmc_rows(valu_csv, "SQ_INSTS_VALU") if valu_csv else {}
    gr = _pmc_rows(valu_csv, "GRBM_GUI_ACTIVE") if valu_csv else {}

    def probe(rows):
        vals = sorted(v for n, v in rows.values() if "copyBuffer" in n)[-3:]
        return (copy_bytes / 1024.0) / float(np.median(vals))

    sf, sw = probe(fe), probe(wr)
    res = {"workload": "c512", "command": command,
           "calibration": {"copy_bytes": copy_bytes, "fetch_scale": sf, "write_scale": sw},
           "kernels": {}}
    for k, (sym, _) in KERNEL_SYMBOL.items():
        f, w = _kernel_values(fe, k), _kernel_values(wr, k)
        if not f or len(f) != len(w):
            continue
        per = [(a * sf + b * sw) * 1024.0 for a, b in zip(f, w)]
        res["kernels"][k] = {"symbol": sym, "launches": len(f), "fetch_kib": f, "write_kib": w,
                             "hbm_bytes_per_launch": float(np.mean(per)),
                             "sources_sha256": source_digest(k)}
        busy = valu_busy(sum(_kernel_values(va, k)), sum(_kernel_values(gr, k)))
        if busy is not None:
            res["kernels"][k]["valu_busy"] = busy
    with open(out_path, "w") as fh:
        json.dump(res, fh, indent=1)
    return res


def measured_pmc(kernel, workload, field):
    """A field of the committed PMC summary for this kernel, or None when there
    is none for this kernel and workload or the kernel's sources changed."""
    try:
        with open(PMC_SUMMARY) as fh:
            pm = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = pm.get("kernels", {}).get(kernel)
    if pm.get("workload") != workload or not ent or kernel not in KERNEL_SYMBOL:
        return None
    if ent.get("sources_sha256") != source_digest(kernel):
        return None
    return ent.get(field)


def workload_description(cfg):
    side = round(cfg.n ** (1.0 / 3.0))
    cube = f"{side}^3" if side ** 3 == cfg.n else f"{cfg.n}"
    return (f"{cfg.name}: {cfg.n} particles ({cube}) in a periodic {cfg.box:g} Mpc/h box, "
            f"{cfg.n_hosts} NFW hosts of {cfg.m_lo:g}-{cfg.m_hi:g} particles (dn/dM ~ M^{cfg.slope}) "
            f"with 0-{cfg.n_sub_max} subhaloes, {cfg.bg_frac:.0%} uniform background; 3D FoF "
            f"b={cfg.b} (ll={cfg.link_len:.6g}), 6D FoF f={cfg.f}, min group/subgroup "
            f"{cfg.min_group}/{cfg.min_sub}; seed 0")


def one_step(arrs, cfg, form, labels, model):
    x, y, z, vx, vy, vz = arrs
    rs.rs_fof3d(x, y, z, cfg.box, cfg.link_len, labels=labels)
    return rs.rs_phase_fof_batch(x, y, z, vx, vy, vz, cfg.box, labels, cfg.min_group,
                                 cfg.min_sub, cfg.f, flags=FLAGS[form],
                                 model=model if form == "learned" else None)


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed(fn, reps=1):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1000.0 / reps, out


def speedups(arrs, cfg, labels, model, ms_learned):
    """Learned over batched and over plain (one group per launch sequence),
    each timed once on the same data."""
    ms_b, _ = timed(lambda: one_step(arrs, cfg, "batched", labels, model))
    ms_p, _ = timed(lambda: one_step(arrs, cfg, "plain", labels, model))
    return {"vs_batched": ms_b / ms_learned, "batched_ms_per_step": ms_b,
            "vs_plain": ms_p / ms_learned, "plain_ms_per_step": ms_p,
            "plain_workload": cfg.name}


def pair_tests(arrs, cfg, form, labels, model, kernel_ms):
    """Pair tests of the searches, counted on one extra (untimed) step with
    the counting kernel builds, per second of the timed step's kernels."""
    rs.rs_profile_enable(False)
    rs.rs_profile_enable(2)
    one_step(arrs, cfg, form, labels, model)
    torch.cuda.synchronize()
    got = {k: rs.rs_profile_get(k)[2] for k in ("pairs_fof3d", "pairs_nn", "pairs_link")}
    rs.rs_profile_enable(False)
    ms = {"pairs_fof3d": kernel_ms["fof3d_link"],
          "pairs_nn": kernel_ms["phase_large_nn"] + kernel_ms["phase_large_nn_fallback"],
          "pairs_link": kernel_ms["phase_large_link"]}
    return {k: {"pairs_per_step": v, "kernel_ms_per_step": ms[k],
                "per_s": v / (ms[k] / 1000.0) if ms[k] > 0 else None} for k, v in got.items()}


def small_node_stats(tree, prof_small, steps):
    """The small-node subtree kernels: members of the subtree roots they load
    (nodes of at most SMALL_MAX members whose parent is larger or absent) and
    member-levels they split, per step, against their event time."""
    size = tree["size"].long()
    parent = tree["parent"].long()
    small = size <= SMALL_MAX
    psize = torch.where(parent >= 0, size[parent.clamp(min=0)],
                        torch.full_like(size, SMALL_MAX + 1))
    roots = small & (psize > SMALL_MAX)
    loaded = int(size[roots].sum().item())
    levels = int(size[small].sum().item())
    ms = sum(v[0] for v in prof_small.values()) / steps
    launches = sum(v[1] for v in prof_small.values()) / steps
    gbs = SMALL_BYTES * loaded / (ms / 1000.0) / 1e9 if ms > 0 else 0.0
    return {"members_loaded": loaded, "member_levels": levels, "ms_per_step": ms,
            "launches_per_step": launches, "algorithmic_bytes": SMALL_BYTES * loaded,
            "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS,
            "note": "side streams, overlapped with the main-stream levels"}


def seed_tests(tree):
    """(particle, seed) tests of rs_seed_assign on a tree: every own particle
    of a node with children against every seed (leaf) below that node."""
    level, parent = tree["level"].long(), tree["parent"].long()
    deepest = tree["deepest"].long()
    m = level.numel()
    if m == 0:
        return 0
    childsum = torch.bincount(parent[parent >= 0], minlength=m)
    leafcnt = (childsum == 0).long()
    for lv in range(int(level.max().item()), 0, -1):   # children before parents
        at = torch.nonzero(level == lv).squeeze(1)
        leafcnt.index_add_(0, parent[at], leafcnt[at])
    own = torch.bincount(deepest[deepest >= 0], minlength=m)
    has = childsum > 0
    return int((own[has] * leafcnt[has]).sum().item())


def subbox_cut(arrs, cfg):
    """One process's share of an 8-way decomposition of the workload: the
    cube [gw, gw + L/2)^3 and its ghost shell of width gw = 1.5 ll, selected
    on the device with the sub-box's own fp32 bounds (owned particles first).
    Returns (x, y, z, n_owned, lo, hi, gw)."""
    gw = 1.5 * cfg.link_len
    side = cfg.box / 2.0
    lo32 = torch.full((3,), gw, dtype=torch.float32)
    hi32 = (torch.full((3,), gw, dtype=torch.float64) + side).float()
    gw64 = float(np.float32(gw))
    x, y, z = arrs[0], arrs[1], arrs[2]
    owned = torch.ones_like(x, dtype=torch.bool)
    shell = torch.ones_like(x, dtype=torch.bool)
    for a, c in enumerate((x, y, z)):
        l, h = float(lo32[a]), float(hi32[a])
        owned &= (c >= l) & (c < h)
        c64 = c.double()
        shell &= (c64 >= l - gw64) & (c64 < h + gw64)
    idx = torch.cat([torch.nonzero(owned).squeeze(1), torch.nonzero(shell & ~owned).squeeze(1)])
    sx, sy, sz = (c[idx].contiguous() for c in (x, y, z))
    n_owned = int(owned.sum().item())
    return sx, sy, sz, n_owned, lo32.tolist(), hi32.tolist(), gw


def subbox_row(arrs, cfg, reps=3):
    """rs_fof3d_subbox on one process's share of an 8-way decomposition
    (subbox_cut), timed."""
    sx, sy, sz, n_owned, lo, hi, gw = subbox_cut(arrs, cfg)
    lo32, hi32 = torch.tensor(lo), torch.tensor(hi)
    labels = torch.empty(sx.numel(), dtype=torch.int32, device=sx.device)
    call = lambda: rs.rs_fof3d_subbox(sx, sy, sz, n_owned, lo32.tolist(), hi32.tolist(), gw,
                                      cfg.link_len, labels=labels)
    call()
    rs.rs_profile_enable(False)
    rs.rs_profile_enable(True)
    ms, (_, links) = timed(call, reps)
    tot, launches, units = rs.rs_profile_get("fof3d_link")
    rs.rs_profile_enable(False)
    avg = tot / max(launches, 1)
    per = KERNEL_BYTES["fof3d_link"] * units / max(launches, 1)
    gbs = per / (avg / 1000.0) / 1e9 if avg > 0 else 0.0
    return {"cube": [float(lo32[0]), float(hi32[0])], "owned": n_owned,
            "ghosts": int(sx.numel()) - n_owned, "ghost_links": int(links.shape[0]),
            "ms_per_call": ms, "owned_per_s": n_owned / (ms / 1000.0),
            "roofline": {"bound": "hbm", "kernel": "fof3d_link", "achieved": gbs,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                         "avg_launch_ms": avg, "algorithmic_bytes_per_launch": per}}


def hierarchy_rows(arrs, cfg, tree, reps=3, subbox=True):
    """Halo properties and seed assignment over the last step's hierarchy,
    and the sub-box pass on one eighth of the box."""
    props = rs.rs_halo_props(*arrs, cfg.box, tree)
    halo = rs.rs_seed_assign(*arrs, cfg.box, tree, props)
    torch.cuda.synchronize()
    rs.rs_profile_enable(True)
    ms_p, _ = timed(lambda: rs.rs_halo_props(*arrs, cfg.box, tree, out=props), reps)
    ms_s, _ = timed(lambda: rs.rs_seed_assign(*arrs, cfg.box, tree, props, out=halo), reps)
    tot, launches, units = rs.rs_profile_get("halo_props")
    st, sl, _ = rs.rs_profile_get("seed_assign")
    rs.rs_profile_enable(False)
    avg = tot / max(launches, 1)
    per = PROPS_BYTES * units / max(launches, 1)
    gbs = per / (avg / 1000.0) / 1e9 if avg > 0 else 0.0
    traffic = measured_pmc("halo_props", cfg.name, "hbm_bytes_per_launch")
    tests = seed_tests(tree)
    sk = st / max(sl, 1)
    tflops = SEED_FLOPS * tests / (sk / 1000.0) / 1e12 if sk > 0 else 0.0
    return {
        "halo_props": {"ms_per_call": ms_p, "nodes": int(tree["level"].numel()),
                       "roofline": {"bound": "hbm", "kernel": "halo_props", "achieved": gbs,
                                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
                                    "avg_launch_ms": avg,
                                    "algorithmic_bytes_per_launch": per,
                                    "member_levels": units / max(launches, 1)}},
        "seed_assign": {"ms_per_call": ms_s, "kernel_ms": sk,
                        "assigned": int((halo >= 0).sum().item()),
                        "roofline": {"bound": "alu", "kernel": "seed_assign",
                                     "achieved": tflops, "peak": ALU_PEAK_TFLOPS,
                                     "unit": "TFLOP/s", "frac": tflops / ALU_PEAK_TFLOPS,
                                     "tests_per_call": tests,
                                     "flops_per_test": SEED_FLOPS}},
        **({"subbox": subbox_row(arrs, cfg, reps)} if subbox else {}),
    }


def cpu_baseline(arrs, cfg, target=1100000, workers=None):
    """The oracle (single-threaded C) on one process's sub-box of the same
    workload, as the paper decomposes the box: the owned particles of a cube
    plus a ghost shell of width 1.5 ll, the sub-box 3D FoF, then the 6D
    hierarchy of its groups.  All-core figure: the same sub-box, its 3D FoF
    single-threaded and its groups' 6D hierarchies dealt to one process per
    core (at most 16), largest groups first; throughput counts owned
    particles."""
    from oracle import baseline
    import tempfile
    host = [a.cpu().numpy() for a in arrs]
    side = cfg.box * (target / cfg.n) ** (1.0 / 3.0)
    gw = 1.5 * cfg.link_len
    sub, no, lo, hi = baseline.cut(host, (gw, gw, gw), side, gw)
    del host
    no, nt, t3, t6, lab, rows = baseline.run_one((sub, no, lo, hi, gw, cfg.box, cfg.link_len,
                                                  cfg.min_group, cfg.min_sub, cfg.f))
    progress(f"oracle on one sub-box: {t3:.1f} s 3D + {t6:.1f} s 6D")
    (tp, ml), (ts, npart) = rows["halo_props"], rows["seed_assign"]
    row_rates = {"subbox": {"value": no / t3, "unit": "owned particles/s", "seconds": t3},
                 "halo_props": {"value": ml / tp, "unit": "member-levels/s", "seconds": tp,
                                "member_levels": ml},
                 "seed_assign": {"value": npart / ts, "unit": "particles/s", "seconds": ts}}
    ncpu = os.cpu_count() or 1
    workers = workers or max(1, min(16, ncpu))
    parts = baseline.split_groups(sub, lab, cfg.min_group, workers)
    res, wall = baseline.run_parts(parts, cfg.box, cfg.min_group, cfg.min_sub, cfg.f,
                                   tempfile.gettempdir(), progress)
    slowest = max(r[1] for r in res)
    return {"value": no / (t3 + t6), "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": (f"one process's sub-box of the same workload: the cube "
                       f"[{lo[0]:.3f}, {hi[0]:.3f})^3 Mpc/h, {no} owned particles and "
                       f"{nt - no} ghosts in a {gw:.4g} Mpc/h shell; sub-box 3D FoF "
                       f"{t3:.2f} s + 6D hierarchy {t6:.2f} s, single-threaded"),
            "rows": row_rates,
            "all_core": {"value": no / (t3 + slowest), "unit": "particles/s",
                         "cores": workers, "host_cpus": ncpu, "kind": "oracle",
                         "sample": (f"the same sub-box: 3D FoF {t3:.2f} s single-threaded, "
                                    f"then its groups' 6D hierarchies in {workers} processes "
                                    f"at once (slowest {slowest:.2f} s; {wall:.2f} s wall "
                                    f"with process start-up)")}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c512")
    ap.add_argument("--form", default="learned", choices=["learned", "batched", "plain"])
    ap.add_argument("--no-speedup", action="store_true", help="skip the form comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the halo-property, seed-assignment and sub-box timings")
    ap.add_argument("--no-pairs", action="store_true",
                    help="skip the extra step that counts pair tests")
    ap.add_argument("--no-subbox", action="store_true",
                    help="skip the sub-box timing (its 3D link launches would mix with the "
                         "step's in a profile)")
    ap.add_argument("--probe-copy", type=int, default=0, metavar="MIB",
                    help="after the run, copy a MIB-sized device buffer 3 times (a plain "
                         "copy kernel of known size, for calibrating byte counters)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "MIB"),
                    help="write the per-launch traffic summary from two rocprofv3 --pmc "
                         "counter_collection.csv files (FETCH_SIZE, WRITE_SIZE) of a run "
                         "with --probe-copy MIB, then exit")
    ap.add_argument("--pmc-valu", default=None, metavar="VALU_CSV",
                    help="with --pmc-summary: counter_collection.csv of a run with "
                         "SQ_INSTS_VALU and GRBM_GUI_ACTIVE")
    ap.add_argument("--pmc-command", default="", help="command recorded in the summary")
    args = ap.parse_args()
    if args.pmc_summary:
        fcsv, wcsv, mib = args.pmc_summary
        res = pmc_summary(fcsv, wcsv, int(mib) << 20, args.pmc_command, PMC_SUMMARY,
                          args.pmc_valu)
        print(json.dumps({k: v["hbm_bytes_per_launch"] for k, v in res["kernels"].items()}))
        return 0
    if args.gpus != 1:
        print("bench.py measures one GPU: the method's hot path runs on a single MI355X; "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        return 2
    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        return 2
    rs.load()
    tuning = rs.load_tuning()
    cfg = synth.CONFIGS[args.config]
    model = learn.load_model()
    dev = torch.device("cuda:0")
    arrs = synth.generate(cfg, 0, device=dev)
    torch.cuda.empty_cache()           # the generator's fp64 temporaries
    labels = torch.empty(cfg.n, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        one_step(arrs, cfg, args.form, labels, model)
    torch.cuda.synchronize()

    rs.rs_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tree = one_step(arrs, cfg, args.form, labels, model)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {k: rs.rs_profile_get(k) for k in KERNEL_BYTES}
    # small subtrees (level 0, and the small children of each large-node level)
    # run on side streams beside the large-node levels; their event spans
    # overlap other work, so they are reported, not ranked
    prof_small = {k: rs.rs_profile_get(k)
                  for k in ("phase_small_level0", "phase_small_children")}
    rs.rs_profile_enable(False)

    ms = (t1 - t0) * 1000.0 / args.steps
    value = cfg.n / (ms / 1000.0)
    n_groups = int((tree["level"] == 0).sum().item())
    dom = max(prof, key=lambda k: prof[k][0])
    tot_ms, launches, units = prof[dom]
    avg_ms = tot_ms / max(launches, 1)
    bytes_per_launch = KERNEL_BYTES[dom] * units / max(launches, 1)
    achieved = bytes_per_launch / (avg_ms / 1000.0) / 1e9 if avg_ms > 0 else 0.0
    traffic = measured_pmc(dom, cfg.name, "hbm_bytes_per_launch")
    line = {
        "metric": METRIC, "value": value, "unit": "particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload_description(cfg), "form": args.form,
                   "tuning": tuning["choice"] if tuning else "compiled defaults",
                   "groups": n_groups, "nodes": int(tree["level"].numel()),
                   "levels": tree["n_levels"],
                   "proposals_accepted": tree["n_accepted"],
                   "proposals_fallback": tree["n_fallback"],
                   "groups_per_s": n_groups / (ms / 1000.0),
                   "nodes_per_s": int(tree["level"].numel()) / (ms / 1000.0),
                   "acceptance_rate": (tree["n_accepted"] /
                                       max(1, tree["n_accepted"] + tree["n_fallback"])),
                   "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()}},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "traffic_gbs": (traffic / (avg_ms / 1000.0) / 1e9
                                     if traffic is not None and avg_ms > 0 else None),
                     "valu_busy": measured_pmc(dom, cfg.name, "valu_busy"),
                     "avg_launch_ms": avg_ms, "launches": launches,
                     "algorithmic_bytes_per_launch": bytes_per_launch},
    }
    progress(f"{args.steps} steps at {ms:.1f} ms")
    line["small_node_kernels"] = small_node_stats(tree, prof_small, args.steps)
    if not args.no_pairs:
        line["pair_tests"] = pair_tests(arrs, cfg, args.form, labels, model,
                                        line["config"]["kernel_ms_per_step"])
        progress("pair tests counted")
    if not args.no_rows:
        line["hierarchy_rows"] = hierarchy_rows(arrs, cfg, tree, subbox=not args.no_subbox)
        progress("halo properties and seed assignment timed")
    if args.form == "learned" and not args.no_speedup:
        line["learned_speedup"] = speedups(arrs, cfg, labels, model, ms)
        progress("batched and plain forms timed")
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(arrs, cfg)
        progress("oracle baseline timed")
        if "hierarchy_rows" in line:
            # the oracle's rate on the same sub-box beside each row's GPU rate
            rr = line["hierarchy_rows"]
            gpu = {"halo_props": (rr["halo_props"]["roofline"]["member_levels"] /
                                  (rr["halo_props"]["ms_per_call"] / 1000.0)),
                   "seed_assign": cfg.n / (rr["seed_assign"]["ms_per_call"] / 1000.0)}
            if "subbox" in rr:
                gpu["subbox"] = rr["subbox"]["owned_per_s"]
            for k, v in line["cpu_baseline"]["rows"].items():
                if k in gpu:
                    rr[k]["oracle_1core"] = v
                    rr[k]["gpu_over_oracle"] = gpu[k] / v["value"]
    if args.probe_copy > 0:
        src = torch.ones(args.probe_copy * (1 << 18), dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["probe_copy_bytes"] = src.numel() * 4
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
