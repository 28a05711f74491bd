"""Host-side logic of bench.py (CPU only): several GPUs are refused, the PMC
summary calibrates the byte counters against the plain copy kernel and
computes the vector-ALU occupancy, and a traffic figure is used only while
its kernel's sources are unchanged."""
import csv
import json
import subprocess
import sys

import pytest

import bench

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(r)
    return str(path)


def _row(d, name, counter, value):
    return {"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter,
            "Counter_Value": value}


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_pmc_summary_calibration_and_occupancy(tmp_path):
    mib = 64
    kib = mib * 1024.0
    link = bench.KERNEL_SYMBOL["phase_large_link"][0] + "true>(rs::TArgs, int, int)"
    # the copy kernel moves `mib` MiB: its FETCH_SIZE reads half of that
    # (scale 2), its WRITE_SIZE all of it (scale 1); a counter is summed over
    # the rows (instances) of one dispatch
    fetch = [_row(d, "__amd_rocclr_copyBuffer", "FETCH_SIZE", kib / 4) for d in (1, 1, 2, 2, 3, 3)]
    write = [_row(d, "__amd_rocclr_copyBuffer", "WRITE_SIZE", kib) for d in (1, 2, 3)]
    fetch += [_row(10, link, "FETCH_SIZE", 600.0), _row(10, link, "FETCH_SIZE", 400.0),
              _row(11, link, "FETCH_SIZE", 3000.0)]
    write += [_row(10, link, "WRITE_SIZE", 10.0), _row(11, link, "WRITE_SIZE", 30.0)]
    valu = [_row(10, link, "SQ_INSTS_VALU", 5.0e6), _row(11, link, "SQ_INSTS_VALU", 3.0e6),
            _row(10, link, "GRBM_GUI_ACTIVE", 8.0e4), _row(11, link, "GRBM_GUI_ACTIVE", 8.0e4)]
    out = tmp_path / "summary.json"
    res = bench.pmc_summary(_write(tmp_path / "f.csv", fetch), _write(tmp_path / "w.csv", write),
                            mib << 20, "cmd", str(out), _write(tmp_path / "v.csv", valu))
    assert res["calibration"]["fetch_scale"] == 2.0
    assert res["calibration"]["write_scale"] == 1.0
    k = res["kernels"]["phase_large_link"]
    assert k["launches"] == 2
    # per launch (fetch x 2 + write x 1) KiB, averaged over the launches
    assert k["hbm_bytes_per_launch"] == ((1000 * 2 + 10) + (3000 * 2 + 30)) / 2 * 1024.0
    # 4 cycles per VALU instruction over 1024 SIMDs x kernel cycles (summed over 8 XCDs)
    assert k["valu_busy"] == pytest.approx(8.0e6 * 4 / (1.6e5 / 8 * 1024))
    assert json.loads(out.read_text())["kernels"]["phase_large_link"]["launches"] == 2


def test_traffic_only_while_sources_unchanged(tmp_path, monkeypatch):
    path = tmp_path / "summary.json"
    entry = {"hbm_bytes_per_launch": 123.0,
             "sources_sha256": bench.source_digest("phase_large_link")}
    path.write_text(json.dumps({"workload": "c512", "kernels": {"phase_large_link": entry}}))
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(path))
    assert bench.measured_pmc("phase_large_link", "c512", "hbm_bytes_per_launch") == 123.0
    assert bench.measured_pmc("phase_large_link", "c256", "hbm_bytes_per_launch") is None
    assert bench.measured_pmc("phase_large_nn", "c512", "hbm_bytes_per_launch") is None
    entry["sources_sha256"] = "0" * 64
    path.write_text(json.dumps({"workload": "c512", "kernels": {"phase_large_link": entry}}))
    assert bench.measured_pmc("phase_large_link", "c512", "hbm_bytes_per_launch") is None


def test_nn_refinement_dispatches_kept_apart(tmp_path):
    # at each level the learned form runs the NN bracket pass, the acceptance
    # of the brackets, then (when some were rejected) the refinement pass with
    # the same kernel; only the bracket passes count as phase_large_nn
    nn = bench.KERNEL_SYMBOL["phase_large_nn"][0] + "true>(rs::TArgs, int, int, float*)"
    seq = [(1, "rs::k_lbracket(int, float const*, rs::LParam*)", 0.0), (2, nn, 900.0),
           (3, "rs::k_lcount(...)", 0.0), (4, "rs::k_laccept(int, int const*, rs::LParam*, int*)", 0.0),
           (5, "__amd_rocclr_copyBuffer", 0.0), (6, nn, 20.0),
           (7, "rs::k_lhist(...)", 0.0), (8, "rs::k_lbracket(int, float const*, rs::LParam*)", 0.0),
           (9, nn, 300.0), (10, "rs::k_laccept(int, int const*, rs::LParam*, int*)", 0.0)]
    rows = {d: (n, v) for d, n, v in seq}
    assert bench._kernel_values(rows, "phase_large_nn") == [900.0, 300.0]
    # the batched form has no brackets: every NN dispatch is the exact pass
    rows = {1: (nn, 5.0), 2: ("rs::k_lhist(...)", 0.0), 3: (nn, 7.0)}
    assert bench._kernel_values(rows, "phase_large_nn") == [5.0, 7.0]


def test_workload_description_names_the_cube():
    from paper_2412_18629_amd import synth
    assert "(512^3)" in bench.workload_description(synth.CONFIGS["c512"])
    assert "(1024^3)" in bench.workload_description(synth.CONFIGS["c1024"])
    odd = synth.scaled(synth.CONFIGS["c32"], 1000001)
    assert "(1000001)" in bench.workload_description(odd)


def test_valu_issue_density():
    # every SIMD issuing a 4-cycle instruction each 4 cycles reads 1
    cycles = 1.0e6
    full = bench.N_SIMD * cycles / bench.VALU_CYCLES
    assert bench.valu_busy(full, cycles * bench.N_XCD) == pytest.approx(1.0)
    assert bench.valu_busy(full / 4, cycles * bench.N_XCD) == pytest.approx(0.25)
    assert bench.valu_busy(0, 1.0) is None


def test_small_node_stats_count_subtree_roots():
    import torch
    # node sizes: a large level-0 node (3000) with a small child (500, a
    # subtree root) that has a child (100, inside the subtree); a small
    # level-0 node (40, a root)
    tree = {"size": torch.tensor([3000, 40, 500, 100]), "parent": torch.tensor([-1, -1, 0, 2])}
    st = bench.small_node_stats(tree, {"a": (10.0, 2, 0.0), "b": (10.0, 1, 0.0)}, steps=2)
    assert st["members_loaded"] == 540 and st["member_levels"] == 640
    assert st["ms_per_step"] == 10.0 and st["launches_per_step"] == 1.5
    assert st["achieved_gbs"] == pytest.approx(32.0 * 540 / 0.01 / 1e9)


def test_seed_tests_counts_pairs_of_own_particles_and_seeds_below():
    # the oracle's hierarchy of a small workload: every particle whose
    # deepest node has children is tested against each leaf below that node
    import numpy as np
    import torch

    import oracle
    from paper_2412_18629_amd import synth
    cfg = synth.scaled(synth.CONFIGS["c32"], 6000)
    h = [a.numpy() for a in synth.generate(cfg, 3)]
    lab = oracle.fof3d(*h[:3], cfg.box, cfg.link_len)
    t = oracle.phase_fof(*h, cfg.box, lab)
    parent, deepest = t["parent"], t["deepest"]
    m = parent.size
    children = [[] for _ in range(m)]
    for r in range(m):
        if parent[r] >= 0:
            children[parent[r]].append(r)

    def leaves(r):
        return 1 if not children[r] else sum(leaves(c) for c in children[r])

    want = sum(leaves(d) for d in deepest if d >= 0 and children[d])
    assert want > 0
    tree = {k: torch.from_numpy(np.asarray(t[k])) for k in ("level", "parent", "deepest")}
    assert bench.seed_tests(tree) == want
