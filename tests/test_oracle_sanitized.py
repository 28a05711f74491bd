"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only) runs its 3D, sub-box, 6D, property and seed paths without a
report (CPU only, in a child process that preloads the sanitizer runtime)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
import numpy as np
sys.path.insert(0, %(root)r)
import oracle
from paper_2412_18629_amd import synth
cfg = synth.scaled(synth.CONFIGS["c32"], 12000)
h = [a.numpy() for a in synth.generate(cfg, 1)]
lab = oracle.fof3d(*h[:3], cfg.box, cfg.link_len)
t = oracle.phase_fof(*h, cfg.box, lab, brute_max=8)
P = oracle.halo_props(*h, cfg.box, t["parent"], t["min_index"], t["deepest"])
s = oracle.seed_assign(*h, cfg.box, t["parent"], t["deepest"], t["a"], t["c"], P)
lo = np.array([2, 2, 2], np.float32); hi = np.array([9, 9, 9], np.float32)
pos = np.stack(h[:3], 1)
own = np.all((pos >= lo) & (pos < hi), 1)
gh = np.all((pos >= lo - 0.4) & (pos < hi + 0.4), 1) & ~own
sub = np.concatenate([pos[own], pos[gh]])
oracle.fof3d_subbox(sub[:, 0], sub[:, 1], sub[:, 2], int(own.sum()), lo, hi, 0.4,
                    cfg.link_len)
print("sanitized run ok", len(t["level"]))
"""


@pytest.mark.slow
def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not asan or not os.path.exists(asan):
        pytest.skip("no libasan")
    lib = str(tmp_path / "liboracle_san.so")
    src = os.path.join(ROOT, "oracle", "fof_oracle.c")
    subprocess.run([gcc, "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                    "-fno-fast-math", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", src, "-o", lib,
                    "-lm"], check=True)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0", RS_ORACLE_LIB=lib,
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-c", SCRIPT % {"root": ROOT}], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized run ok" in r.stdout
    assert "runtime error" not in r.stderr
