"""The launch-shape table: every allowed value of every knob gives the same
tree, bit for bit, as the compiled defaults (only speed may change); a
table written by the autotuner only names allowed values."""
import json
import os

import pytest
import torch

import paper_2412_18629_amd as rs
from paper_2412_18629_amd import autotune, learn, synth

pytestmark = pytest.mark.gpu
FIELDS = ("level", "min_index", "parent", "size", "l2", "a", "c", "sx2", "sv2", "wide", "deepest")


@pytest.fixture(scope="module")
def work():
    defaults = {k: v[0] for k, v in rs.tune_knobs().items()}
    cfg = synth.scaled(synth.CONFIGS["c32"], 400000)
    arrs = [a.cuda() for a in synth.generate(cfg, 41)]
    lab, _ = rs.rs_fof3d(*arrs[:3], cfg.box, cfg.link_len)
    yield cfg, arrs, lab, defaults
    for k, v in defaults.items():
        rs.tune_set(k, v)


def _run(cfg, arrs, lab):
    return rs.rs_phase_fof_batch(*arrs, cfg.box, lab, flags=rs.RS_LEARNED,
                                 model=learn.load_model())


def test_every_knob_value_gives_the_same_tree(work):
    cfg, arrs, lab, defaults = work
    ref = _run(cfg, arrs, lab)
    assert int((ref["size"] > 256).sum()) > 10
    for knob, (_, allowed) in rs.tune_knobs().items():
        for value in allowed:
            rs.tune_set(knob, value)
            got = _run(cfg, arrs, lab)
            for k in FIELDS:
                assert torch.equal(ref[k], got[k]), (knob, value, k)
        rs.tune_set(knob, defaults[knob])


def test_shipped_table_names_allowed_values():
    if not os.path.exists(autotune.DEFAULT_TABLE):
        pytest.skip("no tuning table shipped")
    with open(autotune.DEFAULT_TABLE) as f:
        table = json.load(f)
    knobs = rs.tune_knobs()
    for k, v in table["choice"].items():
        assert v in knobs[k][1], (k, v)
