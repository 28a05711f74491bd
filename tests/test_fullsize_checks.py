"""The full-size checks (tests/fullsize_checks.py) on the oracle's own result
for a small workload: every check passes, and a planted error in any part of
the tree or the labels is caught."""
import numpy as np
import pytest

import oracle
from paper_2412_18629_amd import synth

from fullsize_checks import cell_lists_numpy, check_all


def _oracle_result(cfg, seed):
    h = [a.numpy() for a in synth.generate(cfg, seed)]
    lab = oracle.fof3d(*h[:3], cfg.box, cfg.link_len)
    ref = oracle.phase_fof(*h, cfg.box, lab, cfg.min_group, cfg.min_sub, cfg.f)
    order = np.argsort(lab, kind="stable")
    cperm, cstart, nc, side = cell_lists_numpy(*h[:3], cfg.box)
    props = oracle.halo_props(*h, cfg.box, ref["parent"], ref["min_index"], ref["deepest"])
    halo = oracle.seed_assign(*h, cfg.box, ref["parent"], ref["deepest"], ref["a"], ref["c"],
                              props)
    return dict(host=h, labels=lab, order=order, sorted_labels=lab[order], cperm=cperm,
                cstart=cstart, nc=nc, side=side, tree=ref, props=props, halo=halo)


@pytest.fixture(scope="module")
def small():
    cfg = synth.scaled(synth.CONFIGS["c32"], 60000)
    return cfg, _oracle_result(cfg, 21)


def test_checks_pass_on_oracle_result(small):
    cfg, R = small
    n3, n6 = check_all(R, cfg, n_sample=24, subtree_max=10 ** 9, log=lambda s: None)
    assert n3 == 24 and n6 == 24


def _copy(R):
    S = dict(R)
    S["tree"] = {k: v.copy() for k, v in R["tree"].items()}
    S["labels"] = R["labels"].copy()
    S["props"] = R["props"].copy()
    S["halo"] = R["halo"].copy()
    return S


@pytest.mark.parametrize("what", ["l2", "a", "deepest", "parent", "label_split", "props",
                                  "seed"])
def test_checks_catch_planted_errors(small, what):
    cfg, R = small
    S = _copy(R)
    T = S["tree"]
    if what == "l2":                     # one deeper node's linking length
        v = int(np.flatnonzero(T["level"] == 1)[0])
        T["l2"][v] = np.nextafter(T["l2"][v], np.float32(np.inf))
    elif what == "a":                    # one level-0 metric factor
        T["a"][0] = np.nextafter(T["a"][0], np.float32(0))
    elif what == "deepest":              # a particle assigned one level too shallow
        i = int(np.flatnonzero(T["level"][np.maximum(T["deepest"], 0)] >= 1)[0])
        T["deepest"][i] = T["parent"][T["deepest"][i]]
    elif what == "parent":               # a node re-parented to another level-0 node
        v = int(np.flatnonzero(T["level"] == 1)[0])
        l0 = np.flatnonzero(T["level"] == 0)
        T["parent"][v] = l0[l0 != T["parent"][v]][0]
    elif what == "props":                # every node's xy tensor element, one ulp off
        S["props"][9, :] = np.nextafter(S["props"][9, :], np.float32(np.inf))
    elif what == "seed":                 # particles of a node with children all sent
        kids = np.zeros(T["level"].size, np.int64)   # to one seed
        np.add.at(kids, T["parent"][T["parent"] >= 0], 1)
        own = np.flatnonzero((T["deepest"] >= 0) & (kids[np.maximum(T["deepest"], 0)] > 1))
        S["halo"][own] = S["halo"][own[0]]
    else:                                # a whole group relabelled as its own split
        big = np.bincount(S["labels"]).argmax()
        mem = np.flatnonzero(S["labels"] == big)
        S["labels"][mem[len(mem) // 2:]] = mem[len(mem) // 2]
    with pytest.raises(AssertionError):
        check_all(S, cfg, n_sample=64, subtree_max=10 ** 9, log=lambda s: None)
