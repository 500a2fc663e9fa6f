"""Host-side checks of libtn (no GPU needed): exports, validation, planner."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_2405_14060_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def T():
    import paper_2405_14060_amd as T
    if not os.path.exists(os.path.join(ROOT, "paper_2405_14060_amd", "libtn.so")):
        from paper_2405_14060_amd import build
        build.build()
    T.lib()
    return T


def test_exports_every_declared_symbol(T):
    hdr = open(os.path.join(ROOT, "include", "tn.h")).read()
    names = set(re.findall(r"\b(tn_[a-z_A-Z0-9]+)\s*\(", hdr))
    assert {"tn_load_network", "tn_plan", "tn_logZ", "tn_marginals", "tn_map", "tn_mmap", "tn_sample"} <= names
    L = T.lib()
    for n in sorted(names):
        assert hasattr(L, n), n


def test_load_network_validation(T):
    with pytest.raises(T.TNError):
        T.Network(W.Network(np.array([2, 0], np.int32), [np.array([0], np.int32)], [np.ones(2)], False))
    with pytest.raises(T.TNError):
        T.Network(W.Network(np.array([2], np.int32), [np.array([0], np.int32)], [np.array([1.0, np.nan])], False))
    with pytest.raises(T.TNError):
        T.Network(W.Network(np.array([2], np.int32), [np.array([0], np.int32)], [np.array([1.0, -1.0])], False))
    with pytest.raises(T.TNError):
        T.Network(W.Network(np.array([2], np.int32), [np.array([3], np.int32)], [np.ones(2)], False))


@pytest.mark.parametrize("planner", [0, 1, 2, 3, 4])
def test_planner_tree_is_valid_and_stats_agree(T, planner):
    net = W.random_small_mrf(20, 30, seed=planner, cards=(2, 3))
    pairs, L, info = T.plan_tree_host(T.Network(net), planner=planner, restarts=2)
    lv = oracle.build_leaves(net)
    assert L == len(lv)
    assert pairs.shape == (L - 1, 2)
    used = np.bincount(pairs.ravel(), minlength=2 * L - 1)
    assert np.all(used[:-1] == 1) and used[-1] == 0
    for i, (a, b) in enumerate(pairs):
        assert a < L + i and b < L + i
    st = oracle.tree_stats(lv.labels, pairs, lv.card)
    assert abs(st["sc"] - info["sc"]) < 1e-9
    assert abs(st["tc"] - info["tc"]) < 1e-9


def test_planner_grid20_reaches_sweep_width(T):
    pairs, L, info = T.plan_tree_host(T.Network(W.grid_mrf(20, 20, 0)), restarts=2)
    assert info["sc"] <= 21


def test_planner_slicing_cap(T):
    c = W.config(4, seed=0, small=True)
    pairs, L, info = T.plan_tree_host(T.Network(c["net"]), max_log2_size=6)
    if info["sc"] > 6:
        assert info["n_sliced"] > 0


def test_plan_tree_rejects_bad_tree_on_host(T):
    """Tree validation happens before any device work."""
    from paper_2405_14060_amd._capi import TN_E_INVALID
    net = W.grid_mrf(2, 2, 0)
    N = T.Network(net)
    with pytest.raises(T.TNError) as ei:
        T.Plan(N, tree=np.array([[0, 1]], np.int32))
    assert ei.value.status == TN_E_INVALID


def test_segment_pairs_on_host(T):
    """Consecutive fused segments of a grid's chains run as pairs (one
    carrier pass each) unless asked otherwise: fewer launches, same tree."""
    net = W.grid_mrf(12, 12, 0)
    P = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, host_only=True)
    U = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, host_only=True, pair_segments=False)
    assert np.array_equal(P.tree()[0], U.tree()[0])
    vp = [o["variant"] for o in P.ops(0) + P.ops(1) if o["form"] == 5]
    vu = [o["variant"] for o in U.ops(0) + U.ops(1) if o["form"] == 5]
    assert 5 in vp and 6 in vp and 5 not in vu and 6 not in vu
    # every pair replaces two single-segment passes in each direction
    assert vp.count(5) == vp.count(6) and vu.count(1) == vp.count(1) + 2 * vp.count(5)
    assert P.info()["n_launches_fwd"] < U.info()["n_launches_fwd"]


def test_pairs_moving_an_outer_label_on_host(T):
    """On the 20x20 grid every segment of both fronts is paired: the pairs
    whose tiles would be half empty take a common outer label into one map's
    rows (plan info counts them), which leaves fewer carrier passes than the
    pairs without them would (each such pass then runs two segments)."""
    net = W.grid_mrf(20, 20, 0)
    P = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, host_only=True)
    info = P.info()
    assert info["n_pairs"] > info["n_pairs_moved"] > 0
    # every segment in a pair but one per front (chains of odd length): the
    # forward list holds at most two single-segment passes over a large carrier
    def singles(plan):
        return [o for o in plan.ops(0) if o["form"] == 5 and o["variant"] == 1 and o["x_size"] >= 1 << 16]
    assert len(singles(P)) <= 2
    U = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, host_only=True, pair_segments=False)
    assert U.info()["n_pairs"] == 0 and U.info()["n_pairs_moved"] == 0
    # unpaired, each pair's two segments run alone (the first pair starts on a
    # carrier below 2^16 entries)
    assert len(singles(U)) == len(singles(P)) + 2 * (info["n_pairs"] - 1)


def test_row_batch_form_is_offered(T):
    """The batch-uniform row form is eligible (never the rules' choice) for
    the MMAP slice's batched products with small summed x column blocks."""
    c = W.config(4, 0)
    P = T.Plan(T.Network(c["net"]), semirings=T.SUM_PRODUCT | T.MAX_PLUS, query=c["query"], max_log2_size=28,
               host_only=True, restarts=16)
    ops = P.ops(3)
    elig = [o for o in ops if o["eligible"] & 1024]
    assert elig
    for o in elig:
        assert o["semiring"] == 0 and o["summed"] * o["cols"] <= 128 and o["z_size"] >= 1 << 16
    assert not any(o["form"] == 1 and o["variant"] == 1 for o in ops)  # rules: not chosen


def test_max_plus_pairs_on_host(T):
    """The 20x20 grid's max-plus chain steps over >= 2^12 outputs run two or
    three per pass: fewer launches than with every contraction alone; the
    plan's contraction list (and so its tree) is unchanged."""
    net = W.grid_mrf(20, 20, 0)
    P = T.Plan(T.Network(net), semirings=T.MAX_PLUS, host_only=True)
    U = T.Plan(T.Network(net), semirings=T.MAX_PLUS, host_only=True, fuse=False)
    assert np.array_equal(P.tree()[0], U.tree()[0])
    assert len(P.ops(2)) == len(U.ops(2))
    assert P.info()["n_launches_max"] < 0.6 * U.info()["n_launches_max"]
    small = W.grid_mrf(10, 10, 0)  # below 2^12 outputs: nothing paired
    assert (T.Plan(T.Network(small), semirings=T.MAX_PLUS, host_only=True).info()["n_launches_max"] ==
            T.Plan(T.Network(small), semirings=T.MAX_PLUS, host_only=True, fuse=False).info()["n_launches_max"])


def test_mmap_sum_phase_fuses_chains(T):
    """An MMAP plan's sum phase runs forward only, so its chains of small
    absorptions fuse into segments like the main tree's forward pass (and
    not with no_fuse)."""
    net = W.grid_mrf(14, 14, 0)
    q = [0, 13, 100, 195]
    kw = dict(semirings=T.SUM_PRODUCT | T.MAX_PLUS, query=q, host_only=True, planner=T.PLANNER_NATURAL)
    P = T.Plan(T.Network(net), **kw)
    U = T.Plan(T.Network(net), fuse=False, **kw)
    assert any(o["form"] == 5 for o in P.ops(3))
    assert not any(o["form"] == 5 for o in U.ops(3))
    assert len(P.ops(3)) < len(U.ops(3))
