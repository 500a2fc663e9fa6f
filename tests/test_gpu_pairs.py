"""Two consecutive fused segments of a chain in one carrier pass (forward:
C_0 to C_2 without storing C_1; reverse: C_1 and its adjoint recomputed in
LDS), through the C ABI, against the oracle on the plan's own tree and
against the plan that runs every segment in a pass of its own.

Tolerances as for the other fused-segment tests: log Z relative error
<= 1e-5, marginals max-abs <= 1e-5; the paired and the unpaired plan of the
same tree agree within 2e-6 (both FP32 on the matrix cores; only the
rounding of the intermediate carrier differs)."""
import numpy as np
import pytest

import oracle
from paper_2405_14060_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T(gpu):
    import paper_2405_14060_amd as T
    T.lib()
    return T


def rel(a, b):
    return abs(a - b) / max(1.0, abs(b))


def variants(P, task):
    return {o["variant"] for o in P.ops(task) if o["form"] == 5}


@pytest.mark.parametrize("rows,cols,card,natural", [(12, 12, 2, False), (9, 9, 3, True), (16, 16, 2, False),
                                                    (14, 14, 2, True)])
def test_segment_pairs_against_oracle(T, rows, cols, card, natural):
    """Grids of several sizes and domain sizes (card 3: local sizes that are
    not powers of two), best and natural elimination orders."""
    net = W.grid_mrf(rows, cols, 3, card=card)
    planner = T.PLANNER_NATURAL if natural else T.PLANNER_BEST
    P = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, planner=planner)
    assert 5 in variants(P, 0) and 6 in variants(P, 1)
    lz, m = P.marginals()
    pairs, _ = P.tree()
    lzo, marg, *_ = oracle.marginals(net, pairs=pairs.astype(np.int64))
    assert rel(lz[0], lzo) <= 1e-5
    err = max(np.abs(a - b).max() for a, b in zip(P.split_marginals(m[0]), marg))
    assert err <= 1e-5, err
    U = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, tree=pairs, pair_segments=False)
    assert 5 not in variants(U, 0) and 6 not in variants(U, 1) and U.info()["n_segments"] > 0
    lzu, mu = U.marginals()
    assert rel(lz[0], lzu[0]) <= 2e-6
    assert np.abs(m[0] - mu[0]).max() <= 2e-6


def test_segment_pairs_factor_marginals(T):
    """Factor marginals T_f Tbar_f / Z (theorem thm:diff): the small
    operands' adjoints come from both segments' partial sums of a pair."""
    net = W.grid_mrf(12, 12, 4)
    P = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, want_factor_grad=True)
    assert 6 in variants(P, 1)
    lz, fm = P.factor_marginals()
    pairs, _ = P.tree()
    lzo, want = oracle.factor_marginals(net, None, pairs=pairs.astype(np.int64))
    assert rel(lz[0], lzo) <= 1e-5
    got = P.split_factors(fm[0])
    worst = max(float(np.abs(got[f] - want[f]).max()) for f in range(net.n_factors))
    assert worst <= 1e-5, worst


def test_segment_pairs_graph_replays(T):
    """Captured and eager runs of a paired plan give the same bits, replay
    after replay."""
    net = W.grid_mrf(16, 16, 5)
    G = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, use_graph=True)
    E = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, use_graph=False, tree=G.tree()[0])
    assert 5 in variants(G, 0)
    lze, me = E.marginals()
    for _ in range(3):
        lzg, mg = G.marginals()
        assert lzg[0] == lze[0]
        assert np.array_equal(mg[0], me[0])


@pytest.mark.parametrize("size,seed", [(16, 5), (20, 0)])
def test_segment_pairs_moving_an_outer_label(T, size, seed):
    """Pairs whose tiles would be half empty take the slowest common outer
    label into one map's rows and columns (the map applied as M (x) I over
    it; its S partial the sum of the diagonal blocks): on the 16x16 grid in
    the first map, on the 20x20 grid in the first and in the second.  log Z,
    marginals and factor marginals (theorem thm:diff, through both maps'
    partials) against the oracle on the plan's own tree, and against the
    plan of the same tree that runs every segment in a pass of its own."""
    net = W.grid_mrf(size, size, seed)
    P = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, want_factor_grad=True)
    info = P.info()
    assert info["n_pairs_moved"] > 0 and info["n_pairs"] > info["n_pairs_moved"]
    lz, m = P.marginals()
    lzf, fm = P.factor_marginals()
    pairs, _ = P.tree()
    lzo, marg, *_ = oracle.marginals(net, pairs=pairs.astype(np.int64))
    assert rel(lz[0], lzo) <= 1e-5 and rel(lzf[0], lzo) <= 1e-5
    err = max(np.abs(a - b).max() for a, b in zip(P.split_marginals(m[0]), marg))
    assert err <= 1e-5, err
    _, want = oracle.factor_marginals(net, None, pairs=pairs.astype(np.int64))
    got = P.split_factors(fm[0])
    worst = max(float(np.abs(got[f] - want[f]).max()) for f in range(net.n_factors))
    assert worst <= 1e-5, worst
    U = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, tree=pairs, pair_segments=False)
    assert U.info()["n_pairs"] == 0
    lzu, mu = U.marginals()
    assert rel(lz[0], lzu[0]) <= 2e-6
    assert np.abs(m[0] - mu[0]).max() <= 2e-6
