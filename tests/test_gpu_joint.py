"""Joint marginals of variable sets and factor marginals through the C ABI
(tn_joint_marginals, tn_factor_marginals) against the oracle.

Joint marginals: the adjoint of a unity tensor over each set (the MAR
section's unity tensors over several variables).  Factor marginals:
T_f Tbar_f / Z from the factors' adjoints (theorem thm:diff).  Tolerance
1e-5 max-abs (FP32 storage, FP64 normalisation).
"""
import numpy as np
import pytest

import oracle
from paper_2405_14060_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def T(gpu):
    import paper_2405_14060_amd as T
    T.lib()
    return T


def rel(a, b):
    return abs(a - b) / max(1.0, abs(b))


def some_sets(net, seed):
    rng = np.random.default_rng(seed)
    n = net.n_vars
    sets = [[int(rng.integers(n))], [0, n - 1]]
    for k in (2, 3):
        sets.append([int(v) for v in rng.choice(n, k, replace=False)])
    sets.append([int(v) for v in net.scopes[1]])
    return sets


@pytest.mark.parametrize("seed", range(3))
def test_joint_marginals_no_evidence(T, seed):
    net = W.random_small_mrf(12, 18, seed=seed, cards=(2, 3, 4))
    sets = some_sets(net, seed)
    P = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, joint_sets=sets)
    lz, got = P.joint_marginals()
    lzo, want = oracle.joint_marginals(net, sets)
    assert rel(lz[0], lzo) <= 1e-5
    for g, w in zip(got[0], want):
        assert g.shape == w.shape and np.abs(g - w).max() <= TOL
    # the single-variable marginals of the same plan are unchanged by the sets
    _, m = P.marginals()
    _, marg, *_ = oracle.marginals(net)
    assert max(np.abs(a - b).max() for a, b in zip(P.split_marginals(m[0]), marg)) <= TOL


def test_joint_marginals_sliced_evidence_batch(T):
    """Fixed observed set, two instances in one call; a set holding an
    observed variable (one-hot along it) and a set of observed variables only
    (no unity tensor: a one-hot table)."""
    bn = W.random_bn(60, seed=3)
    obs, ev = W.bn_evidence(bn, seed=4, frac=0.15)
    free = [int(v) for v in np.nonzero(ev < 0)[0]]
    sets = [[free[0], free[5]], [int(obs[0]), free[1], free[2]], [int(obs[1]), int(obs[2])], [free[3]]]
    P = T.Plan(T.Network(bn), semirings=T.SUM_PRODUCT, evidence_mode=T.EVIDENCE_SLICED, observed=obs,
               joint_sets=sets)
    ev2 = np.stack([ev, ev])
    ev2[1, obs[0]] = (ev2[1, obs[0]] + 1) % bn.card[obs[0]]
    lz, got = P.joint_marginals(ev2, batch=2)
    for b in range(2):
        lzo, want = oracle.joint_marginals(bn, sets, ev2[b])
        assert rel(lz[b], lzo) <= 1e-5, b
        for g, w in zip(got[b], want):
            assert g.shape == w.shape and np.abs(g - w).max() <= TOL, (b, g, w)


@pytest.mark.parametrize("layout", ["interleaved", "instance_major"])
def test_joint_marginals_batched_indicators(T, layout):
    bn = W.random_bn(80, seed=6)
    B = 70
    ev = W.bn_evidence_batch(bn, B, seed=9)
    sets = some_sets(bn, 2)
    lay = dict(interleaved=T.LAYOUT_INTERLEAVED, instance_major=T.LAYOUT_INSTANCE_MAJOR)[layout]
    P = T.Plan(T.Network(bn), semirings=T.SUM_PRODUCT, evidence_mode=T.EVIDENCE_INDICATOR, max_batch=B,
               batch_layout=lay, joint_sets=sets)
    lz, got = P.joint_marginals(ev, batch=B)
    for b in (0, 1, 63, 64, B - 1):
        lzo, want = oracle.joint_marginals(bn, sets, ev[b], mode="indicator")
        assert rel(lz[b], lzo) <= 1e-5, b
        for g, w in zip(got[b], want):
            assert np.abs(g - w).max() <= TOL, b


def test_joint_marginals_through_fused_segments(T):
    """A 12x12 grid (its tree holds fused chain segments) with pair sets
    along a row, across rows and far apart; against the oracle on the plan's
    own tree."""
    net = W.grid_mrf(12, 12, 5)
    sets = [[0, 1], [30, 42], [5, 140], [70, 71, 83]]
    P = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, joint_sets=sets, planner=T.PLANNER_NATURAL)
    assert P.info()["n_segments"] > 0
    lz, got = P.joint_marginals()
    pairs, _ = P.tree()
    lzo, want = oracle.joint_marginals(net, sets, pairs=pairs.astype(np.int64))
    assert rel(lz[0], lzo) <= 1e-5
    for g, w in zip(got[0], want):
        assert np.abs(g - w).max() <= TOL


@pytest.mark.parametrize("case", ["none", "sliced", "indicator", "grid"])
def test_factor_marginals_against_oracle(T, case):
    if case == "none":
        net = W.random_small_mrf(12, 18, seed=7, cards=(2, 3, 4))
        P = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, want_factor_grad=True)
        lz, fm = P.factor_marginals()
        runs = [(None, "slice", 0, None)]
    elif case == "sliced":
        net = W.random_bn(60, seed=8)
        obs, ev = W.bn_evidence(net, seed=9, frac=0.2)
        P = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, evidence_mode=T.EVIDENCE_SLICED, observed=obs,
                   want_factor_grad=True)
        ev2 = np.stack([ev, ev])
        ev2[1, obs[0]] = (ev2[1, obs[0]] + 1) % net.card[obs[0]]
        lz, fm = P.factor_marginals(ev2, batch=2)
        runs = [(ev2[0], "slice", 0, None), (ev2[1], "slice", 1, None)]
    elif case == "indicator":
        net = W.random_bn(60, seed=10)
        B = 5
        ev = W.bn_evidence_batch(net, B, seed=11)
        P = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, evidence_mode=T.EVIDENCE_INDICATOR, max_batch=B,
                   want_factor_grad=True, batch_layout=T.LAYOUT_INSTANCE_MAJOR)
        lz, fm = P.factor_marginals(ev, batch=B)
        runs = [(ev[b], "indicator", b, None) for b in (0, B - 1)]
    else:
        net = W.grid_mrf(12, 12, 6)
        P = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, want_factor_grad=True)
        assert P.info()["n_segments"] > 0
        lz, fm = P.factor_marginals()
        pairs, _ = P.tree()
        runs = [(None, "slice", 0, pairs.astype(np.int64))]
    for ev_b, mode, b, pairs in runs:
        lzo, want = oracle.factor_marginals(net, ev_b, mode=mode, pairs=pairs)
        assert rel(lz[b], lzo) <= 1e-5, b
        got = P.split_factors(fm[b])
        for f in range(net.n_factors):
            assert np.abs(got[f] - want[f]).max() <= TOL, (b, f)
            assert abs(got[f].sum() - 1.0) <= 1e-6


def test_joint_and_factor_marginals_errors(T):
    net = W.random_small_mrf(8, 10, seed=1)
    P = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT)
    with pytest.raises(T.TNError):
        P.joint_marginals()
    with pytest.raises(T.TNError):
        P.factor_marginals()
    with pytest.raises(T.TNError):
        T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, joint_sets=[[0, 0]])
    with pytest.raises(T.TNError):
        T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, joint_sets=[[0, net.n_vars]])
