"""Batched sliced evidence: evidence sets that share their observed
variables run as one batch on one tree over the sliced network (the
observed labels are gone, so the tree is smaller than the indicator
network's), every factor touching an observed variable sliced per instance.
Against the oracle per instance and against the one-instance-at-a-time
sliced plan."""
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


@pytest.mark.parametrize("layout", ["interleaved", "instance_major"])
def test_batched_sliced_marginals(T, layout):
    bn = W.random_bn(120, seed=21)
    B = 70
    obs, ev = W.bn_evidence_shared(bn, B, seed=22, frac=0.15)
    lay = dict(interleaved=T.LAYOUT_INTERLEAVED, instance_major=T.LAYOUT_INSTANCE_MAJOR)[layout]
    P = T.Plan(T.Network(bn), semirings=T.SUM_PRODUCT, evidence_mode=T.EVIDENCE_SLICED, observed=obs,
               max_batch=B, batch_layout=lay)
    info = P.info()
    assert info["batch_stride"] == (128 if layout == "interleaved" else 0)
    Q = T.Plan(T.Network(bn), semirings=T.SUM_PRODUCT, evidence_mode=T.EVIDENCE_INDICATOR, max_batch=B,
               batch_layout=lay)
    assert info["tc"] < Q.info()["tc"]  # observed labels sliced out of the tree
    lz, m = P.marginals(ev, batch=B)
    for b in (0, 1, 63, 64, B - 1):
        want_lz, want_m, *_ = oracle.marginals(bn, ev[b])
        assert rel(lz[b], want_lz) <= 1e-5, b
        got = P.split_marginals(m[b])
        assert max(np.abs(x - y).max() for x, y in zip(got, want_m)) <= 1e-5, b
    S = T.Plan(T.Network(bn), semirings=T.SUM_PRODUCT, evidence_mode=T.EVIDENCE_SLICED, observed=obs)
    lz1 = S.log_z(ev, batch=B)
    assert np.abs(lz - lz1).max() <= 1e-5 * max(1.0, np.abs(lz1).max())
    # fewer instances than max_batch: the rows past the batch repeat the first
    lz3 = P.log_z(ev[:3], batch=3)
    assert np.allclose(lz3, lz[:3], rtol=0, atol=1e-9)


def test_batched_sliced_map_and_factor_marginals(T):
    bn = W.random_bn(100, seed=23)
    B = 20
    obs, ev = W.bn_evidence_shared(bn, B, seed=24, frac=0.2)
    Pm = T.Plan(T.Network(bn), semirings=T.MAX_PLUS, evidence_mode=T.EVIDENCE_SLICED, observed=obs, max_batch=B)
    lp, x = Pm.map(ev, batch=B)
    pairs, _ = Pm.tree()
    for b in (0, B // 2, B - 1):
        v32, x32 = oracle.map_assignment(bn, ev[b], pairs=pairs.astype(np.int64), fp32=True)
        assert np.array_equal(x[b], x32), b
        assert np.float32(lp[b]) == np.float32(v32), b
    Pf = T.Plan(T.Network(bn), semirings=T.SUM_PRODUCT, evidence_mode=T.EVIDENCE_SLICED, observed=obs, max_batch=B,
                want_factor_grad=True, joint_sets=[[0, 1], [int(obs[0]), 5]])
    lz, fm = Pf.factor_marginals(ev, batch=B)
    _, jm = Pf.joint_marginals(ev, batch=B)
    for b in (0, B - 1):
        lzo, want = oracle.factor_marginals(bn, ev[b])
        assert rel(lz[b], lzo) <= 1e-5
        got = Pf.split_factors(fm[b])
        for f in range(bn.n_factors):
            assert np.abs(got[f] - want[f]).max() <= 1e-5, (b, f)
        _, jw = oracle.joint_marginals(bn, [[0, 1], [int(obs[0]), 5]], ev[b])
        for g, w in zip(jm[b], jw):
            assert np.abs(g - w).max() <= 1e-5, b
    with pytest.raises(T.TNError):
        Pf.sample(10, seed=1, evidence=ev[0])
