"""The batch-uniform row form (form 1, variant 1) through the C ABI, against
the oracle.

The rows of such a contraction split into batch assignments (labels that Y
holds too) and the rest; a wavefront takes 64 of the latter for one batch
assignment, reads that assignment's summed x columns block of Y once and
keeps its row of X and of Z in registers.  The form is offered to the
autotuner only, so here every contraction that admits it is forced into it
through a decision file (tune_save / tune_load); the process-wide decisions
are cleared afterwards.

Tolerances as for the other FP32 paths: log Z relative error and MMAP
value <= 1e-5, marginals max-abs <= 1e-5; the MMAP answer is certified by
the oracle's log p(Q = answer) (sec. mmap)."""
import warnings

import numpy as np
import pytest

import oracle
from certify import certify_mmap
from paper_2405_14060_amd import workloads as W

pytestmark = pytest.mark.gpu

ROW_BATCH = 1024  # eligible-forms bit of the batch-uniform row form
KEY_FORMS = 15    # position of the eligible forms in a decision's key


@pytest.fixture(scope="module")
def T(gpu):
    import paper_2405_14060_amd as T
    T.lib()
    return T


def rel(a, b):
    return abs(a - b) / max(1.0, abs(b))


def force_row_batch_form(T, path, make_plan):
    """Record the autotuner's decisions for the plans make_plan builds, then
    rewrite those of shapes that admit the batch-uniform row form to take
    it, and load them in place of the recorded ones."""
    T.tune_clear()
    make_plan()
    T.tune_save(path)
    out = []
    n_forced = 0
    for line in open(path):
        parts = line.split()
        n = int(parts[1])
        if int(parts[2 + KEY_FORMS]) & ROW_BATCH:
            parts[2 + n:] = ["1", "1", "1"]
            n_forced += 1
        out.append(" ".join(parts))
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    T.tune_clear()
    T.tune_load(path)
    return n_forced


def row_batch_ops(P, task):
    return [o for o in P.ops(task) if o["form"] == 1 and o["variant"] == 1]


def test_row_batch_form_mmap(T, tmp_path):
    """MMAP on a 100-variable regular graph (10 query variables): the sum
    phase's contractions that admit the form run in it."""
    net = W.random_regular3(100, seed=0, n_query=10)
    q = net.meta["query"]
    try:
        n = force_row_batch_form(T, str(tmp_path / "d.txt"),
                                 lambda: T.Plan(T.Network(net), query=q, autotune=True))
        assert n > 0
        P = T.Plan(T.Network(net), query=q, autotune=True)
        assert row_batch_ops(P, 3)
        val, x = P.mmap()
    finally:
        T.tune_clear()
    ov, ox, _ = oracle.mmap(net, q)
    assert abs(val - ov) <= 1e-5 * max(1, abs(ov))
    if certify_mmap(net, q, x, val):
        warnings.warn("certified MMAP near-tie")
    R = T.Plan(T.Network(net), query=q)  # the rules' forms
    assert not row_batch_ops(R, 3)
    val_r, _ = R.mmap()
    assert abs(val - val_r) <= 1e-5 * max(1, abs(val_r))


@pytest.mark.parametrize("seed", [1, 2])
def test_row_batch_form_marginals(T, tmp_path, seed):
    """log Z and all marginals of 120-variable regular graphs whose forward
    pass holds contractions that admit the form (summed sets of one and two
    entries, 8 and 16 columns)."""
    net = W.random_regular3(120, seed=seed, n_query=10)
    try:
        n = force_row_batch_form(T, str(tmp_path / "d.txt"),
                                 lambda: T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, autotune=True))
        assert n > 0
        P = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, autotune=True)
        assert row_batch_ops(P, 0)
        lz, m = P.marginals()
    finally:
        T.tune_clear()
    pairs, _ = P.tree()
    lzo, marg, *_ = oracle.marginals(net, pairs=pairs.astype(np.int64))
    assert rel(lz[0], lzo) <= 1e-5
    err = max(np.abs(a - b).max() for a, b in zip(P.split_marginals(m[0]), marg))
    assert err <= 1e-5, err
