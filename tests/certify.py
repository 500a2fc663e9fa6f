"""MMAP certificate shared by the GPU tests (test infrastructure)."""
import numpy as np

import oracle


def certify_mmap(net, q, x, val, tol=1e-4, evidence=None):
    """Certify an MMAP answer x (over the sorted query set q) with value val.

    The oracle's log p(Q = x, e) must equal val (FP32 bound of the sum phase)
    and lie within tol of the best entry of the oracle's query table, so an
    answer that differs from the oracle's argmax passes only as a certified
    near-tie.  Returns True for a near-tie (answer differs, gap <= tol)."""
    q = np.asarray(q)
    x = np.asarray(x)
    ev = -np.ones(net.n_vars, np.int32) if evidence is None else np.asarray(evidence, np.int32).copy()
    ev[q] = x
    lp = oracle.log_z(net, ev, mode="slice")
    assert abs(val - lp) <= 1e-5 * max(1.0, abs(lp)), (val, lp)
    _, table = oracle.query_table(net, q, evidence)
    best = float(table.max())
    assert lp >= best - tol, (lp, best)
    shape = tuple(int(net.card[v]) for v in q)
    ox = np.asarray(np.unravel_index(int(np.argmax(table)), shape))
    return not np.array_equal(ox, x)
