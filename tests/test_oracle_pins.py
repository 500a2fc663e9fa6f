"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each check pins the oracle to something other than itself: closed forms,
brute-force enumeration of the plain definitions, the paper's worked example,
published known-answer vectors, invariants (theorem thm:diff, the unity-vector
identity, normalisation), and textbook dynamic programming.  A dropped term,
a wrong index or a transposed operand anywhere in the oracle makes at least
one of them fail.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import oracle.brute as bf
from paper_2405_14060_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

def test_open_chain_closed_form_long():
    """Zero-field Ising chain: Z = 2 prod_i 2cosh(J_i); 10^4 variables
    exercise the power-of-two rescaling (log Z ~ 10^4 >> FP64 range)."""
    rng = np.random.default_rng(1)
    J = rng.normal(0, 1, 9999)
    net = W.chain_mrf(J)
    want = math.log(2) + float(np.sum(np.log(2 * np.cosh(J))))
    got = oracle.log_z(net)
    assert abs(got - want) <= 1e-10 * abs(want)


def test_open_chain_brute_force_matches_closed_form():
    rng = np.random.default_rng(2)
    J = rng.normal(0, 1, 11)
    net = W.chain_mrf(J)
    want = math.log(2) + float(np.sum(np.log(2 * np.cosh(J))))
    assert abs(bf.log_z(net) - want) < 1e-12


@pytest.mark.parametrize("n,J,h", [(12, 0.7, 0.3), (200, -0.4, 0.9), (3000, 0.2, -0.1)])
def test_periodic_chain_transfer_matrix(n, J, h):
    """Homogeneous ring: Z = lp^n + lm^n with
    l(+/-) = e^J cosh h +/- sqrt(e^{2J} sinh^2 h + e^{-2J})."""
    s = np.array([-1.0, 1.0])
    scopes, values = [], []
    for i in range(n):
        scopes.append(np.array([i], np.int32))
        values.append(h * s)
        scopes.append(np.array([i, (i + 1) % n], np.int32))
        values.append(J * np.outer(s, s).ravel())
    net = W.Network(np.full(n, 2, np.int32), scopes, values, True)
    a = math.exp(J) * math.cosh(h)
    r = math.sqrt(math.exp(2 * J) * math.sinh(h) ** 2 + math.exp(-2 * J))
    lp, lm = a + r, a - r
    want = n * math.log(lp) + math.log1p((lm / lp) ** n)
    got = oracle.log_z(net)
    assert abs(got - want) <= 1e-11 * max(1.0, abs(want))
    if n <= 16:
        assert abs(bf.log_z(net) - want) < 1e-11


def test_chain_marginals_and_edge_correlations():
    """Zero-field chain: p(x_v) = 1/2 for all v, and the edge factor marginal
    gives E[s_i s_{i+1}] = tanh J_i (factor adjoints, theorem thm:diff)."""
    rng = np.random.default_rng(3)
    J = rng.normal(0, 1, 40)
    net = W.chain_mrf(J)
    lz, marg, adj, aexp, lv = oracle.marginals(net)
    for m in marg:
        assert np.allclose(m, 0.5, atol=1e-13)
    z_lin = math.exp(lz)
    s = np.array([-1.0, 1.0])
    for i, k in enumerate(lv.kind):
        if k != "factor":
            continue
        f = lv.factor_of[i]
        mu = lv.values[i] * adj[i] * 2.0 ** aexp[i] / z_lin
        e_ss = float(np.sum(mu.reshape(2, 2) * np.outer(s, s)))
        assert abs(mu.sum() - 1) < 1e-12
        assert abs(e_ss - math.tanh(J[f])) < 1e-12


# ---------------------------------------------------------------------------
# Bayesian-network invariants
# ---------------------------------------------------------------------------

def test_bn_without_evidence_has_unit_partition_function():
    bn = W.random_bn(120, seed=5)
    assert abs(oracle.log_z(bn)) < 1e-12


def test_bn_root_evidence_is_product_of_root_tables():
    """Evidence only on parentless variables: p(e) = prod of their tables."""
    bn = W.random_bn(80, seed=6)
    rng = np.random.default_rng(0)
    roots = [v for v in range(bn.n_vars) if len(bn.meta["parents"][v]) == 0]
    ev = np.full(bn.n_vars, -1, np.int32)
    want = 0.0
    for v in roots[:6]:
        ev[v] = int(rng.integers(0, bn.card[v]))
        want += math.log(bn.values[v][ev[v]])
    got = oracle.log_z(bn, ev)
    assert abs(got - want) < 1e-12


# ---------------------------------------------------------------------------
# Brute force on small random models (the plain definitions)
# ---------------------------------------------------------------------------

SMALL = [dict(n=12, f=18, seed=s) for s in range(4)] + [dict(n=9, f=14, seed=10 + s) for s in range(3)]


@pytest.mark.parametrize("cfg", SMALL)
@pytest.mark.parametrize("with_evidence", [False, True])
def test_tree_matches_brute_force(cfg, with_evidence):
    net = W.random_small_mrf(cfg["n"], cfg["f"], cfg["seed"])
    ev = None
    if with_evidence:
        rng = np.random.default_rng(cfg["seed"])
        ev = np.full(net.n_vars, -1, np.int32)
        for v in rng.choice(net.n_vars, 3, replace=False):
            ev[v] = int(rng.integers(0, net.card[v]))
    want = bf.log_z(net, ev)
    for mode in ("slice", "indicator"):
        lz, marg, *_ = oracle.marginals(net, ev, mode=mode)
        assert abs(lz - want) < 1e-12 * max(1, abs(want))
        bm = bf.marginals(net, ev)
        for v in range(net.n_vars):
            assert np.allclose(marg[v], bm[v], atol=1e-12), (mode, v)


def test_grid_4x4_brute_force():
    net = W.grid_mrf(4, 4, 0)
    assert abs(oracle.log_z(net) - bf.log_z(net)) < 1e-12
    lz, marg, *_ = oracle.marginals(net)
    for a, b in zip(marg, bf.marginals(net)):
        assert np.allclose(a, b, atol=1e-13)


def test_result_independent_of_tree():
    """The contraction order changes cost, never the result (section on
    contraction orders)."""
    net = W.grid_mrf(5, 6, 3)
    lv = oracle.build_leaves(net)
    orders = [list(range(net.n_vars)), list(reversed(range(net.n_vars))),
              oracle.min_degree_order(lv.labels, net.n_vars),
              list(np.random.default_rng(0).permutation(net.n_vars))]
    vals = [oracle.sum_forward(lv, oracle.elimination_tree(lv.labels, lv.card, o)) for o in orders]
    lz = [math.log(r[0]) + e * math.log(2) for r, e in vals]
    assert max(lz) - min(lz) < 1e-12 * abs(lz[0])


# ---------------------------------------------------------------------------
# Differentiation (theorem thm:diff, eq. einback, unity-vector identity)
# ---------------------------------------------------------------------------

def test_unity_identity_every_variable():
    """sum_x dZ/d1_v(x) * 1_v(x) = Z for every variable (MAR algorithm)."""
    net = W.grid_mrf(5, 5, 4)
    lz, marg, adj, aexp, lv = oracle.marginals(net)
    for i, k in enumerate(lv.kind):
        if k == "unity":
            tot = math.log(float(np.sum(adj[i]))) + aexp[i] * math.log(2)
            assert abs(tot - lz) < 1e-12 * abs(lz)


def test_theorem_diff_against_brute_force():
    """dZ/dT_f equals the contraction of the network without T_f, with the
    output set to the scope of T_f."""
    net = W.random_small_mrf(10, 14, seed=21)
    lz, marg, adj, aexp, lv = oracle.marginals(net)
    for i, k in enumerate(lv.kind):
        if k != "factor":
            continue
        f = lv.factor_of[i]
        rest = W.Network(net.card, [s for g, s in enumerate(net.scopes) if g != f],
                         [v for g, v in enumerate(net.values) if g != f], net.is_log)
        t = bf.joint_log_table(rest)
        scope = sorted(int(v) for v in net.scopes[f])
        axes = tuple(a for a in range(net.n_vars) if a not in scope)
        want = np.exp(t).sum(axis=axes).ravel()
        got = adj[i] * 2.0 ** aexp[i]
        assert np.allclose(got, want, rtol=1e-11, atol=0)


def test_finite_differences_of_log_z():
    net = W.random_small_mrf(9, 12, seed=22)
    lz, marg, adj, aexp, lv = oracle.marginals(net)
    z = math.exp(lz)
    rng = np.random.default_rng(0)
    for _ in range(6):
        i = int(rng.integers(0, net.n_factors))
        j = int(rng.integers(0, len(lv.values[i])))
        eps = 1e-6 * lv.values[i][j]
        lvp = oracle.build_leaves(net)
        lvp.values[i] = lvp.values[i].copy()
        lvp.values[i][j] += eps
        pairs = oracle.default_tree(lv)
        rp, ep = oracle.sum_forward(lvp, pairs)
        lvp.values[i][j] -= 2 * eps
        rm, em = oracle.sum_forward(lvp, pairs)
        fd = (math.log(rp[0]) + ep * math.log(2) - math.log(rm[0]) - em * math.log(2)) / (2 * eps)
        an = adj[i][j] * 2.0 ** aexp[i] / z
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


# ---------------------------------------------------------------------------
# Max-plus (MPE)
# ---------------------------------------------------------------------------

def viterbi(J, h):
    """Textbook Viterbi on a chain: log-potentials J_i s_i s_{i+1} + h_i s_i."""
    s = np.array([-1.0, 1.0])
    n = len(h)
    best = h[0] * s
    back = []
    for i in range(1, n):
        cand = best[:, None] + J[i - 1] * np.outer(s, s) + h[i] * s[None, :]
        back.append(np.argmax(cand, axis=0))
        best = np.max(cand, axis=0)
    x = [int(np.argmax(best))]
    for b in reversed(back):
        x.append(int(b[x[-1]]))
    return float(np.max(best)), np.array(x[::-1], np.int32)


@pytest.mark.parametrize("fp32", [False, True])
def test_chain_map_matches_viterbi(fp32):
    rng = np.random.default_rng(7)
    n = 300
    J, h = rng.normal(0, 1, n - 1), rng.normal(0, 0.5, n)
    net = W.chain_mrf(J, h)
    want_v, want_x = viterbi(J, h)
    v, x = oracle.map_assignment(net, fp32=fp32)
    assert np.array_equal(x, want_x)
    assert abs(v - want_v) < (1e-3 if fp32 else 1e-10)
    assert abs(oracle.log_joint(net, x) - want_v) < 1e-10


def test_ferromagnetic_chain_tie_break_is_one_of_two_optima():
    net = W.chain_mrf(np.full(30, 0.8))
    v1, x1 = oracle.map_assignment(net)
    v2, x2 = oracle.map_assignment(net)
    assert np.array_equal(x1, x2)
    assert np.all(x1 == 0) or np.all(x1 == 1)
    assert abs(v1 - 30 * 0.8) < 1e-12


@pytest.mark.parametrize("seed", range(5))
def test_map_matches_brute_force(seed):
    net = W.random_small_mrf(12, 18, seed=100 + seed)
    rng = np.random.default_rng(seed)
    ev = np.full(net.n_vars, -1, np.int32)
    for v in rng.choice(net.n_vars, 2, replace=False):
        ev[v] = int(rng.integers(0, net.card[v]))
    best, sols, gap = bf.map_set(net, ev)
    for fp32 in (False, True):
        v, x = oracle.map_assignment(net, ev, fp32=fp32)
        if gap > 1e-4 or not fp32:
            assert any(np.array_equal(x, s) for s in sols)
        assert abs(oracle.log_joint(net, x) - best) < (1e-4 if fp32 else 1e-10)


def test_map_indicator_mode_equals_slice_mode():
    bn = W.random_bn(40, seed=8)
    obs, ev = W.bn_evidence(bn, seed=9, frac=0.2)
    v1, x1 = oracle.map_assignment(bn, ev, mode="slice")
    v2, x2 = oracle.map_assignment(bn, ev, mode="indicator")
    assert np.array_equal(x1, x2)
    assert abs(v1 - v2) < 1e-10


# ---------------------------------------------------------------------------
# MMAP (eq. mmap)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_mmap_matches_brute_force(seed):
    net = W.random_small_mrf(11, 16, seed=200 + seed)
    q = np.sort(np.random.default_rng(seed).choice(net.n_vars, 4, replace=False))
    bv, bx, bgap = bf.mmap(net, q)
    v, x, gap = oracle.mmap(net, q)
    assert np.array_equal(x, bx)
    assert abs(v - bv) < 1e-11 * max(1, abs(bv))


def test_mmap_reductions():
    net = W.random_small_mrf(8, 11, seed=300)
    # Q = all variables: MMAP is the MPE
    v, x, _ = oracle.mmap(net, np.arange(net.n_vars))
    mv, mx = oracle.map_assignment(net)
    assert np.array_equal(x, mx) and abs(v - mv) < 1e-10
    # Q = {}: the value is log Z
    v, x, _ = oracle.mmap(net, np.zeros(0, np.int32))
    assert abs(v - bf.log_z(net)) < 1e-11
    # |Q| = 1: argmax of that variable's marginal
    lz, marg, *_ = oracle.marginals(net)
    for q in range(3):
        v, x, _ = oracle.mmap(net, [q])
        assert int(x[0]) == int(np.argmax(marg[q]))


# ---------------------------------------------------------------------------
# Sampling (eq. sample / eq. condition-prob)
# ---------------------------------------------------------------------------

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    for r in rows:
        w = [int(x, 16) for x in r]
        assert oracle.philox4x32_10(w[0:4], w[4:6]) == w[6:10]


def test_sampler_marginals_within_four_sigma():
    net = W.grid_mrf(4, 5, 11)
    lv = oracle.build_leaves(net)
    pairs = oracle.default_tree(lv)
    n = 20000
    s = oracle.sample_tree(lv, pairs, n, seed=1234)
    assert np.all(s >= 0)
    exact = bf.marginals(net)
    for v in range(net.n_vars):
        p = exact[v][1]
        emp = np.mean(s[:, v] == 1)
        sig = math.sqrt(p * (1 - p) / n)
        assert abs(emp - p) < 4.5 * sig + 1e-12, v


def test_slices_sum_to_the_partition_function():
    """Z = sum over the slices of Z_s (fixing variables splits the sum of
    eq. contraction-definition into disjoint parts), against brute force."""
    net = W.grid_mrf(3, 4, 5)
    lv = oracle.build_leaves(net)
    pairs = oracle.default_tree(lv)
    for sliced in ([0], [1, 6], [2, 5, 11]):
        lz = oracle.slice_log_z(lv, pairs, sliced)
        assert len(lz) == 2 ** len(sliced)
        tot = lz.max() + math.log(np.exp(lz - lz.max()).sum())
        assert abs(tot - bf.log_z(net)) <= 1e-10 * max(1.0, abs(tot))
        # each slice equals the brute-force sum with those variables observed
        for a, lzs in zip(oracle.slice_assignments(sliced, net.card), lz):
            ev = -np.ones(net.n_vars, np.int32)
            for v, x in a.items():
                ev[v] = x
            assert abs(lzs - bf.log_z(net, ev)) <= 1e-10 * max(1.0, abs(lzs))


def test_sampler_counters_follow_ids():
    net = W.grid_mrf(3, 3, 2)
    lv = oracle.build_leaves(net)
    pairs = oracle.default_tree(lv)
    full = oracle.sample_tree(lv, pairs, 50, seed=8)
    assert np.array_equal(oracle.sample_tree(lv, pairs, 50, seed=8, ids=np.arange(50)), full)
    ids = np.array([3, 17, 40])
    assert np.array_equal(oracle.sample_tree(lv, pairs, 3, seed=8, ids=ids), full[ids])


def test_reservoir_slice_frequencies():
    """One pass over the slices keeping slice s with probability
    Z_s / (Z_0 + ... + Z_s) leaves a sample in slice s with probability
    Z_s / Z (weights spanning orders of magnitude, a zero-weight slice)."""
    lz = np.array([math.log(3.0), -math.inf, math.log(0.5), math.log(10.0), math.log(1e-3), 0.0])
    n = 40000
    c = oracle.reservoir_slices(lz, n, seed=5)
    assert np.all(c >= 0) and not np.any(c == 1)
    p = np.exp(lz - np.logaddexp.reduce(lz[np.isfinite(lz)]))
    for s in range(len(lz)):
        emp = np.mean(c == s)
        sig = math.sqrt(p[s] * (1 - p[s]) / n)
        assert abs(emp - p[s]) <= 4.5 * sig + 1e-12, s


def test_sliced_sampler_marginals_within_four_sigma():
    """Each sample ending in slice s with probability Z_s / Z (one pass
    over the slices, weighted reservoir), then sampled inside it, samples the
    joint distribution: marginals against brute force."""
    net = W.grid_mrf(3, 4, 9)
    lv = oracle.build_leaves(net)
    pairs = oracle.default_tree(lv)
    n = 20000
    s = oracle.sample_sliced(lv, pairs, [1, 6], n, seed=31)
    assert np.all(s >= 0)
    exact = bf.marginals(net)
    for v in range(net.n_vars):
        p = exact[v][1]
        emp = np.mean(s[:, v] == 1)
        sig = math.sqrt(p * (1 - p) / n)
        assert abs(emp - p) < 4.5 * sig + 1e-12, v


def test_sampler_joint_chi_square():
    from scipy import stats
    net = W.random_small_mrf(5, 7, seed=400, cards=(2, 3))
    lv = oracle.build_leaves(net)
    pairs = oracle.default_tree(lv)
    n = 100000
    s = oracle.sample_tree(lv, pairs, n, seed=99)
    t = bf.joint_log_table(net)
    p = np.exp(t - t.max())
    p = (p / p.sum()).ravel()
    idx = np.ravel_multi_index(tuple(s.T), t.shape)
    counts = np.bincount(idx, minlength=p.size)
    chi2 = float(np.sum((counts - n * p) ** 2 / (n * p)))
    assert stats.chi2.sf(chi2, p.size - 1) > 1e-4


def test_sampler_respects_evidence():
    bn = W.random_bn(30, seed=12)
    obs, ev = W.bn_evidence(bn, seed=13, frac=0.2)
    lv = oracle.build_leaves(bn, ev)
    pairs = oracle.default_tree(lv)
    s = oracle.sample_tree(lv, pairs, 2000, seed=5)
    free = ev < 0
    assert np.all(s[:, free] >= 0)
    exact = bf.marginals(bn, ev) if bn.n_vars <= 20 else oracle.marginals(bn, ev)[1]
    for v in np.nonzero(free)[0][:8]:
        emp = np.bincount(s[:, v], minlength=bn.card[v]) / 2000
        assert np.all(np.abs(emp - exact[v]) < 4.5 * np.sqrt(exact[v] * (1 - exact[v]) / 2000) + 1e-9)


# ---------------------------------------------------------------------------
# The paper's worked example of contraction orders
# ---------------------------------------------------------------------------

def test_paper_five_tensor_example_ranks():
    g = json.load(open(os.path.join(GOLDEN, "paper_five_tensor_example.json")))
    names = g["leaf_order"]
    labels = [g["leaves"][k] for k in names]
    card = np.full(6, 3, np.int32)
    for key, want in (("tree_a", g["max_intermediate_rank_a"]), ("tree_b", g["max_intermediate_rank_b"])):
        ids = {k: i for i, k in enumerate(names)}
        pairs = []
        for a, b in g[key]:
            pairs.append((ids[a], ids[b]))
            ids[a + b if a + b not in ids else b + a] = len(names) + len(pairs) - 1
            ids.setdefault("".join(sorted(a + b)), len(names) + len(pairs) - 1)
        st = oracle.tree_stats(labels, pairs, card, out=g["output"])
        assert st["rank"] == want
        # both orders give the same contraction result
    rng = np.random.default_rng(0)
    vals = [rng.random(3 ** len(l)) for l in labels]
    lv = oracle.Leaves(card, labels, vals, ["factor"] * 5)
    res = []
    for key in ("tree_a", "tree_b"):
        ids = {k: i for i, k in enumerate(names)}
        pairs = []
        for a, b in g[key]:
            pairs.append((ids[a], ids[b]))
            ids[a + b] = len(names) + len(pairs) - 1
            ids[b + a] = ids[a + b]
        r, e = oracle.sum_forward(lv, pairs, out=g["output"])
        res.append(r * 2.0 ** e)
    # direct definition by einsum over all six labels
    A, B, C, D, E = [v.reshape([3] * len(l)) for v, l in zip(vals, labels)]
    want = np.einsum("il,l,jkl,kmn,jn->im", A, B, C, D, E)
    for r in res:
        assert np.allclose(r.reshape(3, 3), want, rtol=1e-13)
