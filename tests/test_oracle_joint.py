"""Pins of the oracle's joint and factor marginals.

Joint marginals come from the adjoint of a unity tensor over a variable set
(the MAR section's unity tensors, generalised to several variables); factor
marginals from the factors' own adjoints (theorem thm:diff): T_f Tbar_f / Z.
They are pinned to brute-force summation of the joint table, to the
zero-field Ising chain's closed forms E[s_i s_j] = prod of tanh J over the
path between i and j, and to normalisation and consistency with the
single-variable marginals.
"""
import math

import numpy as np
import pytest

import oracle
import oracle.brute as bf
from paper_2405_14060_amd import workloads as W


def sets_for(net, rng):
    """Variable sets of size 1..3, adjacent and not."""
    n = net.n_vars
    out = [[int(rng.integers(n))]]
    for k in (2, 2, 3):
        out.append(sorted(int(v) for v in rng.choice(n, k, replace=False)))
    out.append(sorted(int(v) for v in net.scopes[0]))
    return out


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("mode", ["slice", "indicator"])
def test_joint_marginals_match_brute_force(seed, mode):
    net = W.random_small_mrf(11, 16, seed=60 + seed, cards=(2, 3))
    rng = np.random.default_rng(seed)
    ev = np.full(net.n_vars, -1, np.int32)
    if seed % 2:
        for v in rng.choice(net.n_vars, 2, replace=False):
            ev[v] = int(rng.integers(0, net.card[v]))
    sets = sets_for(net, rng)
    if seed % 2:  # a set holding an observed variable
        sets.append(sorted({int(np.nonzero(ev >= 0)[0][0]), int(np.nonzero(ev < 0)[0][0])}))
    lz, got = oracle.joint_marginals(net, sets, ev if seed % 2 else None, mode=mode)
    assert abs(lz - bf.log_z(net, ev)) <= 1e-10 * max(1.0, abs(lz))
    for s, g in zip(sets, got):
        want = bf.joint_marginal(net, s, ev)
        assert g.shape == want.shape
        assert np.abs(g - want).max() <= 1e-12, s
        assert abs(g.sum() - 1.0) <= 1e-12


def test_joint_marginals_zero_field_chain_correlations():
    """Zero-field Ising chain: E[s_i s_j] = prod_{k=i}^{j-1} tanh J_k for
    any pair i < j (adjacent or not), and every single marginal is 1/2."""
    rng = np.random.default_rng(3)
    J = rng.normal(0, 1, 39)
    net = W.chain_mrf(J)
    pairs = [(0, 1), (4, 5), (2, 7), (10, 30), (38, 39)]
    _, got = oracle.joint_marginals(net, [list(p) for p in pairs])
    s = np.array([-1.0, 1.0])
    for (i, j), g in zip(pairs, got):
        want = float(np.prod(np.tanh(J[i:j])))
        assert abs(float(s @ g @ s) - want) <= 1e-12, (i, j)
        assert np.abs(g.sum(axis=0) - 0.5).max() <= 1e-12


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("mode", ["slice", "indicator"])
def test_factor_marginals_match_brute_force(seed, mode):
    net = W.random_small_mrf(10, 15, seed=80 + seed, cards=(2, 3, 4))
    rng = np.random.default_rng(seed)
    ev = np.full(net.n_vars, -1, np.int32)
    for v in rng.choice(net.n_vars, 2, replace=False):
        ev[v] = int(rng.integers(0, net.card[v]))
    lz, fm = oracle.factor_marginals(net, ev, mode=mode)
    assert abs(lz - bf.log_z(net, ev)) <= 1e-10 * max(1.0, abs(lz))
    marg = bf.marginals(net, ev)
    for f in range(net.n_factors):
        s = [int(v) for v in net.scopes[f]]
        want = bf.joint_marginal(net, s, ev)  # over sorted scope
        want = np.transpose(want, np.argsort(np.argsort(s))).ravel() if len(s) > 1 else want.ravel()
        assert fm[f].shape == want.shape
        assert np.abs(fm[f] - want).max() <= 1e-12, f
        assert abs(fm[f].sum() - 1.0) <= 1e-12
        # summing a factor marginal over all but one variable gives that
        # variable's marginal
        t = fm[f].reshape([int(net.card[v]) for v in s])
        for a, v in enumerate(s):
            other = tuple(b for b in range(len(s)) if b != a)
            assert np.abs(t.sum(axis=other) - marg[v]).max() <= 1e-12


def test_factor_marginals_of_a_bayesian_network_root():
    """A root variable's CPT has no parents: with no evidence its factor
    marginal is the CPT itself."""
    bn = W.random_bn(30, seed=5)
    _, fm = oracle.factor_marginals(bn)
    for f in range(bn.n_factors):
        if len(bn.scopes[f]) == 1:
            assert np.abs(fm[f] - np.asarray(bn.values[f])).max() <= 1e-12
