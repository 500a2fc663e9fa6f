"""Pins of the oracle's max-plus tie-break and of its FP32-emulation bits.

The paper's MPE section asks the Boolean back-propagation to keep exactly one
of several optimal configurations but does not fix which.  The reading used
here (and by the HIP path): at every tree node, among equal maxima the
smallest row-major index over the labels eliminated there wins (labels sorted
by id, last fastest); labels that occur in one child only are reduced in that
child first.  The cases below are built by hand so that this reading implies
one assignment, derived in each docstring without the oracle; the opposite
convention (last maximiser) gives a different one, so a '>' turned into '>='
in any of the oracle's comparisons fails a case.

The FP32-emulation pins use a fact independent of how the oracle organises a
node: IEEE addition is monotone in each operand, so the max-plus value of a
tree computed with one float add per candidate equals the maximum, over all
full assignments x, of the leaves' float32 values added up in the tree's
order (each node adding its two children).  A numpy float32 enumeration of
that sum pins the oracle's FP32 value bit for bit and its assignment to the
set of maximisers.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2405_14060_amd import workloads as W


def leaves(card, labels, tables):
    """Oracle leaves from tables given over sorted label lists (log domain)."""
    vals = [np.asarray(t, np.float64).ravel() for t in tables]
    return oracle.Leaves(card, [np.asarray(l, np.int32) for l in labels], vals, ["factor"] * len(labels))


# ---------------------------------------------------------------------------
# Tie-break: hand-derived answers
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("fp32", [False, True])
def test_private_label_tie_keeps_smallest(fp32):
    """A(x0, x1) is flat in x1 (x1 occurs in A only, so it is reduced inside
    A before the node); B(x0) has a unique maximum at x0 = 1.  The node then
    maximises over x0 alone.  Reading: x0 = 1 (unique), x1 = 0 (first of the
    three tied values).  Last-maximiser convention: x1 = 2."""
    card = [2, 3]
    A = np.array([[0.5, 0.5, 0.5], [1.0, 1.0, 1.0]])
    B = np.array([0.0, 2.0])
    lv = leaves(card, [[0, 1], [0]], [A, B])
    v, x = oracle.max_forward(lv, [(0, 1)], fp32=fp32)
    assert x.tolist() == [1, 0]
    assert v == 3.0


@pytest.mark.parametrize("fp32", [False, True])
def test_shared_label_tie_keeps_smallest(fp32):
    """A(x0) + B(x0) = (0, 3, 3, 1): the node eliminates the shared x0 and
    values 1 and 2 tie.  Reading: x0 = 1.  Last maximiser: x0 = 2."""
    card = [4]
    lv = leaves(card, [[0], [0]], [[0.0, 1.0, 2.0, 0.5], [0.0, 2.0, 1.0, 0.5]])
    v, x = oracle.max_forward(lv, [(0, 1)], fp32=fp32)
    assert x.tolist() == [1]
    assert v == 3.0


@pytest.mark.parametrize("fp32", [False, True])
def test_single_leaf_root_reduction_keeps_smallest_row_major(fp32):
    """One leaf F(x0, x1) (3 x 3), no pairs: the root reduces both labels
    at once.  Maxima at (1, 2) (row-major index 5) and (2, 0) (index 6).
    Reading: (1, 2).  Last maximiser: (2, 0)."""
    F = np.zeros((3, 3))
    F[1, 2] = F[2, 0] = 4.0
    lv = leaves([3, 3], [[0, 1]], [F])
    v, x = oracle.max_forward(lv, np.zeros((0, 2), np.int32), fp32=fp32)
    assert x.tolist() == [1, 2]
    assert v == 4.0


@pytest.mark.parametrize("fp32", [False, True])
def test_tie_break_is_per_node_and_follows_the_tree(fp32):
    """F(x0, x1) with maxima at (1, 2) and (2, 0), plus flat unity vectors
    u0(x0), u1(x1) (leaves 1 and 2).

    Tree ((F, u0), u1): the first node eliminates x0 (x1 is still needed by
    u1): its output is max_x0 F, equal to 4 at x1 = 0 (from x0 = 2) and at
    x1 = 2 (from x0 = 1).  The root eliminates x1: tie between 0 and 2, the
    reading keeps x1 = 0, and the readout of the first node gives x0 = 2:
    (2, 0).

    Tree ((F, u1), u0): x1 is eliminated first; the output over x0 is 4 at
    x0 = 1 and x0 = 2; the root keeps x0 = 1, then x1 = 2: (1, 2).
    Under the last-maximiser convention the two trees give the other answer."""
    F = np.zeros((3, 3))
    F[1, 2] = F[2, 0] = 4.0
    lv = leaves([3, 3], [[0, 1], [0], [1]], [F, np.zeros(3), np.zeros(3)])
    _, x_a = oracle.max_forward(lv, [(0, 1), (3, 2)], fp32=fp32)
    _, x_b = oracle.max_forward(lv, [(0, 2), (3, 1)], fp32=fp32)
    assert x_a.tolist() == [2, 0]
    assert x_b.tolist() == [1, 2]


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("fp32", [False, True])
def test_flat_network_gives_all_zeros_on_any_tree(seed, fp32):
    """All log-potentials 0: every configuration is optimal, so at every
    node every candidate ties and the reading keeps index 0 of the
    eliminated labels: the all-zeros assignment, for any tree (random
    elimination orders here).  Last maximiser: card - 1 everywhere."""
    net = W.random_small_mrf(10, 14, seed=seed, cards=(2, 3, 4))
    for f in range(net.n_factors):
        t = np.asarray(net.values[f], np.float64)
        net.values[f] = np.zeros_like(t) if net.is_log else np.ones_like(t)
    lv = oracle.build_leaves(net, domain="log")
    order = list(np.random.default_rng(seed).permutation(net.n_vars))
    pairs = oracle.elimination_tree(lv.labels, lv.card, order)
    v, x = oracle.max_forward(lv, pairs, fp32=fp32)
    assert v == 0.0
    assert np.all(x == 0)


def test_ferromagnetic_chain_natural_tree_picks_all_zeros():
    """Zero-field ferromagnetic chain: optima all-0 and all-1.  On the
    bucket tree in natural order the last node to decide is the root, over
    the last variable; both of its values tie and the reading keeps 0, and
    the couplings force every other variable to follow: all zeros."""
    net = W.chain_mrf(np.full(30, 0.8))
    lv = oracle.build_leaves(net, domain="log")
    pairs = oracle.elimination_tree(lv.labels, lv.card, list(range(net.n_vars)))
    for fp32 in (False, True):
        v, x = oracle.max_forward(lv, pairs, fp32=fp32)
        assert np.all(x == 0)


# ---------------------------------------------------------------------------
# FP32 emulation: float32 enumeration of the tree-ordered sums
# ---------------------------------------------------------------------------

def tree_ordered_f32_sums(lv, pairs, n_vars):
    """For every full assignment x (row-major, last variable fastest), the
    float32 sum of the leaves' float32 log-values in the tree's order."""
    card = [int(c) for c in lv.card[:n_vars]]
    grid = np.array(list(itertools.product(*[range(c) for c in card])), np.int64).reshape(-1, n_vars)
    vals = []
    for lab, v in zip(lv.labels, lv.values):
        lab = [int(u) for u in lab]
        idx = np.zeros(len(grid), np.int64)
        for u in lab:
            idx = idx * card[u] + grid[:, u]
        vals.append(np.asarray(v, np.float64).astype(np.float32)[idx])
    for a, b in pairs:
        vals.append(np.add(vals[a], vals[b], dtype=np.float32))
    return grid, vals[-1]


@pytest.mark.parametrize("seed", range(6))
def test_fp32_emulation_value_bits_match_float32_enumeration(seed):
    net = W.random_small_mrf(9, 12, seed=40 + seed, cards=(2, 3))
    lv = oracle.build_leaves(net, domain="log")
    pairs = oracle.default_tree(lv)
    grid, s = tree_ordered_f32_sums(lv, pairs, net.n_vars)
    best = s.max()
    v, x = oracle.max_forward(lv, pairs, fp32=True)
    assert np.float32(v) == best and float(np.float32(v)) == v
    k = int(np.ravel_multi_index(tuple(x), tuple(int(c) for c in net.card)))
    assert s[k] == best
    # the FP64 mode differs from the float32 sums in general (rounding)
    v64, _ = oracle.max_forward(lv, pairs, fp32=False)
    assert abs(v64 - float(best)) < 1e-4


def test_fp32_emulation_rounds_each_candidate_once():
    """Leaves whose float32 sum depends on the order of additions:
    1 + 2^-24 + 2^-24 is 1 in float32 when added left to right, but
    1 + 2^-23 when the two small terms are added first.  The tree decides
    which, and the oracle must follow it."""
    e = 2.0 ** -24
    lv = leaves([1], [[0], [0], [0]], [[1.0], [e], [e]])
    v_lr, _ = oracle.max_forward(lv, [(0, 1), (3, 2)], fp32=True)
    v_sm, _ = oracle.max_forward(lv, [(1, 2), (0, 3)], fp32=True)
    assert v_lr == 1.0
    assert v_sm == 1.0 + 2.0 ** -23
