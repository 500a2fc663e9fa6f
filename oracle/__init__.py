"""Plain FP64 CPU reference ("the oracle") for tensor-network inference.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the product library never does, and the
two share no code.  Everything here follows the paper's definitions directly:

* leaves (section "Tensor networks for probabilistic modeling"): the factor
  tables of the model, sliced by the evidence (eq. pr), plus one unity vector
  per query variable (MAR algorithm, step 1) or, for batched evidence, one
  indicator vector per variable (one-hot at the observed value, ones
  otherwise; contracting it equals slicing);
* a binary contraction tree built here by bucket elimination from a
  variable order (its own code, independent of the product's planner);
* contraction along the tree, the reverse pass of eq. einback, the max-plus
  contraction of eq. log-map with argmax readout, and top-down sampling
  (eq. sample / eq. condition-prob), all in ``tn_oracle.c``;
* MMAP by its definition (eq. mmap): the joint table over the query set is
  obtained by one sum contraction with the query labels left open, then its
  argmax is taken.

Parity status of each function is stated in its docstring; the pins live in
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "tn_oracle.c")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C part with gcc (plain -O2, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                               "-shared", "-o", _SO, _SRC, "-lm"])
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER
        i32p, i64p, f64p = P(ctypes.c_int), P(ctypes.c_int64), P(ctypes.c_double)
        L.or_last_error.restype = ctypes.c_char_p
        L.or_sum_forward.argtypes = [ctypes.c_int, i32p, ctypes.c_int, i64p, i32p, f64p,
                                     ctypes.c_int, i32p, ctypes.c_int, i32p, ctypes.c_int,
                                     f64p, i64p, f64p, i64p]
        L.or_max_forward.argtypes = [ctypes.c_int, i32p, ctypes.c_int, i64p, i32p, f64p,
                                     ctypes.c_int, i32p, ctypes.c_int, f64p, i32p]
        L.or_sample.argtypes = [ctypes.c_int, i32p, ctypes.c_int, i64p, i32p, f64p,
                                ctypes.c_int, i32p, ctypes.c_uint64, ctypes.c_int64, i64p, i32p]
        L.or_philox4x32_10.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_set_threads.restype = None
        L.or_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops (each output element of a
    contraction is one sum in a fixed order, so every thread count gives the
    same bits); returns the count now in use."""
    lib().or_set_threads(int(n))
    return int(lib().or_threads())


def threads() -> int:
    return int(lib().or_threads())


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _check(rc):
    if rc != 0:
        raise ValueError("oracle: " + lib().or_last_error().decode())


# ---------------------------------------------------------------------------
# Leaves
# ---------------------------------------------------------------------------

class Leaves:
    """Leaf tensors in the canonical layout: labels sorted ascending,
    row-major, last label fastest.  ``kind[i]`` is 'factor' or 'unity'."""

    def __init__(self, card, labels, values, kind, factor_of=None, var_of=None):
        self.card = np.asarray(card, np.int32)
        self.labels = [np.asarray(l, np.int32) for l in labels]
        self.values = [np.asarray(v, np.float64) for v in values]
        self.kind = list(kind)
        self.factor_of = factor_of or [-1] * len(labels)
        self.var_of = var_of or [-1] * len(labels)

    def __len__(self):
        return len(self.labels)

    def csr(self):
        ptr = np.zeros(len(self) + 1, np.int64)
        for i, l in enumerate(self.labels):
            ptr[i + 1] = ptr[i] + len(l)
        lab = np.concatenate(self.labels).astype(np.int32) if ptr[-1] else np.zeros(1, np.int32)
        vals = np.concatenate(self.values) if len(self) else np.zeros(1)
        return ptr, lab, np.ascontiguousarray(vals, np.float64)


def factor_table(net, f, domain: str) -> np.ndarray:
    """Factor f as an ndarray over its scope order, in the requested domain."""
    s = np.asarray(net.scopes[f])
    t = np.asarray(net.values[f], np.float64).reshape([int(net.card[v]) for v in s])
    if domain == "linear":
        return np.exp(t) if net.is_log else t
    if domain == "log":
        if net.is_log:
            return t
        with np.errstate(divide="ignore"):
            return np.log(t)
    raise ValueError(domain)


def build_leaves(net, evidence=None, mode: str = "slice", domain: str = "linear",
                 unity: bool = True) -> Leaves:
    """Leaves for one evidence instance.

    mode 'slice': factors sliced at the observed values (the sliced set of
    eq. pr), unity vectors for the free variables.  mode 'indicator':
    unsliced factors plus an indicator vector for every variable (one-hot at
    the observed value, all ones if free).  In the log domain unity vectors
    are zeros and indicator entries 0 / -inf.
    """
    n = net.n_vars
    ev = np.full(n, -1, np.int32) if evidence is None else np.asarray(evidence, np.int32)
    one = 1.0 if domain == "linear" else 0.0
    zero = 0.0 if domain == "linear" else -np.inf
    labels, values, kind, fo, vo = [], [], [], [], []
    for f in range(net.n_factors):
        s = np.asarray(net.scopes[f], np.int64)
        t = factor_table(net, f, domain)
        if mode == "slice":
            idx = tuple(int(ev[v]) if ev[v] >= 0 else slice(None) for v in s)
            t = t[idx]
            s = np.array([v for v in s if ev[v] < 0], np.int64)
        perm = np.argsort(s, kind="stable")
        labels.append(s[perm].astype(np.int32))
        values.append(np.ascontiguousarray(np.transpose(t, perm)).ravel())
        kind.append("factor")
        fo.append(f)
        vo.append(-1)
    if unity:
        for v in range(n):
            if mode == "slice" and ev[v] >= 0:
                continue
            vec = np.full(int(net.card[v]), one)
            if mode == "indicator" and ev[v] >= 0:
                vec[:] = zero
                vec[ev[v]] = one
            labels.append(np.array([v], np.int32))
            values.append(vec)
            kind.append("unity")
            fo.append(-1)
            vo.append(v)
    return Leaves(net.card, labels, values, kind, fo, vo)


# ---------------------------------------------------------------------------
# Contraction trees (the oracle's own builder)
# ---------------------------------------------------------------------------

def elimination_tree(labels, card, order) -> np.ndarray:
    """Binary tree by bucket elimination along ``order``.

    For each variable in turn, all current tensors that contain it are merged
    pairwise (smallest first, ties by id) into one.  Remaining tensors are
    merged smallest first at the end.  Returns int32 pairs [L-1, 2] in
    post-order with ids as in the tree convention of ``tn_oracle.c``.
    """
    card = np.asarray(card)
    lg = {v: math.log2(int(card[v])) for v in range(len(card))}
    active = {i: set(int(v) for v in l) for i, l in enumerate(labels)}
    where = {}
    for i, ls in active.items():
        for v in ls:
            where.setdefault(v, set()).add(i)
    nxt = len(labels)
    pairs = []

    def size(i):
        return sum(lg[v] for v in active[i])

    def merge(ids):
        nonlocal nxt
        ids = sorted(ids, key=lambda i: (size(i), i))
        while len(ids) > 1:
            a, b = ids[0], ids[1]
            pairs.append((a, b))
            new = active.pop(a) | active.pop(b)
            for v in new:
                w = where[v]
                w.discard(a)
                w.discard(b)
                w.add(nxt)
            active[nxt] = new
            ids = sorted(ids[2:] + [nxt], key=lambda i: (size(i), i))
            nxt += 1
        return ids[0]

    for v in order:
        ids = list(where.get(v, ()))
        if not ids:
            continue
        keep = merge(ids)
        active[keep].discard(v)
        where[v].discard(keep)
    if len(active) > 1:
        merge(list(active.keys()))
    return np.asarray(pairs, np.int32).reshape(-1, 2)


def min_degree_order(labels, n_vars) -> list:
    """Greedy min-degree elimination order on the interaction graph (ties
    by smallest id), with a lazily updated heap."""
    import heapq
    nbr = [set() for _ in range(n_vars)]
    present = set()
    for l in labels:
        l = [int(v) for v in l]
        present.update(l)
        for a in l:
            nbr[a].update(x for x in l if x != a)
    heap = [(len(nbr[v]), v) for v in present]
    heapq.heapify(heap)
    done, order = set(), []
    while heap:
        d, v = heapq.heappop(heap)
        if v in done or d != len(nbr[v]):
            continue
        nb = nbr[v]
        for a in nb:
            nbr[a].discard(v)
            nbr[a].update(x for x in nb if x != a)
            heapq.heappush(heap, (len(nbr[a]), a))
        done.add(v)
        order.append(v)
    return order


def tree_node_labels(labels, pairs, out=()):
    """Output labels of every node (leaves first), following the tree
    semantics: a node keeps the labels of its children still present in a
    leaf outside its subtree or in the output set."""
    L = len(labels)
    total = {}
    for l in labels:
        for v in l:
            total[int(v)] = total.get(int(v), 0) + 1
    sub = [dict((int(v), 1) for v in l) for l in labels]
    lab = [set(int(v) for v in l) for l in labels]
    out = set(int(v) for v in out)
    for a, b in pairs:
        s = dict(sub[a])
        for v, k in sub[b].items():
            s[v] = s.get(v, 0) + k
        sub.append(s)
        u = lab[a] | lab[b]
        lab.append(set(v for v in u if v in out or total[v] - s.get(v, 0) > 0))
    return lab, L


def tree_stats(labels, pairs, card, out=()) -> dict:
    """Space complexity (log2 of the largest node output), largest label
    union, and time complexity (log2 of sum over nodes of the label-union
    size), the measures used by the paper's benchmark section."""
    card = np.asarray(card)
    lab, L = tree_node_labels(labels, pairs, out)
    sc, su, tc = 0.0, 0.0, 0.0
    for i, (a, b) in enumerate(pairs):
        c = L + i
        sc = max(sc, sum(math.log2(card[v]) for v in lab[c]))
        uu = sum(math.log2(card[v]) for v in lab[a] | lab[b])
        su = max(su, uu)
        tc += 2.0 ** uu
    return dict(sc=sc, union=su, tc=math.log2(tc) if tc else 0.0,
                rank=max((len(lab[L + i]) for i in range(len(pairs))), default=0))


def default_tree(leaves: Leaves, order=None):
    if order is None:
        order = min_degree_order(leaves.labels, len(leaves.card))
    return elimination_tree(leaves.labels, leaves.card, order)


# ---------------------------------------------------------------------------
# Contraction entry points
# ---------------------------------------------------------------------------

def sum_forward(leaves: Leaves, pairs, out=(), want_adj=False):
    """Sum-product contraction; returns (root table over sorted ``out``,
    exponent) and, if requested, (leaf adjoint tables, exponents)."""
    L = lib()
    ptr, lab, vals = leaves.csr()
    pairs = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
    out = np.ascontiguousarray(np.sort(np.asarray(out, np.int32)))
    root = np.zeros(int(np.prod(leaves.card[out])) if len(out) else 1)
    rexp = np.zeros(1, np.int64)
    adj = np.zeros(max(1, vals.size)) if want_adj else np.zeros(1)
    aexp = np.zeros(max(1, len(leaves)), np.int64)
    card = np.ascontiguousarray(leaves.card)
    _check(L.or_sum_forward(len(card), _p(card, ctypes.c_int), len(leaves), _p(ptr, ctypes.c_int64),
                            _p(lab, ctypes.c_int), _p(vals, ctypes.c_double), len(pairs),
                            _p(pairs, ctypes.c_int), len(out), _p(out, ctypes.c_int),
                            1 if want_adj else 0, _p(root, ctypes.c_double),
                            _p(rexp, ctypes.c_int64), _p(adj, ctypes.c_double),
                            _p(aexp, ctypes.c_int64)))
    if not want_adj:
        return root, int(rexp[0])
    per, o = [], 0
    for v in leaves.values:
        per.append(adj[o:o + v.size].copy())
        o += v.size
    return root, int(rexp[0]), per, aexp[:len(leaves)].copy()


def max_forward(leaves: Leaves, pairs, fp32: bool = False):
    """Max-plus contraction of log-domain leaves; returns (value, assignment
    int32[n_vars] with -1 for labels in no leaf)."""
    L = lib()
    ptr, lab, vals = leaves.csr()
    pairs = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
    card = np.ascontiguousarray(leaves.card)
    val = np.zeros(1)
    asg = np.full(len(card), -1, np.int32)
    _check(L.or_max_forward(len(card), _p(card, ctypes.c_int), len(leaves), _p(ptr, ctypes.c_int64),
                            _p(lab, ctypes.c_int), _p(vals, ctypes.c_double), len(pairs),
                            _p(pairs, ctypes.c_int), 1 if fp32 else 0, _p(val, ctypes.c_double),
                            _p(asg, ctypes.c_int)))
    return float(val[0]), asg


def sample_tree(leaves: Leaves, pairs, n: int, seed: int, ids=None) -> np.ndarray:
    """Top-down sampling (eq. sample, eq. condition-prob).  Sample j uses
    ids[j] (default j) as its Philox counter; row j of the result."""
    L = lib()
    ptr, lab, vals = leaves.csr()
    pairs = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
    card = np.ascontiguousarray(leaves.card)
    out = np.full((n, len(card)), -1, np.int32)
    idp = None
    if ids is not None:
        ids = np.ascontiguousarray(np.asarray(ids, np.int64))
        assert ids.size == n
        idp = _p(ids, ctypes.c_int64)
    _check(L.or_sample(len(card), _p(card, ctypes.c_int), len(leaves), _p(ptr, ctypes.c_int64),
                       _p(lab, ctypes.c_int), _p(vals, ctypes.c_double), len(pairs),
                       _p(pairs, ctypes.c_int), ctypes.c_uint64(seed), n, idp, _p(out, ctypes.c_int)))
    return out


# ---------------------------------------------------------------------------
# Slicing (fixed variables per slice) for log Z and sampling
# ---------------------------------------------------------------------------

SLICE_DRAW_NODE = 0xFFFFFFFF  # Philox node word of a sample's slice draw


def fix_leaves(leaves: Leaves, assign: dict) -> Leaves:
    """The same leaves with the variables in ``assign`` fixed at their values
    (each table indexed there, the variables dropped from its labels); the
    leaf count and order are kept, so a tree over the leaves still applies."""
    labels, values = [], []
    for lab, val in zip(leaves.labels, leaves.values):
        t = np.asarray(val).reshape([int(leaves.card[v]) for v in lab]) if len(lab) else np.asarray(val).reshape(())
        idx = tuple(int(assign[int(v)]) if int(v) in assign else slice(None) for v in lab)
        t = t[idx] if len(lab) else t
        labels.append(np.array([v for v in lab if int(v) not in assign], np.int32))
        values.append(np.ascontiguousarray(t).ravel())
    return Leaves(leaves.card, labels, values, leaves.kind, leaves.factor_of, leaves.var_of)


def slice_assignments(sliced, card):
    """Assignments of the sliced variables, row-major (last fastest)."""
    sliced = [int(v) for v in sliced]
    dims = [int(card[v]) for v in sliced]
    for k in range(int(np.prod(dims)) if dims else 1):
        a, r = {}, k
        for v, d in zip(reversed(sliced), reversed(dims)):
            a[v] = r % d
            r //= d
        yield a


def slice_log_z(leaves: Leaves, pairs, sliced) -> np.ndarray:
    """log Z_s of every slice (Z = sum over slices of Z_s)."""
    out = []
    for a in slice_assignments(sliced, leaves.card):
        root, ex = sum_forward(fix_leaves(leaves, a), pairs)
        out.append(math.log(root[0]) + ex * LN2 if root[0] > 0 else -math.inf)
    return np.array(out)


def uniform53(sample: int, node: int, slot: int, seed: int) -> float:
    """Philox uniform in [0, 1): 53 bits of the first two output words."""
    o = philox4x32_10([sample & 0xFFFFFFFF, sample >> 32, node, slot], [seed & 0xFFFFFFFF, seed >> 32])
    return ((o[0] >> 5) * 67108864.0 + (o[1] >> 6)) / 9007199254740992.0


def reservoir_slices(lz, n: int, seed: int) -> np.ndarray:
    """The slice of each of n samples from the slices' log weights lz, in one
    pass over the slices in order: sample i takes slice s when the uniform
    from counter (i, SLICE_DRAW_NODE, s) is below Z_s / (Z_0 + ... + Z_s);
    the last slice taken is kept (-1 if every weight is zero)."""
    choice = np.full(n, -1, np.int64)
    prefix = -math.inf
    for s in range(len(lz)):
        if not lz[s] > -math.inf:
            continue
        prefix = float(np.logaddexp(prefix, lz[s]))
        q = math.exp(lz[s] - prefix)
        for i in range(n):
            if uniform53(i, SLICE_DRAW_NODE, s, seed) < q:
                choice[i] = s
    return choice


def sample_sliced(leaves: Leaves, pairs, sliced, n: int, seed: int) -> np.ndarray:
    """Sampling when the tree is contracted slice by slice, in one pass over
    the slices in order: sample i takes slice s with probability
    Z_s / (Z_0 + ... + Z_s) (uniform from counter (i, SLICE_DRAW_NODE, s)),
    and the last slice it takes is its slice -- with probability Z_s / Z, a
    weighted reservoir of one.  Inside its slice it follows the per-node rule
    with counter i.  Sliced variables take the slice's values."""
    lz = slice_log_z(leaves, pairs, sliced)
    choice = reservoir_slices(lz, n, seed)
    out = np.full((n, len(leaves.card)), -1, np.int32)
    for s, a in enumerate(slice_assignments(sliced, leaves.card)):
        ids = np.nonzero(choice == s)[0]
        if ids.size == 0:
            continue
        rows = sample_tree(fix_leaves(leaves, a), pairs, ids.size, seed, ids)
        for v, x in a.items():
            rows[:, v] = x
        out[ids] = rows
    return out


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(x) for x in o]


# ---------------------------------------------------------------------------
# Inference tasks (one evidence instance each)
# ---------------------------------------------------------------------------

LN2 = math.log(2.0)


def log_z(net, evidence=None, mode="slice", pairs=None) -> float:
    """log p(e) (eq. pr); the partition function when there is no evidence."""
    lv = build_leaves(net, evidence, mode)
    pairs = default_tree(lv) if pairs is None else pairs
    root, ex = sum_forward(lv, pairs)
    if root[0] <= 0:
        return -math.inf
    return math.log(root[0]) + ex * LN2


def marginals(net, evidence=None, mode="slice", pairs=None):
    """All single-variable marginals p(v | e) via the unity-vector adjoints
    (MAR algorithm; theorem thm:diff).  Returns (log Z, list of arrays,
    per-leaf adjoints, exponents, leaves)."""
    lv = build_leaves(net, evidence, mode)
    pairs = default_tree(lv) if pairs is None else pairs
    root, ex, adj, aexp = sum_forward(lv, pairs, want_adj=True)
    ev = np.full(net.n_vars, -1) if evidence is None else np.asarray(evidence)
    marg = [None] * net.n_vars
    for i, k in enumerate(lv.kind):
        if k != "unity":
            continue
        v = lv.var_of[i]
        w = adj[i] * lv.values[i]
        marg[v] = w / w.sum()
    for v in range(net.n_vars):
        if marg[v] is None:  # observed under slicing: one-hot
            m = np.zeros(int(net.card[v]))
            m[int(ev[v])] = 1.0
            marg[v] = m
    lz = math.log(root[0]) + ex * LN2 if root[0] > 0 else -math.inf
    return lz, marg, adj, aexp, lv


def map_assignment(net, evidence=None, mode="slice", pairs=None, fp32=False):
    """MPE (eq. log-map and the unity-vector readout): returns (log p(x*, e),
    assignment with the evidence filled in)."""
    lv = build_leaves(net, evidence, mode, domain="log")
    pairs = default_tree(lv) if pairs is None else pairs
    val, asg = max_forward(lv, pairs, fp32=fp32)
    if evidence is not None:
        ev = np.asarray(evidence)
        asg = np.where(ev >= 0, ev, asg).astype(np.int32)
    return val, asg


def log_joint(net, x) -> float:
    """Direct evaluation of sum_f log T_f(x_f) in FP64."""
    tot = 0.0
    for f in range(net.n_factors):
        t = factor_table(net, f, "log")
        tot += float(t[tuple(int(x[v]) for v in net.scopes[f])])
    return tot


def query_table(net, query, evidence=None, pairs=None):
    """log p(Q, e) as a table over the sorted query set (eq. evidence with
    the query labels as output)."""
    q = np.sort(np.asarray(query, np.int32))
    lv = build_leaves(net, evidence, "slice")
    if pairs is None:
        order = [v for v in min_degree_order(lv.labels, net.n_vars) if v not in set(q.tolist())]
        pairs = elimination_tree(lv.labels, lv.card, order)
    root, ex = sum_forward(lv, pairs, out=q)
    with np.errstate(divide="ignore"):
        return q, np.log(root) + ex * LN2


def mmap(net, query, evidence=None, pairs=None):
    """MMAP by its definition (eq. mmap): argmax over the query table; ties
    keep the smallest row-major index over the sorted query set.  Returns
    (value, assignment of the sorted query set, gap to the runner-up)."""
    q, table = query_table(net, query, evidence, pairs)
    flat = table.ravel()
    k = int(np.argmax(flat))
    srt = np.sort(flat)
    gap = float(srt[-1] - srt[-2]) if flat.size > 1 else math.inf
    idx = np.unravel_index(k, [int(net.card[v]) for v in q]) if len(q) else ()
    return float(flat[k]), np.asarray(idx, np.int32), gap


# ---------------------------------------------------------------------------
# Joint and factor marginals (MAR section: unity tensors over several
# variables; theorem thm:diff for the factors' own adjoints)
# ---------------------------------------------------------------------------

def add_joint_unity(leaves: Leaves, sets, evidence=None, mode: str = "slice") -> Leaves:
    """The leaves plus one unity tensor (all ones) per variable set, over the
    set's sorted variables (in slice mode its observed variables left out:
    they are not labels of the sliced network).  Appended after the other
    leaves, in the order of ``sets``; kind 'joint'."""
    n = len(leaves.card)
    ev = np.full(n, -1, np.int32) if evidence is None else np.asarray(evidence, np.int32)
    labels, values, kind = list(leaves.labels), list(leaves.values), list(leaves.kind)
    fo, vo = list(leaves.factor_of), list(leaves.var_of)
    for s in sets:
        lab = np.array(sorted(int(v) for v in s if not (mode == "slice" and ev[int(v)] >= 0)), np.int32)
        labels.append(lab)
        values.append(np.ones(int(np.prod(leaves.card[lab])) if lab.size else 1))
        kind.append("joint")
        fo.append(-1)
        vo.append(-1)
    return Leaves(leaves.card, labels, values, kind, fo, vo)


def joint_marginals(net, sets, evidence=None, mode="slice", pairs=None):
    """p(x_S | e) for every variable set S (sorted ascending; row-major,
    last variable fastest) from the adjoint of a unity tensor over S: with
    the unity tensor in the network Z is unchanged, and its adjoint is the
    contraction of everything else with S left open, i.e. p(x_S, e) up to
    the common factor.  Observed variables of S (slice mode) are one-hot.
    Returns (log Z, list of arrays shaped by the sorted set's cards)."""
    lv = add_joint_unity(build_leaves(net, evidence, mode), sets, evidence, mode)
    pairs = default_tree(lv) if pairs is None else pairs
    root, ex, adj, aexp = sum_forward(lv, pairs, want_adj=True)
    ev = np.full(net.n_vars, -1) if evidence is None else np.asarray(evidence)
    base = len(lv) - len(sets)
    out = []
    for k, s in enumerate(sets):
        srt = sorted(int(v) for v in s)
        free = [v for v in srt if not (mode == "slice" and ev[v] >= 0)]
        w = adj[base + k] * lv.values[base + k]
        w = w / w.sum()
        full = np.zeros([int(net.card[v]) for v in srt])
        idx = tuple(int(ev[v]) if (mode == "slice" and ev[v] >= 0) else slice(None) for v in srt)
        full[idx] = w.reshape([int(net.card[v]) for v in free]) if free else w[0]
        out.append(full)
    lz = math.log(root[0]) + ex * LN2 if root[0] > 0 else -math.inf
    return lz, out


def factor_marginals(net, evidence=None, mode="slice", pairs=None):
    """p(x_f | e) over every factor's scope (theorem thm:diff: the factor's
    adjoint is dZ/dT_f, so T_f * Tbar_f / Z sums to one over the scope).
    Each result is flattened in the factor's scope order as loaded (last
    variable fastest), with zeros where an observed variable (slice mode)
    takes another value.  Returns (log Z, list of flat arrays)."""
    lv = build_leaves(net, evidence, mode)
    pairs = default_tree(lv) if pairs is None else pairs
    root, ex, adj, aexp = sum_forward(lv, pairs, want_adj=True)
    ev = np.full(net.n_vars, -1) if evidence is None else np.asarray(evidence)
    out = [None] * net.n_factors
    for i, k in enumerate(lv.kind):
        if k != "factor":
            continue
        f = lv.factor_of[i]
        s = [int(v) for v in net.scopes[f]]
        free_sorted = [int(v) for v in lv.labels[i]]
        w = adj[i] * lv.values[i]
        w = w / w.sum()
        # sorted free labels -> scope order, observed axes one-hot
        t = w.reshape([int(net.card[v]) for v in free_sorted]) if free_sorted else w.reshape(())
        perm = [free_sorted.index(v) for v in s if v in free_sorted]
        t = np.transpose(t, perm) if free_sorted else t
        full = np.zeros([int(net.card[v]) for v in s])
        idx = tuple(int(ev[v]) if (mode == "slice" and ev[v] >= 0) else slice(None) for v in s)
        full[idx] = t
        out[f] = full.ravel()
    lz = math.log(root[0]) + ex * LN2 if root[0] > 0 else -math.inf
    return lz, out
