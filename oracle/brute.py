"""Brute-force enumeration (FP64) of the plain definitions, for tiny models.

TEST INFRASTRUCTURE ONLY.  These are the definitions written out over the
full joint table, with no contraction order at all:

* p(e) = sum over all free assignments of the product of the factors
  (eq. pr);
* p(v | e) = p(v, e) / p(e) by summing the joint table (eq. mar-prob);
* the MPE value and the set of maximisers of sum_f log T_f (eq. log-map);
* MMAP: argmax over q of sum over the rest (eq. mmap).

Feasible up to about 2^22 joint states.
"""
from __future__ import annotations

import math

import numpy as np

from . import factor_table


def joint_log_table(net, evidence=None) -> np.ndarray:
    """log of the unnormalised joint over all variables (observed variables
    restricted to their value, so their axis has length one)."""
    n = net.n_vars
    ev = np.full(n, -1) if evidence is None else np.asarray(evidence)
    shape = [1 if ev[v] >= 0 else int(net.card[v]) for v in range(n)]
    if int(np.prod(shape)) > (1 << 23):
        raise ValueError("brute force limited to 2^23 states")
    tab = np.zeros(shape)
    for f in range(net.n_factors):
        s = [int(v) for v in net.scopes[f]]
        t = factor_table(net, f, "log")
        idx = tuple(slice(int(ev[v]), int(ev[v]) + 1) if ev[v] >= 0 else slice(None) for v in s)
        t = t[idx]
        # move axes into variable order and broadcast
        order = np.argsort(s)
        t = np.transpose(t, order)
        full = [1] * n
        for v, d in zip(sorted(s), t.shape):
            full[v] = d
        tab = tab + t.reshape(full)
    return tab


def log_z(net, evidence=None) -> float:
    t = joint_log_table(net, evidence)
    m = np.max(t)
    if not np.isfinite(m):
        return -math.inf
    return float(m + math.log(np.sum(np.exp(t - m))))


def marginals(net, evidence=None):
    t = joint_log_table(net, evidence)
    m = np.max(t)
    p = np.exp(t - m)
    z = p.sum()
    out = []
    ev = np.full(net.n_vars, -1) if evidence is None else np.asarray(evidence)
    for v in range(net.n_vars):
        axes = tuple(a for a in range(net.n_vars) if a != v)
        mv = p.sum(axis=axes) / z
        if ev[v] >= 0:
            full = np.zeros(int(net.card[v]))
            full[int(ev[v])] = 1.0
            mv = full
        out.append(mv)
    return out


def map_set(net, evidence=None, tol: float = 0.0):
    """(best value, list of maximising assignments within tol, runner-up
    gap)."""
    t = joint_log_table(net, evidence)
    flat = t.ravel()
    best = float(np.max(flat))
    ev = np.full(net.n_vars, -1) if evidence is None else np.asarray(evidence)
    hits = np.nonzero(flat >= best - tol)[0]
    sols = []
    for h in hits:
        idx = np.unravel_index(int(h), t.shape)
        x = np.array([int(ev[v]) if ev[v] >= 0 else int(idx[v]) for v in range(net.n_vars)], np.int32)
        sols.append(x)
    srt = np.sort(flat)
    gap = float(srt[-1] - srt[-2]) if flat.size > 1 else math.inf
    return best, sols, gap


def mmap(net, query, evidence=None):
    """(value, assignment of the sorted query set, gap to runner-up)."""
    q = sorted(int(v) for v in query)
    t = joint_log_table(net, evidence)
    axes = tuple(a for a in range(net.n_vars) if a not in q)
    m = np.max(t)
    qt = np.log(np.exp(t - m).sum(axis=axes)) + m if axes else t
    flat = qt.ravel()
    k = int(np.argmax(flat))
    srt = np.sort(flat)
    gap = float(srt[-1] - srt[-2]) if flat.size > 1 else math.inf
    ev = np.full(net.n_vars, -1) if evidence is None else np.asarray(evidence)
    idx = np.unravel_index(k, qt.shape)
    return float(flat[k]), np.asarray(idx, np.int32), gap


def joint_marginal(net, variables, evidence=None):
    """p(x_S | e) over the sorted set S by summing the joint table over every
    other variable; observed variables of S are one-hot."""
    s = sorted(int(v) for v in variables)
    t = joint_log_table(net, evidence)
    m = np.max(t)
    p = np.exp(t - m)
    p /= p.sum()
    axes = tuple(a for a in range(net.n_vars) if a not in s)
    q = p.sum(axis=axes) if axes else p
    ev = np.full(net.n_vars, -1) if evidence is None else np.asarray(evidence)
    full = np.zeros([int(net.card[v]) for v in s])
    idx = tuple(slice(int(ev[v]), int(ev[v]) + 1) if ev[v] >= 0 else slice(None) for v in s)
    full[idx] = q
    return full
