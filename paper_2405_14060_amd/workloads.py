"""Seeded synthetic workloads shaped like the paper's problem families.

This module only draws inputs: factor tables, evidence sets and query sets.
It holds none of the contraction arithmetic, so both the HIP path and the
reference implementation under ``oracle/`` consume the same instances without
sharing any of the method's code.

The paper benchmarks on UAI 2014 problem sets (section "Performance
benchmarks"); those files are not available here.  The generators below are
synthetic stand-ins with the same structure: grid Markov random fields, sparse
Bayesian networks with small domains and observed variables, and random
regular graphs for MMAP.  Every generator takes a seed and uses numpy's PCG64.

Factor convention (the paper's definition of a tensor as a map from the joint
domain of its scope to the element set): ``values[f]`` is the table of factor
``f`` flattened row-major over ``scopes[f]`` in the order given, last variable
fastest.  ``is_log`` tells whether the tables hold log-potentials.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Network:
    """A factorised model p(x) proportional to the product of factor tables."""

    card: np.ndarray                     # int32 [n_vars]
    scopes: list                         # list of int32 arrays
    values: list                         # list of float64 arrays (row-major over scope)
    is_log: bool = False
    meta: dict = field(default_factory=dict)

    @property
    def n_vars(self) -> int:
        return int(self.card.shape[0])

    @property
    def n_factors(self) -> int:
        return len(self.scopes)

    def flat(self):
        """CSR view: (scope_ptr int64, scope_vars int32, value_ptr int64, values float64)."""
        sp = np.zeros(self.n_factors + 1, dtype=np.int64)
        vp = np.zeros(self.n_factors + 1, dtype=np.int64)
        for f, s in enumerate(self.scopes):
            sp[f + 1] = sp[f] + len(s)
            vp[f + 1] = vp[f] + len(self.values[f])
        sv = (np.concatenate([np.asarray(s, np.int32) for s in self.scopes])
              if self.n_factors else np.zeros(0, np.int32))
        vals = (np.concatenate([np.asarray(v, np.float64) for v in self.values])
                if self.n_factors else np.zeros(0, np.float64))
        return sp, sv.astype(np.int32), vp, vals


# ---------------------------------------------------------------------------
# Markov random fields
# ---------------------------------------------------------------------------

def grid_mrf(rows: int, cols: int, seed: int, unary_sd: float = 0.5,
             pair_sd: float = 1.0, card: int = 2) -> Network:
    """Pairwise grid MRF with Gaussian log-potentials (binary by default).

    Variable (r, c) has id r*cols + c.  Factors, in this order: one unary
    table per variable (``card`` entries ~ N(0, unary_sd)), one card x card
    table per horizontal edge (r,c)-(r,c+1), then one per vertical edge
    (r,c)-(r+1,c) (i.i.d. entries ~ N(0, pair_sd)).  ``unary_sd`` is a
    standard deviation.
    """
    rng = np.random.default_rng(seed)
    n = rows * cols
    scopes, values = [], []
    for v in range(n):
        scopes.append(np.array([v], np.int32))
        values.append(rng.normal(0.0, unary_sd, card))
    for r in range(rows):
        for c in range(cols - 1):
            scopes.append(np.array([r * cols + c, r * cols + c + 1], np.int32))
            values.append(rng.normal(0.0, pair_sd, card * card))
    for r in range(rows - 1):
        for c in range(cols):
            scopes.append(np.array([r * cols + c, (r + 1) * cols + c], np.int32))
            values.append(rng.normal(0.0, pair_sd, card * card))
    return Network(np.full(n, card, np.int32), scopes, values, True,
                   dict(kind="grid", rows=rows, cols=cols, seed=seed,
                        unary_sd=unary_sd, pair_sd=pair_sd, card=card))


def random_regular3(n: int, seed: int, pair_sd: float = 1.0,
                    n_query: int = 0) -> Network:
    """Random 3-regular graph on n binary variables, pairwise log-potentials.

    The graph is drawn with the pairing (configuration) model, rejecting
    pairings with self-loops or repeated edges.  Each edge gets a 2x2 table
    of i.i.d. N(0, pair_sd) log-potentials; there are no unary factors.
    ``meta['query']`` holds ``n_query`` variables drawn uniformly without
    replacement (sorted), the max variables of an MMAP query.
    """
    if (3 * n) % 2:
        raise ValueError("3-regular graph needs an even vertex count")
    rng = np.random.default_rng(seed)
    while True:
        stubs = np.repeat(np.arange(n), 3)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        if np.any(pairs[:, 0] == pairs[:, 1]):
            continue
        key = np.sort(pairs, axis=1)
        if len(np.unique(key, axis=0)) != len(key):
            continue
        break
    key = key[np.lexsort((key[:, 1], key[:, 0]))]
    scopes = [np.array(e, np.int32) for e in key]
    values = [rng.normal(0.0, pair_sd, 4) for _ in scopes]
    query = np.sort(rng.choice(n, size=n_query, replace=False)).astype(np.int32)
    return Network(np.full(n, 2, np.int32), scopes, values, True,
                   dict(kind="regular3", n=n, seed=seed, pair_sd=pair_sd,
                        query=query))


def chain_mrf(couplings, fields=None) -> Network:
    """Ising chain in spin variables s = 2x - 1 (x in {0,1}).

    Edge i carries log-potential J_i * s_i * s_{i+1}; an optional unary
    log-potential h_i * s_i.  Used by the closed-form checks.
    """
    J = np.asarray(couplings, np.float64)
    n = len(J) + 1
    scopes, values = [], []
    s = np.array([-1.0, 1.0])
    if fields is not None:
        for i, h in enumerate(np.asarray(fields, np.float64)):
            scopes.append(np.array([i], np.int32))
            values.append(h * s)
    for i, j in enumerate(J):
        scopes.append(np.array([i, i + 1], np.int32))
        values.append(j * np.outer(s, s).ravel())
    return Network(np.full(n, 2, np.int32), scopes, values, True,
                   dict(kind="chain", n=n))


# ---------------------------------------------------------------------------
# Bayesian networks
# ---------------------------------------------------------------------------

def random_bn(n: int, seed: int, window: int = 20, max_parents: int = 3,
              cards=(2, 3, 4)) -> Network:
    """Random Bayesian network with Dirichlet(1) conditional tables.

    Variables are in topological order by id.  Each variable draws its
    domain size uniformly from ``cards`` and a parent count uniformly from
    {0..max_parents} (capped by the candidates available); parents are drawn
    uniformly without replacement from the previous ``window`` variables.
    Each conditional table holds one Dirichlet(1,...,1) draw per parent
    configuration.  Scope order is (sorted parents..., child), child fastest.
    """
    rng = np.random.default_rng(seed)
    card = rng.choice(np.asarray(cards), size=n).astype(np.int32)
    scopes, values, parents = [], [], []
    for v in range(n):
        lo = max(0, v - window)
        k = int(rng.integers(0, max_parents + 1))
        k = min(k, v - lo)
        par = np.sort(rng.choice(np.arange(lo, v), size=k, replace=False)) if k else np.zeros(0, np.int64)
        par = par.astype(np.int32)
        n_rows = int(np.prod(card[par])) if k else 1
        cpt = rng.dirichlet(np.ones(card[v]), size=n_rows)
        scopes.append(np.concatenate([par, [v]]).astype(np.int32))
        values.append(cpt.ravel())
        parents.append(par)
    return Network(card, scopes, values, False,
                   dict(kind="bn", n=n, seed=seed, window=window,
                        max_parents=max_parents, parents=parents))


def ancestral_sample(bn: Network, rng: np.random.Generator) -> np.ndarray:
    """One joint draw from a Bayesian network (variables in id order)."""
    x = np.zeros(bn.n_vars, np.int32)
    for v in range(bn.n_vars):
        par = bn.meta["parents"][v]
        row = 0
        for p in par:
            row = row * int(bn.card[p]) + int(x[p])
        cv = int(bn.card[v])
        probs = bn.values[v][row * cv:(row + 1) * cv]
        x[v] = int(rng.choice(cv, p=probs / probs.sum()))
    return x


def bn_evidence(bn: Network, seed: int, frac: float = 0.1):
    """Fixed observed set: round(frac*n) variables, values from one ancestral draw.

    Returns (observed ids sorted int32, evidence int32[n_vars] with -1 = free).
    """
    rng = np.random.default_rng(seed)
    n = bn.n_vars
    k = int(round(frac * n))
    obs = np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32)
    x = ancestral_sample(bn, rng)
    ev = np.full(n, -1, np.int32)
    ev[obs] = x[obs]
    return obs, ev


def bn_evidence_batch(bn: Network, batch: int, seed: int,
                      frac_lo: float = 0.05, frac_hi: float = 0.20) -> np.ndarray:
    """Batch of evidence sets: per set f ~ U[frac_lo, frac_hi], round(f*n)
    observed variables drawn uniformly, values from a fresh ancestral draw.
    Returns int32 [batch, n_vars] with -1 = free."""
    rng = np.random.default_rng(seed)
    n = bn.n_vars
    out = np.full((batch, n), -1, np.int32)
    for b in range(batch):
        f = rng.uniform(frac_lo, frac_hi)
        k = int(round(f * n))
        obs = rng.choice(n, size=k, replace=False)
        x = ancestral_sample(bn, rng)
        out[b, obs] = x[obs]
    return out


def three_factor_net(n_b: int, n_m: int, n_s: int, n_n: int, card: int, seed: int,
                     sd: float = 1.0) -> Network:
    """Three factors X(B, M, S), Y(B, S, N), Z(B, M, N) over binary batch
    variables B and `card`-valued row (M), summed (S) and column (N)
    variables, i.i.d. N(0, sd) log-potentials: a network whose first
    contraction is one large dense product (batched matrix product, or its
    max-plus counterpart for MAP).  Variable ids: B, then M, S, N."""
    rng = np.random.default_rng(seed)
    c = np.array([2] * n_b + [card] * (n_m + n_s + n_n), np.int32)
    ids = np.arange(c.size)
    B, M = ids[:n_b], ids[n_b:n_b + n_m]
    S, N = ids[n_b + n_m:n_b + n_m + n_s], ids[n_b + n_m + n_s:]
    scopes = [np.concatenate(g).astype(np.int32) for g in ((B, M, S), (B, S, N), (B, M, N))]
    values = [rng.normal(0.0, sd, int(np.prod(c[sc]))) for sc in scopes]
    return Network(c, scopes, values, True, dict(kind="three_factor", seed=seed))


def bn_evidence_shared(bn: Network, batch: int, seed: int, frac: float = 0.1):
    """Batch of evidence sets sharing one observed set: round(frac*n)
    variables drawn uniformly once, values from a fresh ancestral draw per
    set.  Returns (observed ids sorted int32, int32 [batch, n_vars], -1 = free)."""
    rng = np.random.default_rng(seed)
    n = bn.n_vars
    obs = np.sort(rng.choice(n, size=int(round(frac * n)), replace=False)).astype(np.int32)
    out = np.full((batch, n), -1, np.int32)
    for b in range(batch):
        x = ancestral_sample(bn, rng)
        out[b, obs] = x[obs]
    return obs, out


def random_small_mrf(n: int, n_factors: int, seed: int, max_arity: int = 3,
                     cards=(2, 3)) -> Network:
    """Small random factor graph with mixed domain sizes, for exhaustive checks.

    Factor scopes are random subsets (arity 1..max_arity, unsorted order);
    entries are exp(N(0,1)) stored linearly, a few set to exactly zero is not
    done so that every configuration has positive weight.
    """
    rng = np.random.default_rng(seed)
    card = rng.choice(np.asarray(cards), size=n).astype(np.int32)
    scopes, values = [], []
    for _ in range(n_factors):
        a = int(rng.integers(1, max_arity + 1))
        s = rng.choice(n, size=min(a, n), replace=False).astype(np.int32)
        scopes.append(s)
        values.append(np.exp(rng.normal(0.0, 1.0, int(np.prod(card[s])))))
    return Network(card, scopes, values, False, dict(kind="small", n=n, seed=seed))


# ---------------------------------------------------------------------------
# The five workload configurations
# ---------------------------------------------------------------------------

def config(idx: int, seed: int = 0, small: bool = False) -> dict:
    """Instance for workload ``idx`` (0..4); ``small`` shrinks 3 and 4 for CI."""
    if idx == 0:
        return dict(name="grid4x4_mrf", net=grid_mrf(4, 4, seed))
    if idx == 1:
        return dict(name="grid20x20_mrf", net=grid_mrf(20, 20, seed))
    if idx == 2:
        bn = random_bn(300, seed)
        obs, ev = bn_evidence(bn, seed + 1000, 0.1)
        return dict(name="bn300_map", net=bn, observed=obs, evidence=ev)
    if idx == 3:
        n, batch = (120, 16) if small else (500, 512)
        bn = random_bn(n, seed)
        ev = bn_evidence_batch(bn, batch, seed + 2000)
        return dict(name="bn%d_batched%d" % (n, batch), net=bn, evidence=ev)
    if idx == 4:
        n, q = (40, 8) if small else (220, 25)
        net = random_regular3(n, seed, n_query=q)
        return dict(name="regular3_%d_mmap" % n, net=net, query=net.meta["query"])
    raise ValueError(idx)
