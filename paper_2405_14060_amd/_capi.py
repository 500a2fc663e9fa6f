"""ctypes binding of libtn (argument marshalling only).

Every step of inference runs inside libtn's HIP kernels; this module converts
numpy arrays to pointers and status codes to exceptions.  It raises if the
library is not built -- there is no fallback path.

torch, when importable, is imported before the library is opened so that the
process holds a single HIP runtime (torch's copy satisfies libtn's
dependency by soname) and device pointers of torch tensors are valid in libtn.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

try:  # share torch's HIP runtime when torch is present
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtn.so")

TN_OK, TN_E_INVALID, TN_E_NOMEM, TN_E_DEVICE, TN_E_TOO_LARGE, TN_E_ZERO_EVIDENCE, TN_E_UNSUPPORTED = range(7)
TN_F32, TN_BF16, TN_F16 = 0, 1, 2
SUM_PRODUCT, MAX_PLUS = 1, 2
EVIDENCE_NONE, EVIDENCE_SLICED, EVIDENCE_INDICATOR = 0, 1, 2
LAYOUT_AUTO, LAYOUT_INSTANCE_MAJOR, LAYOUT_INTERLEAVED = 0, 1, 2
PLANNER_BEST, PLANNER_GREEDY, PLANNER_MINFILL, PLANNER_NATURAL, PLANNER_MINDEG = range(5)

EXPORTS = ["tn_plan_opts_default", "tn_load_network", "tn_free_network", "tn_plan", "tn_free_plan",
           "tn_plan_info_get", "tn_plan_tree", "tn_plan_sliced", "tn_plan_tree_host", "tn_logZ", "tn_marginals",
           "tn_map", "tn_mmap", "tn_sample", "tn_logZ_dev", "tn_sync", "tn_profile", "tn_profile_kind", "tn_last_error",
           "tn_tune_save", "tn_tune_load", "tn_tune_clear", "tn_sample_noalloc", "tn_joint_marginals",
           "tn_factor_marginals", "tn_load_uai", "tn_read_uai_evidence", "tn_read_uai_query", "tn_network_sizes",
           "tn_network_get", "tn_plan_ops"]

i32p = ctypes.POINTER(ctypes.c_int32)
i64p = ctypes.POINTER(ctypes.c_int64)
f64p = ctypes.POINTER(ctypes.c_double)
f32p = ctypes.POINTER(ctypes.c_float)


class PlanOpts(ctypes.Structure):
    _fields_ = [("semiring_mask", ctypes.c_int32), ("evidence_mode", ctypes.c_int32),
                ("observed", i32p), ("n_observed", ctypes.c_int32),
                ("query", i32p), ("n_query", ctypes.c_int32),
                ("planner", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("max_log2_size", ctypes.c_double),
                ("dtype", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("hip_stream", ctypes.c_void_p),
                ("tree_pairs", i32p), ("n_tree_pairs", ctypes.c_int32),
                ("want_factor_grad", ctypes.c_int32), ("host_only", ctypes.c_int32),
                ("no_fuse", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("batch_layout", ctypes.c_int32), ("joint_ptr", i64p), ("joint_vars", i32p),
                ("n_joint", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_leaves", ctypes.c_int32), ("n_nodes", ctypes.c_int32),
                ("n_kernels_fwd", ctypes.c_int32), ("n_kernels_bwd", ctypes.c_int32),
                ("n_kernels_max", ctypes.c_int32), ("sc", ctypes.c_double),
                ("sc_union", ctypes.c_double), ("tc", ctypes.c_double),
                ("flops_fwd", ctypes.c_double), ("bytes_fwd", ctypes.c_double),
                ("n_sliced", ctypes.c_int32), ("planner_used", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("n_launches_fwd", ctypes.c_int32),
                ("n_launches_bwd", ctypes.c_int32), ("n_launches_max", ctypes.c_int32),
                ("n_segments", ctypes.c_int32), ("n_fused_nodes", ctypes.c_int32),
                ("n_dense", ctypes.c_int32), ("n_wave", ctypes.c_int32),
                ("n_interleaved", ctypes.c_int32), ("batch_stride", ctypes.c_int32),
                ("n_dense_large", ctypes.c_int32), ("two_front", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("n_pairs", ctypes.c_int32),
                ("n_pairs_moved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class OpProfile(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("flops", ctypes.c_double), ("bytes", ctypes.c_double),
                ("ms", ctypes.c_double)]


class OpInfo(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("semiring", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("summed", ctypes.c_int64),
                ("x_size", ctypes.c_int64), ("y_size", ctypes.c_int64), ("z_size", ctypes.c_int64),
                ("eligible", ctypes.c_int32)]


class TNError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("libtn status %d: %s" % (status, msg))
        self.status = status


_lib = None


def lib():
    """Open libtn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libtn.so is not built (run paper_2405_14060_amd.build.build() "
                           "or __graft_entry__.build()); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.tn_last_error.restype = ctypes.c_char_p
    L.tn_plan_opts_default.argtypes = [ctypes.POINTER(PlanOpts)]
    L.tn_plan_opts_default.restype = None
    L.tn_load_network.argtypes = [ctypes.c_int32, i32p, ctypes.c_int32, i64p, i32p, f64p,
                                  ctypes.c_int32, ctypes.POINTER(vp)]
    L.tn_free_network.argtypes = [vp]
    L.tn_free_network.restype = None
    L.tn_plan.argtypes = [vp, ctypes.POINTER(PlanOpts), ctypes.POINTER(vp)]
    L.tn_free_plan.argtypes = [vp]
    L.tn_free_plan.restype = None
    L.tn_plan_info_get.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    L.tn_plan_tree.argtypes = [vp, i32p, ctypes.c_int32, i32p, i32p]
    L.tn_plan_sliced.argtypes = [vp, i32p, ctypes.c_int32, i32p]
    L.tn_plan_tree_host.argtypes = [vp, ctypes.POINTER(PlanOpts), i32p, ctypes.c_int32, i32p, i32p,
                                    ctypes.POINTER(PlanInfo)]
    L.tn_logZ.argtypes = [vp, ctypes.c_int32, i32p, f64p]
    L.tn_marginals.argtypes = [vp, ctypes.c_int32, i32p, f64p, f64p]
    L.tn_map.argtypes = [vp, ctypes.c_int32, i32p, i32p, f64p]
    L.tn_joint_marginals.argtypes = [vp, ctypes.c_int32, i32p, f64p, f64p]
    L.tn_factor_marginals.argtypes = [vp, ctypes.c_int32, i32p, f64p, f64p]
    L.tn_mmap.argtypes = [vp, i32p, i32p, f64p]
    L.tn_sample.argtypes = [vp, i32p, ctypes.c_int64, ctypes.c_uint64, i32p]
    L.tn_sample_noalloc.argtypes = [vp, i32p, ctypes.c_int64, ctypes.c_uint64, i32p]
    L.tn_logZ_dev.argtypes = [vp, i32p, vp, vp, vp]
    L.tn_sync.argtypes = [vp]
    L.tn_profile.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, i32p, ctypes.c_int32,
                             ctypes.POINTER(OpProfile), ctypes.c_int32, i32p]
    L.tn_profile_kind.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, i32p, ctypes.c_int32,
                                  ctypes.POINTER(OpProfile), i32p]
    L.tn_load_uai.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
    L.tn_read_uai_evidence.argtypes = [ctypes.c_char_p, ctypes.c_int32, i32p, i32p, ctypes.c_int32, i32p]
    L.tn_read_uai_query.argtypes = [ctypes.c_char_p, ctypes.c_int32, i32p, ctypes.c_int32, i32p]
    L.tn_network_sizes.argtypes = [vp, i32p, i32p, i64p, i64p]
    L.tn_network_get.argtypes = [vp, i32p, i64p, i32p, f64p, i32p]
    L.tn_plan_ops.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(OpInfo), ctypes.c_int32, i32p]
    L.tn_tune_save.argtypes = [ctypes.c_char_p, i64p]
    L.tn_tune_load.argtypes = [ctypes.c_char_p, i64p]
    L.tn_tune_clear.argtypes = []
    L.tn_tune_clear.restype = None
    for name in ("tn_plan_ops", "tn_load_uai", "tn_read_uai_evidence", "tn_read_uai_query", "tn_network_sizes", "tn_network_get",
                 "tn_tune_save", "tn_tune_load", "tn_load_network", "tn_plan", "tn_plan_info_get", "tn_plan_tree", "tn_plan_sliced", "tn_plan_tree_host",
                 "tn_logZ", "tn_marginals", "tn_joint_marginals", "tn_factor_marginals", "tn_map", "tn_mmap",
                 "tn_sample", "tn_sample_noalloc", "tn_logZ_dev", "tn_sync",
                 "tn_profile", "tn_profile_kind"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(st):
    if st != TN_OK:
        raise TNError(st, lib().tn_last_error().decode())


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct)) if a is not None else None


def tune_save(path) -> int:
    """Write the process's autotuner decisions to a file; returns their count."""
    n = ctypes.c_int64()
    _check(lib().tn_tune_save(os.fsencode(path), ctypes.byref(n)))
    return n.value


def tune_load(path) -> int:
    """Add autotuner decisions from a file written by tune_save; returns their count."""
    n = ctypes.c_int64()
    _check(lib().tn_tune_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


def tune_clear() -> None:
    """Forget every autotuner decision held by the process."""
    lib().tn_tune_clear()


class Network:
    """A model loaded into libtn (copy of the factor tables)."""

    @classmethod
    def from_uai(cls, path):
        """Load a UAI-format model file (MARKOV or BAYES) through tn_load_uai."""
        h = ctypes.c_void_p()
        _check(lib().tn_load_uai(os.fsencode(path), ctypes.byref(h)))
        self = cls.__new__(cls)
        self.h = h
        self._read_back()
        return self

    def _read_back(self):
        """Fill src, card and sizes from the library's copy of the model."""
        from . import workloads as W
        nv, nf, ns, nvals = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().tn_network_sizes(self.h, ctypes.byref(nv), ctypes.byref(nf), ctypes.byref(ns), ctypes.byref(nvals)))
        card = np.zeros(max(1, nv.value), np.int32)
        sp = np.zeros(nf.value + 1, np.int64)
        sv = np.zeros(max(1, ns.value), np.int32)
        vals = np.zeros(max(1, nvals.value))
        is_log = ctypes.c_int32()
        _check(lib().tn_network_get(self.h, _ptr(card, ctypes.c_int32), _ptr(sp, ctypes.c_int64),
                                    _ptr(sv, ctypes.c_int32), _ptr(vals, ctypes.c_double), ctypes.byref(is_log)))
        card = card[:nv.value]
        scopes = [sv[sp[f]:sp[f + 1]].copy() for f in range(nf.value)]
        vp = np.concatenate([[0], np.cumsum([int(np.prod(card[s])) if len(s) else 1 for s in scopes])]).astype(np.int64)
        values = [vals[vp[f]:vp[f + 1]].copy() for f in range(nf.value)]
        self.src = W.Network(card.copy(), scopes, values, bool(is_log.value))
        self.card = np.ascontiguousarray(card, np.int32)
        self.n_vars = int(nv.value)
        self.n_values = int(nvals.value)
        self.value_offsets = vp

    def read_uai_evidence(self, path):
        """Evidence sets of a UAI evidence file: int32 [sets, n_vars], -1 = free."""
        n = ctypes.c_int32()
        _check(lib().tn_read_uai_evidence(os.fsencode(path), self.n_vars, _ptr(self.card, ctypes.c_int32), None, 0,
                                          ctypes.byref(n)))
        ev = np.full((max(1, n.value), max(1, self.n_vars)), -1, np.int32)
        _check(lib().tn_read_uai_evidence(os.fsencode(path), self.n_vars, _ptr(self.card, ctypes.c_int32),
                                          _ptr(ev, ctypes.c_int32), n.value, ctypes.byref(n)))
        return ev[:n.value, :self.n_vars]

    def read_uai_query(self, path):
        """Variables of a UAI query file (in file order)."""
        buf = np.zeros(max(1, self.n_vars), np.int32)
        n = ctypes.c_int32()
        _check(lib().tn_read_uai_query(os.fsencode(path), self.n_vars, _ptr(buf, ctypes.c_int32), buf.size,
                                       ctypes.byref(n)))
        return buf[:n.value].copy()

    def __init__(self, net):
        self.src = net
        sp, sv, vp, vals = net.flat()
        self.card = np.ascontiguousarray(net.card, np.int32)
        self.n_vars = int(self.card.shape[0])
        self.n_values = int(vals.size)
        self.value_offsets = vp
        h = ctypes.c_void_p()
        _check(lib().tn_load_network(self.n_vars, _ptr(self.card, ctypes.c_int32), net.n_factors,
                                     _ptr(sp, ctypes.c_int64), _ptr(sv if sv.size else np.zeros(1, np.int32), ctypes.c_int32),
                                     _ptr(vals if vals.size else np.zeros(1), ctypes.c_double),
                                     1 if net.is_log else 0, ctypes.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.tn_free_network(self.h)
            self.h = None


def make_opts(semirings=SUM_PRODUCT | MAX_PLUS, evidence_mode=EVIDENCE_NONE, observed=None,
              query=None, planner=PLANNER_BEST, restarts=4, seed=0, max_log2_size=0.0,
              dtype=TN_F32, max_batch=1, use_graph=True, stream=None, tree=None,
              want_factor_grad=False, host_only=False, fuse=True, autotune=False, batch_layout=0,
              joint_sets=None, pair_segments=True):
    o = PlanOpts()
    lib().tn_plan_opts_default(ctypes.byref(o))
    keep = []
    o.semiring_mask = semirings
    o.evidence_mode = evidence_mode
    if observed is not None:
        obs = np.ascontiguousarray(observed, np.int32)
        keep.append(obs)
        o.observed = _ptr(obs, ctypes.c_int32)
        o.n_observed = int(obs.size)
    if query is not None and len(query):
        q = np.ascontiguousarray(query, np.int32)
        keep.append(q)
        o.query = _ptr(q, ctypes.c_int32)
        o.n_query = int(q.size)
    o.planner = planner
    o.restarts = restarts
    o.seed = seed
    o.max_log2_size = max_log2_size
    o.dtype = dtype
    o.max_batch = max_batch
    o.use_graph = 1 if use_graph else 0
    o.hip_stream = stream
    if tree is not None:
        t = np.ascontiguousarray(np.asarray(tree, np.int32).reshape(-1, 2))
        keep.append(t)
        o.tree_pairs = _ptr(t, ctypes.c_int32)
        o.n_tree_pairs = int(t.shape[0])
    o.want_factor_grad = 1 if want_factor_grad else 0
    o.host_only = 1 if host_only else 0
    o.no_fuse = (0 if pair_segments else 2) if fuse else 1
    o.autotune = 1 if autotune else 0
    o.batch_layout = batch_layout
    if joint_sets:
        ptr = np.zeros(len(joint_sets) + 1, np.int64)
        for k, st in enumerate(joint_sets):
            ptr[k + 1] = ptr[k] + len(st)
        jv = np.ascontiguousarray(np.concatenate([np.asarray(st, np.int32) for st in joint_sets]), np.int32)
        keep += [ptr, jv]
        o.joint_ptr = _ptr(ptr, ctypes.c_int64)
        o.joint_vars = _ptr(jv, ctypes.c_int32)
        o.n_joint = len(joint_sets)
    return o, keep


def plan_tree_host(network: Network, **kw):
    """Planner only (no device): returns (pairs int32 [L-1,2], n_leaves, info dict)."""
    o, keep = make_opts(**kw)
    cap = 2 * (network.src.n_factors + network.n_vars + 4)
    buf = np.zeros(2 * cap, np.int32)
    n_pairs, n_leaves = ctypes.c_int32(), ctypes.c_int32()
    info = PlanInfo()
    _check(lib().tn_plan_tree_host(network.h, ctypes.byref(o), _ptr(buf, ctypes.c_int32), cap,
                                   ctypes.byref(n_pairs), ctypes.byref(n_leaves), ctypes.byref(info)))
    return buf[:2 * n_pairs.value].reshape(-1, 2).copy(), n_leaves.value, info.as_dict()


class Plan:
    """A compiled plan: contraction tree, kernel descriptors, device arena."""

    def __init__(self, network: Network, **kw):
        self.network = network
        self.kw = kw
        self.n_vars = network.n_vars
        self.card = network.card
        self.max_batch = kw.get("max_batch", 1)
        self.query = np.sort(np.asarray(kw.get("query") if kw.get("query") is not None else [], np.int32))
        o, keep = make_opts(**kw)
        h = ctypes.c_void_p()
        _check(lib().tn_plan(network.h, ctypes.byref(o), ctypes.byref(h)))
        self.h = h
        self.marg_cols = np.concatenate([[0], np.cumsum(self.card)]).astype(np.int64)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.tn_free_plan(self.h)
            self.h = None

    def info(self) -> dict:
        i = PlanInfo()
        _check(lib().tn_plan_info_get(self.h, ctypes.byref(i)))
        return i.as_dict()

    def tree(self):
        cap = 1 << 20
        buf = np.zeros(2 * cap, np.int32)
        n_pairs, n_leaves = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().tn_plan_tree(self.h, _ptr(buf, ctypes.c_int32), cap, ctypes.byref(n_pairs),
                                  ctypes.byref(n_leaves)))
        return buf[:2 * n_pairs.value].reshape(-1, 2).copy(), n_leaves.value

    def _ev(self, evidence, batch):
        if evidence is None:
            return np.full((batch, self.n_vars), -1, np.int32)
        ev = np.ascontiguousarray(np.asarray(evidence, np.int32).reshape(batch, self.n_vars))
        return ev

    def log_z(self, evidence=None, batch=1):
        ev = self._ev(evidence, batch)
        out = np.zeros(batch)
        _check(lib().tn_logZ(self.h, batch, _ptr(ev, ctypes.c_int32), _ptr(out, ctypes.c_double)))
        return out

    def marginals(self, evidence=None, batch=1):
        """Returns (log Z [batch], marginal rows [batch, sum card])."""
        ev = self._ev(evidence, batch)
        lz = np.zeros(batch)
        m = np.zeros((batch, int(self.marg_cols[-1])))
        _check(lib().tn_marginals(self.h, batch, _ptr(ev, ctypes.c_int32), _ptr(lz, ctypes.c_double),
                                  _ptr(m, ctypes.c_double)))
        return lz, m

    def split_marginals(self, row):
        return [row[self.marg_cols[v]:self.marg_cols[v + 1]] for v in range(self.n_vars)]

    def joint_marginals(self, evidence=None, batch=1):
        """Returns (log Z [batch], per instance a list of tables, one per joint
        set, shaped by the cards of the set's variables sorted ascending)."""
        sets = [sorted(int(v) for v in st) for st in self.kw.get("joint_sets") or []]
        sizes = [int(np.prod([int(self.card[v]) for v in st])) for st in sets]
        ev = self._ev(evidence, batch)
        lz = np.zeros(batch)
        out = np.zeros((batch, max(1, sum(sizes))))
        _check(lib().tn_joint_marginals(self.h, batch, _ptr(ev, ctypes.c_int32), _ptr(lz, ctypes.c_double),
                                        _ptr(out, ctypes.c_double)))
        res = []
        for b in range(batch):
            tabs, o = [], 0
            for st, n in zip(sets, sizes):
                tabs.append(out[b, o:o + n].reshape([int(self.card[v]) for v in st]))
                o += n
            res.append(tabs)
        return lz, res

    def factor_marginals(self, evidence=None, batch=1):
        """Returns (log Z [batch], [batch, n_values] factor marginals laid out
        as the network's values)."""
        ev = self._ev(evidence, batch)
        lz = np.zeros(batch)
        out = np.zeros((batch, max(1, self.network.n_values)))
        _check(lib().tn_factor_marginals(self.h, batch, _ptr(ev, ctypes.c_int32), _ptr(lz, ctypes.c_double),
                                         _ptr(out, ctypes.c_double)))
        return lz, out[:, :self.network.n_values]

    def split_factors(self, row):
        """A factor-marginal row split per factor (flat, scope order as loaded)."""
        vp = self.network.value_offsets
        return [row[vp[f]:vp[f + 1]] for f in range(len(vp) - 1)]

    def map(self, evidence=None, batch=1):
        ev = self._ev(evidence, batch)
        a = np.zeros((batch, self.n_vars), np.int32)
        lp = np.zeros(batch)
        _check(lib().tn_map(self.h, batch, _ptr(ev, ctypes.c_int32), _ptr(a, ctypes.c_int32),
                            _ptr(lp, ctypes.c_double)))
        return lp, a

    def mmap(self, evidence=None):
        ev = self._ev(evidence, 1)
        a = np.zeros(max(1, len(self.query)), np.int32)
        val = np.zeros(1)
        _check(lib().tn_mmap(self.h, _ptr(ev, ctypes.c_int32), _ptr(a, ctypes.c_int32),
                             _ptr(val, ctypes.c_double)))
        return float(val[0]), a[:len(self.query)]

    def sample(self, n, seed, evidence=None):
        ev = self._ev(evidence, 1)
        out = np.zeros((n, self.n_vars), np.int32)
        _check(lib().tn_sample(self.h, _ptr(ev, ctypes.c_int32), n, seed, _ptr(out, ctypes.c_int32)))
        return out

    def sample_noalloc(self, n, seed, evidence=None):
        """tn_sample with the device staging in the library's static array
        (no device allocation; n * n_vars <= 2^22)."""
        ev = self._ev(evidence, 1)
        out = np.zeros((n, self.n_vars), np.int32)
        _check(lib().tn_sample_noalloc(self.h, _ptr(ev, ctypes.c_int32), n, seed, _ptr(out, ctypes.c_int32)))
        return out

    def log_z_dev(self, values_ptr, logz_ptr, grad_ptr=None, evidence=None):
        ev = self._ev(evidence, 1)
        _check(lib().tn_logZ_dev(self.h, _ptr(ev, ctypes.c_int32), ctypes.c_void_p(values_ptr),
                                 ctypes.c_void_p(logz_ptr),
                                 ctypes.c_void_p(grad_ptr) if grad_ptr else None))

    def profile(self, task, reps=3, evidence=None, batch=1):
        """Per-launch (kind, flops, bytes, ms) of one task: 0 log Z, 1 marginals, 2 MAP."""
        ev = self._ev(evidence, batch)
        cap = 1 << 16
        buf = (OpProfile * cap)()
        n = ctypes.c_int32()
        _check(lib().tn_profile(self.h, task, batch, _ptr(ev, ctypes.c_int32), reps, buf, cap, ctypes.byref(n)))
        return [(buf[i].kind, buf[i].flops, buf[i].bytes, buf[i].ms) for i in range(min(n.value, cap))]

    def profile_kind(self, task, kind, reps=5, evidence=None, batch=1):
        """Launches of one kind timed back to back: (ms per launch, flops per
        launch, bytes per launch, launches per task)."""
        ev = self._ev(evidence, batch)
        o = OpProfile()
        n = ctypes.c_int32()
        _check(lib().tn_profile_kind(self.h, task, kind, batch, _ptr(ev, ctypes.c_int32), reps,
                                     ctypes.byref(o), ctypes.byref(n)))
        return o.ms, o.flops, o.bytes, n.value

    def ops(self, task):
        """Contractions of a task (0 forward, 1 reverse, 2 max-plus, 3 MMAP
        sum phase) as dicts of form, semiring, variant, label-class sizes and
        operand sizes."""
        n = ctypes.c_int32()
        _check(lib().tn_plan_ops(self.h, task, None, 0, ctypes.byref(n)))
        buf = (OpInfo * max(1, n.value))()
        _check(lib().tn_plan_ops(self.h, task, buf, n.value, ctypes.byref(n)))
        return [{k: getattr(buf[i], k) for k, _ in OpInfo._fields_} for i in range(n.value)]

    def sliced_vars(self):
        """Sliced variables (ascending); slices run over their values, last fastest."""
        buf = np.zeros(max(1, self.n_vars), np.int32)
        n = ctypes.c_int32()
        _check(lib().tn_plan_sliced(self.h, _ptr(buf, ctypes.c_int32), buf.size, ctypes.byref(n)))
        return buf[:n.value].copy()

    def sync(self):
        _check(lib().tn_sync(self.h))
