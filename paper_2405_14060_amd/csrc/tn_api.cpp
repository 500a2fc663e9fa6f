// libtn: C interface, plan construction and execution on one gfx950 GPU.
//
// A plan binds the model's leaves (factor tables, sliced by fixed evidence
// -- paper eq. pr -- plus one unity / indicator vector per variable, the
// auxiliary tensors of the MAR and MPE algorithms) to a binary contraction
// tree, assigns every tensor a slice of one device arena, and lowers every
// tree node to one launch of the generic contraction kernel:
//   forward sum-product  C = sum over eliminated labels of A * B
//   reverse pass         Abar = con(Cbar, B -> Va), Bbar = con(A, Cbar -> Vb)
//                        (eq. einback; leaves' adjoints give the marginals)
//   max-plus             private eliminated labels reduced first, then
//                        C = max_K (A' + B') with argmax indices, read out
//                        top-down (the tropical back-propagation of the MPE
//                        algorithm, realised as argmax backtracking).
// Every call's launches can be captured once into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include <functional>
#include <map>
#include <mutex>
#include <numeric>
#include <string>

#include "tn_plan.h"

using namespace tn;

static thread_local std::string g_err;

extern "C" const char *tn_last_error(void) { return g_err.c_str(); }
void tn::set_last_error(const std::string &m) { g_err = m; }

template <class F>
static tn_status guard(F &&f) {
  try {
    f();
    return TN_OK;
  } catch (const TnError &e) {
    g_err = e.what();
    return e.st;
  } catch (const std::bad_alloc &) {
    g_err = "host allocation failed";
    return TN_E_NOMEM;
  } catch (const std::exception &e) {
    g_err = e.what();
    return TN_E_INVALID;
  }
}

static void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) throw TnError(TN_E_NOMEM, std::string(what) + ": out of device memory");
    throw TnError(TN_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
}

// ---------------------------------------------------------------------------
// network
// ---------------------------------------------------------------------------
extern "C" tn_status tn_load_network(int32_t n_vars, const int32_t *card, int32_t n_factors,
                                     const int64_t *scope_ptr, const int32_t *scope_vars,
                                     const double *values, int32_t values_are_log, tn_net **out) {
  return guard([&] {
    if (!out) throw TnError(TN_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n_vars < 0 || n_factors < 0) throw TnError(TN_E_INVALID, "negative sizes");
    if (n_vars > 0 && !card) throw TnError(TN_E_INVALID, "card is NULL");
    if (n_factors > 0 && (!scope_ptr || !values)) throw TnError(TN_E_INVALID, "factor arrays are NULL");
    auto net = std::make_unique<tn_net>();
    net->n_vars = n_vars;
    net->card.assign(card, card + n_vars);
    for (int v = 0; v < n_vars; ++v)
      if (card[v] < 1) throw TnError(TN_E_INVALID, "domain size of variable " + std::to_string(v) + " < 1");
    net->is_log = values_are_log != 0;
    if (n_factors > 0 && scope_ptr[0] != 0) throw TnError(TN_E_INVALID, "scope_ptr[0] must be 0");
    int64_t voff = 0;
    for (int f = 0; f < n_factors; ++f) {
      if (scope_ptr[f + 1] < scope_ptr[f]) throw TnError(TN_E_INVALID, "scope_ptr not monotone");
      std::vector<int> s(scope_vars + scope_ptr[f], scope_vars + scope_ptr[f + 1]);
      int64_t sz = 1;
      std::vector<char> seen(n_vars, 0);
      for (int v : s) {
        if (v < 0 || v >= n_vars) throw TnError(TN_E_INVALID, "factor " + std::to_string(f) + " has a variable out of range");
        if (seen[v]) throw TnError(TN_E_INVALID, "factor " + std::to_string(f) + " repeats a variable");
        seen[v] = 1;
        sz *= card[v];
        if (sz > (int64_t(1) << 31)) throw TnError(TN_E_TOO_LARGE, "factor table too large");
      }
      std::vector<double> vals(values + voff, values + voff + sz);
      for (double x : vals) {
        if (std::isnan(x)) throw TnError(TN_E_INVALID, "factor " + std::to_string(f) + " has NaN");
        if (net->is_log ? (x == INFINITY) : (x < 0 || !std::isfinite(x)))
          throw TnError(TN_E_INVALID, "factor " + std::to_string(f) +
                                          (net->is_log ? " has +inf log-potential" : " has a negative or non-finite value"));
      }
      net->val_off.push_back(voff);
      voff += sz;
      net->scope.push_back(std::move(s));
      net->vals.push_back(std::move(vals));
    }
    net->n_values = voff;
    *out = net.release();
  });
}

extern "C" void tn_free_network(tn_net *net) { delete net; }

extern "C" void tn_plan_opts_default(tn_plan_opts *o) {
  std::memset(o, 0, sizeof *o);
  o->semiring_mask = TN_SUM_PRODUCT | TN_MAX_PLUS;
  o->evidence_mode = TN_EVIDENCE_NONE;
  o->planner = TN_PLANNER_BEST;
  o->restarts = 4;
  o->seed = 0;
  o->max_log2_size = 0;
  o->dtype = TN_F32;
  o->autotune = 0;
  o->batch_layout = 0;
  o->max_batch = 1;
  o->use_graph = 1;
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
static int64_t numel(const Labels &l, const std::vector<int> &card) {
  int64_t s = 1;
  for (int v : l) s *= card[v];
  return s;
}
static bool has(const Labels &l, int v) { return std::binary_search(l.begin(), l.end(), v); }
static Labels inter(const Labels &a, const Labels &b) {
  Labels o;
  std::set_intersection(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(o));
  return o;
}
static Labels minus(const Labels &a, const Labels &b) {
  Labels o;
  std::set_difference(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(o));
  return o;
}
static Labels unite(const Labels &a, const Labels &b) {
  Labels o;
  std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(o));
  return o;
}
// row-major stride of v in a tensor with sorted labels L (0 if absent)
static int64_t stride_in(const Labels &L, int v, const std::vector<int> &card) {
  int64_t s = 1;
  for (int i = (int)L.size() - 1; i >= 0; --i) {
    if (L[i] == v) return s;
    s *= card[L[i]];
  }
  return 0;
}

static int new_tensor(tn_plan_t *p, const Labels &lab, bool batched, bool scaled) {
  TensorBuf t;
  t.lab = lab;
  t.size = numel(lab, p->card);
  if (t.size >= (int64_t(1) << 31))
    throw TnError(TN_E_TOO_LARGE, "an intermediate tensor has 2^" +
                                      std::to_string(std::log2((double)t.size)) +
                                      " elements; set max_log2_size to slice the network");
  t.batched = batched;
  t.slot = scaled ? 0 : -1;  // real slot assigned at allocation
  p->T.push_back(t);
  return (int)p->T.size() - 1;
}
// a tensor without labels (per-solve scratch of fused segments)
static int new_raw_tensor(tn_plan_t *p, int64_t size, bool scaled) {
  TensorBuf t;
  t.size = size;
  t.slot = scaled ? 0 : -1;
  p->T.push_back(t);
  return (int)p->T.size() - 1;
}
static int new_intbuf(tn_plan_t *p, int64_t size, bool batched) {
  IntBuf b;
  b.size = size;
  b.batched = batched;
  p->IB.push_back(b);
  return (int)p->IB.size() - 1;
}

// split point of a class: trailing labels whose product is <= 1024
static size_t lo_split(const Labels &L, const std::vector<int> &card) {
  size_t s = L.size();
  int64_t prod = 1;
  while (s > 0 && prod * card[L[s - 1]] <= 1024) {
    prod *= card[L[s - 1]];
    --s;
  }
  if (s == L.size() && !L.empty()) s = L.size() - 1;  // a single label larger than 1024
  return s;
}

// append offset tables of class L (split at `split`) for tensor TL
static void add_tabs(tn_plan_t *p, const Labels &L, size_t split, const Labels &TL, int64_t out[2]) {
  const auto &card = p->card;
  Labels hi(L.begin(), L.begin() + split), lo(L.begin() + split, L.end());
  for (int part = 0; part < 2; ++part) {
    const Labels &P = part ? lo : hi;
    std::vector<int64_t> st(P.size());
    for (size_t j = 0; j < P.size(); ++j) st[j] = stride_in(TL, P[j], card);
    int64_t n = numel(P, card);
    out[part] = (int64_t)p->tabs.size();
    std::vector<int> d(P.size(), 0);
    int64_t off = 0;
    for (int64_t i = 0; i < n; ++i) {
      p->tabs.push_back((int32_t)off);
      for (int j = (int)P.size() - 1; j >= 0; --j) {
        if (++d[j] < card[P[j]]) {
          off += st[j];
          break;
        }
        off -= st[j] * (card[P[j]] - 1);
        d[j] = 0;
      }
    }
  }
}

// Lower one contraction Z = X (x) Y to a kernel descriptor.
static Op make_op(tn_plan_t *p, int semi, int X, int Y, int Z, int I) {
  Op op;
  op.semi = semi;
  op.X = X;
  op.Y = Y;
  op.Z = Z;
  op.I = I;
  const auto &card = p->card;
  const Labels &LX = p->T[X].lab, &LZ = p->T[Z].lab;
  const Labels LY = Y >= 0 ? p->T[Y].lab : Labels{};
  const Labels R = inter(LZ, LX), C = minus(LZ, LX), S = minus(unite(LX, LY), LZ);
  if (semi == SEMI_MAX && !minus(C, LY).empty()) throw TnError(TN_E_INVALID, "internal: broadcast in max-plus node");
  const size_t rs = lo_split(R, card), cs = lo_split(C, card), ss = lo_split(S, card);
  for (auto *t : {op.t_rX, op.t_rY, op.t_rZ, op.t_cY, op.t_cZ, op.t_sX, op.t_sY, op.t_gbX, op.t_gbY, op.t_gbZ,
                  op.t_gmX, op.t_gmZ, op.t_oX, op.t_oY})
    t[0] = t[1] = -1;
  add_tabs(p, R, rs, LX, op.t_rX);
  add_tabs(p, R, rs, LZ, op.t_rZ);
  add_tabs(p, C, cs, LZ, op.t_cZ);
  add_tabs(p, S, ss, LX, op.t_sX);
  if (Y >= 0) {
    add_tabs(p, R, rs, LY, op.t_rY);
    add_tabs(p, C, cs, LY, op.t_cY);
    add_tabs(p, S, ss, LY, op.t_sY);
  }
  ContractArgs &a = op.a;
  a.nR = (uint32_t)numel(R, card);
  a.nRl = (uint32_t)numel(Labels(R.begin() + rs, R.end()), card);
  a.nC = (uint32_t)numel(C, card);
  a.nCl = (uint32_t)numel(Labels(C.begin() + cs, C.end()), card);
  a.nS = (uint32_t)numel(S, card);
  a.nSl = (uint32_t)numel(Labels(S.begin() + ss, S.end()), card);
  a.col_fastest = (!LZ.empty() && !C.empty() && LZ.back() == C.back()) ? 1 : 0;
  const bool zb = p->T[Z].batched;
  op.nb = zb ? p->max_batch : 1;
  op.inst = op.nb;
  const uint64_t n_out = (uint64_t)a.nR * a.nC;
  const uint32_t nSh = a.nS / a.nSl;
  if (zb && p->inter) {
    // interleaved plans: every batched contraction takes the interleaved
    // form, rows split into batch labels (held by Y) and M labels
    op.forms = 16;
    a.kind = 4;
    op.nb = p->max_batch / kInterLanes;
    a.nslab = op.nb;
    const Labels Bl = Y >= 0 ? inter(R, LY) : Labels{}, Ml = minus(R, Bl);
    const size_t bs = lo_split(Bl, card), ms = lo_split(Ml, card);
    add_tabs(p, Bl, bs, LX, op.t_gbX);
    if (Y >= 0) add_tabs(p, Bl, bs, LY, op.t_gbY);
    add_tabs(p, Bl, bs, LZ, op.t_gbZ);
    add_tabs(p, Ml, ms, LX, op.t_gmX);
    add_tabs(p, Ml, ms, LZ, op.t_gmZ);
    a.nB = (uint32_t)numel(Bl, card);
    a.nBl = (uint32_t)numel(Labels(Bl.begin() + bs, Bl.end()), card);
    a.nM = (uint32_t)numel(Ml, card);
    a.nMl = (uint32_t)numel(Labels(Ml.begin() + ms, Ml.end()), card);
    // tiles of a wave (forms: 16 = 4 x 4, 32 = 4 x 4 with the summed range
    // split over the workgroup, 64 = 8 x 8, 128 = 16 x 1; the larger tiles
    // for sum-product only): 8 x 8 where rows and columns are wide, 16 x 1
    // for (nearly) column-free contractions, else 4 x 4, split when long
    // sums meet few tiles
    const uint64_t waves = (uint64_t)a.nB * ((a.nM + kInterTile - 1) / kInterTile) *
                           ((a.nC + kInterTile - 1) / kInterTile) * op.nb;
    if (a.nS >= 8) op.forms |= 32;
    if (semi == SEMI_SUM && Y >= 0 && a.nM >= 8 && a.nC >= 8) op.forms |= 64;
    if (semi == SEMI_SUM && a.nM >= 16 && a.nC <= 2) op.forms |= 128;
    a.ksplit = a.nS >= 64 && waves < 4096 ? 4 : 1;
    a.tile = 0;
    if (a.ksplit == 1 && (op.forms & 64)) a.tile = 1;
    else if (a.ksplit == 1 && (op.forms & 128)) a.tile = 2;
    // the variants are not offered to the autotuner: timed alone a variant
    // does not predict its cost inside a grouped stage launch (measured on
    // the 512-set network: per-shape choices by isolated timing were 5 %
    // slower than these rules)
    op.forms = 16;
    op.flops = 2.0 * (double)n_out * (double)a.nS;
    op.bytes = 4.0 * (double)(p->T[X].size + (Y >= 0 ? p->T[Y].size : 0) + p->T[Z].size);
    return op;
  }
  // very few outputs, each a long sum: workgroups reduce chunks of the
  // summed index cooperatively (more outputs, or sums of fewer than 8192
  // entries, go to the wave form below: one wavefront per output takes at
  // most 128 entries per lane there, cheaper than the split form's two
  // launches of their own)
  if (n_out * (uint64_t)op.nb <= 64 && a.nS >= 8192) {
    op.split = true;
    // about 1024 workgroups in total, each reducing at least 1K summed entries
    uint32_t want = std::max<uint32_t>(1, 1024u / (uint32_t)op.nb);
    want = std::min<uint32_t>(want, std::max<uint32_t>(1, a.nS / 1024u));
    a.n_chunks = std::min<uint32_t>(nSh, want);
    // every split contraction owns its partial-sum region: contractions of
    // one stage run concurrently in a grouped launch
    op.part_off = p->part_floats;
    p->part_floats += ((int64_t)op.nb * a.n_chunks * n_out + 63) / 64 * 64;
  }
  // Eligible forms (Op::forms bits: 1 generic, 2 row, 4 dense, 8 wave) and
  // the rule-based choice; the autotuner may later pick another eligible one.
  // dense form: wide row and column sets, a summed set of at least 8 entries
  // (sum-product: or none, an outer product whose tiles still leave through
  // LDS in the order of Z's layout); max-plus runs the same tiles on the
  // vector ALUs
  if (!op.split) {
    op.forms = 1 | 8;
    // generic form in output order: for large outputs whose writes the
    // (rows, columns) enumeration would scatter (labels of X and of Y
    // interleaved in Z's layout); the autotuner may take it
    if (n_out >= (1u << 16)) {
      op.forms |= 512;
      const size_t os = lo_split(LZ, card);
      add_tabs(p, LZ, os, LX, op.t_oX);
      if (Y >= 0) add_tabs(p, LZ, os, LY, op.t_oY);
      a.nOl = (uint32_t)numel(Labels(LZ.begin() + os, LZ.end()), card);
    }
    if (Y >= 0) {
      const Labels Bl = inter(R, LY), Ml = minus(R, LY);
      const int64_t nB = numel(Bl, card), nM = numel(Ml, card);
      // eligible for any summed set (sum-product), or for max-plus (the
      // tiles then run on the vector ALUs) from 8 entries and 2^17
      // candidates over all instances: smaller max-plus products go to the
      // forms of the grouped stage launch instead of a dense launch of their
      // own (on the 300-variable network's tree 8 of its 17 dense launches
      // shared a stage with a grouped one)
      const bool s_ok = semi == SEMI_SUM ? true : a.nS >= 8 && (uint64_t)op.nb * n_out * a.nS >= (1u << 17);
      const bool dense_ok =
          nM >= 16 && a.nC >= 8 && s_ok &&
          nB * ((nM + kGemmTile - 1) / kGemmTile) * (((int64_t)a.nC + kGemmTile - 1) / kGemmTile) < (1LL << 31);
      // batch-uniform row form (sum-product, offered to the autotuner): Y's
      // summed x columns block of a batch assignment fits two entries per
      // lane, and every batch assignment fills wavefronts of M assignments
      const bool rowsb_ok = semi == SEMI_SUM && a.nS <= (uint32_t)kRowMax && a.nC <= (uint32_t)kRowMax &&
                            a.nS * a.nC <= (uint32_t)kRowBlock && nM >= 64 && n_out >= (1u << 16) &&
                            nB * ((nM + 63) / 64) < (1LL << 31);
      if (dense_ok) op.forms |= 4;
      if (rowsb_ok) op.forms |= 1024;
      if (dense_ok || rowsb_ok) {
        const size_t bs = lo_split(Bl, card), ms = lo_split(Ml, card);
        add_tabs(p, Bl, bs, LX, op.t_gbX);
        add_tabs(p, Bl, bs, LY, op.t_gbY);
        add_tabs(p, Bl, bs, LZ, op.t_gbZ);
        add_tabs(p, Ml, ms, LX, op.t_gmX);
        add_tabs(p, Ml, ms, LZ, op.t_gmZ);
        a.nB = (uint32_t)nB;
        a.nBl = (uint32_t)numel(Labels(Bl.begin() + bs, Bl.end()), card);
        a.nM = (uint32_t)nM;
        a.nMl = (uint32_t)numel(Labels(Ml.begin() + ms, Ml.end()), card);
        a.nBlo = 1;
        for (auto it = LZ.rbegin(); it != LZ.rend() && has(Bl, *it) && a.nBlo * card[*it] <= 16; ++it)
          a.nBlo *= (uint32_t)card[*it];
        a.x_s_fast = (!LX.empty() && has(S, LX.back())) ? 1 : 0;
        a.y_n_fast = (!LY.empty() && has(C, LY.back())) ? 1 : 0;
        a.s_pair = a.x_s_fast && has(S, LY.back()) && card[LX.back()] == 2 && a.nS % 2 == 0 ? 1 : 0;
        a.z_n_fast = (!LZ.empty() && has(C, LZ.back())) ? 1 : 0;
      }
    }
    // row form for skinny contractions: few summed entries and columns
    const bool row_ok = a.nS <= (uint32_t)kRowFormMax && a.nC <= (uint32_t)kRowFormMax && a.nS * a.nC <= 64;
    if (row_ok) op.forms |= 2;
    if (row_ok || (op.forms & 1024)) {
      a.ns = (int32_t)a.nS;
      a.nc = (int32_t)a.nC;
      auto offsets = [&](const Labels &L, const Labels &TL, int32_t *dst) {
        const int64_t n = numel(L, card);
        std::vector<int> d(L.size(), 0);
        for (int64_t i = 0; i < n; ++i) {
          int64_t off = 0;
          for (size_t j = 0; j < L.size(); ++j) off += (int64_t)d[j] * stride_in(TL, L[j], card);
          dst[i] = (int32_t)off;
          for (int j = (int)L.size() - 1; j >= 0; --j) {
            if (++d[j] < card[L[j]]) break;
            d[j] = 0;
          }
        }
      };
      offsets(S, LX, a.sx);
      offsets(S, LY, a.sy);
      offsets(C, LY, a.cy);
      offsets(C, LZ, a.cz);
      // runs of four adjacent, 16-byte aligned entries (every other offset
      // of the operand a multiple of 4): vector loads of X's row and stores
      // of Z's row in the batch-uniform row form
      auto runs = [&](const int32_t *o, int64_t n, const Labels &L, const Labels &TL, int r) {
        if (n % r != 0 || n > kRowMax) return false;
        for (int64_t i = 0; i < n; ++i)
          if (o[i] != o[i - i % r] + i % r || o[i - i % r] % r != 0) return false;
        for (int v : minus(TL, L))
          if (stride_in(TL, v, card) % r != 0) return false;
        return true;
      };
      a.row_vx = !(op.forms & 1024) ? 0 : runs(a.sx, a.nS, S, LX, 4) ? 1 : runs(a.sx, a.nS, S, LX, 2) ? 2 : 0;
      a.row_vz = (op.forms & 1024) && runs(a.cz, a.nC, C, LZ, 4) ? 1 : 0;
      if ((a.nRl & (a.nRl - 1)) == 0) {
        int sh = 0;
        while ((1u << sh) < a.nRl) ++sh;
        a.rl_shift = sh;
      }
    }
    // large dense tiles (FP32 sum-product): 128 x 128 output tiles where
    // rows and columns are wide; the rules take them where the summed set
    // fills a chunk of 16, the autotuner may take them for shorter sums
    // (operands below 2^29 entries per instance: 32-bit byte offsets)
    if ((op.forms & 4) && semi == SEMI_SUM && p->opts.dtype == TN_F32 && a.nM >= 128 && a.nC >= 128 &&
        p->T[X].size < (int64_t(1) << 29) && p->T[Y].size < (int64_t(1) << 29))
      op.forms |= 256;
    // rules: dense (large tiles where eligible), else wave for long sums,
    // else row, else generic
    if ((op.forms & 4) && (a.nS >= 8 || a.nS == 1)) a.kind = 2;
    else if (a.nS >= 64) a.kind = 3;
    else if (op.forms & 2) a.kind = 1;
    else a.kind = 0;
    // the generic form writes runs of Z as long as the trailing labels of Z
    // of the class it enumerates fastest; below 16 entries it takes the
    // output order
    if (a.kind == 0 && (op.forms & 512)) {
      const Labels &fast = a.col_fastest ? C : R;
      int64_t run = 1;
      for (auto it = LZ.rbegin(); it != LZ.rend() && has(fast, *it); ++it) run *= card[*it];
      if (run < 16) a.tile = 1;
    }
    if (a.kind == 2 && (op.forms & 256) && a.nS >= 16) a.tile = 1;
  }
  op.flops = 2.0 * (double)n_out * (double)a.nS;
  op.bytes = 4.0 * (double)(p->T[X].size + (Y >= 0 ? p->T[Y].size : 0) + p->T[Z].size);
  return op;
}

// ---------------------------------------------------------------------------
// plan construction
// ---------------------------------------------------------------------------

// leaves of the main tree for the plan's evidence mode
static void build_leaves(tn_plan_t *p, const tn_net *net) {
  const int n = p->n_vars;
  for (int f = 0; f < (int)net->scope.size(); ++f) {
    Labels lab;
    for (int v : net->scope[f])
      if (!p->is_obs[v]) lab.push_back(v);
    std::sort(lab.begin(), lab.end());
    p->leaf_lab.push_back(lab);
    p->leaf_kind.push_back(0);
    p->leaf_var.push_back(-1);
    p->leaf_factor.push_back(f);
  }
  for (int v = 0; v < n; ++v) {
    if (p->mode == TN_EVIDENCE_SLICED && p->is_obs[v]) continue;
    p->leaf_lab.push_back(Labels{v});
    p->leaf_kind.push_back(p->mode == TN_EVIDENCE_INDICATOR ? 2 : 1);
    p->leaf_var.push_back(v);
    p->leaf_factor.push_back(-1);
  }
  // one unity tensor (all ones) per joint set, over its unobserved variables
  for (const auto &set : p->joint_sets) {
    Labels lab;
    for (int v : set)
      if (!(p->mode == TN_EVIDENCE_SLICED && p->is_obs[v])) lab.push_back(v);
    if (lab.empty()) continue;
    p->leaf_lab.push_back(lab);
    p->leaf_kind.push_back(3);
    p->leaf_var.push_back(-1);
    p->leaf_factor.push_back(-1);
  }
}

// gather map of factor f restricted to its unobserved variables (sorted),
// and (var, stride) pairs of its observed variables, strides in load order;
// true when the map is the identity (the unobserved variables trail the
// scope in sorted order), so that the leaf is a contiguous copy
static bool factor_gather(tn_plan_t *p, const tn_net *net, int f, const std::vector<char> &fixed,
                          int32_t &gmap_off, int32_t &obs_b, int32_t &obs_e) {
  const auto &sc = net->scope[f];
  std::vector<int64_t> st(sc.size());
  int64_t s = 1;
  for (int i = (int)sc.size() - 1; i >= 0; --i) {
    st[i] = s;
    s *= p->card[sc[i]];
  }
  Labels lab;
  for (int v : sc)
    if (!fixed[v]) lab.push_back(v);
  std::sort(lab.begin(), lab.end());
  std::vector<int64_t> ls(lab.size());
  for (size_t j = 0; j < lab.size(); ++j)
    for (size_t i = 0; i < sc.size(); ++i)
      if (sc[i] == lab[j]) ls[j] = st[i];
  gmap_off = (int32_t)p->gmap.size();
  int64_t n = numel(lab, p->card);
  std::vector<int> d(lab.size(), 0);
  int64_t off = 0;
  for (int64_t i = 0; i < n; ++i) {
    p->gmap.push_back((int32_t)off);
    for (int j = (int)lab.size() - 1; j >= 0; --j) {
      if (++d[j] < p->card[lab[j]]) {
        off += ls[j];
        break;
      }
      off -= ls[j] * (p->card[lab[j]] - 1);
      d[j] = 0;
    }
  }
  obs_b = (int32_t)(p->obs.size() / 2);
  for (size_t i = 0; i < sc.size(); ++i)
    if (fixed[sc[i]]) {
      p->obs.push_back(sc[i]);
      p->obs.push_back((int32_t)st[i]);
    }
  obs_e = (int32_t)(p->obs.size() / 2);
  for (int64_t i = 0; i < n; ++i)
    if (p->gmap[gmap_off + i] != i) return false;
  return true;
}

// Forward ops of a tree whose leaf tensors exist: creates node tensors.
// For max-plus, labels eliminated at a node that only one child holds are
// reduced in that child first (with their own argmax), so that the node
// itself maximises over the shared labels only.
static void build_forward(tn_plan_t *p, TreeExec &t, int semi) {
  const int L = (int)t.leaf_tensor.size();
  t.node_tensor = t.leaf_tensor;
  t.node_tensor.resize(L + t.pairs.size(), -1);
  t.node_ops.assign(t.pairs.size(), {});
  t.root_op = -1;
  const bool sum = semi == SEMI_SUM;
  for (size_t q = 0; q < t.pairs.size(); ++q) {
    const int c = L + (int)q, l = t.pairs[q][0], r = t.pairs[q][1];
    int tl = t.node_tensor[l], tr = t.node_tensor[r];
    const Labels &Lc = t.lab[c];
    if (!sum) {
      for (int side = 0; side < 2; ++side) {
        int &tc = side ? tr : tl;
        const Labels mine = p->T[tc].lab, other = p->T[side ? tl : tr].lab;
        Labels keep;
        for (int v : mine)
          if (has(other, v) || has(Lc, v)) keep.push_back(v);
        if (keep.size() == mine.size()) continue;
        int red = new_tensor(p, keep, p->T[tc].batched, false);
        int ib = new_intbuf(p, p->T[red].size, p->T[red].batched);
        t.node_ops[q].push_back((int)t.ops.size());
        t.ops.push_back(make_op(p, SEMI_MAX, tc, -1, red, ib));
        tc = red;
      }
    }
    const bool bat = p->T[tl].batched || p->T[tr].batched;
    int z = new_tensor(p, Lc, bat, sum);
    int X = tl, Y = tr;
    const int64_t wl = p->T[tl].size * (p->T[tl].batched ? 2 : 1), wr = p->T[tr].size * (p->T[tr].batched ? 2 : 1);
    if (wr > wl) std::swap(X, Y);
    int ib = sum ? -1 : new_intbuf(p, p->T[z].size, bat);
    t.node_ops[q].push_back((int)t.ops.size());
    t.ops.push_back(make_op(p, semi, X, Y, z, ib));
    t.node_tensor[c] = z;
  }
  const int root_node = L + (int)t.pairs.size() - 1;
  const int rt = t.node_tensor[root_node];
  if (p->T[rt].lab != t.out) {
    // single leaf (or labels left at the root): reduce to the output labels
    int z = new_tensor(p, t.out, p->T[rt].batched, sum);
    int ib = sum ? -1 : new_intbuf(p, p->T[z].size, p->T[z].batched);
    t.root_op = (int)t.ops.size();
    t.ops.push_back(make_op(p, semi, rt, -1, z, ib));
    t.root = z;
  } else {
    t.root = rt;
  }
}

// Readout steps for a max-plus tree: top-down, each node's main argmax
// first, then the argmax of its children's private reductions.
// Chains of two or three consecutive max-plus contractions (each one's X is
// the previous one's output, which nothing else reads) run as one pass
// (kKindMaxPair): pairs where each step sums over at most four assignments
// and the second adds at most four columns, triples where every step sums
// over at most two and the third adds at most two; every later step's
// summed labels come from the previous output.  The intermediate values
// stay in registers (the same FP32 values and first maximisers as the
// contractions alone), and the last step's index array holds, per output,
// every step's choice as one index over (S1, S2[, S3]), the last fastest —
// the readout takes the whole chain with one read, and the other index
// arrays are not written.  Contractions of >= 2^12 outputs of one instance
// only (below, a separate launch class costs more than the pass saves).  Fills t.fops (a chain sits at its last contraction's place, after
// every producer of its operands), t.chain_prev and t.chain_inner; t.fused
// when a chain formed.
static void build_max_pairs(tn_plan_t *p, TreeExec &t) {
  const auto &card = p->card;
  const int n = (int)t.ops.size();
  std::map<int, int> uses, reader;  // tensor -> ops reading it; op reading it as X
  for (int i = 0; i < n; ++i) {
    uses[t.ops[i].X]++;
    if (t.ops[i].Y >= 0) uses[t.ops[i].Y]++;
    reader[t.ops[i].X] = i;
  }
  auto ok = [&](const Op &op) {
    return op.semi == SEMI_MAX && op.Y >= 0 && !op.split && op.nb == 1 && op.inst == 1 && op.seg < 0 && op.I >= 0;
  };
  // offsets of the assignments of L (row-major, last fastest) in a tensor
  // with labels TL (0 for labels it lacks)
  auto offs = [&](const Labels &L, const Labels &TL) {
    std::vector<int32_t> o;
    std::vector<int> d(L.size(), 0);
    for (int64_t i = 0, m = numel(L, card); i < m; ++i) {
      int64_t v = 0;
      for (size_t k = 0; k < L.size(); ++k) v += (int64_t)d[k] * stride_in(TL, L[k], card);
      o.push_back((int32_t)v);
      for (int k = (int)L.size() - 1; k >= 0; --k) {
        if (++d[k] < card[L[k]]) break;
        d[k] = 0;
      }
    }
    return o;
  };
  auto elim = [&](const Op &op) { return minus(unite(p->T[op.X].lab, p->T[op.Y].lab), p->T[op.Z].lab); };
  // the contraction reading op i's output as its X, if op i may start or
  // continue a chain
  auto next = [&](int i) {
    const Op &a = t.ops[i];
    if (!ok(a) || a.Z == t.root || uses[a.Z] != 1 || !reader.count(a.Z)) return -1;
    const int j = reader[a.Z];
    return j > i && ok(t.ops[j]) ? j : -1;
  };
  std::vector<std::vector<int>> chain_at(n);  // last contraction -> the chain
  std::vector<char> used(n, 0);
  for (int i = 0; i < n; ++i) {
    if (used[i]) continue;
    const int j = next(i);
    if (j < 0 || used[j]) continue;
    const Op &a = t.ops[i], &b = t.ops[j];
    const Labels &LZ1 = p->T[a.Z].lab, &LZ2 = p->T[b.Z].lab;
    const Labels S1 = elim(a), S2 = elim(b);
    const int k = next(j);
    if (k >= 0 && !used[k]) {  // three steps, each of at most two summed assignments
      const Op &c = t.ops[k];
      const Labels &LZ3 = p->T[c.Z].lab;
      const Labels S3 = elim(c), C3 = minus(LZ3, LZ2), R3 = inter(LZ3, LZ2);
      if (minus(S2, LZ1).empty() && minus(S3, LZ2).empty() && numel(S1, card) <= kTripleMax &&
          numel(S2, card) <= kTripleMax && numel(S3, card) <= kTripleMax && numel(C3, card) <= kTripleMax &&
          numel(LZ3, card) >= kChainMinOut && numel(R3, card) < (int64_t(1) << 31)) {
        used[i] = used[j] = used[k] = 1;
        chain_at[k] = {i, j, k};
        continue;
      }
    }
    const Labels R2 = inter(LZ2, LZ1), C2 = minus(LZ2, LZ1);
    if (!minus(S2, LZ1).empty() || numel(S1, card) > kPairMax || numel(S2, card) > kPairMax ||
        numel(C2, card) > kPairMax || numel(LZ2, card) < kChainMinOut || numel(R2, card) >= (int64_t(1) << 31))
      continue;
    used[i] = used[j] = 1;
    chain_at[j] = {i, j};
  }
  t.fops.clear();
  t.fused = false;
  t.chain_prev.assign(n, -1);
  t.chain_inner.assign(n, 0);
  for (int j = 0; j < n; ++j) {
    const std::vector<int> &ch = chain_at[j];
    for (size_t q = 0; q < ch.size(); ++q) {
      if (q > 0) t.chain_prev[ch[q]] = ch[q - 1];
      if (q + 1 < ch.size()) t.chain_inner[ch[q]] = 1;
    }
  }
  for (int j = 0; j < n; ++j) {
    if (used[j] && chain_at[j].empty()) continue;  // emitted with its chain's last contraction
    if (chain_at[j].empty()) {
      t.fops.push_back(t.ops[j]);
      continue;
    }
    const std::vector<int> &ch = chain_at[j];
    const bool three = ch.size() == 3;
    const Op &a = t.ops[ch[0]], &b = t.ops[ch[1]], &last = t.ops[j];
    const Labels &LX = p->T[a.X].lab, &LY1 = p->T[a.Y].lab, &LZ1 = p->T[a.Z].lab, &LY2 = p->T[b.Y].lab;
    const Labels &LZ2 = p->T[b.Z].lab, &LZ = p->T[last.Z].lab;
    const Labels &LY3 = p->T[last.Y].lab;
    const Labels &Lprev = three ? LZ2 : LZ1;  // the last step's X
    const Labels R = inter(LZ, Lprev), C = minus(LZ, Lprev);
    const Labels S1 = elim(a), S2 = elim(b), S3 = three ? elim(last) : Labels{};
    Op f;
    f.semi = SEMI_MAX;
    f.X = a.X;
    f.Y = a.Y;
    f.Z = last.Z;
    f.I = last.I;
    f.Y2 = b.Y;
    f.ins.push_back(b.Y);
    if (three) {
      f.Y3 = last.Y;
      f.ins.push_back(last.Y);
    }
    for (auto *tb : {f.t_rX, f.t_rY, f.t_rZ, f.t_cY, f.t_cZ, f.t_sX, f.t_sY, f.t_gbX, f.t_gbY, f.t_gbZ, f.t_gmX,
                     f.t_gmZ, f.t_oX, f.t_oY})
      tb[0] = tb[1] = -1;
    const size_t rs = lo_split(R, card);
    add_tabs(p, R, rs, LX, f.t_rX);
    add_tabs(p, R, rs, LY1, f.t_rY);
    add_tabs(p, R, rs, LZ, f.t_rZ);
    add_tabs(p, R, rs, LY2, f.t_gbY);
    if (three) add_tabs(p, R, rs, LY3, f.t_gmX);
    ContractArgs &c = f.a;
    c.kind = kKindMaxPair;
    c.steps = three ? 3 : 2;
    c.nR = (uint32_t)numel(R, card);
    c.nRl = (uint32_t)numel(Labels(R.begin() + rs, R.end()), card);
    if ((c.nRl & (c.nRl - 1)) == 0) {
      int sh = 0;
      while ((1u << sh) < c.nRl) ++sh;
      c.rl_shift = sh;
    }
    c.ns = (int32_t)numel(S1, card);
    c.ns2 = (int32_t)numel(S2, card);
    c.ns3 = three ? (int32_t)numel(S3, card) : 1;
    c.nc = (int32_t)numel(C, card);
    c.nS = (uint32_t)c.ns;
    c.nC = (uint32_t)c.nc;
    const std::vector<int32_t> xs1 = offs(S1, LX), ys1 = offs(S1, LY1), xs2 = offs(S2, LX), ys2 = offs(S2, LY1);
    const std::vector<int32_t> zc = offs(C, LZ);
    if (!three) {
      const std::vector<int32_t> y2s2 = offs(S2, LY2), y2c = offs(C, LY2);
      for (int u = 0; u < c.ns2; ++u) {
        for (int v = 0; v < c.ns; ++v) {
          c.sx[kPairMax * u + v] = xs2[u] + xs1[v];
          c.sy[kPairMax * u + v] = ys2[u] + ys1[v];
        }
        for (int w = 0; w < c.nc; ++w) c.cy[kPairMax * w + u] = y2s2[u] + y2c[w];
      }
    } else {
      const std::vector<int32_t> xs3 = offs(S3, LX), ys3 = offs(S3, LY1), y2s2 = offs(S2, LY2), y2s3 = offs(S3, LY2);
      const std::vector<int32_t> y3s3 = offs(S3, LY3), y3c = offs(C, LY3);
      constexpr int K = kTripleMax;
      for (int u3 = 0; u3 < c.ns3; ++u3) {
        for (int u2 = 0; u2 < c.ns2; ++u2) {
          for (int u1 = 0; u1 < c.ns; ++u1) {
            c.sx[(K * u3 + u2) * K + u1] = xs3[u3] + xs2[u2] + xs1[u1];
            c.sy[(K * u3 + u2) * K + u1] = ys3[u3] + ys2[u2] + ys1[u1];
          }
          c.cy[K * u3 + u2] = y2s3[u3] + y2s2[u2];
        }
        for (int w = 0; w < c.nc; ++w) c.cz[K * w + u3] = y3c[w] + y3s3[u3];
      }
    }
    for (int w = 0; w < c.nc; ++w) c.cz[kPairZ + w] = zc[w];
    // X's entries of a lane adjacent and 16-byte aligned (every step sums two
    // assignments, the summed labels X's fastest ones in step order):
    // vector loads
    {
      const int box = three ? c.ns * c.ns2 * c.ns3 : c.ns * c.ns2;
      bool adj = c.ns == 2 && c.ns2 == 2 && (!three || c.ns3 == 2);
      for (int u = 0; adj && u < box; ++u) {
        const int k = three ? u : kPairMax * (u / 2) + u % 2;
        adj = c.sx[k] == c.sx[0] + u;
      }
      if (adj && c.sx[0] % 4 == 0)
        for (int v : R)
          if (stride_in(LX, v, card) % 4 != 0) adj = false;
      c.row_vx = adj ? 1 : 0;
    }
    f.flops = 0;
    f.bytes = 4.0 * (double)(p->T[a.X].size + p->T[a.Y].size + p->T[b.Y].size + p->T[last.Z].size);
    for (int q : ch) f.flops += t.ops[q].flops;
    if (three) f.bytes += 4.0 * (double)p->T[last.Y].size;
    t.fops.push_back(f);
    t.fused = true;
  }
  if (!t.fused) {
    t.fops.clear();
    t.chain_prev.clear();
    t.chain_inner.clear();
  }
}

static void build_backtrack(tn_plan_t *p, TreeExec &t) {
  t.back.clear();
  t.back_meta.clear();
  // a step reads the op's argmax at its output's assignment and assigns its
  // eliminated variables; the last contraction of a max-plus chain run in
  // one pass assigns every step's (its index runs over all of them, the
  // last step's fastest), and the earlier ones have no step of their own
  auto eliminated = [&](const Op &op) {
    Labels U = p->T[op.X].lab;
    if (op.Y >= 0) U = unite(U, p->T[op.Y].lab);
    return minus(U, p->T[op.Z].lab);
  };
  auto add_step = [&](int id) {
    if (!t.chain_inner.empty() && t.chain_inner[id]) return;
    const Op &op = t.ops[id];
    BackStep s{};
    s.arg = op.I;  // IntBuf id; converted to an offset at allocation
    const Labels &LZ = p->T[op.Z].lab;
    s.in_begin = (int32_t)(t.back_meta.size() / 2);
    for (int v : LZ) {
      t.back_meta.push_back(v);
      t.back_meta.push_back((int32_t)stride_in(LZ, v, p->card));
    }
    s.in_end = (int32_t)(t.back_meta.size() / 2);
    s.out_begin = s.in_end;
    std::vector<int> chain{id};  // the chain ending at this op, first contraction first
    while (!t.chain_prev.empty() && t.chain_prev[chain.front()] >= 0) chain.insert(chain.begin(), t.chain_prev[chain.front()]);
    Labels out;
    for (int q : chain) {
      const Labels e = eliminated(t.ops[q]);
      out.insert(out.end(), e.begin(), e.end());
    }
    for (int v : out) {
      t.back_meta.push_back(v);
      t.back_meta.push_back(p->card[v]);
    }
    s.out_end = (int32_t)(t.back_meta.size() / 2);
    t.back.push_back(s);
  };
  if (t.root_op >= 0) add_step(t.root_op);
  for (int q = (int)t.pairs.size() - 1; q >= 0; --q) {
    const auto &ids = t.node_ops[q];
    add_step(ids.back());
    for (size_t k = 0; k + 1 < ids.size(); ++k) add_step(ids[k]);
  }
  // Readout levels: a step needs the variables of its node's output, which
  // earlier steps assign; level = 1 + the largest level among the steps that
  // assigned them.  Steps of one level read only lower levels and write
  // disjoint variables, so each level runs in parallel.
  std::vector<int> lev_of_var(p->n_vars, -1), lev(t.back.size());
  int n_lev = 0;
  for (size_t i = 0; i < t.back.size(); ++i) {
    const BackStep &s = t.back[i];
    int l = 0;
    for (int k = s.in_begin; k < s.in_end; ++k) l = std::max(l, lev_of_var[t.back_meta[2 * k]] + 1);
    for (int k = s.out_begin; k < s.out_end; ++k) lev_of_var[t.back_meta[2 * k]] = l;
    lev[i] = l;
    n_lev = std::max(n_lev, l + 1);
  }
  // steps in level order, each step's pairs laid out in that order too
  std::vector<BackStep> sorted;
  std::vector<int32_t> meta;
  t.back_lev.assign(1, 0);
  for (int l = 0; l < n_lev; ++l) {
    for (size_t i = 0; i < t.back.size(); ++i)
      if (lev[i] == l) {
        BackStep s = t.back[i];
        const int32_t b = (int32_t)(meta.size() / 2);
        meta.insert(meta.end(), t.back_meta.begin() + 2 * s.in_begin, t.back_meta.begin() + 2 * s.out_end);
        s.in_end = b + (s.in_end - s.in_begin);
        s.out_begin = b + (s.out_begin - s.in_begin);
        s.out_end = b + (s.out_end - s.in_begin);
        s.in_begin = b;
        sorted.push_back(s);
      }
    t.back_lev.push_back((int32_t)sorted.size());
  }
  t.back = std::move(sorted);
  t.back_meta = std::move(meta);
  // chunks of whole levels for the readout kernel's LDS staging
  t.n_back_lev = n_lev;
  std::vector<int32_t> chunks;
  auto pairs_of = [&](int l0, int l1) {
    const int s0 = t.back_lev[l0], s1 = t.back_lev[l1];
    return s1 > s0 ? t.back[s1 - 1].out_end - t.back[s0].in_begin : 0;
  };
  for (int l0 = 0; l0 < n_lev;) {
    int l1 = l0 + 1;
    while (l1 < n_lev && t.back_lev[l1 + 1] - t.back_lev[l0] <= kBackChunkSteps &&
           pairs_of(l0, l1 + 1) <= kBackChunkPairs)
      ++l1;
    const int s0 = t.back_lev[l0], s1 = t.back_lev[l1];
    chunks.insert(chunks.end(), {l0, l1, s0, s1, s1 > s0 ? t.back[s0].in_begin : 0,
                                 s1 > s0 ? t.back[s1 - 1].out_end : 0});
    l0 = l1;
  }
  t.n_back_chunks = (int32_t)(chunks.size() / kBackChunkInts);
  t.back_lev.insert(t.back_lev.end(), chunks.begin(), chunks.end());
}

// Top-down sampling steps (eq. sample, eq. condition-prob): at every node the
// shared eliminated labels are drawn with weights Ar[z, k] * Br[z, k], where
// Ar, Br are the children summed over their private eliminated labels
// (reduction contractions run after the forward pass when sampling), then
// each child's private labels are drawn from the child itself.
static void build_sampling(tn_plan_t *p, const TreeExec &t) {
  p->samp.clear();
  p->samp_meta.clear();
  p->samp_ops.clear();
  const int L = (int)t.leaf_tensor.size();
  auto quad = [&](int v, int c, int64_t sa, int64_t sb) {
    p->samp_meta.push_back(v);
    p->samp_meta.push_back(c);
    p->samp_meta.push_back((int32_t)sa);
    p->samp_meta.push_back((int32_t)sb);
  };
  if (t.pairs.empty()) {
    SampleStep st{};
    st.A = t.leaf_tensor[0];
    st.B = -1;
    st.Ar = st.A;
    st.Br = -1;
    st.node = L;
    const Labels &la = p->T[t.leaf_tensor[0]].lab;
    st.pa_b = (int32_t)(p->samp_meta.size() / 4);
    for (int v : la) quad(v, p->card[v], stride_in(la, v, p->card), 0);
    st.pa_e = (int32_t)(p->samp_meta.size() / 4);
    p->samp.push_back(st);
    return;
  }
  for (int q = (int)t.pairs.size() - 1; q >= 0; --q) {
    const int c = L + q, l = t.pairs[q][0], r = t.pairs[q][1];
    const Labels &La = t.lab[l], &Lb = t.lab[r], &Lc = t.lab[c];
    SampleStep st{};
    st.A = t.node_tensor[l];
    st.B = t.node_tensor[r];
    st.node = c;
    const Labels K = minus(inter(La, Lb), Lc);
    const Labels Pa = minus(minus(La, Lb), Lc), Pb = minus(minus(Lb, La), Lc);
    // reduced children (only needed when shared labels are drawn)
    auto reduced = [&](int child, const Labels &Lx, const Labels &P) -> int {
      if (K.empty() || P.empty()) return child;
      const int red = new_tensor(p, minus(Lx, P), false, true);
      p->samp_ops.push_back(make_op(p, SEMI_SUM, child, -1, red, -1));
      return red;
    };
    const int ar = reduced((int)st.A, La, Pa), br = reduced((int)st.B, Lb, Pb);
    st.Ar = ar;
    st.Br = br;
    const Labels &LAr = p->T[ar].lab, &LBr = p->T[br].lab;
    auto beg = [&] { return (int32_t)(p->samp_meta.size() / 4); };
    st.aIn_b = beg();
    for (int v : inter(La, Lc)) quad(v, p->card[v], stride_in(La, v, p->card), stride_in(LAr, v, p->card));
    st.aIn_e = beg();
    st.bIn_b = beg();
    for (int v : inter(Lb, Lc)) quad(v, p->card[v], stride_in(Lb, v, p->card), stride_in(LBr, v, p->card));
    st.bIn_e = beg();
    st.k_b = beg();
    for (int v : K) quad(v, p->card[v], stride_in(La, v, p->card), stride_in(Lb, v, p->card));
    st.k_e = beg();
    st.kr_b = beg();
    for (int v : K) quad(v, p->card[v], stride_in(LAr, v, p->card), stride_in(LBr, v, p->card));
    st.kr_e = beg();
    st.pa_b = beg();
    for (int v : Pa) quad(v, p->card[v], stride_in(La, v, p->card), 0);
    st.pa_e = beg();
    st.pb_b = beg();
    for (int v : Pb) quad(v, p->card[v], 0, stride_in(Lb, v, p->card));
    st.pb_e = beg();
    p->samp.push_back(st);
  }
}

template <class T>
static T *dalloc(tn_plan_t *p, size_t n) {
  if (n == 0) n = 1;
  void *ptr = nullptr;
  hip_check(hipMalloc(&ptr, n * sizeof(T)), "hipMalloc");
  p->allocs.push_back(ptr);
  p->device_bytes += (int64_t)(n * sizeof(T));
  return (T *)ptr;
}
template <class T>
static T *dupload(tn_plan_t *p, const std::vector<T> &v) {
  T *d = dalloc<T>(p, v.size());
  if (!v.empty()) hip_check(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "upload");
  return d;
}

template <class T>
static T *dalloc_vec(tn_plan_t *p, const std::vector<T> &v) {
  return dupload(p, v);
}

static void fill_args(tn_plan_t *p, Op &op) {
  ContractArgs &a = op.a;
  auto tab = [&](const int64_t t[2]) {
    Tab2 r;
    if (t[0] >= 0) {
      r.hi = p->d_tabs + t[0];
      r.lo = p->d_tabs + t[1];
    }
    return r;
  };
  a.rX = tab(op.t_rX);
  a.rY = tab(op.t_rY);
  a.rZ = tab(op.t_rZ);
  a.cY = tab(op.t_cY);
  a.cZ = tab(op.t_cZ);
  a.sX = tab(op.t_sX);
  a.sY = tab(op.t_sY);
  a.gbX = tab(op.t_gbX);
  a.gbY = tab(op.t_gbY);
  a.gbZ = tab(op.t_gbZ);
  a.gmX = tab(op.t_gmX);
  a.gmZ = tab(op.t_gmZ);
  a.oX = tab(op.t_oX);
  a.oY = tab(op.t_oY);
  const TensorBuf &X = p->T[op.X], &Z = p->T[op.Z];
  // instance stride bs and element stride es of an operand
  auto strides = [&](const TensorBuf &t, int64_t &bs, int32_t &es) {
    bs = t.batched ? (p->inter ? 1 : t.size) : 0;
    es = t.batched && p->inter ? p->max_batch : 1;
  };
  a.X = p->arena + X.off;
  strides(X, a.bsX, a.esX);
  if (op.Y >= 0) {
    const TensorBuf &Y = p->T[op.Y];
    a.Y = p->arena + Y.off;
    strides(Y, a.bsY, a.esY);
    a.slotY = Y.slot;
    a.batY = Y.batched;
  }
  a.Z = p->arena + Z.off;
  strides(Z, a.bsZ, a.esZ);
  a.I = op.I >= 0 ? p->iarena + p->IB[op.I].off : nullptr;
  if (op.Y2 >= 0) a.Y2 = p->arena + p->T[op.Y2].off;
  if (op.Y3 >= 0) a.Y3 = p->arena + p->T[op.Y3].off;
  a.mx = p->mx;
  a.ex = p->ex;
  a.mx_stride = std::max(1, p->n_slots);
  a.slotX = X.slot;
  a.batX = X.batched;
  a.slotZ = Z.slot;
  a.batZ = Z.batched;
  a.part = p->d_part + (op.part_off >= 0 ? op.part_off : 0);
  a.parti = p->d_parti + (op.part_off >= 0 ? op.part_off : 0);
  a.prec = a.kind == 2 ? p->opts.dtype : 0;
}


// ---------------------------------------------------------------------------
// schedules (stages of independent contractions)
// ---------------------------------------------------------------------------
static Schedule build_schedule(tn_plan_t *p, const std::vector<Op> &ops, bool alap) {
  Schedule sc;
  const int n = (int)ops.size();
  if (n == 0) return sc;
  std::map<int, int> producer;  // tensor id -> op index
  for (int i = 0; i < n; ++i) {
    producer[ops[i].Z] = i;
    for (int t : ops[i].outs) producer[t] = i;
  }
  std::vector<int> stage(n, 0);
  std::vector<std::vector<int>> consumers(n);
  for (int i = 0; i < n; ++i) {
    int st = 0;
    std::vector<int> inputs = ops[i].ins;
    inputs.push_back(ops[i].X);
    inputs.push_back(ops[i].Y);
    for (int t : inputs) {
      if (t < 0) continue;
      auto it = producer.find(t);
      if (it != producer.end() && it->second < i) {
        st = std::max(st, stage[it->second] + 1);
        consumers[it->second].push_back(i);
      }
    }
    stage[i] = st;
  }
  int smax = *std::max_element(stage.begin(), stage.end());
  if (alap) {
    for (int i = n - 1; i >= 0; --i) {
      int st = smax;
      for (int c : consumers[i]) st = std::min(st, stage[c] - 1);
      stage[i] = st;
    }
  }
  sc.n_stages = smax + 1;
  // launches: per stage, map ops of each semiring together, split ops
  // together, segment sweeps of one kind together, carrier transforms alone
  for (int st = 0; st <= smax; ++st) {
    for (int kind = 3; kind <= 4; ++kind) {  // composed maps / adjoint sweeps of a stage together
      Launch L;
      L.seg = true;
      L.seg_kind = kind;
      for (int i = 0; i < n; ++i)
        if (stage[i] == st && ops[i].seg >= 0 && ops[i].seg_kind == kind) L.ops.push_back(i);
      if (!L.ops.empty()) sc.launches.push_back(std::move(L));
    }
    for (int kind : {1, 2, 5, 6}) {  // carrier passes: two independent ones of a kind per launch
      std::vector<int> ids;
      for (int i = 0; i < n; ++i)
        if (stage[i] == st && ops[i].seg >= 0 && ops[i].seg_kind == kind) ids.push_back(i);
      for (size_t j = 0; j < ids.size(); j += 2) {
        Launch L;
        L.seg = true;
        L.seg_kind = kind;
        L.ops.push_back(ids[j]);
        if (j + 1 < ids.size()) L.ops.push_back(ids[j + 1]);
        sc.launches.push_back(std::move(L));
      }
    }
    for (int semi = 0; semi < 2; ++semi)
      for (int cls = 0; cls < 5; ++cls) {  // one-lane-per-output forms, split reductions, dense, interleaved,
                                           // max-plus pairs
        Launch L;
        L.semi = semi;
        L.split = cls == 1;
        L.gemm = cls == 2;
        L.inter = cls == 3;
        L.mpair = cls == 4;
        for (int i = 0; i < n; ++i) {
          const Op &op = ops[i];
          const int c = op.split ? 1
                                 : (op.a.kind == 2 ? 2 : (op.a.kind == 4 ? 3 : (op.a.kind == kKindMaxPair ? 4 : 0)));
          if (stage[i] == st && op.seg < 0 && op.semi == semi && c == cls) {
            // large dense tiles and the batch-uniform row form: a launch of their own
            if ((c == 2 || (op.a.kind == 1 && c == 0)) && op.a.tile == 1) {
              Launch one;
              one.semi = semi;
              one.gemm = c == 2;
              one.ops.push_back(i);
              sc.launches.push_back(std::move(one));
            } else {
              L.ops.push_back(i);
            }
          }
        }
        if (!L.ops.empty()) sc.launches.push_back(std::move(L));
      }
  }
  (void)p;
  return sc;
}

static void upload_schedule(tn_plan_t *p, Schedule &sc, const std::vector<Op> &ops) {
  for (Launch &L : sc.launches) {
    if (L.seg && (L.seg_kind == 3 || L.seg_kind == 4)) {
      std::vector<int32_t> ids;
      L.lds = 0;
      for (int i : L.ops) {
        ids.push_back(ops[i].seg);
        const SegPlan &sp = p->segs[ops[i].seg];
        L.lds = std::max(L.lds, L.seg_kind == 3 ? sp.mat_lds : sp.fin_lds);
      }
      L.d_ids = dalloc_vec(p, ids);
      continue;
    }
    if (L.seg || L.ops.size() < 2) continue;
    std::vector<ContractArgs> args;
    std::vector<uint32_t> nb, nb2;
    std::vector<GroupBlock> bl, bl2;
    for (int i : L.ops) {
      const Op &op = ops[i];
      const uint32_t k = (uint32_t)args.size();
      args.push_back(op.a);
      const uint32_t per = L.split ? op.a.n_chunks : map_blocks(op.a);
      nb.push_back(per);
      for (uint32_t b = 0; b < per * (uint32_t)op.nb; ++b) bl.push_back(GroupBlock{k, b});
      if (L.split) {
        const uint32_t per2 = op.a.nR * op.a.nC;
        nb2.push_back(per2);
        for (uint32_t b = 0; b < per2 * (uint32_t)op.nb; ++b) bl2.push_back(GroupBlock{k, b});
      }
    }
    L.total = (uint32_t)bl.size();
    L.total2 = (uint32_t)bl2.size();
    L.d_args = dalloc_vec(p, args);
    L.d_blk = dalloc_vec(p, bl);
    L.d_nblk = dalloc_vec(p, nb);
    if (L.split) {
      L.d_blk2 = dalloc_vec(p, bl2);
      L.d_nblk2 = dalloc_vec(p, nb2);
    }
  }
}

tn_plan_impl::~tn_plan_impl() {
  for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
  if (stream) (void)hipStreamSynchronize(stream);
  for (void *ptr : allocs) (void)hipFree(ptr);
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

// Autotuner: for every distinct contraction shape with more than one
// eligible kernel form, time each form on the device (its own arguments,
// three launches between two events after a warm-up) and keep the fastest.
// The forms sum in different orders, so a decision changes the FP32
// rounding of a result: decisions are kept process-wide, keyed by the GPU
// architecture and the shape, and every later plan with that shape reuses
// them (two plans of one model built in one process run the same launches
// and give bit-identical results).  tn_tune_save / tn_tune_load carry the
// decisions across processes.  Operand contents do not matter for the
// timing (every access is at table offsets).
namespace {
using TuneKey = std::vector<int64_t>;
struct TuneCache {
  std::mutex mu;
  std::map<std::pair<std::string, TuneKey>, std::array<int, 3>> dec;
};
TuneCache &tune_cache() {
  static TuneCache c;
  return c;
}
std::string device_arch() {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  hipDeviceProp_t prop;
  hip_check(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
  std::string a = prop.gcnArchName;
  return a.substr(0, a.find(':'));
}
}  // namespace

static void set_form(tn_plan_t *p, Op *op, const std::array<int, 3> &f) {
  op->a.kind = f[0];
  op->a.ksplit = f[1];
  op->a.tile = f[2];
  op->a.prec = f[0] == 2 ? p->opts.dtype : 0;  // matrix-core operand precision of the dense form only
}

static void autotune_ops(tn_plan_t *p, const std::vector<Op *> &ops) {
  TuneCache &tc = tune_cache();
  const std::string arch = device_arch();
  hipEvent_t e0, e1;
  hip_check(hipEventCreate(&e0), "event");
  hip_check(hipEventCreate(&e1), "event");
  // (form bit, kind, workgroup split of the summed range, tile variant)
  static const int kForm[11][4] = {{1, 0, 1, 0},    {2, 1, 1, 0},   {4, 2, 1, 0},    {8, 3, 1, 0},
                                   {16, 4, 1, 0},   {32, 4, 4, 0},  {64, 4, 1, 1},   {128, 4, 1, 2},
                                   {256, 2, 1, 1},  {512, 0, 1, 1}, {1024, 1, 1, 1}};
  for (Op *op : ops) {
    if (op->split || op->seg >= 0) continue;
    std::vector<std::array<int, 3>> cands;
    for (auto &f : kForm)
      if (op->forms & f[0]) cands.push_back({f[1], f[2], f[3]});
    if (cands.size() < 2) continue;
    const ContractArgs &a = op->a;
    const TuneKey key = {op->semi, op->Y >= 0, op->nb, a.nR, a.nRl, a.nC, a.nCl, a.nS, a.nSl,
                         a.col_fastest, a.nB, a.nM, a.x_s_fast, a.y_n_fast, a.z_n_fast, op->forms,
                         a.batX, a.batY, p->opts.dtype};
    std::array<int, 3> best{-1, 1, 0};
    bool known = false;
    {
      std::lock_guard<std::mutex> lk(tc.mu);
      auto it = tc.dec.find({arch, key});
      if (it != tc.dec.end()) {
        best = it->second;
        known = std::find(cands.begin(), cands.end(), best) != cands.end();
      }
    }
    if (!known) {
      float best_ms = 0.f;
      best = {-1, 1, 0};
      for (auto cand : cands) {
        set_form(p, op, cand);
        hip_check(hipMemcpy(op->d_a, &op->a, sizeof(ContractArgs), hipMemcpyHostToDevice), "autotune");
        launch_contract(op->semi, op->Y >= 0, false, op->a, op->d_a, op->nb, p->stream);
        hip_check(hipEventRecord(e0, p->stream), "event");
        for (int r = 0; r < 3; ++r) launch_contract(op->semi, op->Y >= 0, false, op->a, op->d_a, op->nb, p->stream);
        hip_check(hipEventRecord(e1, p->stream), "event");
        hip_check(hipEventSynchronize(e1), "autotune");
        hip_check(hipGetLastError(), "autotune launch");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        if (best[0] < 0 || ms < best_ms) {
          best = cand;
          best_ms = ms;
        }
      }
      std::lock_guard<std::mutex> lk(tc.mu);
      auto ins = tc.dec.emplace(std::make_pair(arch, key), best);
      best = ins.first->second;  // another thread's decision for the shape wins if it came first
    }
    set_form(p, op, best);
    hip_check(hipMemcpy(op->d_a, &op->a, sizeof(ContractArgs), hipMemcpyHostToDevice), "autotune");
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// Decision file: one line per decision, "arch n k_0 ... k_{n-1} kind ksplit tile".
extern "C" tn_status tn_tune_save(const char *path, int64_t *n_saved) {
  return guard([&] {
    if (!path) throw TnError(TN_E_INVALID, "NULL path");
    TuneCache &tc = tune_cache();
    std::lock_guard<std::mutex> lk(tc.mu);
    FILE *f = std::fopen(path, "w");
    if (!f) throw TnError(TN_E_INVALID, std::string("cannot write ") + path);
    for (auto &kv : tc.dec) {
      std::fprintf(f, "%s %zu", kv.first.first.c_str(), kv.first.second.size());
      for (int64_t k : kv.first.second) std::fprintf(f, " %lld", (long long)k);
      std::fprintf(f, " %d %d %d\n", kv.second[0], kv.second[1], kv.second[2]);
    }
    const bool ok = std::fclose(f) == 0;
    if (!ok) throw TnError(TN_E_INVALID, std::string("cannot write ") + path);
    if (n_saved) *n_saved = (int64_t)tc.dec.size();
  });
}

extern "C" tn_status tn_tune_load(const char *path, int64_t *n_loaded) {
  return guard([&] {
    if (!path) throw TnError(TN_E_INVALID, "NULL path");
    FILE *f = std::fopen(path, "r");
    if (!f) throw TnError(TN_E_INVALID, std::string("cannot read ") + path);
    std::vector<std::pair<std::pair<std::string, TuneKey>, std::array<int, 3>>> got;
    char arch[64];
    size_t n = 0;
    bool bad = false;
    while (std::fscanf(f, "%63s %zu", arch, &n) == 2) {
      if (n > 64) { bad = true; break; }
      TuneKey key(n);
      for (size_t i = 0; i < n && !bad; ++i) {
        long long k = 0;
        if (std::fscanf(f, "%lld", &k) != 1) bad = true;
        key[i] = k;
      }
      std::array<int, 3> d{};
      if (bad || std::fscanf(f, "%d %d %d", &d[0], &d[1], &d[2]) != 3) { bad = true; break; }
      if (d[0] < 0 || d[0] > 4 || (d[1] != 1 && d[1] != 4) || d[2] < 0 || d[2] > 2) { bad = true; break; }
      got.push_back({{std::string(arch), key}, d});
    }
    const bool at_end = std::feof(f);
    std::fclose(f);
    if (bad || !at_end) throw TnError(TN_E_INVALID, std::string("malformed decision file ") + path);
    TuneCache &tc = tune_cache();
    std::lock_guard<std::mutex> lk(tc.mu);
    for (auto &g : got) tc.dec[g.first] = g.second;
    if (n_loaded) *n_loaded = (int64_t)got.size();
  });
}

extern "C" void tn_tune_clear(void) {
  TuneCache &tc = tune_cache();
  std::lock_guard<std::mutex> lk(tc.mu);
  tc.dec.clear();
}

static void build_mmap(tn_plan_t *p, const tn_net *net);
static void allocate_mmap(tn_plan_t *p);
static void upload_segments(tn_plan_t *p);

static void allocate(tn_plan_t *p, const tn_net *net) {
  // device work starts here: everything above is host-side planning
  hip_check(hipGetDevice(&p->device), "hipGetDevice");
  if (p->opts.hip_stream) {
    p->stream = (hipStream_t)p->opts.hip_stream;
  } else {
    hip_check(hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking), "hipStreamCreate");
    p->own_stream = true;
  }
  // slots: prepared leaves first, then constants, then everything reset per solve
  int slot = 0;
  std::vector<char> prepared(p->T.size(), 0), constant(p->T.size(), 0);
  for (auto &d : p->leaves_sum) prepared[d.slot] = 1;  // d.slot holds the tensor id here
  for (auto &gl : p->group_leaves)
    for (auto &d : gl) prepared[d.slot] = 1;
  if (p->seed_tensor >= 0) constant[p->seed_tensor] = 1;
  auto give = [&](int i) {
    p->T[i].slot = slot;
    slot += p->T[i].batched ? p->max_batch : 1;
  };
  for (size_t i = 0; i < p->T.size(); ++i)
    if (p->T[i].slot >= 0 && prepared[i]) give((int)i);
  for (size_t i = 0; i < p->T.size(); ++i)
    if (p->T[i].slot >= 0 && constant[i]) give((int)i);
  p->reset_begin = slot;
  for (size_t i = 0; i < p->T.size(); ++i)
    if (p->T[i].slot >= 0 && !prepared[i] && !constant[i]) give((int)i);
  p->reset_end = slot;
  p->n_slots = slot;
  for (auto &d : p->leaves_sum) d.slot = p->T[d.slot].slot;
  for (auto &gl : p->group_leaves)
    for (auto &d : gl) d.slot = p->T[d.slot].slot;
  // arena: factor stores, then tensors (256-byte aligned)
  int64_t off = 0;
  auto take = [&](int64_t n) {
    int64_t o = off;
    off += (n + 63) / 64 * 64;
    return o;
  };
  const int64_t fs_lin = take(net->n_values), fs_log = take(net->n_values);
  for (auto &t : p->T) t.off = take(t.size * (t.batched ? p->max_batch : 1));
  p->arena_floats = off;
  int64_t ioff = 0;
  for (auto &b : p->IB) {
    b.off = ioff;
    ioff += (b.size * (b.batched ? p->max_batch : 1) + 63) / 64 * 64;
  }
  p->iarena_ints = ioff;
  p->arena = dalloc<float>(p, (size_t)p->arena_floats);
  p->iarena = dalloc<int32_t>(p, (size_t)p->iarena_ints + 64);
  p->mx = dalloc<uint32_t>(p, (size_t)kMaxSubSlots * std::max(1, p->n_slots));
  p->ex = dalloc<int32_t>(p, (size_t)std::max(1, p->n_slots));
  hip_check(hipMemset(p->mx, 0, sizeof(uint32_t) * kMaxSubSlots * std::max(1, p->n_slots)), "memset");
  hip_check(hipMemset(p->ex, 0, sizeof(int32_t) * std::max(1, p->n_slots)), "memset");
  // factor stores: linear FP32 and log FP32 (host FP64 conversion, rounded once)
  std::vector<float> lin(net->n_values), lg(net->n_values);
  for (size_t f = 0; f < net->vals.size(); ++f)
    for (size_t i = 0; i < net->vals[f].size(); ++i) {
      const double x = net->vals[f][i];
      const int64_t o = net->val_off[f] + (int64_t)i;
      if (net->is_log) {
        lin[o] = (float)std::exp(x);
        lg[o] = (float)x;
      } else {
        lin[o] = (float)x;
        lg[o] = x > 0 ? (float)std::log(x) : -INFINITY;
      }
    }
  if (!lin.empty()) {
    hip_check(hipMemcpy(p->arena + fs_lin, lin.data(), lin.size() * 4, hipMemcpyHostToDevice), "upload");
    hip_check(hipMemcpy(p->arena + fs_log, lg.data(), lg.size() * 4, hipMemcpyHostToDevice), "upload");
  }
  auto fix_leaf = [&](LeafDesc &d, int tensor, bool maxdom) {
    d.dst = p->T[tensor].off;
    if (d.kind == 0) d.src += maxdom ? fs_log : fs_lin;
  };
  // the largest leaves of a set (up to kPrepBig, above 2^14 entries, not
  // interleaved) are prepared by several workgroups, one per 2^14 entries
  auto split_large = [&](std::vector<LeafDesc> &set) {
    std::vector<size_t> idx;
    for (size_t i = 0; i < set.size(); ++i) {
      set[i].nsub = 1;
      if (set[i].size > (1 << 14) && !(set[i].batched && p->inter)) idx.push_back(i);
    }
    std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return set[x].size > set[y].size; });
    for (size_t k = 0; k < idx.size() && k < (size_t)kPrepBig; ++k)
      set[idx[k]].nsub = std::min<int32_t>(kMaxSubSlots, (set[idx[k]].size + (1 << 14) - 1) >> 14);
  };
  // leaf descriptors carry the tensor id in dst until here
  for (auto &d : p->leaves_sum) fix_leaf(d, (int)d.dst, false);
  for (auto &d : p->leaves_max) fix_leaf(d, (int)d.dst, true);
  for (auto &gl : p->group_leaves)
    for (auto &d : gl) fix_leaf(d, (int)d.dst, false);
  for (auto &d : p->qleaves) fix_leaf(d, (int)d.dst, true);
  split_large(p->leaves_sum);
  split_large(p->leaves_max);
  for (auto &gl : p->group_leaves) split_large(gl);
  split_large(p->qleaves);
  p->d_tabs = dupload(p, p->tabs);
  p->d_gmap = dupload(p, p->gmap);
  p->d_obs = dupload(p, p->obs);
  p->d_evidence = dalloc<int32_t>(p, (size_t)p->max_batch * std::max(1, p->n_vars));
  if (!p->sliced.empty() || !p->groups.empty()) {
    p->d_slice_rows = dalloc<int32_t>(p, (size_t)kSliceChunk * std::max(1, p->n_vars));
    p->d_slice_lz = dalloc<double>(p, (size_t)kSliceChunk);
  }
  p->d_assign = dalloc<int32_t>(p, (size_t)p->max_batch * std::max(1, p->n_vars));
  p->d_out = dalloc<double>(p, (size_t)p->max_batch);
  p->d_part = dalloc<float>(p, (size_t)std::max<int64_t>(1, p->part_floats));
  p->d_parti = dalloc<int32_t>(p, (size_t)std::max<int64_t>(1, p->part_floats));
  for (auto &op : p->sum_tree.ops) fill_args(p, op);
  for (auto &op : p->max_tree.ops) fill_args(p, op);
  for (auto &op : p->bwd) fill_args(p, op);
  for (auto &g : p->groups)
    for (auto &op : g.ops) fill_args(p, op);
  for (auto &op : p->qtree.ops) fill_args(p, op);
  for (auto &op : p->samp_ops) fill_args(p, op);
  {
    std::vector<Op *> all;
    for (auto &op : p->sum_tree.ops) all.push_back(&op);
    for (auto &op : p->max_tree.ops) all.push_back(&op);
    for (auto &op : p->bwd) all.push_back(&op);
    for (auto &g : p->groups)
      for (auto &op : g.ops) all.push_back(&op);
    for (auto &op : p->qtree.ops) all.push_back(&op);
    for (auto &op : p->samp_ops) all.push_back(&op);
    std::vector<ContractArgs> host;
    for (Op *op : all) host.push_back(op->a);
    ContractArgs *d = dupload(p, host);
    for (size_t i = 0; i < all.size(); ++i) all[i]->d_a = d + i;
    if (p->opts.autotune) {
      autotune_ops(p, all);
      // the fused lists hold copies of the unfused contractions: same choice
      std::map<int, std::array<int, 3>> kind_of;  // output tensor -> form
      for (Op *op : all) kind_of[op->Z] = {op->a.kind, op->a.ksplit, op->a.tile};
      std::vector<std::vector<Op> *> lists{&p->ffwd, &p->fbwd, &p->max_tree.fops};
      for (auto &g : p->groups) lists.push_back(&g.fops);
      for (auto *L : lists)
        for (Op &op : *L)
          if (op.seg < 0 && op.a.kind != kKindMaxPair && kind_of.count(op.Z)) {
            op.a.kind = kind_of[op.Z][0];
            op.a.ksplit = kind_of[op.Z][1];
            op.a.tile = kind_of[op.Z][2];
          }
    }
  }
  p->sched_fwd = build_schedule(p, p->sum_tree.ops, false);
  p->sched_bwd = build_schedule(p, p->bwd, true);
  if (p->max_tree.fused) {  // arguments of the list with max-plus pairs
    std::vector<ContractArgs> host;
    for (auto &op : p->max_tree.fops) {
      fill_args(p, op);
      host.push_back(op.a);
    }
    ContractArgs *d = dupload(p, host);
    for (size_t k = 0; k < p->max_tree.fops.size(); ++k) p->max_tree.fops[k].d_a = d + k;
  }
  const std::vector<Op> &max_list = p->max_tree.fused ? p->max_tree.fops : p->max_tree.ops;
  p->sched_max = build_schedule(p, max_list, false);
  p->sched_q = build_schedule(p, p->qtree.ops, false);
  p->sched_samp = build_schedule(p, p->samp_ops, false);
  upload_schedule(p, p->sched_fwd, p->sum_tree.ops);
  upload_schedule(p, p->sched_bwd, p->bwd);
  upload_schedule(p, p->sched_max, max_list);
  upload_schedule(p, p->sched_q, p->qtree.ops);
  upload_schedule(p, p->sched_samp, p->samp_ops);
  for (auto &g : p->groups) {
    if (g.fused) {  // contraction arguments of the fused list's unfused ops
      std::vector<ContractArgs> host;
      for (auto &op : g.fops)
        if (op.seg < 0) {
          fill_args(p, op);
          host.push_back(op.a);
        }
      ContractArgs *d = dupload(p, host);
      size_t k = 0;
      for (auto &op : g.fops)
        if (op.seg < 0) op.d_a = d + k++;
    }
    const std::vector<Op> &gl = g.fused ? g.fops : g.ops;
    p->sched_groups.push_back(build_schedule(p, gl, false));
    upload_schedule(p, p->sched_groups.back(), gl);
  }
  if (!p->fused && !p->segs.empty()) upload_segments(p);
  if (p->fused) {
    for (auto &op : p->ffwd)
      if (op.seg < 0) fill_args(p, op);
    for (auto &op : p->fbwd)
      if (op.seg < 0) fill_args(p, op);
    std::vector<Op *> all;
    for (auto &op : p->ffwd)
      if (op.seg < 0) all.push_back(&op);
    for (auto &op : p->fbwd)
      if (op.seg < 0) all.push_back(&op);
    std::vector<ContractArgs> host;
    for (Op *op : all) host.push_back(op->a);
    ContractArgs *d = dupload(p, host);
    for (size_t i = 0; i < all.size(); ++i) all[i]->d_a = d + i;
    upload_segments(p);
    p->sched_ffwd = build_schedule(p, p->ffwd, false);
    p->sched_fbwd = build_schedule(p, p->fbwd, true);
    upload_schedule(p, p->sched_ffwd, p->ffwd);
    upload_schedule(p, p->sched_fbwd, p->fbwd);
  }
  p->d_leaves_sum = dupload(p, p->leaves_sum);
  p->d_leaves_max = dupload(p, p->leaves_max);
  p->d_qleaves = dupload(p, p->qleaves);
  for (auto &gl : p->group_leaves) p->d_group_leaves.push_back(dupload(p, gl));
  // seed of the reverse pass: ones, maximum 1, exponent 0
  if (p->seed_tensor >= 0) {
    const TensorBuf &s = p->T[p->seed_tensor];
    const int64_t n = s.size * (s.batched ? p->max_batch : 1);
    std::vector<float> ones(n, 1.f);
    hip_check(hipMemcpy(p->arena + s.off, ones.data(), n * 4, hipMemcpyHostToDevice), "upload");
    const int ns = s.batched ? p->max_batch : 1;
    std::vector<uint32_t> m(ns, 0x3f800000u);
    hip_check(hipMemcpy(p->mx + s.slot, m.data(), ns * 4, hipMemcpyHostToDevice), "upload");
  }
  // marginal / gradient descriptors
  for (auto &m : p->marg) {
    const TensorBuf &A = p->T[(int)m.adj], &Lf = p->T[(int)m.leaf];
    m.adj = A.off;
    m.leaf = Lf.off;
    m.adj_batched = A.batched;
    m.leaf_batched = Lf.batched;
    m.adj_bs = p->inter ? 1 : A.size;
    m.leaf_bs = p->inter ? 1 : Lf.size;
    m.adj_es = A.batched && p->inter ? p->max_batch : 1;
    m.leaf_es = Lf.batched && p->inter ? p->max_batch : 1;
  }
  p->d_marg_desc = dupload(p, p->marg);
  p->d_marg = dalloc<double>(p, (size_t)p->max_batch * std::max(1, p->marg_row));
  for (auto &g : p->grads) {
    const TensorBuf &A = p->T[(int)g.adj];
    g.slot = A.slot;
    g.adj = A.off;
    const TensorBuf &Lf = p->T[(int)g.leaf];
    g.leaf = Lf.off;
    g.leaf_batched = Lf.batched;
    g.leaf_bs = p->inter ? 1 : Lf.size;
    g.leaf_es = Lf.batched && p->inter ? p->max_batch : 1;
    g.adj_batched = A.batched;
    g.adj_bs = p->inter ? 1 : A.size;
    g.adj_es = A.batched && p->inter ? p->max_batch : 1;
  }
  p->d_grad_desc = dupload(p, p->grads);
  if (!p->grads.empty()) p->d_fmarg = dalloc<double>(p, (size_t)p->max_batch * std::max<int64_t>(1, net->n_values));
  for (auto &j : p->joint) {
    if (j.adj < 0) continue;
    const TensorBuf &A = p->T[(int)j.adj];
    j.adj = A.off;
    j.adj_batched = A.batched;
    j.adj_bs = p->inter ? 1 : A.size;
    j.adj_es = A.batched && p->inter ? p->max_batch : 1;
  }
  if (!p->joint.empty()) {
    p->d_joint_desc = dupload(p, p->joint);
    p->d_joint_tab = dupload(p, p->joint_tab);
    p->d_joint = dalloc<double>(p, (size_t)p->max_batch * std::max(1, p->joint_row));
  }
  auto fix_back = [&](TreeExec &t) {
    for (auto &s : t.back) {
      const IntBuf &b = p->IB[(int)s.arg];
      s.arg = b.off;
      s.bs = b.batched ? (p->inter ? 1 : b.size) : 0;
      s.es = b.batched && p->inter ? p->max_batch : 1;
    }
  };
  fix_back(p->max_tree);
  fix_back(p->qtree);
  p->d_back = dupload(p, p->max_tree.back);
  p->d_back_meta = dupload(p, p->max_tree.back_meta);
  p->d_back_lev = dupload(p, p->max_tree.back_lev);
  p->d_qback_lev = dupload(p, p->qtree.back_lev);
  p->d_qback = dupload(p, p->qtree.back);
  p->d_qback_meta = dupload(p, p->qtree.back_meta);
  for (auto &s : p->samp) {
    s.A = p->T[(int)s.A].off;
    if (s.B >= 0) s.B = p->T[(int)s.B].off;
    s.Ar = p->T[(int)s.Ar].off;
    if (s.Br >= 0) s.Br = p->T[(int)s.Br].off;
  }
  p->d_samp = dupload(p, p->samp);
  p->d_samp_meta = dupload(p, p->samp_meta);
  if (p->is_mmap) allocate_mmap(p);
}


// ---------------------------------------------------------------------------
// fused chain segments
// ---------------------------------------------------------------------------
static int64_t index_in(const Labels &L, const std::vector<int> &val, const std::vector<int> &card) {
  int64_t k = 0;
  for (int v : L) k = k * card[v] + val[v];
  return k;
}

// Try to describe ops[first..] (chain order) as one segment; fills sp and
// returns true if all size limits hold.
static bool describe_segment(tn_plan_t *p, const std::vector<Op> &ops, const std::vector<int> &chain, SegPlan &sp,
                             bool commit) {
  const auto &card = p->card;
  const int L = (int)chain.size();
  std::vector<Labels> V(L + 1), U(L);
  V[0] = p->T[ops[chain[0]].X].lab;
  for (int j = 0; j < L; ++j) {
    U[j] = p->T[ops[chain[j]].Y].lab;
    V[j + 1] = p->T[ops[chain[j]].Z].lab;
  }
  Labels T;
  for (int j = 0; j < L; ++j) {
    Labels E = minus(unite(V[j], U[j]), V[j + 1]);
    T = unite(T, unite(U[j], E));
    Labels d1 = minus(V[j], V[j + 1]), d2 = minus(V[j + 1], V[j]);
    T = unite(T, unite(d1, d2));
  }
  const Labels O = minus(V[0], T);
  if (minus(O, V[L]).size()) return false;  // outer labels must survive
  std::vector<Labels> Loc(L + 1);
  for (int j = 0; j <= L; ++j) Loc[j] = inter(V[j], T);
  for (int j = 0; j <= L; ++j)
    if (numel(Loc[j], card) > kSegMaxLocal) return false;
  for (int j = 0; j < L; ++j)
    if (numel(unite(Loc[j], U[j]), card) > 1024) return false;  // triples of a step
  const int64_t nO = numel(O, card);
  if (nO < 256) return false;
  // LDS of the sweeps: 32 x 32 work areas (two for the composed map, three
  // for the adjoints), P_0 .. P_{L-1} (adjoints), 64 floats of small operand
  // per step and the index lists (three CSR orders of every step's triples)
  const int64_t n_in0 = numel(Loc[0], card);
  int64_t lists = 0, pstore = 0;
  for (int j = 0; j < L; ++j) {
    const int64_t nnz = numel(unite(Loc[j], U[j]), card);
    lists += numel(Loc[j + 1], card) + numel(Loc[j], card) + numel(U[j], card) + 3 + 6 * nnz;
    pstore += numel(Loc[j], card) * n_in0;
  }
  const int64_t fin_lds = 3 * 1024 + pstore + 64 * L + lists;
  if (fin_lds > 15 * 1024) return false;
  if (!commit) return true;
  sp.ops = chain;
  sp.loc_in = Loc[0];
  sp.loc_out = Loc[L];
  sp.outer = O;
  sp.c0 = ops[chain[0]].X;
  sp.cL = ops[chain[L - 1]].Z;
  sp.nO = (uint32_t)nO;
  sp.fin_lds = (int32_t)fin_lds;
  sp.mat_lds = (int32_t)(2 * 1024 + 64 * L + lists);
  const size_t os = lo_split(O, card);
  sp.nOl = (uint32_t)numel(Labels(O.begin() + os, O.end()), card);
  add_tabs(p, O, os, V[0], sp.oX);
  add_tabs(p, O, os, V[L], sp.oZ);
  auto local_tab = [&](const Labels &Lc, const Labels &TL) {
    int64_t off = (int64_t)p->tabs.size();
    const int64_t n = numel(Lc, card);
    std::vector<int> d(Lc.size(), 0);
    for (int64_t i = 0; i < n; ++i) {
      int64_t o = 0;
      for (size_t k = 0; k < Lc.size(); ++k) o += (int64_t)d[k] * stride_in(TL, Lc[k], card);
      p->tabs.push_back((int32_t)o);
      for (int k = (int)Lc.size() - 1; k >= 0; --k) {
        if (++d[k] < card[Lc[k]]) break;
        d[k] = 0;
      }
    }
    return off;
  };
  // carrier labels faster than its fastest outer label (all local): the
  // tile moves take them fastest, then the outer assignment; a count that is
  // not a power of two takes every local entry fastest
  auto lo_shift = [&](const Labels &Vc) {
    int64_t n = 1;
    for (int v : Vc)
      if (v > O.back()) n *= card[v];
    int sh = 0;
    while ((int64_t(1) << sh) < n) ++sh;
    return (int64_t(1) << sh) == n && sh <= 5 ? sh : 5;
  };
  sp.in_lo_shift = lo_shift(V[0]);
  sp.out_lo_shift = lo_shift(V[L]);
  sp.inX = local_tab(Loc[0], V[0]);
  sp.outZ = local_tab(Loc[L], V[L]);
  sp.n_in0 = (int32_t)numel(Loc[0], card);
  sp.n_outL = (int32_t)numel(Loc[L], card);
  sp.steps.clear();
  std::vector<int32_t> blk;  // the segment's lists, offsets relative to its start
  std::vector<int> val(p->n_vars, 0);
  for (int j = 0; j < L; ++j) {
    SegStep st{};
    st.y = ops[chain[j]].Y;  // tensor id until allocation
    st.ny = (int32_t)numel(U[j], card);
    st.n_in = (int32_t)numel(Loc[j], card);
    st.n_out = (int32_t)numel(Loc[j + 1], card);
    const Labels W = unite(Loc[j], U[j]);
    const int64_t nW = numel(W, card);
    std::vector<std::array<int32_t, 3>> tri;  // (in, out, s), enumeration order
    std::vector<int> d(W.size(), 0);
    for (int64_t w = 0; w < nW; ++w) {
      for (size_t k = 0; k < W.size(); ++k) val[W[k]] = d[k];
      int64_t so = 0;
      for (int v : U[j]) so += (int64_t)val[v] * stride_in(U[j], v, card);
      tri.push_back({(int32_t)index_in(Loc[j], val, card), (int32_t)index_in(Loc[j + 1], val, card), (int32_t)so});
      for (int k = (int)W.size() - 1; k >= 0; --k) {
        if (++d[k] < card[W[k]]) break;
        d[k] = 0;
      }
    }
    st.nnz = (int32_t)tri.size();
    // CSR lists grouped by key (stable: enumeration order within a group,
    // so every sum runs in a fixed order)
    auto csr = [&](int key, int n, int a1, int a2, int32_t &ptr, int32_t &l1, int32_t &l2) {
      std::vector<int32_t> cnt(n + 1, 0);
      for (auto &t : tri) cnt[t[key] + 1]++;
      for (int i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
      ptr = (int32_t)blk.size();
      blk.insert(blk.end(), cnt.begin(), cnt.end());
      std::vector<int32_t> x1(tri.size()), x2(tri.size()), pos(cnt.begin(), cnt.end() - 1);
      for (auto &t : tri) {
        const int32_t q = pos[t[key]]++;
        x1[q] = t[a1];
        x2[q] = t[a2];
      }
      l1 = (int32_t)blk.size();
      blk.insert(blk.end(), x1.begin(), x1.end());
      l2 = (int32_t)blk.size();
      blk.insert(blk.end(), x2.begin(), x2.end());
    };
    csr(1, st.n_out, 0, 2, st.fo_ptr, st.fo_in, st.fo_s);
    csr(0, st.n_in, 1, 2, st.bi_ptr, st.bi_out, st.bi_s);
    csr(2, st.ny, 0, 1, st.bs_ptr, st.bs_in, st.bs_out);
    sp.steps.push_back(st);
  }
  sp.list_off = (int64_t)p->tabs.size();
  sp.list_len = (int32_t)blk.size();
  if (sp.list_len != lists) throw TnError(TN_E_INVALID, "internal: segment list size");
  p->tabs.insert(p->tabs.end(), blk.begin(), blk.end());
  double b = 4.0 * (double)(p->T[sp.c0].size + p->T[sp.cL].size);
  sp.bytes_fwd = b;
  sp.bytes_bwd = 4.0 * (double)(2 * p->T[sp.c0].size + p->T[sp.cL].size);
  for (int i : chain) sp.flops += ops[i].flops;
  return true;
}

// Labels faster in a carrier (labels TL) than all of the tile's column
// labels `cols`: log2 of their assignments, when a power of two up to 2^5,
// else 5 (every local entry fastest).
static int32_t tile_lo_shift(const Labels &loc, const Labels &cols, const std::vector<int> &card) {
  const int fc = cols.empty() ? -1 : cols.back();
  int64_t n = 1;
  for (int v : loc)
    if (v > fc) n *= card[v];
  int sh = 0;
  while ((int64_t(1) << sh) < n) ++sh;
  return (int64_t(1) << sh) == n && sh <= 5 ? sh : 5;
}

// Segments s1 and s2 (s2's input carrier is s1's output) as one carrier
// pass: the labels of the pass (DSegArgs), the workgroup shape and the
// tables.  False when a tile would not fit (at most 32 assignments of Q and
// of R, at least four outer assignments per workgroup) or would leave the
// large carriers' tiles mostly empty.  Where one map's local sets are small
// enough, the slowest common outer label o* joins its rows and columns (the
// map becomes M (x) I; in the first map o* also joins R, in the second Q):
// the tiles then hold more local entries and fewer outer assignments,
// which fills them where the local sets alone would fill half.
static bool describe_pair(tn_plan_t *p, int s1, int s2, DSegPlan &dp, bool commit) {
  const SegPlan &a = p->segs[s1], &b = p->segs[s2];
  const auto &card = p->card;
  const Labels &V0 = p->T[a.c0].lab, &V2 = p->T[b.cL].lab;
  const Labels &A = a.loc_in, &B = a.loc_out, &C = b.loc_in, &D = b.loc_out;
  const Labels P = inter(C, B), Q = inter(C, a.outer), R = minus(B, C);
  Labels O = minus(a.outer, Q);
  if (unite(P, Q) != C || !minus(O, V2).empty()) return false;
  const int64_t nQ = numel(Q, card), nR = numel(R, card);
  if (nQ > kSegMaxLocal || nR > kSegMaxLocal || O.empty()) return false;
  // a large carrier in a tile it fills less than three quarters of runs
  // faster in a pass of its own
  const bool lx = p->T[a.c0].size >= (1 << 16), lz = p->T[b.cL].size >= (1 << 16);
  // workgroup shape with o* (k1 or k2 assignments) in the first or second
  // map; false when it does not fit or does not fill the tiles
  auto shape = [&](int64_t k1, int64_t k2, int &nob) {
    const int64_t q = nQ * k2, r = nR * k1;
    if (a.n_in0 * k1 > kSegMaxLocal || a.n_outL * k1 > kSegMaxLocal || r > kSegMaxLocal ||
        b.n_in0 * k2 > kSegMaxLocal || b.n_outL * k2 > kSegMaxLocal || q > kSegMaxLocal)
      return false;
    nob = kSegOuterBlock;
    while ((int64_t)nob * std::max(q, r) > kSegOuterBlock) nob >>= 1;
    const double use_x = (double)a.n_in0 * k1 * q * nob / (kSegMaxLocal * kSegOuterBlock);
    const double use_z = (double)b.n_outL * k2 * r * nob / (kSegMaxLocal * kSegOuterBlock);
    return nob >= 4 && !((use_x < 0.75 && lx) || (use_z < 0.75 && lz));
  };
  int nob = 0;
  int64_t aug1 = 1, aug2 = 1;
  if (!shape(1, 1, nob)) {
    if (O.size() < 2) return false;
    const int64_t k = card[O.front()];
    if (shape(k, 1, nob)) aug1 = k;
    else if (shape(1, k, nob)) aug2 = k;
    else return false;
  }
  const int ostar = O.front();
  if (aug1 > 1 || aug2 > 1) O.erase(O.begin());
  const int64_t nO = numel(O, card);
  if (nO >= (int64_t(1) << 31)) return false;
  if (!commit) return true;
  // the tiles' row orders, with o* (when moved) slowest
  auto with = [&](bool moved, const Labels &L) {
    Labels o;
    if (moved) o.push_back(ostar);
    o.insert(o.end(), L.begin(), L.end());
    return o;
  };
  const Labels Ao = with(aug1 > 1, A), Bo = with(aug1 > 1, B), Ro = with(aug1 > 1, R);
  const Labels Co = with(aug2 > 1, C), Do = with(aug2 > 1, D), Qo = with(aug2 > 1, Q);
  const Labels Rs = aug1 > 1 ? unite(R, Labels{ostar}) : R, Qs = aug2 > 1 ? unite(Q, Labels{ostar}) : Q;
  dp.s1 = s1;
  dp.s2 = s2;
  dp.aug1 = (int32_t)aug1;
  dp.aug2 = (int32_t)aug2;
  dp.nO = (uint32_t)nO;
  const size_t os = lo_split(O, card);
  dp.nOl = (uint32_t)numel(Labels(O.begin() + os, O.end()), card);
  add_tabs(p, O, os, V0, dp.oX);
  add_tabs(p, O, os, V2, dp.oZ);
  dp.nob = nob;
  dp.nQ = (int32_t)(nQ * aug2);
  dp.nR = (int32_t)(nR * aug1);
  // column order: the tile's fastest column label decides which part of a
  // column runs fastest
  const Labels colX = unite(Qs, O), colZ = unite(Rs, O);
  dp.q_fast = !Qs.empty() && Qs.back() == colX.back();
  dp.r_fast = !Rs.empty() && Rs.back() == colZ.back();
  dp.in_lo_shift = tile_lo_shift(A, colX, card);
  dp.out_lo_shift = tile_lo_shift(D, colZ, card);
  dp.n_part = (int32_t)((nO + nob - 1) / nob);
  std::vector<int32_t> t(kDSegTab * kSegMaxLocal, 0);
  std::vector<int> val(p->n_vars, 0);
  // offsets of the assignments of Lc (row-major) in a carrier with labels TL
  auto offsets = [&](const Labels &Lc, const Labels &TL, int row) {
    const int64_t n = numel(Lc, card);
    std::vector<int> d(Lc.size(), 0);
    for (int64_t i = 0; i < n; ++i) {
      int64_t o = 0;
      for (size_t k = 0; k < Lc.size(); ++k) o += (int64_t)d[k] * stride_in(TL, Lc[k], card);
      t[row * kSegMaxLocal + i] = (int32_t)o;
      for (int k = (int)Lc.size() - 1; k >= 0; --k) {
        if (++d[k] < card[Lc[k]]) break;
        d[k] = 0;
      }
    }
  };
  offsets(Ao, V0, 0);
  offsets(Do, V2, 1);
  offsets(Qo, V0, 2);
  offsets(Ro, V2, 3);
  offsets(Ro, Bo, 6);  // per r: its part of the row in the first map's output tile
  {  // per c in C: the P part of its row in the first map's output tile and its index in Q
    const int64_t n = numel(Co, card);
    std::vector<int> d(Co.size(), 0);
    for (int64_t i = 0; i < n; ++i) {
      for (size_t k = 0; k < Co.size(); ++k) val[Co[k]] = d[k];
      int64_t pb = 0, qi = 0;
      for (int v : P) pb += (int64_t)val[v] * stride_in(Bo, v, card);
      for (int v : Qo) qi += (int64_t)val[v] * stride_in(Qo, v, card);
      t[4 * kSegMaxLocal + i] = (int32_t)pb;
      t[5 * kSegMaxLocal + i] = (int32_t)qi;
      for (int k = (int)Co.size() - 1; k >= 0; --k) {
        if (++d[k] < card[Co[k]]) break;
        d[k] = 0;
      }
    }
  }
  dp.tab = (int64_t)p->tabs.size();
  p->tabs.insert(p->tabs.end(), t.begin(), t.end());
  dp.bytes_fwd = 4.0 * (double)(p->T[a.c0].size + p->T[b.cL].size);
  dp.bytes_bwd = 4.0 * (double)(2 * p->T[a.c0].size + p->T[b.cL].size);
  dp.flops = a.flops + b.flops;
  return true;
}

// Pairs of consecutive segments along each chain, from its start (segments
// s_begin.. of the plan).
static void plan_pairs(tn_plan_t *p, size_t s_begin) {
  std::map<int, int> by_input;  // input carrier -> segment
  for (size_t si = s_begin; si < p->segs.size(); ++si) by_input[p->segs[si].c0] = (int)si;
  std::vector<char> has_prev(p->segs.size(), 0);
  for (size_t si = s_begin; si < p->segs.size(); ++si) {
    auto it = by_input.find(p->segs[si].cL);
    if (it != by_input.end()) has_prev[it->second] = 1;
  }
  for (size_t s0 = s_begin; s0 < p->segs.size(); ++s0) {
    if (has_prev[s0]) continue;
    int cur = (int)s0;
    while (cur >= 0) {
      auto it = by_input.find(p->segs[cur].cL);
      const int nxt = it == by_input.end() ? -1 : it->second;
      DSegPlan dp;
      if (nxt >= 0 && describe_pair(p, cur, nxt, dp, false)) {
        describe_pair(p, cur, nxt, dp, true);
        p->segs[cur].pair = p->segs[nxt].pair = (int)p->dsegs.size();
        p->dsegs.push_back(dp);
        auto it2 = by_input.find(p->segs[nxt].cL);
        cur = it2 == by_input.end() ? -1 : it2->second;
      } else {
        cur = nxt;
      }
    }
  }
}

// Fused segments over a forward op list: chains of sum-product contractions
// that absorb small operands (<= 64 entries) into a large carrier (>= 4096),
// among the ops that `allowed` admits.  Appends the segments (and pairs of
// consecutive ones) to the plan, writes the fused forward list to `fwd` and
// returns every op's segment (-1: none); fwd stays empty without segments.
static std::vector<int> fuse_forward(tn_plan_t *p, const std::vector<Op> &ops, const std::vector<char> &allowed,
                                     std::vector<Op> &fwd) {
  const int n = (int)ops.size();
  const size_t s_begin = p->segs.size();
  std::map<int, int> prod;
  for (int i = 0; i < n; ++i) prod[ops[i].Z] = i;
  std::vector<char> chainable(n, 0);
  for (int i = 0; i < n; ++i) {
    const Op &op = ops[i];
    chainable[i] = allowed[i] && op.semi == SEMI_SUM && op.Y >= 0 && !op.split && p->T[op.Y].size <= 64 &&
                   p->T[op.X].size >= 4096 && !p->T[op.X].batched && !p->T[op.Y].batched;
  }
  std::vector<int> next(n, -1), has_prev(n, 0);
  for (int i = 0; i < n; ++i) {
    if (!chainable[i]) continue;
    auto it = prod.find(ops[i].X);
    if (it != prod.end() && chainable[it->second]) {
      next[it->second] = i;
      has_prev[i] = 1;
    }
  }
  std::vector<int> seg_of(n, -1);
  for (int s0 = 0; s0 < n; ++s0) {
    if (!chainable[s0] || has_prev[s0]) continue;
    int cur = s0;
    while (cur >= 0) {
      std::vector<int> chain{cur};
      SegPlan probe;
      while (next[chain.back()] >= 0 && (int)chain.size() < kSegMaxSteps) {
        chain.push_back(next[chain.back()]);
        if (!describe_segment(p, ops, chain, probe, false)) {
          chain.pop_back();
          break;
        }
      }
      int after = next[chain.back()];
      if (chain.size() >= 2 && describe_segment(p, ops, chain, probe, false)) {
        SegPlan sp;
        describe_segment(p, ops, chain, sp, true);
        for (int i : chain) seg_of[i] = (int)p->segs.size();
        p->segs.push_back(std::move(sp));
      }
      cur = after;
    }
  }
  if (p->segs.size() == s_begin) return seg_of;
  if (p->opts.no_fuse == 0) plan_pairs(p, s_begin);
  // forward list: at the position of a segment's last node, the composed
  // map (it reads the small operands only, so the schedule hoists it) and
  // the carrier transform
  for (size_t si = s_begin; si < p->segs.size(); ++si) {
    SegPlan &sp = p->segs[si];
    sp.mt = new_raw_tensor(p, (int64_t)sp.n_outL * sp.n_in0, true);
  }
  for (int i = 0; i < n; ++i) {
    if (seg_of[i] < 0) {
      fwd.push_back(ops[i]);
      continue;
    }
    SegPlan &sp = p->segs[seg_of[i]];
    if (i != sp.ops.back()) continue;
    const int pr = sp.pair;
    Op m;
    m.seg = seg_of[i];
    m.seg_kind = 3;
    m.Z = sp.mt;
    for (int j : sp.ops) m.ins.push_back(ops[j].Y);
    for (int j : sp.ops) m.flops += 2.0 * p->T[ops[j].Y].size * sp.n_in0;
    m.bytes = 4.0 * sp.n_outL * sp.n_in0;
    fwd.push_back(m);
    if (pr >= 0 && p->dsegs[pr].s1 == seg_of[i]) continue;  // its carrier pass is the pair's
    Op op;
    if (pr >= 0) {  // both segments of the pair: C_0 -> C_2
      const DSegPlan &dp = p->dsegs[pr];
      op.seg = pr;
      op.seg_kind = 5;
      op.X = p->segs[dp.s1].c0;
      op.Z = sp.cL;
      op.ins.push_back(p->segs[dp.s1].mt);
      op.ins.push_back(sp.mt);
      op.flops = dp.flops;
      op.bytes = dp.bytes_fwd;
    } else {
      op.seg = seg_of[i];
      op.seg_kind = 1;
      op.X = sp.c0;
      op.Z = sp.cL;
      op.ins.push_back(sp.mt);
      op.flops = sp.flops;
      op.bytes = sp.bytes_fwd;
    }
    fwd.push_back(op);
  }
  return seg_of;
}

static void build_fusion(tn_plan_t *p, std::vector<char> &need, int L_leaves) {
  const std::vector<Op> &ops = p->sum_tree.ops;
  const int n = (int)ops.size();
  std::map<int, int> node_of;  // node of the sum tree that holds each tensor
  for (size_t c = 0; c < p->sum_tree.node_tensor.size(); ++c) node_of[p->sum_tree.node_tensor[c]] = (int)c;
  std::vector<char> allowed(n, 0);
  for (int i = 0; i < n; ++i)  // the reverse segment needs the carriers' adjoints
    allowed[i] = ops[i].X >= 0 && node_of.count(ops[i].X) && need[node_of.at(ops[i].X)];
  fuse_forward(p, ops, allowed, p->ffwd);
  if (p->segs.empty()) return;
  p->fused = true;
  // reverse list: the two adjoint contractions of every fused node are
  // replaced by one reverse segment at the position of the first of them
  std::map<int, int> adj_to_seg;  // adjoint tensor produced by a replaced op -> segment
  for (size_t si = 0; si < p->segs.size(); ++si) {
    SegPlan &sp = p->segs[si];
    sp.g = p->adj_tensor[node_of.at(sp.cL)];
    sp.c0bar = p->adj_tensor[node_of.at(sp.c0)];
    bool any = false;
    for (size_t j = 0; j < sp.ops.size(); ++j) {
      const Op &fo = ops[sp.ops[j]];
      const int ynode = node_of.at(fo.Y), xnode = node_of.at(fo.X);
      const int ybar = need[ynode] ? p->adj_tensor[ynode] : -1;
      sp.ybar_tensor.push_back(ybar);
      if (ybar >= 0) {
        any = true;
        adj_to_seg[ybar] = (int)si;
      }
      if (p->adj_tensor[xnode] >= 0) adj_to_seg[p->adj_tensor[xnode]] = (int)si;
    }
    if (any) {
      sp.n_part = sp.pair >= 0 ? p->dsegs[sp.pair].n_part : (int32_t)((sp.nO + kSegOuterBlock - 1) / kSegOuterBlock);
      sp.spt = new_raw_tensor(p, (int64_t)sp.n_part * sp.n_outL * sp.n_in0, true);
    }
  }
  std::vector<char> emitted(p->segs.size(), 0), pair_emitted(p->dsegs.size(), 0);
  for (const Op &op : p->bwd) {
    auto it = adj_to_seg.find(op.Z);
    if (it == adj_to_seg.end()) {
      p->fbwd.push_back(op);
      continue;
    }
    const int si = it->second;
    if (emitted[si]) continue;
    emitted[si] = 1;
    SegPlan &sp = p->segs[si];
    if (sp.pair < 0) {
      Op b;
      b.seg = si;
      b.seg_kind = 2;
      b.X = sp.g;
      b.Z = sp.c0bar;
      b.ins.push_back(sp.c0);
      b.ins.push_back(sp.mt);
      if (sp.spt >= 0) b.outs.push_back(sp.spt);
      b.flops = 2 * sp.flops;
      b.bytes = sp.bytes_bwd;
      p->fbwd.push_back(b);
    } else if (!pair_emitted[sp.pair]) {  // the pair's reverse pass: adjoint of C_2 -> adjoint of C_0
      pair_emitted[sp.pair] = 1;
      const DSegPlan &dp = p->dsegs[sp.pair];
      const SegPlan &s1 = p->segs[dp.s1], &s2 = p->segs[dp.s2];
      Op b;
      b.seg = sp.pair;
      b.seg_kind = 6;
      b.X = s2.g;
      b.Z = s1.c0bar;
      b.ins.push_back(s1.c0);
      b.ins.push_back(s1.mt);
      b.ins.push_back(s2.mt);
      if (s1.spt >= 0) b.outs.push_back(s1.spt);
      if (s2.spt >= 0) b.outs.push_back(s2.spt);
      b.flops = 2 * dp.flops;
      b.bytes = dp.bytes_bwd;
      p->fbwd.push_back(b);
    }
    if (sp.spt < 0) continue;
    Op f;
    f.seg = si;
    f.seg_kind = 4;
    f.X = sp.spt;
    for (size_t j = 0; j < sp.ops.size(); ++j) {
      f.ins.push_back(ops[sp.ops[j]].Y);
      if (sp.ybar_tensor[j] >= 0) {
        if (f.Z < 0) f.Z = sp.ybar_tensor[j];
        f.outs.push_back(sp.ybar_tensor[j]);
      }
    }
    f.bytes = 4.0 * (double)sp.n_part * sp.n_outL * sp.n_in0;
    f.flops = 2.0 * (double)sp.n_part * sp.n_outL * sp.n_in0;
    p->fbwd.push_back(f);
  }
  // a pair never writes its intermediate carrier C_1 nor its adjoint: no
  // other contraction may read them
  for (const DSegPlan &dp : p->dsegs) {
    const int c1 = p->segs[dp.s1].cL, c1bar = p->segs[dp.s1].g;
    for (const auto *L : {&p->ffwd, &p->fbwd})
      for (const Op &op : *L) {
        if (op.seg >= 0 && op.seg_kind != 1 && op.seg_kind != 2) continue;  // small operands / pairs
        bool reads = op.X == c1 || op.Y == c1 || op.X == c1bar || op.Y == c1bar;
        for (int t : op.ins) reads = reads || t == c1 || t == c1bar;
        if (reads) throw TnError(TN_E_INVALID, "internal: a paired segments' carrier has another reader");
      }
  }
  (void)L_leaves;
}

static void upload_segments(tn_plan_t *p) {
  for (SegPlan &sp : p->segs) {
    for (size_t j = 0; j < sp.steps.size(); ++j) {
      SegStep &st = sp.steps[j];
      const int yt = (int)st.y;
      st.y = p->T[yt].off;
      st.yslot = p->T[yt].slot;
      if (j < sp.ybar_tensor.size() && sp.ybar_tensor[j] >= 0) {
        st.ybar = p->T[sp.ybar_tensor[j]].off;
        st.ybar_slot = p->T[sp.ybar_tensor[j]].slot;
      }
    }
  }
  for (int kind = 0; kind < 2; ++kind) {
    std::vector<SegArgs> &H = kind ? p->seg_bwd_h : p->seg_fwd_h;
    for (SegPlan &sp : p->segs) {
      SegArgs a;
      a.arena = p->arena;
      a.mx = p->mx;
      a.ex = p->ex;
      a.mx_stride = std::max(1, p->n_slots);
      a.nO = sp.nO;
      a.nOl = sp.nOl;
      if ((sp.nOl & (sp.nOl - 1)) == 0) {
        int sh = 0;
        while ((1u << sh) < sp.nOl) ++sh;
        a.ol_shift = sh;
      }
      a.oX = Tab2{p->d_tabs + sp.oX[0], p->d_tabs + sp.oX[1]};
      a.oZ = Tab2{p->d_tabs + sp.oZ[0], p->d_tabs + sp.oZ[1]};
      a.inX = p->d_tabs + sp.inX;
      a.outZ = p->d_tabs + sp.outZ;
      a.n_in0 = sp.n_in0;
      a.n_outL = sp.n_outL;
      a.in_lo_shift = sp.in_lo_shift;
      a.out_lo_shift = sp.out_lo_shift;
      a.lists = p->d_tabs + sp.list_off;
      a.n_steps = (int32_t)sp.steps.size();
      a.list_len = sp.list_len;
      a.prec = p->opts.dtype;
      a.mat_lds = sp.mat_lds;
      a.fin_lds = sp.fin_lds;
      a.M = p->T[sp.mt].off;
      a.slotM = p->T[sp.mt].slot;
      a.X = p->T[sp.c0].off;
      a.slotX = p->T[sp.c0].slot;
      std::vector<SegStep> st = sp.steps;
      if (!kind) {
        for (auto &x : st) x.ybar = -1;
        a.Z = p->T[sp.cL].off;
        a.slotZ = p->T[sp.cL].slot;
      } else if (sp.g >= 0) {  // segments of a forward-only list have no reverse step
        a.G = p->T[sp.g].off;
        a.slotG = p->T[sp.g].slot;
        a.Z = p->T[sp.c0bar].off;
        a.slotZ = p->T[sp.c0bar].slot;
        if (sp.spt >= 0) {
          a.Sp = p->T[sp.spt].off;
          a.slotSp = p->T[sp.spt].slot;
          a.n_part = sp.n_part;
        }
      }
      a.steps = dupload(p, st);
      H.push_back(a);
    }
    SegArgs *d = dupload(p, H);
    if (kind) p->d_seg_bwd = d;
    else p->d_seg_fwd = d;
  }
  for (int kind = 0; kind < 2; ++kind) {
    std::vector<DSegArgs> &H = kind ? p->dseg_bwd_h : p->dseg_fwd_h;
    for (const DSegPlan &dp : p->dsegs) {
      const SegPlan &s1 = p->segs[dp.s1], &s2 = p->segs[dp.s2];
      DSegArgs a;
      a.arena = p->arena;
      a.mx = p->mx;
      a.ex = p->ex;
      a.mx_stride = std::max(1, p->n_slots);
      a.X = p->T[s1.c0].off;
      a.slotX = p->T[s1.c0].slot;
      a.M1 = p->T[s1.mt].off;
      a.slotM1 = p->T[s1.mt].slot;
      a.M2 = p->T[s2.mt].off;
      a.slotM2 = p->T[s2.mt].slot;
      a.nO = dp.nO;
      a.nOl = dp.nOl;
      if ((dp.nOl & (dp.nOl - 1)) == 0) {
        int sh = 0;
        while ((1u << sh) < dp.nOl) ++sh;
        a.ol_shift = sh;
      }
      a.oX = Tab2{p->d_tabs + dp.oX[0], p->d_tabs + dp.oX[1]};
      a.oZ = Tab2{p->d_tabs + dp.oZ[0], p->d_tabs + dp.oZ[1]};
      a.nob = dp.nob;
      a.aug1 = dp.aug1;
      a.aug2 = dp.aug2;
      a.nA = s1.n_in0 * dp.aug1;
      a.nB = s1.n_outL * dp.aug1;
      a.nC = s2.n_in0 * dp.aug2;
      a.nD = s2.n_outL * dp.aug2;
      a.nQ = dp.nQ;
      a.nR = dp.nR;
      a.q_fast = dp.q_fast;
      a.r_fast = dp.r_fast;
      a.in_lo_shift = dp.in_lo_shift;
      a.out_lo_shift = dp.out_lo_shift;
      a.tab = p->d_tabs + dp.tab;
      a.prec = p->opts.dtype;
      if (!kind) {
        a.Z = p->T[s2.cL].off;
        a.slotZ = p->T[s2.cL].slot;
      } else if (s2.g >= 0) {
        a.G = p->T[s2.g].off;
        a.slotG = p->T[s2.g].slot;
        a.Z = p->T[s1.c0bar].off;
        a.slotZ = p->T[s1.c0bar].slot;
        if (s1.spt >= 0) {
          if (s1.n_part != dp.n_part) throw TnError(TN_E_INVALID, "internal: pair partial count");
          a.Sp1 = p->T[s1.spt].off;
          a.slotSp1 = p->T[s1.spt].slot;
        }
        if (s2.spt >= 0) {
          if (s2.n_part != dp.n_part) throw TnError(TN_E_INVALID, "internal: pair partial count");
          a.Sp2 = p->T[s2.spt].off;
          a.slotSp2 = p->T[s2.spt].slot;
        }
      }
      H.push_back(a);
    }
  }
}

static void make_plan(tn_plan_t *p, const tn_net *net, const tn_plan_opts *o) {
  p->opts = *o;
  p->n_vars = net->n_vars;
  p->card = net->card;
  p->mode = o->evidence_mode;
  if (p->mode < 0 || p->mode > 2) throw TnError(TN_E_INVALID, "unknown evidence mode");
  p->max_batch = p->mode == TN_EVIDENCE_NONE ? 1 : std::max(1, o->max_batch);
  p->batched_ev = p->mode == TN_EVIDENCE_INDICATOR || (p->mode == TN_EVIDENCE_SLICED && p->max_batch > 1);
  if (o->batch_layout < 0 || o->batch_layout > 2) throw TnError(TN_E_INVALID, "unknown batch layout");
  p->inter = p->batched_ev && p->max_batch > 1 &&
             (o->batch_layout == 2 || (o->batch_layout == 0 && o->dtype == TN_F32));
  if (p->inter) p->max_batch = (p->max_batch + kInterLanes - 1) / kInterLanes * kInterLanes;
  p->want_sum = (o->semiring_mask & TN_SUM_PRODUCT) != 0;
  p->want_max = (o->semiring_mask & TN_MAX_PLUS) != 0;
  p->want_grad = o->want_factor_grad != 0;
  if (o->no_fuse < 0 || o->no_fuse > 2) throw TnError(TN_E_INVALID, "no_fuse: 0, 1 or 2");
  if (o->dtype < TN_F32 || o->dtype > TN_F16) throw TnError(TN_E_INVALID, "unknown dtype");
  p->is_obs.assign(p->n_vars, 0);
  if (p->mode == TN_EVIDENCE_SLICED) {
    for (int i = 0; i < o->n_observed; ++i) {
      int v = o->observed[i];
      if (v < 0 || v >= p->n_vars) throw TnError(TN_E_INVALID, "observed variable out of range");
      if (p->is_obs[v]) throw TnError(TN_E_INVALID, "observed variable listed twice");
      p->is_obs[v] = 1;
      p->observed.push_back(v);
    }
  }
  if (o->n_joint > 0) {
    if (!o->joint_ptr || !o->joint_vars) throw TnError(TN_E_INVALID, "joint sets: NULL arrays");
    if (o->query && o->n_query > 0) throw TnError(TN_E_UNSUPPORTED, "joint marginals in an MMAP plan");
    for (int k = 0; k < o->n_joint; ++k) {
      const int64_t b = o->joint_ptr[k], e = o->joint_ptr[k + 1];
      if (b < 0 || e <= b) throw TnError(TN_E_INVALID, "joint set " + std::to_string(k) + " is empty or malformed");
      std::vector<int> set;
      double log2n = 0;
      for (int64_t i = b; i < e; ++i) {
        const int v = o->joint_vars[i];
        if (v < 0 || v >= p->n_vars) throw TnError(TN_E_INVALID, "joint set variable out of range");
        set.push_back(v);
        log2n += std::log2((double)p->card[v]);
      }
      std::sort(set.begin(), set.end());
      if (std::adjacent_find(set.begin(), set.end()) != set.end())
        throw TnError(TN_E_INVALID, "joint set lists a variable twice");
      if (log2n > 24) throw TnError(TN_E_TOO_LARGE, "joint set table above 2^24 entries");
      p->joint_sets.push_back(std::move(set));
    }
  }
  if (o->query && o->n_query > 0) {
    p->is_mmap = true;
    if (p->batched_ev) throw TnError(TN_E_UNSUPPORTED, "MMAP with batched evidence");
    build_mmap(p, net);
    if (!o->host_only) allocate(p, net);
    return;
  }
  // stream
  build_leaves(p, net);
  const int L = (int)p->leaf_lab.size();
  if (o->tree_pairs && o->n_tree_pairs > 0) {
    for (int i = 0; i < o->n_tree_pairs; ++i) p->pairs.push_back({o->tree_pairs[2 * i], o->tree_pairs[2 * i + 1]});
    validate_tree(L, p->pairs);
    p->stats = tree_stats(p->leaf_lab, p->pairs, {}, p->card);
    p->planner_used = -1;
  } else {
    PlanChoice pc = plan_tree(p->leaf_lab, p->card, {}, o->planner, o->restarts, o->seed,
                              p->batched_ev ? 0.0 : o->max_log2_size);
    // chains of nodes below the fused-segment size (2^12 outputs) in fewer levels
    p->pairs = rebalance_small_chains(p->leaf_lab, pc.pairs, {}, p->card, 11.0);
    p->stats = tree_stats(p->leaf_lab, p->pairs, {}, p->card);
    p->planner_used = pc.planner;
    p->two_front = pc.two_front;
  }
  auto lab = node_labels(p->leaf_lab, p->pairs, {}, p->n_vars);
  if (p->inter) {
    // interleaved rows are addressed with 32-bit byte offsets: every batched
    // tensor (largest node or leaf, all instances) must stay below 2 GiB
    double big = std::exp2(p->stats.sc);
    for (const auto &l : p->leaf_lab) big = std::max(big, (double)numel(l, p->card));
    if (big * p->max_batch * 4.0 >= 2147483648.0) {
      if (o->batch_layout == 2)
        throw TnError(TN_E_TOO_LARGE, "interleaved layout: a batched tensor would exceed 2 GiB");
      p->inter = false;
      p->max_batch = std::max(1, o->max_batch);
    }
  }
  std::vector<char> fixed = p->is_obs;
  if (o->max_log2_size > 0 && p->stats.sc > o->max_log2_size + 1e-9) {
    // sliced sum-product plan (log Z and sampling): the chosen variables are
    // fixed per slice like evidence; the tree over the leaves stays, its
    // labels lose the sliced variables
    if (p->batched_ev || p->want_max || p->want_grad)
      throw TnError(TN_E_UNSUPPORTED, "slicing: sum-product plans without batched evidence or gradients");
    p->sliced = choose_slices(p->leaf_lab, p->pairs, {}, p->card, o->max_log2_size);
    for (int v : p->sliced) fixed[v] = 1;
    for (auto &l : p->leaf_lab) l.erase(std::remove_if(l.begin(), l.end(), [&](int v) { return (bool)fixed[v]; }), l.end());
    TreeStats st = tree_stats(p->leaf_lab, p->pairs, {}, p->card);
    double n_slices = 1;
    for (int v : p->sliced) n_slices *= p->card[v];
    st.flops *= n_slices;
    st.bytes *= n_slices;
    st.tc = st.flops > 0 ? std::log2(st.flops / 2) : 0;
    p->stats = st;
    lab = node_labels(p->leaf_lab, p->pairs, {}, p->n_vars);
  }
  // leaf tensors and descriptors
  std::vector<int> leaf_sum(L, -1), leaf_max(L, -1);
  for (int i = 0; i < L; ++i) {
    LeafDesc d{};
    d.kind = p->leaf_kind[i] == 3 ? 1 : p->leaf_kind[i];  // joint-set unity tensors: constant ones
    d.var = p->leaf_var[i];
    d.size = (int32_t)numel(p->leaf_lab[i], p->card);
    if (d.kind == 0) {
      const int f = p->leaf_factor[i];
      d.ident = factor_gather(p, net, f, fixed, d.gmap, d.obs_begin, d.obs_end) ? 1 : 0;
      d.src = net->val_off[f];
    }
    // batched: indicator vectors, and under batched sliced evidence every
    // factor sliced at an observed variable (one slice per instance)
    const bool bat = p->leaf_kind[i] == 2 ||
                     (p->mode == TN_EVIDENCE_SLICED && p->batched_ev && d.kind == 0 && d.obs_end > d.obs_begin);
    d.batched = bat;
    if (p->want_sum) {
      leaf_sum[i] = new_tensor(p, p->leaf_lab[i], bat, true);
      LeafDesc s = d;
      s.dst = leaf_sum[i];
      s.slot = leaf_sum[i];
      s.maxdom = 0;
      p->leaves_sum.push_back(s);
    }
    if (p->want_max) {
      leaf_max[i] = new_tensor(p, p->leaf_lab[i], bat, false);
      LeafDesc m = d;
      m.dst = leaf_max[i];
      m.slot = -1;
      m.maxdom = 1;
      p->leaves_max.push_back(m);
    }
  }
  if (p->want_sum) {
    TreeExec &t = p->sum_tree;
    t.leaf_tensor = leaf_sum;
    t.pairs = p->pairs;
    t.lab = lab;
    build_forward(p, t, SEMI_SUM);
    // reverse pass
    std::vector<char> need(L + p->pairs.size(), 0);
    for (int i = 0; i < L; ++i) need[i] = p->leaf_kind[i] != 0 || p->want_grad;
    for (size_t q = 0; q < p->pairs.size(); ++q)
      need[L + q] = need[p->pairs[q][0]] || need[p->pairs[q][1]];
    p->adj_tensor.assign(L + p->pairs.size(), -1);
    const int rootn = L + (int)p->pairs.size() - 1;
    p->seed_tensor = new_tensor(p, p->T[t.root].lab, p->batched_ev, true);
    if (t.root != t.node_tensor[rootn]) {
      // root reduction: its adjoint is a broadcast of the seed
      int a = new_tensor(p, p->T[t.node_tensor[rootn]].lab, p->T[p->seed_tensor].batched, true);
      p->bwd.push_back(make_op(p, SEMI_SUM, p->seed_tensor, -1, a, -1));
      p->adj_tensor[rootn] = a;
    } else {
      p->adj_tensor[rootn] = p->seed_tensor;
    }
    for (int q = (int)p->pairs.size() - 1; q >= 0; --q) {
      const int c = L + q;
      if (!need[c]) continue;
      for (int side = 0; side < 2; ++side) {
        const int ch = p->pairs[q][side], sib = p->pairs[q][1 - side];
        if (!need[ch]) continue;
        const int cbar = p->adj_tensor[c], sbt = t.node_tensor[sib];
        const bool bat = p->T[cbar].batched || p->T[sbt].batched;
        int a = new_tensor(p, lab[ch], bat, true);
        int X = cbar, Y = sbt;
        if (p->T[Y].size > p->T[X].size) std::swap(X, Y);
        p->bwd.push_back(make_op(p, SEMI_SUM, X, Y, a, -1));
        p->adj_tensor[ch] = a;
      }
    }
    int col = 0;
    p->marg_col.assign(p->n_vars, 0);
    for (int v = 0; v < p->n_vars; ++v) {
      p->marg_col[v] = col;
      col += p->card[v];
    }
    p->marg_row = col;
    for (int i = 0; i < L; ++i) {
      if (p->leaf_kind[i] == 3) {
        continue;  // joint sets: below
      } else if (p->leaf_kind[i] != 0) {
        MargDesc m{};
        m.adj = p->adj_tensor[i];
        m.leaf = leaf_sum[i];
        m.card = p->card[p->leaf_var[i]];
        m.out = p->marg_col[p->leaf_var[i]];
        p->marg.push_back(m);
      } else if (p->want_grad) {
        GradDesc g{};
        g.adj = p->adj_tensor[i];
        g.size = (int32_t)numel(p->leaf_lab[i], p->card);
        const int f = p->leaf_factor[i];
        g.dst = net->val_off[f];
        const LeafDesc &ld = p->leaves_sum[i];
        g.gmap = ld.gmap;
        g.obs_begin = ld.obs_begin;
        g.obs_end = ld.obs_end;
        g.leaf = leaf_sum[i];
        int64_t full = 1;
        for (int v : net->scope[f]) full *= p->card[v];
        g.full = (int32_t)full;
        p->grads.push_back(g);
      }
    }
    // joint sets: the unity tensor of each (leaves after the unity vectors,
    // in set order) and the layout of its table
    {
      int li = 0;
      while (li < L && p->leaf_kind[li] != 3) ++li;
      int col = 0;
      for (const auto &set : p->joint_sets) {
        JointDesc j;
        j.out = col;
        j.v_begin = (int32_t)(p->joint_tab.size() / 3);
        Labels lab;
        for (int v : set)
          if (!(p->mode == TN_EVIDENCE_SLICED && p->is_obs[v])) lab.push_back(v);
        int64_t n_full = 1;
        for (int v : set) {
          n_full *= p->card[v];
          p->joint_tab.push_back(v);
          p->joint_tab.push_back(p->card[v]);
          p->joint_tab.push_back(has(lab, v) ? (int32_t)stride_in(lab, v, p->card) : -1);
        }
        j.v_end = (int32_t)(p->joint_tab.size() / 3);
        j.n_full = (int32_t)n_full;
        if (!lab.empty()) j.adj = p->adj_tensor[li++];  // tensor id until allocation
        p->joint.push_back(j);
        col += (int)n_full;
      }
      p->joint_row = col;
    }
    if (!p->batched_ev) build_sampling(p, t);
    if (p->opts.no_fuse != 1 && !p->batched_ev) build_fusion(p, need, L);
  }
  if (p->want_max) {
    TreeExec &t = p->max_tree;
    t.leaf_tensor = leaf_max;
    t.pairs = p->pairs;
    t.lab = lab;
    build_forward(p, t, SEMI_MAX);
    if (p->opts.no_fuse != 1 && !p->batched_ev && p->max_batch == 1) build_max_pairs(p, t);
    build_backtrack(p, t);
  }
  if (o->host_only) return;
  allocate(p, net);
}

extern "C" tn_status tn_plan(const tn_net *net, const tn_plan_opts *opts, tn_plan_t **out) {
  return guard([&] {
    if (!net || !out) throw TnError(TN_E_INVALID, "NULL argument");
    *out = nullptr;
    tn_plan_opts o;
    if (opts) o = *opts;
    else tn_plan_opts_default(&o);
    auto p = std::make_unique<tn_plan_impl>();
    p->net_src = net;
    make_plan(p.get(), net, &o);
    if (!o.host_only) hip_check(hipDeviceSynchronize(), "plan upload");
    *out = p.release();
  });
}

extern "C" void tn_free_plan(tn_plan_t *p) { delete p; }

extern "C" tn_status tn_plan_info_get(const tn_plan_t *p, tn_plan_info *info) {
  return guard([&] {
    if (!p || !info) throw TnError(TN_E_INVALID, "NULL argument");
    std::memset(info, 0, sizeof *info);
    info->n_leaves = (int32_t)p->leaf_lab.size();
    info->n_nodes = (int32_t)(p->leaf_lab.size() + p->pairs.size());
    info->n_kernels_fwd = (int32_t)p->sum_tree.ops.size();
    info->n_kernels_bwd = (int32_t)p->bwd.size();
    info->n_kernels_max = (int32_t)p->max_tree.ops.size();
    info->sc = p->stats.sc;
    info->sc_union = p->stats.sc_union;
    info->tc = p->stats.tc;
    info->flops_fwd = p->stats.flops;
    info->bytes_fwd = p->stats.bytes;
    info->n_sliced = (int32_t)p->sliced.size();
    info->planner_used = p->planner_used;
    info->two_front = p->two_front ? 1 : 0;
    if (!p->pairs.empty()) stage_time(p->leaf_lab, p->pairs, {}, p->card, &info->n_levels);
    info->device_bytes = p->device_bytes;
    if (p->opts.host_only)  // planned only: the float arena the plan would hold
      for (const auto &t : p->T) info->device_bytes += 4 * t.size * (t.batched ? p->max_batch : 1);
    auto count = [](const Schedule &sc) {
      int n = 0;
      for (const Launch &L : sc.launches) n += L.split ? 2 : 1;
      return n;
    };
    info->n_launches_fwd = count(p->sched_fwd);
    info->n_launches_bwd = count(p->sched_bwd);
    info->n_launches_max = count(p->sched_max);
    if (p->opts.host_only) {  // schedules are built at allocation: build them here (host only)
      tn_plan_t *q = const_cast<tn_plan_t *>(p);
      info->n_launches_fwd = count(p->fused ? build_schedule(q, p->ffwd, false) : build_schedule(q, p->sum_tree.ops, false));
      info->n_launches_bwd = count(p->fused ? build_schedule(q, p->fbwd, true) : build_schedule(q, p->bwd, true));
      info->n_launches_max =
          count(build_schedule(q, p->max_tree.fused ? p->max_tree.fops : p->max_tree.ops, false));
    } else if (p->fused) {
      info->n_launches_fwd = count(p->sched_ffwd);
      info->n_launches_bwd = count(p->sched_fbwd);
    }
    info->n_segments = (int32_t)p->segs.size();
    info->n_pairs = (int32_t)p->dsegs.size();
    for (const auto &dp : p->dsegs) info->n_pairs_moved += dp.aug1 > 1 || dp.aug2 > 1 ? 1 : 0;
    for (const auto &sp : p->segs) info->n_fused_nodes += (int32_t)sp.ops.size();
    for (const auto *L : {&p->sum_tree.ops, &p->bwd, &p->qtree.ops, &p->max_tree.ops})
      for (const Op &op : *L) {
        info->n_dense += op.a.kind == 2 ? 1 : 0;
        info->n_dense_large += op.a.kind == 2 && op.a.tile == 1 ? 1 : 0;
        info->n_wave += op.a.kind == 3 ? 1 : 0;
        info->n_interleaved += op.a.kind == 4 ? 1 : 0;
      }
    info->batch_stride = p->inter ? p->max_batch : 0;
    for (const auto &g : p->groups)
      for (const Op &op : g.ops) {
        info->n_dense += op.a.kind == 2 ? 1 : 0;
        info->n_dense_large += op.a.kind == 2 && op.a.tile == 1 ? 1 : 0;
        info->n_wave += op.a.kind == 3 ? 1 : 0;
      }
  });
}

extern "C" tn_status tn_plan_tree(const tn_plan_t *p, int32_t *pairs, int32_t cap, int32_t *n_pairs,
                                  int32_t *n_leaves) {
  return guard([&] {
    if (!p) throw TnError(TN_E_INVALID, "NULL plan");
    if (n_pairs) *n_pairs = (int32_t)p->pairs.size();
    if (n_leaves) *n_leaves = (int32_t)p->leaf_lab.size();
    for (int i = 0; i < (int)p->pairs.size() && i < cap; ++i) {
      pairs[2 * i] = p->pairs[i][0];
      pairs[2 * i + 1] = p->pairs[i][1];
    }
  });
}

extern "C" tn_status tn_plan_ops(const tn_plan_t *p, int32_t task, tn_op_info *out, int32_t cap, int32_t *n) {
  return guard([&] {
    if (!p || !n) throw TnError(TN_E_INVALID, "NULL argument");
    std::vector<const Op *> ops;
    auto add = [&](const std::vector<Op> &v) {
      for (const Op &op : v) ops.push_back(&op);
    };
    if (task == 0) add(p->fused ? p->ffwd : p->sum_tree.ops);
    else if (task == 1) add(p->fused ? p->fbwd : p->bwd);
    else if (task == 2) add(p->max_tree.ops);
    else if (task == 3)
      for (const auto &g : p->groups) add(g.fused ? g.fops : g.ops);
    else throw TnError(TN_E_INVALID, "unknown task");
    *n = (int32_t)ops.size();
    for (size_t i = 0; i < ops.size() && (int32_t)i < cap; ++i) {
      const Op &op = *ops[i];
      tn_op_info o{};
      o.form = op.seg >= 0 ? 5 : op.a.kind;
      o.semiring = op.semi;
      o.variant = op.seg >= 0 ? op.seg_kind : op.a.tile;
      o.rows = op.a.nR;
      o.cols = op.a.nC;
      o.summed = op.a.nS;
      o.x_size = op.X >= 0 ? p->T[op.X].size : 0;
      o.y_size = op.Y >= 0 ? p->T[op.Y].size : 0;
      o.z_size = op.Z >= 0 ? p->T[op.Z].size : 0;
      o.eligible = op.seg >= 0 ? 0 : op.forms;
      out[i] = o;
    }
  });
}

extern "C" tn_status tn_plan_sliced(const tn_plan_t *p, int32_t *vars, int32_t cap, int32_t *n) {
  return guard([&] {
    if (!p) throw TnError(TN_E_INVALID, "NULL plan");
    if (n) *n = (int32_t)p->sliced.size();
    for (int i = 0; i < (int)p->sliced.size() && i < cap; ++i) vars[i] = p->sliced[i];
  });
}

extern "C" tn_status tn_plan_tree_host(const tn_net *net, const tn_plan_opts *opts, int32_t *pairs,
                                       int32_t cap, int32_t *n_pairs, int32_t *n_leaves,
                                       tn_plan_info *stats) {
  return guard([&] {
    if (!net) throw TnError(TN_E_INVALID, "NULL network");
    tn_plan_opts o;
    if (opts) o = *opts;
    else tn_plan_opts_default(&o);
    tn_plan_impl p;
    p.n_vars = net->n_vars;
    p.card = net->card;
    p.mode = o.evidence_mode;
    p.is_obs.assign(p.n_vars, 0);
    if (p.mode == TN_EVIDENCE_SLICED)
      for (int i = 0; i < o.n_observed; ++i) {
        if (o.observed[i] < 0 || o.observed[i] >= p.n_vars) throw TnError(TN_E_INVALID, "observed variable out of range");
        p.is_obs[o.observed[i]] = 1;
      }
    build_leaves(&p, net);
    const bool batched = p.mode == TN_EVIDENCE_INDICATOR || (p.mode == TN_EVIDENCE_SLICED && o.max_batch > 1);
    PlanChoice pc = plan_tree(p.leaf_lab, p.card, {}, o.planner, o.restarts, o.seed,
                              batched ? 0.0 : o.max_log2_size);
    if (n_pairs) *n_pairs = (int32_t)pc.pairs.size();
    if (n_leaves) *n_leaves = (int32_t)p.leaf_lab.size();
    for (int i = 0; i < (int)pc.pairs.size() && i < cap; ++i) {
      pairs[2 * i] = pc.pairs[i][0];
      pairs[2 * i + 1] = pc.pairs[i][1];
    }
    if (stats) {
      std::memset(stats, 0, sizeof *stats);
      stats->n_leaves = (int32_t)p.leaf_lab.size();
      stats->n_nodes = (int32_t)(p.leaf_lab.size() + pc.pairs.size());
      stats->sc = pc.stats.sc;
      stats->sc_union = pc.stats.sc_union;
      stats->tc = pc.stats.tc;
      stats->flops_fwd = pc.stats.flops;
      stats->bytes_fwd = pc.stats.bytes;
      stats->planner_used = pc.planner;
      stats->two_front = pc.two_front ? 1 : 0;
      if (!pc.pairs.empty()) stage_time(p.leaf_lab, pc.pairs, {}, p.card, &stats->n_levels);
      if (o.max_log2_size > 0) {
        Labels sl = choose_slices(p.leaf_lab, pc.pairs, {}, p.card, o.max_log2_size);
        stats->n_sliced = (int32_t)sl.size();
      }
    }
  });
}

// ---------------------------------------------------------------------------
// execution
// ---------------------------------------------------------------------------
namespace tn {

void run_ops(tn_plan_t *p, const std::vector<Op> &ops) {
  for (const Op &op : ops) launch_contract(op.semi, op.Y >= 0, op.split, op.a, op.d_a, op.nb, p->stream);
}

void run_sched(tn_plan_t *p, const std::vector<Op> &ops, const Schedule &sc) {
  for (const Launch &L : sc.launches) {
    if (L.seg) {
      const Op &op = ops[L.ops[0]];
      const int seg2 = L.ops.size() > 1 ? ops[L.ops[1]].seg : -1;
      switch (L.seg_kind) {
        case 1:
          if (seg2 >= 0) launch_seg_fwd2(p->seg_fwd_h[op.seg], p->seg_fwd_h[seg2], p->stream);
          else launch_seg_fwd(p->seg_fwd_h[op.seg], p->stream);
          break;
        case 2:
          if (seg2 >= 0) launch_seg_bwd2(p->seg_bwd_h[op.seg], p->seg_bwd_h[seg2], p->stream);
          else launch_seg_bwd(p->seg_bwd_h[op.seg], p->stream);
          break;
        case 5: launch_dseg_fwd(p->dseg_fwd_h[op.seg], seg2 >= 0 ? &p->dseg_fwd_h[seg2] : nullptr, p->stream); break;
        case 6: launch_dseg_bwd(p->dseg_bwd_h[op.seg], seg2 >= 0 ? &p->dseg_bwd_h[seg2] : nullptr, p->stream); break;
        case 3: launch_seg_mat(p->d_seg_fwd, L.d_ids, (int)L.ops.size(), L.lds, p->stream); break;
        default: launch_seg_fin(p->d_seg_bwd, L.d_ids, (int)L.ops.size(), L.lds, p->stream); break;
      }
    } else if (L.ops.size() == 1) {
      const Op &op = ops[L.ops[0]];
      launch_contract(op.semi, op.Y >= 0, op.split, op.a, op.d_a, op.nb, p->stream);
    } else if (L.gemm) {
      launch_group(L.semi, 3 + (L.semi == SEMI_SUM ? p->opts.dtype : 0), L.d_args, L.d_blk, L.d_nblk,
                   (int)L.ops.size(), L.total, p->stream);
    } else if (L.inter) {
      launch_group(L.semi, 6, L.d_args, L.d_blk, L.d_nblk, (int)L.ops.size(), L.total, p->stream);
    } else if (L.mpair) {
      launch_group(L.semi, 7, L.d_args, L.d_blk, L.d_nblk, (int)L.ops.size(), L.total, p->stream);
    } else if (!L.split) {
      launch_group(L.semi, 0, L.d_args, L.d_blk, L.d_nblk, (int)L.ops.size(), L.total, p->stream);
    } else {
      launch_group(L.semi, 1, L.d_args, L.d_blk, L.d_nblk, (int)L.ops.size(), L.total, p->stream);
      launch_group(L.semi, 2, L.d_args, L.d_blk2, L.d_nblk2, (int)L.ops.size(), L.total2, p->stream);
    }
  }
}

static PrepareArgs prep_args(tn_plan_t *p, const std::vector<LeafDesc> &h, const LeafDesc *d, bool reset) {
  PrepareArgs a;
  a.arena = p->arena;
  a.leaves = d;
  a.n_leaves = (int)h.size();
  a.gmap = p->d_gmap;
  a.obs = p->d_obs;
  a.evidence = p->d_evidence;
  a.n_vars = p->n_vars;
  a.mx = p->mx;
  a.ex = p->ex;
  a.mx_stride = std::max(1, p->n_slots);
  a.reset_begin = reset ? p->reset_begin : 0;
  a.reset_end = reset ? p->reset_end : 0;
  a.batch = p->max_batch;
  a.max_batch = p->max_batch;
  a.interleaved = p->inter ? 1 : 0;
  for (size_t i = 0; i < h.size() && a.n_big < kPrepBig; ++i)
    if (h[i].nsub > 1) {
      a.big_leaf[a.n_big] = (int32_t)i;
      a.big_blk0[a.n_big + 1] = a.big_blk0[a.n_big] + h[i].nsub;
      ++a.n_big;
    }
  return a;
}

void launch_prepare_set(tn_plan_t *p, const std::vector<LeafDesc> &h, const LeafDesc *d, bool reset) {
  launch_prepare(prep_args(p, h, d, reset), p->stream);
}

// Run `body` directly, or replay its captured graph.
template <class F>
void run_graph(tn_plan_t *p, const std::string &key, F &&body) {
  if (!p->opts.use_graph || p->eager) {
    body();
    hip_check(hipGetLastError(), "kernel launch");
    return;
  }
  auto it = p->graphs.find(key);
  if (it == p->graphs.end()) {
    hipGraph_t g = nullptr;
    hip_check(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    body();
    hipError_t le = hipGetLastError();
    hip_check(hipStreamEndCapture(p->stream, &g), "end capture");
    hip_check(le, "kernel launch during capture");
    hipGraphExec_t ge = nullptr;
    hip_check(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0), "graph instantiate");
    (void)hipGraphDestroy(g);
    it = p->graphs.emplace(key, ge).first;
  }
  hip_check(hipGraphLaunch(it->second, p->stream), "graph launch");
}

}  // namespace tn

static void upload_evidence(tn_plan_t *p, int batch, const int32_t *ev) {
  std::vector<int32_t> h((size_t)p->max_batch * p->n_vars, -1);
  for (int b = 0; b < batch; ++b)
    for (int v = 0; v < p->n_vars; ++v) {
      int e = ev ? ev[(int64_t)b * p->n_vars + v] : -1;
      if (e < -1 || e >= p->card[v]) throw TnError(TN_E_INVALID, "evidence value out of range");
      if (p->mode == TN_EVIDENCE_NONE && e >= 0) throw TnError(TN_E_INVALID, "plan has no evidence; pass -1");
      if (p->mode == TN_EVIDENCE_SLICED && (e >= 0) != (bool)p->is_obs[v])
        throw TnError(TN_E_INVALID, "evidence must give exactly the plan's observed variables");
      h[(size_t)b * p->n_vars + v] = e;
    }
  // sliced leaves gather at the observed values of every row, so rows past
  // the batch repeat the first one
  if (p->mode == TN_EVIDENCE_SLICED)
    for (int b = std::max(1, batch); b < p->max_batch; ++b)
      std::copy(h.begin(), h.begin() + p->n_vars, h.begin() + (size_t)b * p->n_vars);
  hip_check(hipMemcpyAsync(p->d_evidence, h.data(), h.size() * 4, hipMemcpyHostToDevice, p->stream), "evidence upload");
  hip_check(hipStreamSynchronize(p->stream), "evidence upload");
}

// Sliced sum-product plans: the caller's evidence row with the sliced
// variables at slice s (slices in row-major order over the sliced variables,
// last fastest), uploaded as the plan's evidence.
static int64_t n_slices_of(const tn_plan_t *p) {
  int64_t n = 1;
  for (int v : p->sliced) n *= p->card[v];
  return n;
}
static std::vector<int32_t> slice_row(const tn_plan_t *p, const int32_t *ev, int64_t s) {
  std::vector<int32_t> row(p->n_vars, -1);
  for (int v = 0; v < p->n_vars; ++v) {
    const int e = ev ? ev[v] : -1;
    if (e < -1 || e >= p->card[v]) throw TnError(TN_E_INVALID, "evidence value out of range");
    if (p->mode == TN_EVIDENCE_NONE && e >= 0) throw TnError(TN_E_INVALID, "plan has no evidence; pass -1");
    if (p->mode == TN_EVIDENCE_SLICED && (e >= 0) != (bool)p->is_obs[v])
      throw TnError(TN_E_INVALID, "evidence must give exactly the plan's observed variables");
    row[v] = e;
  }
  for (int i = (int)p->sliced.size() - 1; i >= 0; --i) {
    const int v = p->sliced[i];
    row[v] = (int32_t)(s % p->card[v]);
    s /= p->card[v];
  }
  return row;
}
static void forward_sum(tn_plan_t *p, bool with_bwd, bool allow_fused);
// Slices [s0, s0 + n) of a run (n <= kSliceChunk): their evidence rows
// (row(s) fills one) go to the device in one copy; per slice, body(j) runs
// after a stream-ordered copy of row j into the plan's evidence row.  The
// host waits once per chunk (before `rows` is rebuilt), not once per slice.
template <class Row, class Body>
static void slice_chunk(tn_plan_t *p, std::vector<int32_t> &rows, int64_t s0, int64_t n, Row row, Body body) {
  const size_t nv = (size_t)p->n_vars;
  hip_check(hipStreamSynchronize(p->stream), "slice chunk");
  rows.resize((size_t)n * nv);
  for (int64_t j = 0; j < n; ++j) row(s0 + j, rows.data() + j * nv);
  hip_check(hipMemcpyAsync(p->d_slice_rows, rows.data(), rows.size() * 4, hipMemcpyHostToDevice, p->stream), "slice");
  for (int64_t j = 0; j < n; ++j) {
    hip_check(hipMemcpyAsync(p->d_evidence, p->d_slice_rows + j * nv, nv * 4, hipMemcpyDeviceToDevice, p->stream),
              "slice row");
    body(j);
  }
}
// log Z_s of every slice (FP64 per slice)
static std::vector<double> slice_log_z(tn_plan_t *p, const int32_t *ev, bool unfused) {
  const int64_t ns = n_slices_of(p);
  std::vector<double> lz(ns);
  const std::vector<int32_t> base = slice_row(p, ev, 0);
  std::vector<int32_t> rows;
  for (int64_t s0 = 0; s0 < ns; s0 += kSliceChunk) {
    const int64_t n = std::min(kSliceChunk, ns - s0);
    slice_chunk(
        p, rows, s0, n,
        [&](int64_t s, int32_t *r) {
          std::copy(base.begin(), base.end(), r);
          for (int i = (int)p->sliced.size() - 1; i >= 0; --i) {
            const int v = p->sliced[i];
            r[v] = (int32_t)(s % p->card[v]);
            s /= p->card[v];
          }
        },
        [&](int64_t j) {
          forward_sum(p, false, !unfused);
          hip_check(hipMemcpyAsync(p->d_slice_lz + j, p->d_out, sizeof(double), hipMemcpyDeviceToDevice, p->stream),
                    "D2D");
        });
    hip_check(hipMemcpyAsync(&lz[s0], p->d_slice_lz, n * sizeof(double), hipMemcpyDeviceToHost, p->stream), "D2H");
  }
  hip_check(hipStreamSynchronize(p->stream), "slices");
  return lz;
}
static double log_sum_exp(const std::vector<double> &v) {
  double m = -INFINITY;
  for (double x : v) m = std::max(m, x);
  if (!(m > -INFINITY)) return -INFINITY;
  double t = 0;
  for (double x : v) t += std::exp(x - m);
  return m + std::log(t);
}

static void check_batch(tn_plan_t *p, int batch) {
  if (batch < 1) throw TnError(TN_E_INVALID, "batch must be >= 1");
  if (p->batched_ev && batch > p->max_batch) throw TnError(TN_E_INVALID, "batch exceeds max_batch");
  if (p->mode == TN_EVIDENCE_NONE && batch != 1) throw TnError(TN_E_INVALID, "mode NONE takes batch 1");
}

// Sum-product forward (and reverse pass).  Fused chain segments skip the
// intermediate carriers; sampling reads every node, so it runs unfused.
static void forward_sum(tn_plan_t *p, bool with_bwd, bool allow_fused = true) {
  const bool fz = p->fused && allow_fused;
  run_graph(p, std::string(with_bwd ? "sum+bwd" : "sum") + (fz ? "" : "-unfused"), [&] {
    launch_prepare_set(p, p->leaves_sum, p->d_leaves_sum, true);
    if (fz) run_sched(p, p->ffwd, p->sched_ffwd);
    else run_sched(p, p->sum_tree.ops, p->sched_fwd);
    const TensorBuf &r = p->T[p->sum_tree.root];
    launch_logz(p->arena + r.off, r.batched ? (p->inter ? 1 : r.size) : 0, p->ex, r.slot, r.batched, p->max_batch, p->d_out, p->stream);
    if (with_bwd) {
      if (fz) run_sched(p, p->fbwd, p->sched_fbwd);
      else run_sched(p, p->bwd, p->sched_bwd);
      launch_marg(p->arena, p->d_marg_desc, (int)p->marg.size(), p->max_batch, p->marg_row, p->d_marg, p->stream);
      launch_joint(p->arena, p->d_joint_desc, (int)p->joint.size(), p->d_joint_tab, p->d_evidence, p->n_vars,
                   p->max_batch, p->joint_row, p->d_joint, p->stream);
    }
  });
}

template <class F>
static void per_instance(tn_plan_t *p, int batch, const int32_t *ev, F &&f) {
  // one pass over the batch, except SLICED plans built for one instance:
  // one pass each
  if (!p->batched_ev && p->mode == TN_EVIDENCE_SLICED) {
    for (int b = 0; b < batch; ++b) f(b, 1, ev ? ev + (int64_t)b * p->n_vars : nullptr);
  } else {
    f(0, batch, ev);
  }
}

extern "C" tn_status tn_logZ(tn_plan_t *p, int32_t batch, const int32_t *evidence, double *logz) {
  return guard([&] {
    if (!p || !logz) throw TnError(TN_E_INVALID, "NULL argument");
    if (!p->want_sum || p->is_mmap) throw TnError(TN_E_UNSUPPORTED, "plan has no sum-product pass");
    check_batch(p, batch);
    if (!p->sliced.empty()) {  // Z = sum over the slices of Z_s
      for (int b = 0; b < batch; ++b)
        logz[b] = log_sum_exp(slice_log_z(p, evidence ? evidence + (int64_t)b * p->n_vars : nullptr, false));
    } else {
      per_instance(p, batch, evidence, [&](int b0, int nb, const int32_t *ev) {
        upload_evidence(p, nb, ev);
        forward_sum(p, false);
        hip_check(hipMemcpyAsync(logz + b0, p->d_out, nb * sizeof(double), hipMemcpyDeviceToHost, p->stream), "D2H");
        hip_check(hipStreamSynchronize(p->stream), "logZ");
      });
    }
    for (int b = 0; b < batch; ++b)
      if (!(logz[b] > -INFINITY)) throw TnError(TN_E_ZERO_EVIDENCE, "p(e) = 0 for instance " + std::to_string(b));
  });
}

extern "C" tn_status tn_marginals(tn_plan_t *p, int32_t batch, const int32_t *evidence, double *logz,
                                  double *marg) {
  return guard([&] {
    if (!p || !marg) throw TnError(TN_E_INVALID, "NULL argument");
    if (!p->want_sum || p->is_mmap) throw TnError(TN_E_UNSUPPORTED, "plan has no sum-product pass");
    if (!p->sliced.empty()) throw TnError(TN_E_UNSUPPORTED, "marginals of sliced plans");
    check_batch(p, batch);
    std::vector<double> lz(batch);
    per_instance(p, batch, evidence, [&](int b0, int nb, const int32_t *ev) {
      upload_evidence(p, nb, ev);
      forward_sum(p, true);
      hip_check(hipMemcpyAsync(lz.data() + b0, p->d_out, nb * sizeof(double), hipMemcpyDeviceToHost, p->stream), "D2H");
      hip_check(hipMemcpyAsync(marg + (int64_t)b0 * p->marg_row, p->d_marg, (size_t)nb * p->marg_row * sizeof(double),
                               hipMemcpyDeviceToHost, p->stream), "D2H");
      hip_check(hipStreamSynchronize(p->stream), "marginals");
      if (p->mode == TN_EVIDENCE_SLICED)
        for (int b = 0; b < nb; ++b)
          for (int v : p->observed) {
            double *row = marg + (int64_t)(b0 + b) * p->marg_row + p->marg_col[v];
            const int e = ev[(int64_t)b * p->n_vars + v];
            for (int x = 0; x < p->card[v]; ++x) row[x] = x == e ? 1.0 : 0.0;
          }
    });
    if (logz) std::copy(lz.begin(), lz.end(), logz);
    for (int b = 0; b < batch; ++b)
      if (!(lz[b] > -INFINITY)) throw TnError(TN_E_ZERO_EVIDENCE, "p(e) = 0 for instance " + std::to_string(b));
  });
}

extern "C" tn_status tn_joint_marginals(tn_plan_t *p, int32_t batch, const int32_t *evidence, double *logz,
                                        double *joint) {
  return guard([&] {
    if (!p || !joint) throw TnError(TN_E_INVALID, "NULL argument");
    if (!p->want_sum || p->is_mmap) throw TnError(TN_E_UNSUPPORTED, "plan has no sum-product pass");
    if (p->joint.empty()) throw TnError(TN_E_UNSUPPORTED, "plan has no joint sets");
    if (!p->sliced.empty()) throw TnError(TN_E_UNSUPPORTED, "joint marginals of sliced plans");
    check_batch(p, batch);
    std::vector<double> lz(batch);
    per_instance(p, batch, evidence, [&](int b0, int nb, const int32_t *ev) {
      upload_evidence(p, nb, ev);
      forward_sum(p, true);
      hip_check(hipMemcpyAsync(lz.data() + b0, p->d_out, nb * sizeof(double), hipMemcpyDeviceToHost, p->stream), "D2H");
      hip_check(hipMemcpyAsync(joint + (int64_t)b0 * p->joint_row, p->d_joint,
                               (size_t)nb * p->joint_row * sizeof(double), hipMemcpyDeviceToHost, p->stream), "D2H");
      hip_check(hipStreamSynchronize(p->stream), "joint marginals");
    });
    if (logz) std::copy(lz.begin(), lz.end(), logz);
    for (int b = 0; b < batch; ++b)
      if (!(lz[b] > -INFINITY)) throw TnError(TN_E_ZERO_EVIDENCE, "p(e) = 0 for instance " + std::to_string(b));
  });
}

extern "C" tn_status tn_factor_marginals(tn_plan_t *p, int32_t batch, const int32_t *evidence, double *logz,
                                         double *fmarg) {
  return guard([&] {
    if (!p || !fmarg) throw TnError(TN_E_INVALID, "NULL argument");
    if (!p->want_sum || p->is_mmap) throw TnError(TN_E_UNSUPPORTED, "plan has no sum-product pass");
    if (!p->want_grad) throw TnError(TN_E_UNSUPPORTED, "plan built without want_factor_grad");
    if (!p->sliced.empty()) throw TnError(TN_E_UNSUPPORTED, "factor marginals of sliced plans");
    check_batch(p, batch);
    const int64_t nv = p->net_src->n_values;
    std::vector<double> lz(batch);
    per_instance(p, batch, evidence, [&](int b0, int nb, const int32_t *ev) {
      upload_evidence(p, nb, ev);
      forward_sum(p, true);
      launch_factor_marg(p->arena, p->d_grad_desc, (int)p->grads.size(), p->d_gmap, p->d_obs, p->d_evidence,
                         p->n_vars, nb, nv, p->d_fmarg, p->stream);
      hip_check(hipGetLastError(), "factor marginal launch");
      hip_check(hipMemcpyAsync(lz.data() + b0, p->d_out, nb * sizeof(double), hipMemcpyDeviceToHost, p->stream), "D2H");
      hip_check(hipMemcpyAsync(fmarg + b0 * nv, p->d_fmarg, (size_t)nb * nv * sizeof(double), hipMemcpyDeviceToHost,
                               p->stream), "D2H");
      hip_check(hipStreamSynchronize(p->stream), "factor marginals");
    });
    if (logz) std::copy(lz.begin(), lz.end(), logz);
    for (int b = 0; b < batch; ++b)
      if (!(lz[b] > -INFINITY)) throw TnError(TN_E_ZERO_EVIDENCE, "p(e) = 0 for instance " + std::to_string(b));
  });
}

extern "C" tn_status tn_map(tn_plan_t *p, int32_t batch, const int32_t *evidence, int32_t *assign, double *logp) {
  return guard([&] {
    if (!p || !assign) throw TnError(TN_E_INVALID, "NULL argument");
    if (!p->want_max || p->is_mmap) throw TnError(TN_E_UNSUPPORTED, "plan has no max-plus pass");
    check_batch(p, batch);
    per_instance(p, batch, evidence, [&](int b0, int nb, const int32_t *ev) {
      upload_evidence(p, nb, ev);
      hip_check(hipMemcpyAsync(p->d_assign, p->d_evidence, (size_t)p->max_batch * p->n_vars * 4,
                               hipMemcpyDeviceToDevice, p->stream), "init");
      run_graph(p, "max", [&] {
        launch_prepare_set(p, p->leaves_max, p->d_leaves_max, false);
        run_sched(p, p->max_tree.fused ? p->max_tree.fops : p->max_tree.ops, p->sched_max);
        launch_backtrack(p->iarena, p->d_back, p->d_back_lev, p->max_tree.n_back_lev, p->max_tree.n_back_chunks, p->d_back_meta,
                         p->n_vars, p->max_batch, p->d_assign, p->stream);
      });
      hip_check(hipMemcpyAsync(assign + (int64_t)b0 * p->n_vars, p->d_assign, (size_t)nb * p->n_vars * 4,
                               hipMemcpyDeviceToHost, p->stream), "D2H");
      const TensorBuf &r = p->T[p->max_tree.root];
      std::vector<float> rv(nb);
      for (int b = 0; b < nb; ++b)
        hip_check(hipMemcpyAsync(&rv[b], p->arena + r.off + (r.batched ? (int64_t)b * (p->inter ? 1 : r.size) : 0), 4,
                                 hipMemcpyDeviceToHost, p->stream), "D2H");
      hip_check(hipStreamSynchronize(p->stream), "map");
      if (logp)
        for (int b = 0; b < nb; ++b) logp[b0 + b] = (double)rv[b];
    });
  });
}

static void ensure_sample_buffer(tn_plan_t *p, int64_t n) {
  if (n <= p->samp_cap) return;
  if (p->d_samp_out) {
    hip_check(hipFree(p->d_samp_out), "hipFree");
    p->allocs.erase(std::find(p->allocs.begin(), p->allocs.end(), (void *)p->d_samp_out));
  }
  p->d_samp_out = dalloc<int32_t>(p, (size_t)n * p->n_vars);
  p->samp_cap = n;
}

// Device staging of one sampling call: the sample rows [n][n_vars] and, on
// sliced plans, the ids of the samples drawn in one slice.
struct SampleStaging {
  int32_t *rows = nullptr;
  int64_t *ids = nullptr;
};

// Sampling a sliced plan (reading of the paper's sampling step under
// slicing), in one pass over the slices in order: sample i
// takes slice s with probability Z_s / (Z_0 + ... + Z_s) (uniform from
// counter (i, kSliceDrawNode, s)); the last slice it takes is its slice,
// with probability Z_s / Z (a weighted reservoir of one).  A sample is drawn
// inside every slice it takes, right after that slice's forward pass; its
// row ends as the draw of its last slice (the per-node counters follow the
// sample id, so that draw equals drawing the slice first).
static void sample_sliced(tn_plan_t *p, const int32_t *evidence, int64_t n, uint64_t seed, int32_t *samples,
                          const SampleStaging &stg) {
  const int64_t ns = n_slices_of(p);
  double prefix = -INFINITY;
  std::vector<int64_t> ids;
  ids.reserve((size_t)n);
  for (int64_t s = 0; s < ns; ++s) {
    const std::vector<int32_t> row = slice_row(p, evidence, s);
    hip_check(hipMemcpyAsync(p->d_evidence, row.data(), row.size() * 4, hipMemcpyHostToDevice, p->stream), "slice");
    forward_sum(p, false, false);
    double lz = -INFINITY;
    hip_check(hipMemcpyAsync(&lz, p->d_out, sizeof(double), hipMemcpyDeviceToHost, p->stream), "D2H");
    hip_check(hipStreamSynchronize(p->stream), "slice");
    if (!(lz > -INFINITY)) continue;
    const double m = std::max(prefix, lz);
    prefix = m + std::log(std::exp(prefix - m) + std::exp(lz - m));
    if (n == 0) continue;
    const double q = std::exp(lz - prefix);
    ids.clear();
    for (int64_t i = 0; i < n; ++i)
      if (sample_uniform((uint64_t)i, kSliceDrawNode, (uint32_t)s, seed) < q) ids.push_back(i);
    if (ids.empty()) continue;
    hip_check(hipMemcpyAsync(stg.ids, ids.data(), ids.size() * 8, hipMemcpyHostToDevice, p->stream), "ids");
    run_sched(p, p->samp_ops, p->sched_samp);
    launch_sample(p->arena, p->d_samp, (int)p->samp.size(), p->d_samp_meta, p->n_vars, (int64_t)ids.size(), seed,
                  p->d_evidence, stg.ids, stg.rows, p->stream);
    hip_check(hipGetLastError(), "sample launch");
    hip_check(hipStreamSynchronize(p->stream), "sample");
  }
  if (!(prefix > -INFINITY)) throw TnError(TN_E_ZERO_EVIDENCE, "p(e) = 0");
  if (n == 0) return;
  hip_check(hipMemcpyAsync(samples, stg.rows, (size_t)n * p->n_vars * 4, hipMemcpyDeviceToHost, p->stream), "D2H");
  hip_check(hipStreamSynchronize(p->stream), "sample");
}

static void check_sample_args(tn_plan_t *p, int64_t n, int32_t *samples) {
  if (!p || (!samples && n > 0)) throw TnError(TN_E_INVALID, "NULL argument");
  if (n < 0) throw TnError(TN_E_INVALID, "negative sample count");
  if (!p->want_sum || p->is_mmap || p->batched_ev)
    throw TnError(TN_E_UNSUPPORTED, "sampling needs a sum-product plan without batched evidence");
}

// n samples into the staging rows, then to the host (stg.rows holds
// n * n_vars int32; stg.ids n int64 on sliced plans).
static void sample_impl(tn_plan_t *p, const int32_t *evidence, int64_t n, uint64_t seed, int32_t *samples,
                        const SampleStaging &stg) {
  if (!p->sliced.empty()) {
    sample_sliced(p, evidence, n, seed, samples, stg);
    return;
  }
  upload_evidence(p, 1, evidence);
  forward_sum(p, false, false);
  run_sched(p, p->samp_ops, p->sched_samp);
  std::vector<double> lz(1);
  hip_check(hipMemcpyAsync(lz.data(), p->d_out, sizeof(double), hipMemcpyDeviceToHost, p->stream), "D2H");
  hip_check(hipStreamSynchronize(p->stream), "sample forward");
  if (!(lz[0] > -INFINITY)) throw TnError(TN_E_ZERO_EVIDENCE, "p(e) = 0");
  if (n == 0) return;
  launch_sample(p->arena, p->d_samp, (int)p->samp.size(), p->d_samp_meta, p->n_vars, n, seed, p->d_evidence,
                nullptr, stg.rows, p->stream);
  hip_check(hipGetLastError(), "sample launch");
  hip_check(hipMemcpyAsync(samples, stg.rows, (size_t)n * p->n_vars * 4, hipMemcpyDeviceToHost, p->stream), "D2H");
  hip_check(hipStreamSynchronize(p->stream), "sample");
}

extern "C" tn_status tn_sample(tn_plan_t *p, const int32_t *evidence, int64_t n, uint64_t seed, int32_t *samples) {
  return guard([&] {
    check_sample_args(p, n, samples);
    SampleStaging stg;
    int64_t *d_ids = nullptr;
    if (n > 0) {
      ensure_sample_buffer(p, n);
      stg.rows = p->d_samp_out;
      if (!p->sliced.empty()) d_ids = stg.ids = dalloc<int64_t>(p, (size_t)n);
    }
    struct FreeIds {  // the id list lives for this call only
      tn_plan_t *p;
      int64_t *d;
      ~FreeIds() {
        if (!d) return;
        (void)hipStreamSynchronize(p->stream);
        (void)hipFree(d);
        p->allocs.erase(std::find(p->allocs.begin(), p->allocs.end(), (void *)d));
      }
    } free_ids{p, d_ids};
    sample_impl(p, evidence, n, seed, samples, stg);
  });
}

extern "C" tn_status tn_sample_noalloc(tn_plan_t *p, const int32_t *evidence, int64_t n, uint64_t seed,
                                       int32_t *samples) {
  return guard([&] {
    check_sample_args(p, n, samples);
    // rows first, then the id list 256-byte aligned behind them
    const int64_t row_ints = n * (int64_t)p->n_vars;
    const int64_t id_off = (row_ints + 63) / 64 * 64;
    const int64_t need = p->sliced.empty() ? row_ints : id_off + 2 * n;
    if (p->n_vars > 0 && (n > kScratchInts / p->n_vars || need > kScratchInts))
      throw TnError(TN_E_TOO_LARGE, "tn_sample_noalloc: " + std::to_string(n) + " samples of " +
                                        std::to_string(p->n_vars) + " variables exceed the static staging of " +
                                        std::to_string(kScratchInts) + " int32 (" +
                                        std::to_string(kScratchInts * 4 >> 20) + " MiB)");
    std::string err;
    int32_t *base = scratch_ptr(p->device, err);
    if (!base) throw TnError(TN_E_DEVICE, err);
    SampleStaging stg;
    stg.rows = base;
    stg.ids = reinterpret_cast<int64_t *>(base + id_off);
    struct Eager {  // no graph capture or instantiation in this call
      tn_plan_t *p;
      bool was;
      ~Eager() { p->eager = was; }
    } eager{p, p->eager};
    p->eager = true;
    sample_impl(p, evidence, n, seed, samples, stg);
  });
}

extern "C" tn_status tn_logZ_dev(tn_plan_t *p, const int32_t *evidence, const float *values_dev, double *logz_dev,
                                 float *grad_dev) {
  return guard([&] {
    if (!p || !values_dev || !logz_dev) throw TnError(TN_E_INVALID, "NULL argument");
    if (!p->want_sum || p->is_mmap || p->batched_ev)
      throw TnError(TN_E_UNSUPPORTED, "tn_logZ_dev needs a sum-product plan in mode NONE or SLICED (one instance)");
    if (grad_dev && !p->want_grad) throw TnError(TN_E_UNSUPPORTED, "plan built without want_factor_grad");
    if (!p->sliced.empty()) throw TnError(TN_E_UNSUPPORTED, "tn_logZ_dev on a sliced plan");
    const tn_net *net = p->net_src;
    upload_evidence(p, 1, evidence);
    // factor store (linear) lives at arena offset 0
    hip_check(hipMemcpyAsync(p->arena, values_dev, (size_t)net->n_values * 4, hipMemcpyDeviceToDevice, p->stream), "values");
    forward_sum(p, grad_dev != nullptr);
    hip_check(hipMemcpyAsync(logz_dev, p->d_out, sizeof(double), hipMemcpyDeviceToDevice, p->stream), "logz");
    if (grad_dev) {
      hip_check(hipMemsetAsync(grad_dev, 0, (size_t)net->n_values * 4, p->stream), "grad clear");
      const TensorBuf &r = p->T[p->sum_tree.root];
      launch_factor_grad(p->arena, p->d_grad_desc, (int)p->grads.size(), p->d_gmap, p->d_obs, p->d_evidence, p->ex,
                         p->arena + r.off, r.slot, net->n_values, grad_dev, p->stream);
      hip_check(hipGetLastError(), "grad launch");
    }
  });
}

extern "C" tn_status tn_sync(tn_plan_t *p) {
  return guard([&] {
    if (!p) throw TnError(TN_E_INVALID, "NULL plan");
    hip_check(hipStreamSynchronize(p->stream), "sync");
  });
}

// ---------------------------------------------------------------------------
// MMAP (paper: section on maximum marginal a posteriori, eq. mmap)
//   1. partition the factor tables so that every summed variable has all of
//      its tables in one group (union-find over summed variables);
//   2. contract every group with its query variables left open (sliced when
//      an intermediate would exceed the size cap; slice results are summed);
//   3. solve the MPE of the network of group results and query-only tables.
// ---------------------------------------------------------------------------
static int uf_find(std::vector<int> &u, int x) {
  while (u[x] != x) x = u[x] = u[u[x]];
  return x;
}

static void build_mmap(tn_plan_t *p, const tn_net *net) {
  const tn_plan_opts &o = p->opts;
  std::vector<char> isq(p->n_vars, 0);
  for (int i = 0; i < o.n_query; ++i) {
    int v = o.query[i];
    if (v < 0 || v >= p->n_vars) throw TnError(TN_E_INVALID, "query variable out of range");
    if (isq[v]) throw TnError(TN_E_INVALID, "query variable listed twice");
    if (p->is_obs[v]) throw TnError(TN_E_INVALID, "query and evidence variables must be disjoint");
    isq[v] = 1;
  }
  for (int v = 0; v < p->n_vars; ++v)
    if (isq[v]) p->query.push_back(v);
  const int F = (int)net->scope.size();
  std::vector<int> uf(F);
  std::iota(uf.begin(), uf.end(), 0);
  std::vector<int> first(p->n_vars, -1);
  std::vector<char> summed_in_factor(p->n_vars, 0);
  for (int f = 0; f < F; ++f)
    for (int v : net->scope[f]) {
      if (isq[v] || p->is_obs[v]) continue;
      summed_in_factor[v] = 1;
      if (first[v] < 0) first[v] = f;
      else uf[uf_find(uf, f)] = uf_find(uf, first[v]);
    }
  for (int v = 0; v < p->n_vars; ++v)
    if (!isq[v] && !p->is_obs[v] && !summed_in_factor[v]) p->mmap_const += std::log((double)p->card[v]);
  std::map<int, std::vector<int>> comp;
  std::vector<int> qonly;
  for (int f = 0; f < F; ++f) {
    bool has_summed = false;
    for (int v : net->scope[f])
      if (!isq[v] && !p->is_obs[v]) has_summed = true;
    if (has_summed) comp[uf_find(uf, f)].push_back(f);
    else qonly.push_back(f);
  }
  std::vector<int> qleaf_tensor;
  std::vector<Labels> qleaf_lab;
  p->stats = TreeStats{};
  for (auto &kv : comp) {
    const std::vector<int> &fs = kv.second;
    TreeExec t;
    std::vector<Labels> labs;
    Labels outq;
    for (int f : fs) {
      Labels l;
      for (int v : net->scope[f])
        if (!p->is_obs[v]) l.push_back(v);
      std::sort(l.begin(), l.end());
      for (int v : l)
        if (isq[v]) outq.push_back(v);
      labs.push_back(l);
    }
    std::sort(outq.begin(), outq.end());
    outq.erase(std::unique(outq.begin(), outq.end()), outq.end());
    PlanChoice pc = plan_tree(labs, p->card, outq, o.planner, o.restarts, o.seed, o.max_log2_size);
    Labels sl;
    if (o.max_log2_size > 0 && pc.stats.sc > o.max_log2_size + 1e-9)
      sl = choose_slices(labs, pc.pairs, outq, p->card, o.max_log2_size);
    std::vector<char> fixed = p->is_obs;
    for (int v : sl) fixed[v] = 1;
    p->group_sliced_ptr.push_back((int)p->group_sliced_vars.size());
    for (int v : sl) p->group_sliced_vars.push_back(v);
    for (int v : sl) p->sliced.push_back(v);
    std::vector<Labels> slabs;
    std::vector<LeafDesc> gl;
    for (size_t i = 0; i < fs.size(); ++i) {
      Labels l;
      for (int v : labs[i])
        if (!fixed[v]) l.push_back(v);
      slabs.push_back(l);
      int tid = new_tensor(p, l, false, true);
      LeafDesc d{};
      d.kind = 0;
      d.var = -1;
      d.size = (int32_t)numel(l, p->card);
      d.ident = factor_gather(p, net, fs[i], fixed, d.gmap, d.obs_begin, d.obs_end) ? 1 : 0;
      d.src = net->val_off[fs[i]];
      d.dst = tid;
      d.slot = tid;
      gl.push_back(d);
      t.leaf_tensor.push_back(tid);
    }
    t.pairs = pc.pairs;
    t.out = outq;
    t.lab = node_labels(slabs, t.pairs, outq, p->n_vars);
    TreeStats st = tree_stats(slabs, t.pairs, outq, p->card);
    p->stats.sc = std::max(p->stats.sc, st.sc);
    p->stats.sc_union = std::max(p->stats.sc_union, st.sc_union);
    const double nsl = std::exp2(std::accumulate(sl.begin(), sl.end(), 0.0,
                                                 [&](double a, int v) { return a + std::log2((double)p->card[v]); }));
    p->stats.flops += st.flops * nsl;
    p->stats.bytes += st.bytes * nsl;
    build_forward(p, t, SEMI_SUM);
    if (o.no_fuse != 1) {  // the sum phase runs forward only: every chain may fuse
      fuse_forward(p, t.ops, std::vector<char>(t.ops.size(), 1), t.fops);
      t.fused = !t.fops.empty();
    }
    // log-domain copy of the group result: a leaf of the max phase
    int lg = new_tensor(p, outq, false, false);
    p->group_log.push_back(lg);
    qleaf_tensor.push_back(lg);
    qleaf_lab.push_back(outq);
    p->groups.push_back(std::move(t));
    p->group_leaves.push_back(std::move(gl));
  }
  p->group_sliced_ptr.push_back((int)p->group_sliced_vars.size());
  p->stats.tc = p->stats.flops > 0 ? std::log2(p->stats.flops / 2) : 0;
  // max phase leaves: query-only tables, then one zero vector per query
  // variable so that every query variable is read out
  for (int f : qonly) {
    Labels l;
    for (int v : net->scope[f])
      if (!p->is_obs[v]) l.push_back(v);
    std::sort(l.begin(), l.end());
    int tid = new_tensor(p, l, false, false);
    LeafDesc d{};
    d.kind = 0;
    d.size = (int32_t)numel(l, p->card);
    d.ident = factor_gather(p, net, f, p->is_obs, d.gmap, d.obs_begin, d.obs_end) ? 1 : 0;
    d.src = net->val_off[f];
    d.dst = tid;
    d.slot = -1;
    d.maxdom = 1;
    p->qleaves.push_back(d);
    qleaf_tensor.push_back(tid);
    qleaf_lab.push_back(l);
  }
  for (int v : p->query) {
    int tid = new_tensor(p, Labels{v}, false, false);
    LeafDesc d{};
    d.kind = 1;
    d.var = v;
    d.size = p->card[v];
    d.dst = tid;
    d.slot = -1;
    d.maxdom = 1;
    p->qleaves.push_back(d);
    qleaf_tensor.push_back(tid);
    qleaf_lab.push_back(Labels{v});
  }
  TreeExec &q = p->qtree;
  q.leaf_tensor = qleaf_tensor;
  PlanChoice qc = plan_tree(qleaf_lab, p->card, {}, o.planner, o.restarts, o.seed);
  q.pairs = qc.pairs;
  q.out = {};
  q.lab = node_labels(qleaf_lab, q.pairs, {}, p->n_vars);
  build_forward(p, q, SEMI_MAX);
  build_backtrack(p, q);
}

static void allocate_mmap(tn_plan_t *p) {
  int64_t mx = 1;
  for (size_t g = 0; g < p->groups.size(); ++g) mx = std::max(mx, p->T[p->groups[g].root].size);
  p->d_acc = dalloc<double>(p, (size_t)mx + 64);
}

static void run_mmap(tn_plan_t *p, const int32_t *evidence, int32_t *assign_q, double *value) {
  std::vector<int32_t> row(p->n_vars, -1);
  for (int v = 0; v < p->n_vars; ++v) {
    int e = evidence ? evidence[v] : -1;
    if (e < -1 || e >= p->card[v]) throw TnError(TN_E_INVALID, "evidence value out of range");
    if ((e >= 0) != (bool)p->is_obs[v]) throw TnError(TN_E_INVALID, "evidence must give exactly the plan's observed variables");
    row[v] = e;
  }
  int32_t *acc_ex = p->iarena + p->iarena_ints;  // one int past the index arena
  std::vector<int32_t> rows;
  for (size_t g = 0; g < p->groups.size(); ++g) {
    const TreeExec &t = p->groups[g];
    const int sb = p->group_sliced_ptr[g], se = p->group_sliced_ptr[g + 1];
    int64_t n_slices = 1;
    for (int i = sb; i < se; ++i) n_slices *= p->card[p->group_sliced_vars[i]];
    const TensorBuf &r = p->T[t.root];
    for (int64_t s0 = 0; s0 < n_slices; s0 += kSliceChunk) {
      slice_chunk(
          p, rows, s0, std::min(kSliceChunk, n_slices - s0),
          [&](int64_t s, int32_t *rw) {
            std::copy(row.begin(), row.end(), rw);
            for (int i = se - 1; i >= sb; --i) {
              const int v = p->group_sliced_vars[i];
              rw[v] = (int32_t)(s % p->card[v]);
              s /= p->card[v];
            }
          },
          [&](int64_t j) {
            launch_prepare_set(p, p->group_leaves[g], p->d_group_leaves[g], true);
            run_sched(p, t.fused ? t.fops : t.ops, p->sched_groups[g]);
            launch_slice_acc(p->arena + r.off, p->mx, p->ex, r.slot, p->d_acc, acc_ex, r.size, s0 + j == 0 ? 1 : 0,
                             p->stream);
          });
    }
    launch_acc_tolog(p->d_acc, acc_ex, r.size, p->arena + p->T[p->group_log[g]].off, p->stream);
  }
  hip_check(hipMemcpyAsync(p->d_evidence, row.data(), row.size() * 4, hipMemcpyHostToDevice, p->stream), "evidence");
  hip_check(hipMemcpyAsync(p->d_assign, row.data(), row.size() * 4, hipMemcpyHostToDevice, p->stream), "init");
  launch_prepare_set(p, p->qleaves, p->d_qleaves, false);
  run_sched(p, p->qtree.ops, p->sched_q);
  launch_backtrack(p->iarena, p->d_qback, p->d_qback_lev, p->qtree.n_back_lev, p->qtree.n_back_chunks, p->d_qback_meta,
                   p->n_vars, 1, p->d_assign,
                   p->stream);
  hip_check(hipGetLastError(), "mmap launch");
  std::vector<int32_t> a(p->n_vars);
  float rv = 0;
  hip_check(hipMemcpyAsync(a.data(), p->d_assign, a.size() * 4, hipMemcpyDeviceToHost, p->stream), "D2H");
  hip_check(hipMemcpyAsync(&rv, p->arena + p->T[p->qtree.root].off, 4, hipMemcpyDeviceToHost, p->stream), "D2H");
  hip_check(hipStreamSynchronize(p->stream), "mmap");
  for (size_t i = 0; i < p->query.size(); ++i) assign_q[i] = a[p->query[i]];
  if (value) *value = (double)rv + p->mmap_const;
}

extern "C" tn_status tn_mmap(tn_plan_t *p, const int32_t *evidence, int32_t *assign_q, double *log_value) {
  return guard([&] {
    if (!p || !assign_q) throw TnError(TN_E_INVALID, "NULL argument");
    if (!p->is_mmap) throw TnError(TN_E_UNSUPPORTED, "plan has no query set");
    double v = -INFINITY;
    run_mmap(p, evidence, assign_q, &v);
    if (!(v > -INFINITY)) throw TnError(TN_E_ZERO_EVIDENCE, "p(e) = 0");
    if (log_value) *log_value = v;
  });
}

// ---------------------------------------------------------------------------
// per-launch profile (events around every launch of one task)
// ---------------------------------------------------------------------------
static tn_status profile_impl(tn_plan_t *p, int32_t task, int32_t batch, const int32_t *evidence, int32_t reps,
                              tn_op_profile *out, int32_t cap, int32_t *n_ops, int32_t kind_only) {
  return guard([&] {
    if (!p || reps < 1) throw TnError(TN_E_INVALID, "bad argument");
    if (p->is_mmap != (task == 3)) throw TnError(TN_E_UNSUPPORTED, "task 3 is the profile of MMAP plans");
    if ((task <= 1 && !p->want_sum) || (task == 2 && !p->want_max)) throw TnError(TN_E_UNSUPPORTED, "task not in plan");
    std::vector<int32_t> slice_row;
    if (task == 3) {
      // sum phase of every group for its first slice (sliced variables at 0)
      slice_row.assign(p->n_vars, -1);
      for (int v = 0; v < p->n_vars; ++v) {
        const int e = evidence ? evidence[v] : -1;
        if (e < -1 || e >= p->card[v] || (e >= 0) != (bool)p->is_obs[v])
          throw TnError(TN_E_INVALID, "evidence must give exactly the plan's observed variables");
        slice_row[v] = e;
      }
      for (int v : p->sliced) slice_row[v] = 0;
      hip_check(hipMemcpyAsync(p->d_evidence, slice_row.data(), slice_row.size() * 4, hipMemcpyHostToDevice, p->stream),
                "slice");
      hip_check(hipStreamSynchronize(p->stream), "slice");
    } else {
      check_batch(p, batch);
      if (p->mode == TN_EVIDENCE_SLICED && !p->batched_ev && batch != 1)
        throw TnError(TN_E_INVALID, "profile one instance at a time");
      upload_evidence(p, batch, evidence);
    }
    // launch list: (kind, flops, bytes, launcher)
    struct L {
      int kind;
      double flops, bytes;
      std::function<void()> go;
    };
    std::vector<L> ls;
    // one entry per launch of the schedule actually run by the task (grouped
    // stages included), with the algorithmic work of the ops it covers
    auto add_ops = [&](const std::vector<Op> &ops, const Schedule &sc) {
      for (const Launch &L : sc.launches) {
        double fl = 0, by = 0;
        for (int i : L.ops) {
          const Op &op = ops[i];
          fl += op.seg >= 0 ? op.flops : op.flops * op.inst;
          by += op.seg >= 0 ? op.bytes : (op.bytes + (op.semi == SEMI_MAX ? 4.0 * p->T[op.Z].size : 0.0)) * op.inst;
        }
        int kind;
        if (L.seg) kind = L.seg_kind >= 5 ? L.seg_kind + 1 : 5 + L.seg_kind;  // 6 carrier forward (one segment
                                                                               // or a pair), 7 carrier reverse,
                                                                               // 8 composed maps, 9 adjoint sweeps
        else if (L.gemm) kind = L.semi == SEMI_MAX ? 11 : 10;
        else if (L.inter) kind = L.semi == SEMI_MAX ? 13 : 12;
        else kind = (L.split ? 2 : 0) + (L.semi == SEMI_MAX ? 1 : 0);
        const Launch *lp = &L;
        const std::vector<Op> *opsp = &ops;
        ls.push_back({kind, fl, by, [p, lp, opsp] {
                        Schedule one;
                        one.launches.push_back(*lp);
                        run_sched(p, *opsp, one);
                      }});
      }
    };
    if (task <= 1) {
      ls.push_back({4, 0, 0, [p] { launch_prepare_set(p, p->leaves_sum, p->d_leaves_sum, true); }});
      if (p->fused) add_ops(p->ffwd, p->sched_ffwd);
      else add_ops(p->sum_tree.ops, p->sched_fwd);
      ls.push_back({5, 0, 0, [p] {
                      const TensorBuf &r = p->T[p->sum_tree.root];
                      launch_logz(p->arena + r.off, r.batched ? (p->inter ? 1 : r.size) : 0, p->ex, r.slot, r.batched, p->max_batch,
                                  p->d_out, p->stream);
                    }});
      if (task == 1) {
        if (p->fused) add_ops(p->fbwd, p->sched_fbwd);
        else add_ops(p->bwd, p->sched_bwd);
        ls.push_back({5, 0, 0, [p] {
                        launch_marg(p->arena, p->d_marg_desc, (int)p->marg.size(), p->max_batch, p->marg_row,
                                    p->d_marg, p->stream);
                      }});
      }
    } else if (task == 3) {
      int32_t *acc_ex = p->iarena + p->iarena_ints;
      for (size_t g = 0; g < p->groups.size(); ++g) {
        ls.push_back({4, 0, 0, [p, g] { launch_prepare_set(p, p->group_leaves[g], p->d_group_leaves[g], true); }});
        add_ops(p->groups[g].fused ? p->groups[g].fops : p->groups[g].ops, p->sched_groups[g]);
        ls.push_back({5, 0, 0, [p, g, acc_ex] {
                        const TensorBuf &r = p->T[p->groups[g].root];
                        launch_slice_acc(p->arena + r.off, p->mx, p->ex, r.slot, p->d_acc, acc_ex, r.size, 1, p->stream);
                      }});
      }
    } else {
      ls.push_back({4, 0, 0, [p] { launch_prepare_set(p, p->leaves_max, p->d_leaves_max, false); }});
      add_ops(p->max_tree.fused ? p->max_tree.fops : p->max_tree.ops, p->sched_max);
      ls.push_back({5, 0, 0, [p] {
                      launch_backtrack(p->iarena, p->d_back, p->d_back_lev, p->max_tree.n_back_lev,
                                       p->max_tree.n_back_chunks, p->d_back_meta, p->n_vars, p->max_batch, p->d_assign, p->stream);
                    }});
    }
    if (kind_only >= 0) {
      // the launches of one kind back to back, bracketed by two events
      std::vector<size_t> sel;
      for (size_t i = 0; i < ls.size(); ++i)
        if (ls[i].kind == kind_only) sel.push_back(i);
      hipEvent_t e0, e1;
      hip_check(hipEventCreate(&e0), "event");
      hip_check(hipEventCreate(&e1), "event");
      for (size_t i : sel) ls[i].go();  // warm
      hip_check(hipEventRecord(e0, p->stream), "event");
      for (int r = 0; r < reps; ++r)
        for (size_t i : sel) ls[i].go();
      hip_check(hipEventRecord(e1, p->stream), "event");
      hip_check(hipEventSynchronize(e1), "event sync");
      hip_check(hipGetLastError(), "profile launch");
      float ms = 0;
      hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      if (n_ops) *n_ops = (int32_t)sel.size();
      if (cap > 0 && !sel.empty()) {
        out[0].kind = kind_only;
        out[0].flops = 0;
        out[0].bytes = 0;
        for (size_t i : sel) {
          out[0].flops += ls[i].flops;
          out[0].bytes += ls[i].bytes;
        }
        out[0].ms = ms / reps / (double)sel.size();
        out[0].flops /= (double)sel.size();
        out[0].bytes /= (double)sel.size();
      }
      return;
    }
    std::vector<hipEvent_t> ev(ls.size() + 1);
    for (auto &e : ev) hip_check(hipEventCreate(&e), "event");
    std::vector<double> acc(ls.size(), 0.0);
    for (int r = 0; r < reps; ++r) {
      hip_check(hipEventRecord(ev[0], p->stream), "event");
      for (size_t i = 0; i < ls.size(); ++i) {
        ls[i].go();
        hip_check(hipEventRecord(ev[i + 1], p->stream), "event");
      }
      hip_check(hipEventSynchronize(ev.back()), "event sync");
      hip_check(hipGetLastError(), "profile launch");
      for (size_t i = 0; i < ls.size(); ++i) {
        float ms = 0;
        hip_check(hipEventElapsedTime(&ms, ev[i], ev[i + 1]), "elapsed");
        acc[i] += ms;
      }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (n_ops) *n_ops = (int32_t)ls.size();
    for (size_t i = 0; i < ls.size() && (int)i < cap; ++i) {
      out[i].kind = ls[i].kind;
      out[i].flops = ls[i].flops;
      out[i].bytes = ls[i].bytes;
      out[i].ms = acc[i] / reps;
    }
  });
}

extern "C" tn_status tn_profile(tn_plan_t *p, int32_t task, int32_t batch, const int32_t *evidence, int32_t reps,
                                tn_op_profile *out, int32_t cap, int32_t *n_ops) {
  return profile_impl(p, task, batch, evidence, reps, out, cap, n_ops, -1);
}

extern "C" tn_status tn_profile_kind(tn_plan_t *p, int32_t task, int32_t kind, int32_t batch, const int32_t *evidence,
                                     int32_t reps, tn_op_profile *avg, int32_t *n_launches) {
  if (kind < 0) {
    g_err = "kind must be >= 0";
    return TN_E_INVALID;
  }
  return profile_impl(p, task, batch, evidence, reps, avg, 1, n_launches, kind);
}
