// Contraction-tree construction and analysis (host).
//
// The paper (section on contraction orders) treats the order of pairwise
// contractions as a binary tree whose leaves are the input tensors; the
// order changes the cost -- space complexity (largest intermediate) and time
// complexity -- but not the result, and finding the best order is NP-hard,
// so heuristics are used.  This file holds the tree semantics (which labels
// every node keeps), complexity measures, and the heuristics: bucket
// elimination along a variable order (natural, min-degree, min-fill, with
// randomised tie-breaks) and a pairwise greedy on output size, run as a
// best-of search, plus the choice of labels to slice under a size cap.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <functional>
#include <limits>
#include <numeric>
#include <queue>
#include <random>
#include <unordered_map>

#include "tn_internal.h"

namespace tn {

static double log2size(const Labels &l, const std::vector<int> &card) {
  double s = 0;
  for (int v : l) s += std::log2((double)card[v]);
  return s;
}

static Labels merge_sorted(const Labels &a, const Labels &b) {
  Labels u;
  u.reserve(a.size() + b.size());
  std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(u));
  return u;
}

void validate_tree(int n_leaves, const std::vector<Pair> &pairs) {
  if (n_leaves < 1) throw TnError(TN_E_INVALID, "contraction tree needs at least one leaf");
  if ((int)pairs.size() != n_leaves - 1)
    throw TnError(TN_E_INVALID, "contraction tree over " + std::to_string(n_leaves) +
                                    " leaves needs " + std::to_string(n_leaves - 1) + " pairs");
  std::vector<char> used(n_leaves + pairs.size(), 0);
  for (size_t p = 0; p < pairs.size(); ++p) {
    int c = n_leaves + (int)p;
    for (int k = 0; k < 2; ++k) {
      int x = pairs[p][k];
      if (x < 0 || x >= c) throw TnError(TN_E_INVALID, "tree pair refers to a later or invalid node");
      if (used[x]) throw TnError(TN_E_INVALID, "tree uses a node twice");
      used[x] = 1;
    }
    if (pairs[p][0] == pairs[p][1]) throw TnError(TN_E_INVALID, "tree pair joins a node with itself");
  }
}

std::vector<Labels> node_labels(const std::vector<Labels> &leaves, const std::vector<Pair> &pairs,
                                const Labels &out, int n_vars) {
  std::vector<int> total(n_vars, 0);
  std::vector<char> keep(n_vars, 0);
  for (int v : out) keep[v] = 1;
  for (auto &l : leaves)
    for (int v : l) total[v]++;
  std::vector<Labels> lab(leaves.begin(), leaves.end());
  // per node: number of leaves of its subtree holding each kept label
  std::vector<std::vector<int>> cnt(leaves.size());
  for (size_t i = 0; i < leaves.size(); ++i) cnt[i].assign(leaves[i].size(), 1);
  lab.reserve(leaves.size() + pairs.size());
  for (auto &p : pairs) {
    const Labels &A = lab[p[0]], &B = lab[p[1]];
    const std::vector<int> &ca = cnt[p[0]], &cb = cnt[p[1]];
    Labels L;
    std::vector<int> C;
    size_t i = 0, j = 0;
    while (i < A.size() || j < B.size()) {
      int v, k;
      if (j == B.size() || (i < A.size() && A[i] < B[j])) { v = A[i]; k = ca[i]; ++i; }
      else if (i == A.size() || B[j] < A[i]) { v = B[j]; k = cb[j]; ++j; }
      else { v = A[i]; k = ca[i] + cb[j]; ++i; ++j; }
      if (keep[v] || total[v] > k) { L.push_back(v); C.push_back(k); }
    }
    lab.push_back(std::move(L));
    cnt.push_back(std::move(C));
  }
  return lab;
}

TreeStats tree_stats(const std::vector<Labels> &leaves, const std::vector<Pair> &pairs,
                     const Labels &out, const std::vector<int> &card) {
  TreeStats s;
  auto lab = node_labels(leaves, pairs, out, (int)card.size());
  const int L = (int)leaves.size();
  double tc = 0;
  if (pairs.empty()) {
    double u = log2size(leaves[0], card);
    s.sc = log2size(out, card);
    s.sc_union = u;
    tc = std::exp2(u);
    s.bytes = 4.0 * (std::exp2(u) + std::exp2(s.sc));
  }
  for (size_t p = 0; p < pairs.size(); ++p) {
    const Labels &A = lab[pairs[p][0]], &B = lab[pairs[p][1]], &C = lab[L + p];
    double u = log2size(merge_sorted(A, B), card);
    s.sc = std::max(s.sc, log2size(C, card));
    s.sc_union = std::max(s.sc_union, u);
    tc += std::exp2(u);
    s.bytes += 4.0 * (std::exp2(log2size(A, card)) + std::exp2(log2size(B, card)) +
                      std::exp2(log2size(C, card)));
  }
  s.flops = 2.0 * tc;
  s.tc = tc > 0 ? std::log2(tc) : 0;
  return s;
}

// ---------------------------------------------------------------------------
// Bucket elimination along an order
// ---------------------------------------------------------------------------

struct Forest {
  const std::vector<int> &card;
  std::vector<Labels> lab;
  std::vector<double> lsz;
  std::vector<char> alive;
  std::vector<int> count;      // alive tensors holding each label
  std::vector<char> keep;
  std::vector<Pair> pairs;
  int n_leaves;

  Forest(const std::vector<Labels> &leaves, const std::vector<int> &c, const Labels &out)
      : card(c), lab(leaves), alive(leaves.size(), 1), count(c.size(), 0), keep(c.size(), 0),
        n_leaves((int)leaves.size()) {
    for (auto &l : lab) {
      lsz.push_back(log2size(l, card));
      for (int v : l) count[v]++;
    }
    for (int v : out) keep[v] = 1;
  }
  // labels of the merge of a and b under the tree semantics
  Labels merged(int a, int b) const {
    Labels u = merge_sorted(lab[a], lab[b]);
    Labels o;
    for (int v : u) {
      int inside = (std::binary_search(lab[a].begin(), lab[a].end(), v) ? 1 : 0) +
                   (std::binary_search(lab[b].begin(), lab[b].end(), v) ? 1 : 0);
      if (keep[v] || count[v] > inside) o.push_back(v);
    }
    return o;
  }
  int merge(int a, int b) {
    Labels o = merged(a, b);
    for (int v : lab[a]) count[v]--;
    for (int v : lab[b]) count[v]--;
    for (int v : o) count[v]++;
    alive[a] = alive[b] = 0;
    pairs.push_back({a, b});
    lab.push_back(std::move(o));
    lsz.push_back(log2size(lab.back(), card));
    alive.push_back(1);
    return (int)lab.size() - 1;
  }
  // merge a set of tensors smallest first (ties by the given keys)
  int merge_all(std::vector<int> ids, std::mt19937_64 *rng) {
    auto key = [&](int i) { return lsz[i]; };
    std::vector<uint64_t> tie(lab.size() + ids.size() + 4, 0);
    while (ids.size() > 1) {
      std::sort(ids.begin(), ids.end(), [&](int x, int y) {
        if (key(x) != key(y)) return key(x) < key(y);
        return x < y;
      });
      if (rng && ids.size() > 2 && key(ids[1]) == key(ids[2])) {
        // randomise among equal-size candidates for the second slot
        size_t e = 2;
        while (e < ids.size() && key(ids[e]) == key(ids[1])) ++e;
        std::uniform_int_distribution<size_t> d(1, e - 1);
        std::swap(ids[1], ids[d(*rng)]);
      }
      int c = merge(ids[0], ids[1]);
      ids.erase(ids.begin(), ids.begin() + 2);
      ids.push_back(c);
    }
    return ids.empty() ? -1 : ids[0];
  }
};

static std::vector<Pair> bucket_tree(const std::vector<Labels> &leaves, const std::vector<int> &card,
                                     const Labels &out, const std::vector<int> &order,
                                     std::mt19937_64 *rng) {
  Forest F(leaves, card, out);
  std::vector<std::vector<int>> where(card.size());
  for (int i = 0; i < (int)leaves.size(); ++i)
    for (int v : leaves[i]) where[v].push_back(i);
  for (int v : order) {
    std::vector<int> ids;
    for (int i : where[v])
      if (F.alive[i]) ids.push_back(i);
    if (ids.size() < 2) continue;
    size_t before = F.lab.size();
    F.merge_all(ids, rng);
    for (size_t c = before; c < F.lab.size(); ++c)
      for (int u : F.lab[c]) where[u].push_back((int)c);
  }
  std::vector<int> rest;
  for (int i = 0; i < (int)F.lab.size(); ++i)
    if (F.alive[i]) rest.push_back(i);
  F.merge_all(rest, rng);
  return F.pairs;
}

// Greedy elimination orders on the interaction graph.  kind 0 = min-degree,
// 1 = min-fill.  Labels in `out` are never eliminated.
static std::vector<int> greedy_order(const std::vector<Labels> &leaves, int n_vars,
                                     const Labels &out, int kind, std::mt19937_64 *rng) {
  std::vector<std::vector<char>> adj(n_vars, std::vector<char>(n_vars, 0));
  std::vector<char> present(n_vars, 0), keep(n_vars, 0), gone(n_vars, 0);
  for (int v : out) keep[v] = 1;
  for (auto &l : leaves)
    for (int a : l) {
      present[a] = 1;
      for (int b : l)
        if (a != b) adj[a][b] = 1;
    }
  auto nbrs = [&](int v) {
    std::vector<int> r;
    for (int u = 0; u < n_vars; ++u)
      if (adj[v][u] && !gone[u]) r.push_back(u);
    return r;
  };
  auto score = [&](int v) -> double {
    auto nb = nbrs(v);
    if (kind == 0) return (double)nb.size();
    double f = 0;
    for (size_t i = 0; i < nb.size(); ++i)
      for (size_t j = i + 1; j < nb.size(); ++j)
        if (!adj[nb[i]][nb[j]]) f += 1;
    return f;
  };
  std::vector<double> sc(n_vars, 0);
  std::vector<uint64_t> tie(n_vars);
  std::vector<int> cand;
  for (int v = 0; v < n_vars; ++v)
    if (present[v] && !keep[v]) {
      cand.push_back(v);
      sc[v] = score(v);
      tie[v] = rng ? (*rng)() : (uint64_t)v;
    }
  std::vector<int> order;
  std::vector<char> dirty(n_vars, 0);
  while (!cand.empty()) {
    size_t best = 0;
    for (size_t i = 1; i < cand.size(); ++i) {
      int a = cand[i], b = cand[best];
      if (sc[a] < sc[b] || (sc[a] == sc[b] && tie[a] < tie[b])) best = i;
    }
    int v = cand[best];
    cand.erase(cand.begin() + best);
    auto nb = nbrs(v);
    for (size_t i = 0; i < nb.size(); ++i)
      for (size_t j = 0; j < nb.size(); ++j)
        if (i != j) adj[nb[i]][nb[j]] = 1;
    gone[v] = 1;
    order.push_back(v);
    for (int u : nb) {
      dirty[u] = 1;
      for (int w : nbrs(u)) dirty[w] = 1;
    }
    for (int u : cand)
      if (dirty[u]) {
        sc[u] = score(u);
        dirty[u] = 0;
      }
    std::fill(dirty.begin(), dirty.end(), 0);
  }
  return order;
}

// Pairwise greedy: repeatedly merge the pair of tensors sharing a label whose
// merge has the smallest size(out) - size(a) - size(b); randomised restarts
// perturb the output size.
static std::vector<Pair> greedy_pairs(const std::vector<Labels> &leaves, const std::vector<int> &card,
                                      const Labels &out, std::mt19937_64 *rng) {
  Forest F(leaves, card, out);
  std::vector<std::vector<int>> where(card.size());
  for (int i = 0; i < (int)leaves.size(); ++i)
    for (int v : leaves[i]) where[v].push_back(i);
  struct Cand {
    double cost;
    int a, b;
    bool operator<(const Cand &o) const {
      if (cost != o.cost) return cost > o.cost;
      if (a != o.a) return a > o.a;
      return b > o.b;
    }
  };
  std::priority_queue<Cand> pq;
  std::uniform_real_distribution<double> U(0.0, 1.0);
  auto cost = [&](int a, int b) {
    Labels o = F.merged(a, b);
    double so = std::exp2(log2size(o, card));
    if (rng) so *= 1.0 + 0.5 * U(*rng);
    return so - std::exp2(F.lsz[a]) - std::exp2(F.lsz[b]);
  };
  auto push_for = [&](int a) {
    std::vector<int> seen;
    for (int v : F.lab[a])
      for (int b : where[v])
        if (b != a && F.alive[b]) seen.push_back(b);
    std::sort(seen.begin(), seen.end());
    seen.erase(std::unique(seen.begin(), seen.end()), seen.end());
    for (int b : seen) pq.push({cost(std::min(a, b), std::max(a, b)), std::min(a, b), std::max(a, b)});
  };
  for (int i = 0; i < (int)leaves.size(); ++i) push_for(i);
  while (!pq.empty()) {
    Cand c = pq.top();
    pq.pop();
    if (!F.alive[c.a] || !F.alive[c.b]) continue;
    int n = F.merge(c.a, c.b);
    for (int v : F.lab[n]) where[v].push_back(n);
    push_for(n);
  }
  std::vector<int> rest;
  for (int i = 0; i < (int)F.lab.size(); ++i)
    if (F.alive[i]) rest.push_back(i);
  F.merge_all(rest, nullptr);
  return F.pairs;
}

// Two-front variant of an elimination order: the first half in order and the
// second half from its end, interleaved (v_0, v_{n-1}, v_1, v_{n-2}, ...).
// Bucket elimination then grows two intermediates from the two ends of the
// order, independent until they meet, so their contractions pair up in
// stages (half the sequential levels of a sweep).
static std::vector<int> two_front(const std::vector<int> &order) {
  const size_t n = order.size(), h = (n + 1) / 2;
  std::vector<int> r;
  r.reserve(n);
  for (size_t i = 0; i < h; ++i) {
    r.push_back(order[i]);
    if (n - 1 - i >= h) r.push_back(order[n - 1 - i]);
  }
  return r;
}

double roofline_time(const std::vector<Labels> &leaves, const std::vector<Pair> &pairs, const Labels &out,
                     const std::vector<int> &card) {
  const int L = (int)leaves.size();
  const auto lab = node_labels(leaves, pairs, out, (int)card.size());
  auto has = [](const Labels &l, int v) { return std::binary_search(l.begin(), l.end(), v); };
  double t = 0;
  for (size_t q = 0; q < pairs.size(); ++q) {
    const Labels &A = lab[pairs[q][0]], &B = lab[pairs[q][1]], &C = lab[L + q];
    const Labels U = merge_sorted(A, B);
    double m = 0, n = 0, s = 0;  // log2 entries of rows, columns and summed labels
    for (int v : U) {
      const bool a = has(A, v), b = has(B, v), c = has(C, v);
      const double lc = std::log2((double)card[v]);
      if (a && !b && c) m += lc;
      else if (b && !a && c) n += lc;
      else if (a && b && !c) s += lc;
    }
    // the dense form's eligibility: >= 16 rows, >= 8 columns, >= 8 summed
    // entries or none
    const bool dense = m >= 4 - 1e-9 && n >= 3 - 1e-9 && (s >= 3 - 1e-9 || s < 1e-9);
    const double flops = 2.0 * std::exp2(log2size(U, card));
    const double bytes = 4.0 * (std::exp2(log2size(A, card)) + std::exp2(log2size(B, card)) +
                                std::exp2(log2size(C, card)));
    t += kNodeLaunchSeconds + std::max(flops / (dense ? kDenseFlopRate : kVectorFlopRate),
                                       bytes / (dense ? kDenseByteRate : kVectorByteRate));
  }
  return t;
}

double stage_time(const std::vector<Labels> &leaves, const std::vector<Pair> &pairs, const Labels &out,
                  const std::vector<int> &card, int *n_levels) {
  const int L = (int)leaves.size(), P = (int)pairs.size();
  const auto lab = node_labels(leaves, pairs, out, (int)card.size());
  std::vector<int> level(L + P, 0);
  std::vector<double> worst;  // per level: the slowest node
  for (int q = 0; q < P; ++q) {
    const int c = L + q, a = pairs[q][0], b = pairs[q][1];
    level[c] = 1 + std::max(level[a], level[b]);
    const double mac = std::exp2(log2size(merge_sorted(lab[a], lab[b]), card));
    const double t = kStageLaunchSeconds + mac / kStageMacRate;
    if ((int)worst.size() < level[c]) worst.resize(level[c], 0.0);
    worst[level[c] - 1] = std::max(worst[level[c] - 1], t);
  }
  if (n_levels) *n_levels = (int)worst.size();
  double t = 0;
  for (double w : worst) t += w;
  return t;
}

PlanChoice plan_tree(const std::vector<Labels> &leaves, const std::vector<int> &card,
                     const Labels &out, int strategy, int restarts, uint64_t seed, double cap) {
  const int n_vars = (int)card.size();
  std::vector<char> isout(n_vars, 0);
  for (int v : out) isout[v] = 1;
  PlanChoice best;
  std::pair<double, double> best_key;
  bool have = false;
  auto consider = [&](std::vector<Pair> pairs, int which, bool twofront = false) {
    TreeStats st = tree_stats(leaves, pairs, out, card);
    std::pair<double, double> key(std::round(2 * st.sc) / 2, st.tc);
    if (cap <= 0) {
      // unsliced: among trees of one space-complexity class, the estimated
      // time of the stage schedule (every stage costs its slowest node)
      key.second = stage_time(leaves, pairs, out, card, nullptr);
    } else if (st.sc > cap + 1e-9) {
      // total work once sliced below the cap
      Labels sl;
      try {
        sl = choose_slices(leaves, pairs, out, card, cap);
      } catch (const TnError &) {
        return;  // cannot be sliced below the cap (output labels)
      }
      std::vector<char> fixed(n_vars, 0);
      for (int v : sl) fixed[v] = 1;
      std::vector<Labels> lv(leaves.size());
      for (size_t i = 0; i < leaves.size(); ++i)
        for (int v : leaves[i])
          if (!fixed[v]) lv[i].push_back(v);
      double ns = 1;
      for (int v : sl) ns *= card[v];
      // every slice runs the sliced tree: its roofline time, launches included
      key = std::make_pair(std::round(2 * cap) / 2, std::log2(ns * roofline_time(lv, pairs, out, card)));
    } else {
      key = std::make_pair(std::round(2 * cap) / 2, std::log2(roofline_time(leaves, pairs, out, card)));
    }
    if (!have || key < best_key) {
      best.pairs = std::move(pairs);
      best.stats = st;
      best.planner = which;
      best.two_front = twofront;
      best_key = key;
      have = true;
    }
  };
  // unsliced plans also try the two-front variant of each order (ties of its
  // bucket merges are not randomised, so the restarts' random streams stay
  // those of the base orders)
  auto consider_order = [&](const std::vector<int> &order, std::mt19937_64 *R, int which) {
    consider(bucket_tree(leaves, card, out, order, R), which);
    if (cap <= 0) consider(bucket_tree(leaves, card, out, two_front(order), nullptr), which, true);
  };
  if (leaves.size() == 1) {
    consider({}, strategy);
    return best;
  }
  restarts = std::max(1, restarts);
  if (strategy == TN_PLANNER_BEST || strategy == TN_PLANNER_NATURAL) {
    std::vector<int> order;
    for (int v = 0; v < n_vars; ++v)
      if (!isout[v]) order.push_back(v);
    consider_order(order, nullptr, TN_PLANNER_NATURAL);
  }
  for (int r = 0; r < restarts; ++r) {
    std::mt19937_64 rng(seed * 1000003ull + (uint64_t)r);
    std::mt19937_64 *R = r ? &rng : nullptr;
    if (strategy == TN_PLANNER_BEST || strategy == TN_PLANNER_MINFILL)
      consider_order(greedy_order(leaves, n_vars, out, 1, R), R, TN_PLANNER_MINFILL);
    if (strategy == TN_PLANNER_BEST || strategy == TN_PLANNER_MINDEG)
      consider_order(greedy_order(leaves, n_vars, out, 0, R), R, TN_PLANNER_MINDEG);
    if (strategy == TN_PLANNER_BEST || strategy == TN_PLANNER_GREEDY)
      consider(greedy_pairs(leaves, card, out, R), TN_PLANNER_GREEDY);
  }
  if (!have) throw TnError(TN_E_INVALID, "unknown planner");
  return best;
}

// Tree refinement for launch count: a chain of small nodes, each absorbing
// one side input into the previous node's result, takes one launch per node
// however little work it does.  The same inputs contracted as a balanced tree
// (adjacent inputs first, order kept) give the same result in log2(length)
// levels, and the levels' independent nodes share launches.  A chain is
// rebalanced only if the tree's largest intermediate does not grow and its
// work grows by at most 10 %.
std::vector<Pair> rebalance_small_chains(const std::vector<Labels> &leaves, const std::vector<Pair> &pairs,
                                         const Labels &out, const std::vector<int> &card, double max_log2) {
  const int L = (int)leaves.size(), P = (int)pairs.size(), N = L + P;
  if (P < 3) return pairs;
  const auto lab = node_labels(leaves, pairs, out, (int)card.size());
  std::vector<int> left(N, -1), right(N, -1), parent(N, -1), nleaf(N, 1);
  for (int q = 0; q < P; ++q) {
    const int c = L + q;
    left[c] = pairs[q][0];
    right[c] = pairs[q][1];
    parent[left[c]] = parent[right[c]] = c;
    nleaf[c] = nleaf[left[c]] + nleaf[right[c]];
  }
  auto small = [&](int c) { return c >= L && log2size(lab[c], card) <= max_log2 + 1e-9; };
  // carrier child of a small internal node: its small internal child with
  // more leaves (the other child is a side input)
  auto carrier = [&](int c) {
    const int a = left[c], b = right[c];
    const bool sa = small(a), sb = small(b);
    if (sa && sb) return nleaf[a] >= nleaf[b] ? a : b;
    return sa ? a : (sb ? b : -1);
  };
  // new tree: item lists per rebuilt chain top, emitted recursively
  std::vector<std::vector<int>> items_of(N);
  std::vector<char> rebuilt(N, 0);
  for (int c = L; c < N; ++c) {
    if (!small(c)) continue;
    const int pc = parent[c];
    if (pc >= 0 && small(pc) && carrier(pc) == c) continue;  // not a chain top
    std::vector<int> chain;  // top down
    for (int x = c; x >= 0 && small(x); x = carrier(x)) chain.push_back(x);
    if (chain.size() < 3) continue;
    std::vector<int> items;
    const int bottom = chain.back();
    items.push_back(left[bottom]);
    items.push_back(right[bottom]);
    for (int i = (int)chain.size() - 2; i >= 0; --i) {
      const int x = chain[i], cx = chain[i + 1];
      items.push_back(left[x] == cx ? right[x] : left[x]);
    }
    items_of[c] = items;
    rebuilt[c] = 1;
  }
  std::vector<Pair> np;
  std::function<int(int)> emit;
  std::function<int(const std::vector<int> &, int, int)> balanced = [&](const std::vector<int> &it, int lo, int hi) {
    if (hi - lo == 1) return emit(it[lo]);
    const int mid = (lo + hi + 1) / 2;
    const int a = balanced(it, lo, mid), b = balanced(it, mid, hi);
    np.push_back({a, b});
    return L + (int)np.size() - 1;
  };
  emit = [&](int c) -> int {
    if (c < L) return c;
    if (rebuilt[c]) return balanced(items_of[c], 0, (int)items_of[c].size());
    const int a = emit(left[c]), b = emit(right[c]);
    np.push_back({a, b});
    return L + (int)np.size() - 1;
  };
  emit(N - 1);
  const TreeStats s0 = tree_stats(leaves, pairs, out, card), s1 = tree_stats(leaves, np, out, card);
  if (s1.sc > s0.sc + 1e-9 || s1.flops > 1.1 * s0.flops) return pairs;
  return np;
}

Labels choose_slices(const std::vector<Labels> &leaves, const std::vector<Pair> &pairs,
                     const Labels &out, const std::vector<int> &card, double cap) {
  Labels sliced;
  std::vector<char> isout(card.size(), 0), isl(card.size(), 0);
  for (int v : out) isout[v] = 1;
  for (;;) {
    std::vector<Labels> lv(leaves.size());
    for (size_t i = 0; i < leaves.size(); ++i)
      for (int v : leaves[i])
        if (!isl[v]) lv[i].push_back(v);
    auto lab = node_labels(lv, pairs, out, (int)card.size());
    std::vector<double> score(card.size(), 0);
    bool over = false;
    for (size_t c = leaves.size(); c < lab.size(); ++c) {
      double s = log2size(lab[c], card);
      if (s > cap + 1e-9) {
        over = true;
        for (int v : lab[c])
          if (!isout[v]) score[v] += s;
      }
    }
    if (!over) break;
    int best = -1;
    for (int v = 0; v < (int)card.size(); ++v)
      if (score[v] > 0 && (best < 0 || score[v] > score[best])) best = v;
    if (best < 0) throw TnError(TN_E_TOO_LARGE, "cannot slice the output labels below the cap");
    isl[best] = 1;
    sliced.push_back(best);
  }
  std::sort(sliced.begin(), sliced.end());
  return sliced;
}

}  // namespace tn
