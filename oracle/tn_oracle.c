/*
 * Plain FP64 CPU reference for tensor-network contraction along a binary
 * contraction tree.  TEST INFRASTRUCTURE ONLY: it is called by the tests, by
 * the smoke check and by the CPU-baseline leg of the benchmark, never by the
 * product library, and it shares no code with it.
 *
 * What it computes (paper, "Tensor networks" section, definition of a
 * tensor network and eq. contraction-definition): a tensor is a table over
 * the joint domain of its labels; a pairwise contraction of A (labels Va) and
 * B (labels Vb) to output labels Vc is the sum, over every assignment of the
 * labels in Va u Vb that are not in Vc, of the product of the two slices.
 * A binary contraction tree (paper, discussion of contraction orders) fixes
 * the order: leaves are the input tensors, each internal node contracts its
 * two children and keeps exactly the labels still needed by tensors outside
 * its subtree or by the requested output V0.
 *
 * Everything here is written as direct loops over all assignments of a
 * node's label union, with no blocking or reordering:
 *   or_sum_forward   sum-product contraction (eq. pr / eq. evidence) with
 *                    per-tensor power-of-two rescaling of each node output,
 *                    and, on request, the reverse pass of eq. einback
 *                    (the adjoint of every leaf: theorem thm:diff).
 *   or_max_forward   max-plus contraction (eq. tropical, eq. log-map) in FP64
 *                    or in FP32 emulation, followed by the top-down argmax
 *                    readout of the maximising assignment.
 *   or_sample        top-down sampling along the tree (eq. sample,
 *                    eq. condition-prob) with Philox4x32-10 uniforms.
 *   or_philox4x32_10 the counter-based generator of Salmon, Moraes, Dror and
 *                    Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 *                    SC'11, written from its published definition.
 *
 * Conventions shared with the callers (interface only):
 *   - labels of every tensor are sorted ascending and distinct; the table is
 *     row-major over them, last label fastest;
 *   - the tree is given as pairs (l, r) in post-order: ids < n_leaves are
 *     leaves, id n_leaves + i is the result of pair i; the last pair is the
 *     root;
 *   - at a node, labels eliminated that occur in only one child are reduced
 *     in that child first (the private-label rule), then the shared
 *     eliminated labels K are reduced; for max-plus, ties keep the smallest
 *     row-major index over the eliminated labels (sorted ascending, last
 *     fastest).  The paper asks that ties keep exactly one configuration but
 *     does not fix which; this is the reading used on both sides.
 * Return value of every entry point: 0 on success, a negative code on
 * invalid input (message in or_last_error()).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static char g_err[512];
const char *or_last_error(void) { return g_err; }
static int fail(const char *msg) {
  snprintf(g_err, sizeof g_err, "%s", msg);
  return -1;
}

/* ------------------------------------------------------------------------ */
/* Tensors                                                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
  int nl;
  int *lab;      /* sorted ascending */
  int64_t size;
  double *v;
  int64_t ex;    /* true value = v * 2^ex (sum-product only) */
} Ten;

static int64_t size_of(int nl, const int *lab, const int *card) {
  int64_t s = 1;
  for (int i = 0; i < nl; ++i) s *= card[lab[i]];
  return s;
}

static void ten_init(Ten *t, int nl, const int *lab, const int *card) {
  t->nl = nl;
  t->lab = (int *)malloc(sizeof(int) * (nl > 0 ? nl : 1));
  for (int i = 0; i < nl; ++i) t->lab[i] = lab[i];
  t->size = size_of(nl, lab, card);
  t->v = (double *)calloc((size_t)t->size, sizeof(double));
  t->ex = 0;
}

static void ten_free(Ten *t) {
  free(t->lab);
  free(t->v);
  t->lab = NULL;
  t->v = NULL;
}

static int has_label(const Ten *t, int v) {
  for (int i = 0; i < t->nl; ++i)
    if (t->lab[i] == v) return 1;
  return 0;
}

/* stride of label v inside t, 0 if absent */
static int64_t stride_of(const Ten *t, int v, const int *card) {
  int64_t s = 1;
  for (int i = t->nl - 1; i >= 0; --i) {
    if (t->lab[i] == v) return s;
    s *= card[t->lab[i]];
  }
  return 0;
}

/* sorted union of two sorted label lists */
static int label_union(const Ten *a, const Ten *b, int *out) {
  int i = 0, j = 0, n = 0;
  while (i < a->nl || j < b->nl) {
    if (j >= b->nl || (i < a->nl && a->lab[i] < b->lab[j])) out[n++] = a->lab[i++];
    else if (i >= a->nl || b->lab[j] < a->lab[i]) out[n++] = b->lab[j++];
    else { out[n++] = a->lab[i]; ++i; ++j; }
  }
  return n;
}

/* Divide by the power of two of the largest magnitude; record it in ex. */
static void rescale(Ten *t) {
  double mx = 0.0;
  for (int64_t i = 0; i < t->size; ++i)
    if (fabs(t->v[i]) > mx) mx = fabs(t->v[i]);
  if (mx == 0.0 || !isfinite(mx)) return;
  int e;
  frexp(mx, &e);
  for (int64_t i = 0; i < t->size; ++i) t->v[i] = ldexp(t->v[i], -e);
  t->ex += e;
}

/* Odometer over all assignments of the labels U (sorted), tracking the
 * row-major offsets into up to three tensors.  Visits assignments in
 * row-major order over U, last label fastest. */
typedef struct {
  int n;
  int digit[64];
  int cardu[64];
  int64_t s[3][64];
  int64_t off[3];
} Odo;

static int odo_init(Odo *o, int nu, const int *U, const int *card, const Ten *t0,
                    const Ten *t1, const Ten *t2) {
  if (nu > 64) return fail("too many labels in one contraction");
  o->n = nu;
  const Ten *ts[3] = {t0, t1, t2};
  for (int j = 0; j < nu; ++j) {
    o->digit[j] = 0;
    o->cardu[j] = card[U[j]];
    for (int k = 0; k < 3; ++k) o->s[k][j] = ts[k] ? stride_of(ts[k], U[j], card) : 0;
  }
  o->off[0] = o->off[1] = o->off[2] = 0;
  return 0;
}

/* advance; returns 0 when the odometer wrapped past the last assignment */
static int odo_next(Odo *o) {
  for (int j = o->n - 1; j >= 0; --j) {
    if (++o->digit[j] < o->cardu[j]) {
      for (int k = 0; k < 3; ++k) o->off[k] += o->s[k][j];
      return 1;
    }
    o->digit[j] = 0;
    for (int k = 0; k < 3; ++k) o->off[k] -= o->s[k][j] * (o->cardu[j] - 1);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Tree analysis                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
  int n_leaves, n_pairs, n_nodes;
  int *left, *right;     /* per node (leaves: -1) */
  int **lab;             /* output labels per node, sorted */
  int *nl;
} Tree;

static void tree_free(Tree *t) {
  if (t->lab)
    for (int i = 0; i < t->n_nodes; ++i) free(t->lab[i]);
  free(t->lab);
  free(t->nl);
  free(t->left);
  free(t->right);
}

/* Output labels of every node: labels of the children's union that still
 * occur in a leaf outside the subtree, or that belong to V0.  Each node
 * carries, for each of its output labels, how many leaves of its subtree
 * hold that label (a label missing from a child's output cannot occur in
 * that child's subtree unless it was eliminated there, and then it occurs
 * nowhere else). */
static int tree_build(Tree *t, int n_vars, int n_leaves, const int64_t *leaf_ptr,
                      const int *leaf_lab, int n_pairs, const int *pairs, int n_out,
                      const int *out_lab) {
  memset(t, 0, sizeof *t);
  if (n_leaves < 1) return fail("no leaves");
  if (n_pairs != n_leaves - 1) return fail("a binary tree over L leaves has L-1 pairs");
  t->n_leaves = n_leaves;
  t->n_pairs = n_pairs;
  t->n_nodes = n_leaves + n_pairs;
  t->left = (int *)malloc(sizeof(int) * t->n_nodes);
  t->right = (int *)malloc(sizeof(int) * t->n_nodes);
  t->lab = (int **)calloc(t->n_nodes, sizeof(int *));
  t->nl = (int *)calloc(t->n_nodes, sizeof(int));
  int **cnt = (int **)calloc(t->n_nodes, sizeof(int *));
  char *used = (char *)calloc(t->n_nodes, 1);
  int *total = (int *)calloc(n_vars, sizeof(int));
  char *isout = (char *)calloc(n_vars, 1);
  int rc = 0;
  for (int i = 0; i < n_out; ++i) {
    if (out_lab[i] < 0 || out_lab[i] >= n_vars) { rc = fail("output label out of range"); goto done; }
    isout[out_lab[i]] = 1;
  }
  for (int l = 0; l < n_leaves; ++l) {
    t->left[l] = t->right[l] = -1;
    int nl = (int)(leaf_ptr[l + 1] - leaf_ptr[l]);
    t->nl[l] = nl;
    t->lab[l] = (int *)malloc(sizeof(int) * (nl ? nl : 1));
    cnt[l] = (int *)malloc(sizeof(int) * (nl ? nl : 1));
    for (int j = 0; j < nl; ++j) {
      int v = leaf_lab[leaf_ptr[l] + j];
      if (v < 0 || v >= n_vars) { rc = fail("leaf label out of range"); goto done; }
      if (j && v <= leaf_lab[leaf_ptr[l] + j - 1]) { rc = fail("leaf labels must be sorted and distinct"); goto done; }
      t->lab[l][j] = v;
      cnt[l][j] = 1;
      total[v]++;
    }
  }
  for (int p = 0; p < n_pairs; ++p) {
    int c = n_leaves + p, a = pairs[2 * p], b = pairs[2 * p + 1];
    if (a < 0 || b < 0 || a >= c || b >= c || a == b) { rc = fail("pair ids must refer to earlier nodes"); goto done; }
    if (used[a] || used[b]) { rc = fail("a node is used twice in the tree"); goto done; }
    used[a] = used[b] = 1;
    t->left[c] = a;
    t->right[c] = b;
    int na = t->nl[a], nb = t->nl[b];
    int *buf = (int *)malloc(sizeof(int) * (na + nb + 1));
    int *cb = (int *)malloc(sizeof(int) * (na + nb + 1));
    int i = 0, j = 0, n = 0;
    while (i < na || j < nb) {
      int v, k;
      if (j >= nb || (i < na && t->lab[a][i] < t->lab[b][j])) { v = t->lab[a][i]; k = cnt[a][i]; ++i; }
      else if (i >= na || t->lab[b][j] < t->lab[a][i]) { v = t->lab[b][j]; k = cnt[b][j]; ++j; }
      else { v = t->lab[a][i]; k = cnt[a][i] + cnt[b][j]; ++i; ++j; }
      if (isout[v] || total[v] - k > 0) { buf[n] = v; cb[n] = k; ++n; }
    }
    t->lab[c] = buf;
    cnt[c] = cb;
    t->nl[c] = n;
  }
  for (int i = 0; i + 1 < t->n_nodes; ++i)
    if (!used[i]) { rc = fail("tree does not cover every node"); goto done; }
  for (int i = 0; i < n_out; ++i)
    if (!total[out_lab[i]]) { rc = fail("output label occurs in no leaf"); goto done; }
done:
  for (int i = 0; i < t->n_nodes; ++i) free(cnt[i]);
  free(cnt);
  free(used);
  free(total);
  free(isout);
  if (rc) tree_free(t);
  return rc;
}

static int root_id(const Tree *t) { return t->n_nodes - 1; }

/* ------------------------------------------------------------------------ */
/* Sum-product                                                               */
/* ------------------------------------------------------------------------ */

/* out[x_o] = sum over the assignments of the labels of P and Q not in out
 * (row-major, last fastest) of P[x_p] * Q[x_q]; out's labels are a subset
 * of P's and Q's.  Each output element is one independent sum taken in that
 * order, so the elements may be computed in parallel (OpenMP) with the same
 * result as one sequential pass over the whole label union. */
static int sum_into(const Ten *P, const Ten *Q, Ten *out, const int *card) {
  int U[128], E[128];
  if (P->nl + Q->nl > 128) return fail("label union too large");
  const int nu = label_union(P, Q, U);
  int ne = 0;
  for (int j = 0; j < nu; ++j)
    if (!has_label(out, U[j])) E[ne++] = U[j];
  if (ne > 64 || out->nl > 64) return fail("too many labels in one contraction");
  int64_t sPo[64], sQo[64], sPe[64], sQe[64];
  int co[64], ce[64];
  for (int j = 0; j < out->nl; ++j) {
    co[j] = card[out->lab[j]];
    sPo[j] = stride_of(P, out->lab[j], card);
    sQo[j] = stride_of(Q, out->lab[j], card);
  }
  int64_t n_e = 1;
  for (int j = 0; j < ne; ++j) {
    ce[j] = card[E[j]];
    sPe[j] = stride_of(P, E[j], card);
    sQe[j] = stride_of(Q, E[j], card);
    n_e *= ce[j];
  }
  const int64_t n_o = out->size;
#pragma omp parallel
  {
    /* a contiguous range of output elements per thread: decode its first
     * element, then step through the rest in row-major order */
    int nt = 1, it = 0;
#ifdef _OPENMP
    nt = omp_get_num_threads();
    it = omp_get_thread_num();
#endif
    const int64_t lo = n_o * it / nt, hi = n_o * (it + 1) / nt;
    int dout[64], d[64];
    int64_t k = lo, p0 = 0, q0 = 0;
    for (int j = out->nl - 1; j >= 0; --j) {
      dout[j] = (int)(k % co[j]);
      k /= co[j];
      p0 += dout[j] * sPo[j];
      q0 += dout[j] * sQo[j];
    }
    for (int64_t oc = lo; oc < hi; ++oc) {
      for (int j = 0; j < ne; ++j) d[j] = 0;
      int64_t p = p0, q = q0;
      double acc = 0.0;
      for (int64_t e = 0; e < n_e; ++e) {
        acc += P->v[p] * Q->v[q];
        for (int j = ne - 1; j >= 0; --j) { /* next assignment of E */
          if (++d[j] < ce[j]) { p += sPe[j]; q += sQe[j]; break; }
          d[j] = 0;
          p -= sPe[j] * (ce[j] - 1);
          q -= sQe[j] * (ce[j] - 1);
        }
      }
      out->v[oc] = acc;
      for (int j = out->nl - 1; j >= 0; --j) { /* next output element */
        if (++dout[j] < co[j]) { p0 += sPo[j]; q0 += sQo[j]; break; }
        dout[j] = 0;
        p0 -= sPo[j] * (co[j] - 1);
        q0 -= sQo[j] * (co[j] - 1);
      }
    }
  }
  return 0;
}

/* C[x_c] = sum over the labels of A and B not in C of A[x_a] * B[x_b]
 * (B may be NULL for a single operand). */
static int contract_sum(const Ten *A, const Ten *B, Ten *C, const int *card) {
  static double one_v = 1.0;
  static const Ten one = {0, NULL, 1, &one_v, 0};
  if (sum_into(A, B ? B : &one, C, card)) return -1;
  C->ex = A->ex + (B ? B->ex : 0);
  rescale(C);
  return 0;
}

/* Reverse rule (eq. einback): Abar = con(Cbar, B -> labels of A),
 * Bbar = con(Cbar, A -> labels of B). */
static int adjoint_sum(const Ten *A, const Ten *B, const Ten *Cbar, Ten *Abar, Ten *Bbar,
                       const int *card) {
  if (Abar && sum_into(Cbar, B, Abar, card)) return -1;
  if (Bbar && sum_into(Cbar, A, Bbar, card)) return -1;
  if (Abar) { Abar->ex = Cbar->ex + B->ex; rescale(Abar); }
  if (Bbar) { Bbar->ex = Cbar->ex + A->ex; rescale(Bbar); }
  return 0;
}

/* Threads of the parallel loops (OpenMP); n <= 0 leaves the default. */
void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
int or_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/*
 * Sum-product contraction of the tree.
 *   leaf_vals: concatenated leaf tables (row-major over sorted labels).
 *   root_vals: out, the root table over out_lab (sorted), scaled;
 *   root_exp:  out, its power-of-two exponent (true = vals * 2^exp).
 *   want_adj:  if nonzero (requires n_out == 0), leaf_adj / leaf_adj_exp
 *              receive d(root)/d(leaf) for every leaf, scaled the same way
 *              (leaf_adj has the layout of leaf_vals, leaf_adj_exp one entry
 *              per leaf).
 */
int or_sum_forward(int n_vars, const int *card, int n_leaves, const int64_t *leaf_ptr,
                   const int *leaf_lab, const double *leaf_vals, int n_pairs, const int *pairs,
                   int n_out, const int *out_lab, int want_adj, double *root_vals,
                   int64_t *root_exp, double *leaf_adj, int64_t *leaf_adj_exp) {
  for (int v = 0; v < n_vars; ++v)
    if (card[v] < 1) return fail("domain sizes must be >= 1");
  if (want_adj && n_out) return fail("adjoints are defined for a scalar root");
  Tree t;
  if (tree_build(&t, n_vars, n_leaves, leaf_ptr, leaf_lab, n_pairs, pairs, n_out, out_lab)) return -1;
  Ten *T = (Ten *)calloc(t.n_nodes, sizeof(Ten));
  int64_t voff = 0;
  int rc = 0;
  for (int l = 0; l < n_leaves; ++l) {
    ten_init(&T[l], t.nl[l], t.lab[l], card);
    memcpy(T[l].v, leaf_vals + voff, sizeof(double) * T[l].size);
    voff += T[l].size;
  }
  for (int p = 0; p < n_pairs; ++p) {
    int c = n_leaves + p;
    ten_init(&T[c], t.nl[c], t.lab[c], card);
    if ((rc = contract_sum(&T[t.left[c]], &T[t.right[c]], &T[c], card))) goto done;
  }
  /* the root's output must be exactly V0 (a single leaf still needs its
   * labels outside V0 summed) */
  int r = root_id(&t);
  Ten R;
  ten_init(&R, n_out, out_lab, card);
  if ((rc = contract_sum(&T[r], NULL, &R, card))) { ten_free(&R); goto done; }
  memcpy(root_vals, R.v, sizeof(double) * R.size);
  *root_exp = R.ex;
  if (want_adj) {
    Ten *G = (Ten *)calloc(t.n_nodes, sizeof(Ten));
    for (int i = 0; i < t.n_nodes; ++i) ten_init(&G[i], t.nl[i], t.lab[i], card);
    /* d root / d T_root: the root-level reduction is a sum, so ones */
    for (int64_t i = 0; i < G[r].size; ++i) G[r].v[i] = 1.0;
    G[r].ex = 0;
    for (int p = n_pairs - 1; p >= 0 && !rc; --p) {
      int c = n_leaves + p, a = t.left[c], b = t.right[c];
      rc = adjoint_sum(&T[a], &T[b], &G[c], &G[a], &G[b], card);
    }
    int64_t o = 0;
    for (int l = 0; l < n_leaves && !rc; ++l) {
      memcpy(leaf_adj + o, G[l].v, sizeof(double) * G[l].size);
      leaf_adj_exp[l] = G[l].ex;
      o += G[l].size;
    }
    for (int i = 0; i < t.n_nodes; ++i) ten_free(&G[i]);
    free(G);
  }
  ten_free(&R);
done:
  for (int i = 0; i < t.n_nodes; ++i) ten_free(&T[i]);
  free(T);
  tree_free(&t);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Max-plus                                                                  */
/* ------------------------------------------------------------------------ */
static double rnd(double x, int fp32) { return fp32 ? (double)(float)x : x; }
static double padd(double a, double b, int fp32) {
  if (fp32) {
    volatile float fa = (float)a, fb = (float)b;
    volatile float s = fa + fb;
    return (double)s;
  }
  return a + b;
}

/* sorted difference a \ b */
static int label_minus(const int *a, int na, const int *b, int nb, int *out) {
  int n = 0;
  for (int i = 0; i < na; ++i) {
    int f = 0;
    for (int j = 0; j < nb; ++j)
      if (a[i] == b[j]) f = 1;
    if (!f) out[n++] = a[i];
  }
  return n;
}

/* Row-major index of the assignment restricted to labels L (sorted). */
static int64_t flat_index(int nl, const int *L, const int *x, const int *card) {
  int64_t k = 0;
  for (int i = 0; i < nl; ++i) k = k * card[L[i]] + x[L[i]];
  return k;
}
static void decode_index(int64_t k, int nl, const int *L, int *x, const int *card) {
  for (int i = nl - 1; i >= 0; --i) {
    x[L[i]] = (int)(k % card[L[i]]);
    k /= card[L[i]];
  }
}

/* Reduce A over its labels not in keep (sorted list): out has labels keep,
 * arg stores the row-major index over the reduced labels of the first
 * maximiser.  A's table is visited row-major over its sorted labels, so for
 * a fixed kept assignment the reduced assignments arrive in increasing
 * row-major order and a strict comparison keeps the smallest maximiser. */
static int reduce_max(const Ten *A, const int *keep, int nkeep, Ten *out, int64_t **arg,
                      const int *card) {
  ten_init(out, nkeep, keep, card);
  *arg = (int64_t *)calloc((size_t)out->size, sizeof(int64_t));
  char *seen = (char *)calloc((size_t)out->size, 1);
  int P[128];
  int np = label_minus(A->lab, A->nl, keep, nkeep, P);
  int64_t pw[64];
  for (int j = 0; j < A->nl; ++j) {
    pw[j] = 0;
    int64_t w = 1;
    for (int i = np - 1; i >= 0; --i) {
      if (P[i] == A->lab[j]) pw[j] = w;
      w *= card[P[i]];
    }
  }
  Odo o;
  if (odo_init(&o, A->nl, A->lab, card, A, out, NULL)) { free(seen); return -1; }
  do {
    int64_t p = 0;
    for (int j = 0; j < A->nl; ++j) p += (int64_t)o.digit[j] * pw[j];
    double val = A->v[o.off[0]];
    int64_t oo = o.off[1];
    if (!seen[oo] || val > out->v[oo]) {
      out->v[oo] = val;
      (*arg)[oo] = p;
      seen[oo] = 1;
    }
  } while (odo_next(&o));
  free(seen);
  return 0;
}

static int in_list(int v, const int *lab, int n) {
  for (int i = 0; i < n; ++i)
    if (lab[i] == v) return 1;
  return 0;
}

/*
 * Max-plus contraction with V0 = {} and readout of the maximising
 * assignment.  leaf_vals are log-values (-inf allowed).  fp32 != 0 emulates
 * FP32: leaves are rounded to float and every candidate is one IEEE float
 * addition.  assign[v] receives the value of every label that occurs in some
 * leaf (others are left untouched).
 */
int or_max_forward(int n_vars, const int *card, int n_leaves, const int64_t *leaf_ptr,
                   const int *leaf_lab, const double *leaf_vals, int n_pairs, const int *pairs,
                   int fp32, double *root_val, int *assign) {
  if (n_vars > 4096) return fail("too many variables for the max-plus reference");
  Tree t;
  if (tree_build(&t, n_vars, n_leaves, leaf_ptr, leaf_lab, n_pairs, pairs, 0, NULL)) return -1;
  Ten *T = (Ten *)calloc(t.n_nodes, sizeof(Ten));
  Ten *Ap = (Ten *)calloc(t.n_nodes, sizeof(Ten)); /* pre-reduced left child per node */
  Ten *Bp = (Ten *)calloc(t.n_nodes, sizeof(Ten));
  int64_t **argA = (int64_t **)calloc(t.n_nodes, sizeof(int64_t *));
  int64_t **argB = (int64_t **)calloc(t.n_nodes, sizeof(int64_t *));
  int64_t **argK = (int64_t **)calloc(t.n_nodes, sizeof(int64_t *));
  int *x = (int *)malloc(sizeof(int) * n_vars);
  int rc = 0;
  int64_t voff = 0;
  for (int l = 0; l < n_leaves; ++l) {
    ten_init(&T[l], t.nl[l], t.lab[l], card);
    for (int64_t i = 0; i < T[l].size; ++i) T[l].v[i] = rnd(leaf_vals[voff + i], fp32);
    voff += T[l].size;
  }
  for (int p = 0; p < n_pairs && !rc; ++p) {
    int c = n_leaves + p, a = t.left[c], b = t.right[c];
    const Ten *A = &T[a], *B = &T[b];
    /* kept labels of each child: the ones shared with the sibling or kept
     * by the node */
    int ka[128], kb[128], nka = 0, nkb = 0;
    for (int j = 0; j < A->nl; ++j)
      if (has_label(B, A->lab[j]) || in_list(A->lab[j], t.lab[c], t.nl[c])) ka[nka++] = A->lab[j];
    for (int j = 0; j < B->nl; ++j)
      if (has_label(A, B->lab[j]) || in_list(B->lab[j], t.lab[c], t.nl[c])) kb[nkb++] = B->lab[j];
    if ((rc = reduce_max(A, ka, nka, &Ap[c], &argA[c], card))) break;
    if ((rc = reduce_max(B, kb, nkb, &Bp[c], &argB[c], card))) break;
    /* shared eliminated labels K, then C = max_K (A' + B') */
    Ten *C = &T[c];
    ten_init(C, t.nl[c], t.lab[c], card);
    argK[c] = (int64_t *)calloc((size_t)C->size, sizeof(int64_t));
    char *seen = (char *)calloc((size_t)C->size, 1);
    int U[128];
    int nu = label_union(&Ap[c], &Bp[c], U);
    int K[128];
    int nk = label_minus(U, nu, C->lab, C->nl, K);
    Odo o;
    if ((rc = odo_init(&o, nu, U, card, &Ap[c], &Bp[c], C))) { free(seen); break; }
    int *xv = (int *)calloc(n_vars, sizeof(int));
    do {
      for (int j = 0; j < nu; ++j) xv[U[j]] = o.digit[j];
      double cand = padd(Ap[c].v[o.off[0]], Bp[c].v[o.off[1]], fp32);
      if (!seen[o.off[2]] || cand > C->v[o.off[2]]) {
        /* the union is visited row-major, so for a fixed output element the
         * K assignments come in increasing row-major order: the first
         * maximiser is the smallest index */
        C->v[o.off[2]] = cand;
        argK[c][o.off[2]] = flat_index(nk, K, xv, card);
        seen[o.off[2]] = 1;
      }
    } while (odo_next(&o));
    free(xv);
    free(seen);
  }
  if (!rc) {
    int r = root_id(&t);
    /* root-level reduction of any labels left (single-leaf trees) */
    Ten Rr;
    int64_t *argR = NULL;
    if ((rc = reduce_max(&T[r], NULL, 0, &Rr, &argR, card)) == 0) {
      *root_val = Rr.v[0];
      for (int v = 0; v < n_vars; ++v) x[v] = -1;
      decode_index(argR[0], T[r].nl, T[r].lab, x, card);
      for (int p = n_pairs - 1; p >= 0; --p) {
        int c = n_leaves + p;
        const Ten *C = &T[c];
        int64_t off = 0;
        for (int j = 0; j < C->nl; ++j) off += (int64_t)x[C->lab[j]] * stride_of(C, C->lab[j], card);
        int U[128], K[128];
        int nu = label_union(&Ap[c], &Bp[c], U);
        int nk = label_minus(U, nu, C->lab, C->nl, K);
        decode_index(argK[c][off], nk, K, x, card);
        for (int side = 0; side < 2; ++side) {
          const Ten *ch = &T[side ? t.right[c] : t.left[c]];
          const Ten *cp = side ? &Bp[c] : &Ap[c];
          int64_t *arg = side ? argB[c] : argA[c];
          int P[128];
          int np = label_minus(ch->lab, ch->nl, cp->lab, cp->nl, P);
          if (!np) continue;
          int64_t o2 = 0;
          for (int j = 0; j < cp->nl; ++j) o2 += (int64_t)x[cp->lab[j]] * stride_of(cp, cp->lab[j], card);
          decode_index(arg[o2], np, P, x, card);
        }
      }
      for (int v = 0; v < n_vars; ++v)
        if (x[v] >= 0) assign[v] = x[v];
      ten_free(&Rr);
      free(argR);
    }
  }
  for (int i = 0; i < t.n_nodes; ++i) {
    ten_free(&T[i]);
    if (Ap[i].v) ten_free(&Ap[i]);
    if (Bp[i].v) ten_free(&Bp[i]);
    free(argA[i]);
    free(argB[i]);
    free(argK[i]);
  }
  free(T); free(Ap); free(Bp); free(argA); free(argB); free(argK); free(x);
  tree_free(&t);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11)                                      */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform double in [0,1) from the first two output words (53 bits) */
static double philox_uniform(uint64_t sample, uint32_t node, uint32_t slot, uint64_t seed) {
  uint32_t ctr[4] = {(uint32_t)sample, (uint32_t)(sample >> 32), node, slot};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t o[4];
  or_philox4x32_10(ctr, key, o);
  uint64_t a = o[0] >> 5, b = o[1] >> 6;
  return ((double)a * 67108864.0 + (double)b) / 9007199254740992.0;
}

/* ------------------------------------------------------------------------ */
/* Sampling along the tree                                                   */
/* ------------------------------------------------------------------------ */

/* Draw the assignment of labels P (sorted) with weight w(p) given by a
 * callback-free table: weights[p] already filled.  Inverse CDF in row-major
 * order of P. */
static int64_t draw(const double *w, int64_t n, double u) {
  double tot = 0.0;
  for (int64_t i = 0; i < n; ++i) tot += w[i];
  double target = u * tot, cum = 0.0;
  int64_t last = -1;
  for (int64_t i = 0; i < n; ++i) {
    if (w[i] > 0) last = i;
    cum += w[i];
    if (cum > target && w[i] > 0) return i;
  }
  return last < 0 ? 0 : last;
}

/* sum-reduce A over labels not in keep */
static int reduce_sum(const Ten *A, const int *keep, int nkeep, Ten *out, const int *card) {
  ten_init(out, nkeep, keep, card);
  Odo o;
  if (odo_init(&o, A->nl, A->lab, card, A, out, NULL)) return -1;
  do {
    out->v[o.off[1]] += A->v[o.off[0]];
  } while (odo_next(&o));
  return 0;
}

/*
 * n samples from the distribution proportional to the contraction of the
 * leaves (all labels summed), drawn top-down along the tree: at each node,
 * given the labels already drawn (the node's output labels), first the
 * shared eliminated labels K from w(k) = A'(.,k) B'(.,k) with Philox counter
 * (sample, node, 0), then the left child's private labels from A with
 * counter (sample, node, 1), then the right child's with (sample, node, 2).
 * A' and B' are the children with their private labels summed out.  For a
 * single-leaf tree, its labels are drawn from the leaf with counter
 * (sample, n_leaves, 1).  samples is [n][n_vars]; labels that occur in no
 * leaf are left untouched.
 */
int or_sample(int n_vars, const int *card, int n_leaves, const int64_t *leaf_ptr,
              const int *leaf_lab, const double *leaf_vals, int n_pairs, const int *pairs,
              uint64_t seed, int64_t n, const int64_t *ids, int *samples) {
  Tree t;
  if (tree_build(&t, n_vars, n_leaves, leaf_ptr, leaf_lab, n_pairs, pairs, 0, NULL)) return -1;
  Ten *T = (Ten *)calloc(t.n_nodes, sizeof(Ten));
  Ten *Ap = (Ten *)calloc(t.n_nodes, sizeof(Ten));
  Ten *Bp = (Ten *)calloc(t.n_nodes, sizeof(Ten));
  int rc = 0;
  int64_t voff = 0;
  for (int l = 0; l < n_leaves; ++l) {
    ten_init(&T[l], t.nl[l], t.lab[l], card);
    memcpy(T[l].v, leaf_vals + voff, sizeof(double) * T[l].size);
    voff += T[l].size;
  }
  for (int p = 0; p < n_pairs && !rc; ++p) {
    int c = n_leaves + p, a = t.left[c], b = t.right[c];
    int ka[128], kb[128], nka = 0, nkb = 0;
    for (int j = 0; j < T[a].nl; ++j)
      if (has_label(&T[b], T[a].lab[j]) || in_list(T[a].lab[j], t.lab[c], t.nl[c])) ka[nka++] = T[a].lab[j];
    for (int j = 0; j < T[b].nl; ++j)
      if (has_label(&T[a], T[b].lab[j]) || in_list(T[b].lab[j], t.lab[c], t.nl[c])) kb[nkb++] = T[b].lab[j];
    if ((rc = reduce_sum(&T[a], ka, nka, &Ap[c], card))) break;
    if ((rc = reduce_sum(&T[b], kb, nkb, &Bp[c], card))) break;
    rescale(&Ap[c]);
    rescale(&Bp[c]);
    ten_init(&T[c], t.nl[c], t.lab[c], card);
    if ((rc = contract_sum(&Ap[c], &Bp[c], &T[c], card))) break;
  }
  int *x = (int *)malloc(sizeof(int) * n_vars);
  int64_t wcap = 1;
  for (int i = 0; i < t.n_nodes; ++i)
    if (T[i].size > wcap) wcap = T[i].size;
  double *w = (double *)malloc(sizeof(double) * wcap);
  for (int64_t j = 0; j < n && !rc; ++j) {
    /* sample j draws with counter ids[j] (its index among all samples when
       the caller samples a subset, e.g. one slice's samples) */
    const int64_t s = ids ? ids[j] : j;
    for (int v = 0; v < n_vars; ++v) x[v] = -1;
    int r = root_id(&t);
    if (T[r].nl) {
      /* labels left at the root (single-leaf tree): draw them from it */
      for (int64_t i = 0; i < T[r].size; ++i) w[i] = T[r].v[i];
      int64_t k = draw(w, T[r].size, philox_uniform((uint64_t)s, (uint32_t)n_leaves, 1, seed));
      decode_index(k, T[r].nl, T[r].lab, x, card);
    }
    for (int p = n_pairs - 1; p >= 0; --p) {
      int c = n_leaves + p;
      const Ten *A = &Ap[c], *B = &Bp[c], *C = &T[c];
      int U[128], K[128];
      int nu = label_union(A, B, U);
      int nk = label_minus(U, nu, C->lab, C->nl, K);
      if (nk) {
        int64_t nK = size_of(nk, K, card);
        for (int64_t k = 0; k < nK; ++k) {
          decode_index(k, nk, K, x, card);
          int64_t oa = 0, ob = 0;
          for (int j = 0; j < A->nl; ++j) oa += (int64_t)x[A->lab[j]] * stride_of(A, A->lab[j], card);
          for (int j = 0; j < B->nl; ++j) ob += (int64_t)x[B->lab[j]] * stride_of(B, B->lab[j], card);
          w[k] = A->v[oa] * B->v[ob];
        }
        int64_t k = draw(w, nK, philox_uniform((uint64_t)s, (uint32_t)c, 0, seed));
        decode_index(k, nk, K, x, card);
      }
      for (int side = 0; side < 2; ++side) {
        const Ten *ch = &T[side ? t.right[c] : t.left[c]];
        const Ten *cp = side ? B : A;
        int P[128];
        int np = label_minus(ch->lab, ch->nl, cp->lab, cp->nl, P);
        if (!np) continue;
        int64_t nP = size_of(np, P, card);
        for (int64_t q = 0; q < nP; ++q) {
          decode_index(q, np, P, x, card);
          int64_t o2 = 0;
          for (int j = 0; j < ch->nl; ++j) o2 += (int64_t)x[ch->lab[j]] * stride_of(ch, ch->lab[j], card);
          w[q] = ch->v[o2];
        }
        int64_t q = draw(w, nP, philox_uniform((uint64_t)s, (uint32_t)c, (uint32_t)(1 + side), seed));
        decode_index(q, np, P, x, card);
      }
    }
    for (int v = 0; v < n_vars; ++v) samples[j * n_vars + v] = x[v];
  }
  free(w);
  free(x);
  for (int i = 0; i < t.n_nodes; ++i) {
    ten_free(&T[i]);
    if (Ap[i].v) ten_free(&Ap[i]);
    if (Bp[i].v) ten_free(&Bp[i]);
  }
  free(T); free(Ap); free(Bp);
  tree_free(&t);
  return rc;
}
