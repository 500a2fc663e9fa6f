// Internal declarations shared by the host planner, the runtime and the
// kernel launchers of libtn.
#pragma once

#include <array>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/tn.h"

struct TnError : std::runtime_error {
  tn_status st;
  TnError(tn_status s, const std::string &m) : std::runtime_error(m), st(s) {}
};

struct tn_net {
  int n_vars = 0;
  std::vector<int> card;
  std::vector<std::vector<int>> scope;   // scope order as loaded
  std::vector<std::vector<double>> vals; // linear or log, as loaded
  std::vector<int64_t> val_off;          // offset of each factor in the flat store
  int64_t n_values = 0;
  bool is_log = false;
};

namespace tn {

// The thread-local message returned by tn_last_error().
void set_last_error(const std::string &m);

using Labels = std::vector<int>;  // variable ids, sorted ascending
using Pair = std::array<int, 2>;

// ---------------------------------------------------------------------------
// Trees and planning (tn_planner.cpp)
// ---------------------------------------------------------------------------

// Output labels of every node of a binary tree (leaves first, then pairs in
// post-order): a node keeps the labels of its children that still occur in a
// leaf outside its subtree or in the requested output set.
std::vector<Labels> node_labels(const std::vector<Labels> &leaves, const std::vector<Pair> &pairs,
                                const Labels &out, int n_vars);

struct TreeStats {
  double sc = 0, sc_union = 0, tc = 0;  // log2
  double flops = 0;                     // 2 * sum of union sizes
  double bytes = 0;                     // 4 * sum over nodes (|A| + |B| + |C|)
};
TreeStats tree_stats(const std::vector<Labels> &leaves, const std::vector<Pair> &pairs,
                     const Labels &out, const std::vector<int> &card);

void validate_tree(int n_leaves, const std::vector<Pair> &pairs);

struct PlanChoice {
  std::vector<Pair> pairs;
  TreeStats stats;
  int planner = 0;
  bool two_front = false;  // the two-front variant of the planner's order won
};

// Time model of a tree under the stage schedule (contractions grouped by
// level, a level costs its slowest node): sum over levels of
// max(launch cost + multiply-adds / rate).  n_levels (optional) = levels.
static constexpr double kStageLaunchSeconds = 4e-6;
static constexpr double kStageMacRate = 2e13;
// Roofline estimate of one pass over a tree (seconds): per node a launch
// plus the slower of its flops at its kernel form's rate and its operand and
// output bytes at that form's HBM rate (rates measured on this GPU: the
// matrix-core form on scattered tiles, and the one-lane-per-output forms).
static constexpr double kNodeLaunchSeconds = 5e-6;
static constexpr double kDenseFlopRate = 2.5e13, kDenseByteRate = 3e12;
static constexpr double kVectorFlopRate = 8e12, kVectorByteRate = 1.8e12;
double roofline_time(const std::vector<Labels> &leaves, const std::vector<Pair> &pairs, const Labels &out,
                     const std::vector<int> &card);
double stage_time(const std::vector<Labels> &leaves, const std::vector<Pair> &pairs, const Labels &out,
                  const std::vector<int> &card, int *n_levels);

// Choose a contraction tree over the leaves; labels in `out` are never
// eliminated.  `strategy` is a TN_PLANNER_* value.  Without a slicing cap,
// candidates (every order and its two-front variant) are ranked by (largest
// intermediate to half a power of two, stage_time); with a cap (cap > 0)
// by (largest intermediate, work), and a candidate that
// exceeds it is ranked by its total work once sliced below the cap (the
// work of one slice plus a launch cost per node, times the number of
// slices), so that a tree with larger intermediates but much less sliced
// work wins.
PlanChoice plan_tree(const std::vector<Labels> &leaves, const std::vector<int> &card,
                     const Labels &out, int strategy, int restarts, uint64_t seed, double cap = 0);

// Rebalance chains of nodes with at most 2^max_log2 outputs into balanced
// trees over the same inputs (fewer sequential levels), when the largest
// intermediate does not grow and the work grows by at most 10 %.
std::vector<Pair> rebalance_small_chains(const std::vector<Labels> &leaves, const std::vector<Pair> &pairs,
                                         const Labels &out, const std::vector<int> &card, double max_log2);

// Pick labels to slice (fix per slice) so that every node output and every
// node label union is at most 2^cap elements.
Labels choose_slices(const std::vector<Labels> &leaves, const std::vector<Pair> &pairs,
                     const Labels &out, const std::vector<int> &card, double cap);

// ---------------------------------------------------------------------------
// Kernel launch descriptors (tn_kernels.hip)
// ---------------------------------------------------------------------------

// Offset tables of one index class (rows, columns or summed labels) for one
// tensor: offset(i) = hi[i / nlo] + lo[i % nlo].
struct Tab2 {
  const int32_t *hi = nullptr, *lo = nullptr;
};

static constexpr int kRowMax = 32;      // summed entries and columns held by a row-form lane
static constexpr int kRowFormMax = 16;  // of which the row form with per-lane operand reads takes 16
static constexpr int kRowBlock = 128;   // batch-uniform row form: Y entries per batch (summed x columns)
static constexpr int kMaxSubSlots = 64;  // sub-slots per recorded maximum

struct ContractArgs {
  const float *X = nullptr, *Y = nullptr;
  float *Z = nullptr;
  int32_t *I = nullptr;  // argmax output (max-plus)
  int64_t bsX = 0, bsY = 0, bsZ = 0;
  Tab2 rX, rY, rZ;  // rows: labels of Z that X holds
  Tab2 cY, cZ;      // columns: labels of Z that X lacks
  Tab2 sX, sY;      // summed: labels of X or Y not in Z
  uint32_t nR = 1, nRl = 1, nC = 1, nCl = 1, nS = 1, nSl = 1;
  int col_fastest = 0;
  // power-of-two scaling slots (sum-product)
  uint32_t *mx = nullptr;
  int32_t *ex = nullptr;
  int32_t mx_stride = 0;  // sub-slot stride of mx (number of slots)
  int32_t slotX = -1, slotY = -1, slotZ = -1;
  int32_t batX = 0, batY = 0, batZ = 0;  // 1 if the slot is per instance
  // split reduction scratch
  float *part = nullptr;
  int32_t *parti = nullptr;
  uint32_t n_chunks = 1;
  // row form (kind 1): one lane per row, all summed entries and columns in
  // registers; offsets of the summed entries in X, Y and of the columns in
  // Y, Z, in canonical order.  tile 1 (sum-product): the rows split into
  // batch and M labels as in the dense form (gb*, gm* tables); a wavefront
  // takes 64 M assignments of one batch assignment and reads that batch's
  // summed x columns block of Y once
  int32_t kind = 0;  // 0 generic, 1 row form, 2 dense matrix-core form, 3 wave per output,
                     // 4 interleaved instances (lane = instance)
  int32_t ns = 0, nc = 0;
  int32_t rl_shift = -1;  // log2(nRl) when nRl is a power of two
  int32_t row_vx = 0;     // tile 1: summed entries 4k..4k+3 adjacent in X, 16-byte aligned
                          // (2: entries 2k, 2k+1 adjacent, 8-byte aligned)
  int32_t row_vz = 0;     // tile 1: columns 4k..4k+3 adjacent in Z, 16-byte aligned
  int32_t sx[kRowMax], sy[kRowMax], cy[kRowMax], cz[kRowMax];
  // dense form (kind 2, sum-product): the rows split into batch labels
  // (held by Y too) and M labels (not held by Y); for every batch
  // assignment Z[M, N] = sum_S X[M, S] Y[S, N] with N the columns, as
  // 64 x 64 output tiles on the matrix cores
  Tab2 gbX, gbY, gbZ;       // batch labels in X, Y, Z
  Tab2 gmX, gmZ;            // M labels in X, Z
  uint32_t nB = 1, nBl = 1, nM = 1, nMl = 1;
  uint32_t nBlo = 1;        // batch assignments of the batch labels faster in Z than every
                            // M and column label: tiles of those batches are dealt together
                            // (they share cache lines of every operand)
  int32_t x_s_fast = 0;     // X's stride-1 label is summed (else an M or batch label)
  int32_t y_n_fast = 0;     // Y's stride-1 label is a column label
  int32_t z_n_fast = 0;     // Z's stride-1 label is a column label
  int32_t s_pair = 0;       // X's and Y's stride-1 label is a summed label of two values (and
                            // the summed set even): the summed entries come in adjacent pairs
  int32_t prec = 0;         // matrix-core operands: 0 FP32, 1 BF16, 2 FP16 (FP32 accumulation)
  // interleaved form (kind 4): element e of instance b of a batched tensor
  // sits at e * es + b (es = instances held); a shared operand has es = 1
  // and bs = 0.  Rows are split into batch labels and M labels as in the
  // dense form (gb*, gm* tables; no Y: M = rows).
  int32_t esX = 1, esY = 1, esZ = 1;
  int32_t ksplit = 1;       // 4: the waves of a workgroup split the summed range of one tile
  int32_t tile = 0;         // tile of a wave: 0 = 4 x 4, 1 = 8 x 8, 2 = 16 x 1 (rows x columns)
  int32_t nslab = 1;        // groups of 64 instances
  // generic form in output order (kind 0, tile 1): outputs enumerated in
  // Z's memory order (lane o writes Z[o]); offsets of X and Y for every
  // output through tables over Z's labels (stride 0 for labels they lack)
  Tab2 oX, oY;
  uint32_t nOl = 1;         // entries of the low tables
  // two consecutive max-plus contractions in one pass (kind kKindMaxPair):
  // Z1 = X (x) Y, then Z = Z1 (x) Y2, Z1 kept in registers; I gets, per
  // output of Z, the index s1 * ns2 + s2 of both steps' first maximisers.  A
  // lane takes one assignment r of R2 = Z's labels held by Z1; rX, rY, rZ:
  // its offsets in X, Y, Z; gbY: in Y2.  Per summed assignment s2 of the
  // second step (ns2 <= 4) and s1 of the first (ns <= 4), k = 4 s2 + s1:
  // sx[k], sy[k] offsets in X and Y; per column c (nc <= 4) cy[4 c + s2]
  // in Y2 and cz[kPairZ + c] in Z.
  // steps = 3 (three contractions, each summing <= 2 assignments, <= 2
  // columns): Z1 = X (x) Y, Z2 = Z1 (x) Y2, Z = Z2 (x) Y3; a lane takes r of
  // R3 = Z's labels held by Z2; rX, rY, gbY, gmX, rZ: its offsets in X, Y,
  // Y2, Y3, Z; k = 4 s3 + 2 s2 + s1: sx[k], sy[k]; cy[2 s3 + s2] in Y2;
  // cz[2 c + s3] in Y3, cz[kPairZ + c] in Z; I gets (s1 ns2 + s2) ns3 + s3.
  const float *Y2 = nullptr, *Y3 = nullptr;
  int32_t ns2 = 0, ns3 = 0, steps = 2;
};
static constexpr int kKindMaxPair = 7;
static constexpr int kPairMax = 4;    // summed assignments of either step, columns of the second
static constexpr int kTripleMax = 2;  // the same for each step of a three-step chain
static constexpr int64_t kChainMinOut = 1 << 12;  // outputs of a chain's last step
static constexpr int kPairZ = 16;     // cz[kPairZ + c]: Z offsets of the second step's columns
static constexpr int kGemmTile = 64;  // output tile edge of the dense form
static constexpr int kInterTile = 4;  // output tile edge (rows x columns) of the interleaved form
static constexpr int kInterLanes = 64;  // instances per wavefront of the interleaved form

enum Semiring { SEMI_SUM = 0, SEMI_MAX = 1 };

// a: host copy (grid shape); d_a: the same arguments in device memory
void launch_contract(int semi, bool has_y, bool split, const ContractArgs &a, const ContractArgs *d_a, int nb,
                     void *stream);
// blocks per instance (interleaved form: per 64 instances) of a launch
uint32_t map_blocks(const ContractArgs &a);
// phase 0: map, 1: split partials, 2: split finish, 3 + p: dense form with
// operand precision p, 6: interleaved form
// blk: per workgroup of the launch, its contraction and its workgroup index
// within that contraction (one read instead of a search over the ops)
struct GroupBlock {
  uint32_t op, local;
};
void launch_group(int semi, int phase, const ContractArgs *ops, const GroupBlock *blk,
                  const uint32_t *nblk, int n, uint32_t total_blocks, void *stream);

// Fused chain segment: consecutive tree nodes that each contract the
// previous node's output (the carrier) with a small tensor.  The labels the
// chain touches (local labels) are few; on them the chain is a product of
// small linear maps, one per step, and the labels it never touches (outer
// labels) are carried along.  The composed map M (local entries of the
// output carrier x local entries of the input carrier, at most 32 x 32) is
// built once per solve from the small operands (k_seg_mat), and the carrier
// is transformed by one batched matrix product per segment on the matrix
// cores: C_L[:, o] = M C_0[:, o] for every outer assignment o.  The reverse
// pass applies M^T to the output adjoint and accumulates
// S = sum_o Gbar[:, o] C_0[:, o]^T, from which every small operand's adjoint
// follows by sweeps over the steps (k_seg_fin, eq. einback per step).
// A step's triples (in, out, s) say: out-entry += in-entry * small[s].
struct SegStep {
  int64_t y = -1;         // float offset of the small operand
  int32_t yslot = -1;     // its scaling slot
  int32_t ny = 0;         // its elements
  int32_t n_in = 0, n_out = 0;   // local entries before / after the step
  int32_t nnz = 0;        // index triples of the step
  // the step's triples in three orders (int32 offsets into the lists):
  // by output entry (CSR: ptr[n_out + 1], in[], s[]), by input entry
  // (ptr[n_in + 1], out[], s[]) and by small-operand entry (ptr[ny + 1],
  // in[], out[])
  int32_t fo_ptr = 0, fo_in = 0, fo_s = 0;
  int32_t bi_ptr = 0, bi_out = 0, bi_s = 0;
  int32_t bs_ptr = 0, bs_in = 0, bs_out = 0;
  int64_t ybar = -1;      // reverse pass: adjoint of the small operand (-1 = not needed)
  int32_t ybar_slot = -1;
};

static constexpr int64_t kSliceChunk = 256;  // slices whose evidence rows are uploaded at once
static constexpr int kSegMaxLocal = 32;   // local entries of a carrier in a segment
static constexpr int kSegOuterBlock = 128; // outer assignments per workgroup (4 waves x 32)
static constexpr int kSegMaxSteps = 16;    // steps of a segment

struct SegArgs {
  float *arena = nullptr;
  uint32_t *mx = nullptr;
  int32_t *ex = nullptr;
  int32_t mx_stride = 0;
  int64_t X = 0, Z = 0, G = 0;   // forward: X = input carrier, Z = output carrier;
                                 // reverse: G = adjoint of the output carrier,
                                 //          X = input carrier, Z = its adjoint
  int32_t slotX = -1, slotZ = -1, slotG = -1;
  int64_t M = 0;                 // composed map, n_outL x n_in0 row-major (raw, max in [0.5, 1))
  int32_t slotM = -1;            // its exponent slot
  int64_t Sp = 0;                // reverse: per-workgroup partials of S (n_part x n_outL x n_in0)
  int32_t slotSp = -1;           // exponent of S
  int32_t n_part = 0;            // reverse: workgroups of the carrier kernel
  uint32_t nO = 1, nOl = 1;      // outer assignments; split of the outer tables
  int32_t ol_shift = -1;         // log2(nOl) when nOl is a power of two
  Tab2 oX, oZ;                   // outer offsets in the input / output carrier
  const int32_t *inX = nullptr;  // local offsets of the input carrier
  const int32_t *outZ = nullptr; // local offsets of the output carrier
  int32_t n_in0 = 0, n_outL = 0;
  const SegStep *steps = nullptr;
  int32_t n_steps = 0;
  const int32_t *lists = nullptr;  // the steps' CSR lists (offsets in SegStep are relative)
  int32_t list_len = 0;            // int32 entries of the lists
  int32_t in_lo_shift = 5;       // log2 of the input carrier's local entries below its fastest
                                 // outer label (tile load order: those, then outer, then the rest)
  int32_t out_lo_shift = 5;      // same for the output carrier
  int32_t mat_lds = 0, fin_lds = 0;  // floats of LDS of the sweep kernels
  int32_t prec = 0;              // matrix-core operands: 0 FP32, 1 BF16, 2 FP16 (FP32 accumulation)
};
// carrier kernels: the arguments are passed by value
void launch_seg_fwd(const SegArgs &a, void *stream);
void launch_seg_bwd(const SegArgs &a, void *stream);
// two independent segments (same precision) in one launch
struct SegPair {
  SegArgs a[2];
  uint32_t split = 0;  // workgroups of the first segment
};
void launch_seg_fwd2(const SegArgs &a, const SegArgs &b, void *stream);
void launch_seg_bwd2(const SegArgs &a, const SegArgs &b, void *stream);
// one workgroup per listed segment; lds_floats = the largest mat_lds / fin_lds of them
void launch_seg_mat(const SegArgs *d_base, const int32_t *d_ids, int n, int lds_floats, void *stream);
void launch_seg_fin(const SegArgs *d_base, const int32_t *d_ids, int n, int lds_floats, void *stream);
unsigned seg_blocks(const SegArgs &a);  // workgroups of a carrier launch

// Two consecutive segments of a chain in one carrier pass.  Segment 1 maps
// C_0 to C_1 on local labels A -> B (map M1), segment 2 maps C_1 to C_2 on
// C -> D (map M2).  C splits into P (labels of B) and Q (outer labels of
// segment 1), R = B \ C passes through segment 2 and O, the other outer
// labels, is common to C_0, C_1 and C_2.  The forward pass forms C_2 from
// C_0 without writing C_1; the reverse pass recomputes C_1 and its adjoint
// in LDS.
struct DSegArgs {
  float *arena = nullptr;
  uint32_t *mx = nullptr;
  int32_t *ex = nullptr;
  int32_t mx_stride = 0;
  int64_t X = 0, Z = 0, G = 0;     // forward: X = C_0, Z = C_2; reverse: G = adjoint of C_2,
                                   // X = C_0, Z = adjoint of C_0
  int32_t slotX = -1, slotZ = -1, slotG = -1;
  int64_t M1 = 0, M2 = 0;          // composed maps (B x A and D x C, row-major)
  int32_t slotM1 = -1, slotM2 = -1;
  int64_t Sp1 = 0, Sp2 = 0;        // reverse: per-workgroup partials of each segment's S
  int32_t slotSp1 = -1, slotSp2 = -1;  // (-1: that segment needs none)
  uint32_t nO = 1, nOl = 1;        // assignments of O; split of its tables
  int32_t ol_shift = -1;           // log2(nOl) when nOl is a power of two
  Tab2 oX, oZ;                     // offsets of O's assignments in C_0 / C_2
  int32_t nob = 1;                 // assignments of O per workgroup (power of two)
  int32_t nA = 0, nB = 0, nC = 0, nD = 0, nQ = 1, nR = 1;  // local entries of the tiles
  int32_t aug1 = 1, aug2 = 1;      // the first map is M1 (x) I_aug1 over (o*, A) -> (o*, B),
                                   // the second M2 (x) I_aug2 over (o*, C) -> (o*, D), for a
                                   // common outer label o* of aug assignments placed slowest
                                   // in the rows (nA, nB and nR, or nC, nD and nQ count it)
  int32_t q_fast = 0, r_fast = 0;  // tile column order: 1 = the Q (R) assignment fastest
  int32_t in_lo_shift = 5, out_lo_shift = 5;  // as in SegArgs, for C_0 and C_2
  const int32_t *tab = nullptr;    // kDSegTab x 32 int32: offsets of A in C_0, of D in C_2,
                                   // of Q in C_0, of R in C_2; per c in C its P part of the
                                   // index in B and its Q index; per r its part of the index in B
  int32_t prec = 0;
};
static constexpr int kDSegTab = 7;
struct DSegPair {
  DSegArgs a[2];
  uint32_t split = 0;  // workgroups of the first
};
unsigned dseg_blocks(const DSegArgs &a);
// one or two (b != nullptr) independent pairs of segments per launch
void launch_dseg_fwd(const DSegArgs &a, const DSegArgs *b, void *stream);
void launch_dseg_bwd(const DSegArgs &a, const DSegArgs *b, void *stream);

struct LeafDesc {
  int32_t kind;      // 0 factor gather, 1 constant one-vector, 2 indicator
  int32_t var;       // indicator variable
  int32_t size;      // elements per instance
  int32_t batched;   // 1: one copy per instance
  int64_t dst;       // float offset of the leaf tensor in the arena
  int64_t src;       // float offset of the factor table in the arena
  int32_t gmap;      // int32 offset of the gather map (size entries)
  int32_t obs_begin, obs_end;  // (var, stride) pairs in the observation list
  int32_t slot;      // mx slot (ex slot is the same index)
  int32_t maxdom;    // 1: log domain (zero = -inf, one = 0)
  int32_t nsub;      // workgroups preparing the leaf (> 1: a large leaf, each
                     // workgroup's maximum in its own sub-slot)
  int32_t ident;     // 1: the gather map is the identity (element i at src + base + i)
};

static constexpr int kPrepBig = 16;  // leaves per launch prepared by several workgroups

struct PrepareArgs {
  float *arena = nullptr;
  const LeafDesc *leaves = nullptr;
  int n_leaves = 0;
  const int32_t *gmap = nullptr;
  const int32_t *obs = nullptr;      // pairs (var, stride)
  const int32_t *evidence = nullptr; // [batch][n_vars]
  int n_vars = 0;
  uint32_t *mx = nullptr;
  int32_t *ex = nullptr;
  int32_t mx_stride = 0;
  int reset_begin = 0, reset_end = 0;  // slots zeroed each solve
  int batch = 1;
  int max_batch = 1;
  int interleaved = 0;  // batched leaves: element i of instance b at i * max_batch + b
  // large leaves (nsub > 1): their indices and first workgroup (after the
  // n_leaves one-per-leaf workgroups, which skip them)
  int n_big = 0;
  int32_t big_leaf[kPrepBig] = {};
  int32_t big_blk0[kPrepBig + 1] = {};
};
void launch_prepare(const PrepareArgs &a, void *stream);

void launch_logz(const float *root, int64_t bs, const int32_t *ex, int slot, int batched,
                 int batch, double *out, void *stream);

struct MargDesc {
  int64_t adj;    // float offset of the unity/indicator adjoint
  int64_t leaf;   // float offset of the unity/indicator leaf
  int32_t card;
  int32_t out;    // column offset in the marginal row
  int32_t adj_batched, leaf_batched;
  int64_t adj_bs, leaf_bs;  // instance strides
  int64_t adj_es, leaf_es;  // element strides
};
void launch_marg(const float *arena, const MargDesc *d, int n, int batch, int row, double *out,
                 void *stream);

struct GradDesc {
  int64_t adj;       // float offset of the factor-leaf adjoint
  int32_t size;      // leaf elements
  int32_t slot;      // adjoint slot (exponent)
  int64_t dst;       // offset of the factor in the gradient array
  int32_t gmap;      // gather map of the leaf (leaf element -> table entry)
  int32_t obs_begin, obs_end;
  int64_t leaf;      // float offset of the factor leaf (sliced table)
  int32_t full;      // entries of the factor's whole table
  int32_t adj_batched;
  int64_t adj_bs, adj_es;  // instance and element strides of the adjoint
  int32_t leaf_batched;    // the leaf holds one slice per instance (batched sliced evidence)
  int64_t leaf_bs, leaf_es;
};
void launch_factor_grad(const float *arena, const GradDesc *d, int n, const int32_t *gmap,
                        const int32_t *obs, const int32_t *evidence, const int32_t *ex,
                        const float *root, int root_slot, int64_t n_values, float *grad,
                        void *stream);

// Factor marginals T_f Tbar_f / sum over the leaf, scattered into the
// factor's whole table (zeros elsewhere): out[b * row + dst + entry], FP64.
void launch_factor_marg(const float *arena, const GradDesc *d, int n, const int32_t *gmap, const int32_t *obs,
                        const int32_t *evidence, int n_vars, int batch, int64_t row, double *out, void *stream);

// Joint marginal of a variable set from its unity tensor's adjoint.  The
// set's variables (sorted) are (var, card, stride of the variable in the
// unity tensor, -1 if observed and sliced out) triples at tab[3 * v_begin ..].
struct JointDesc {
  int64_t adj = -1;          // float offset of the unity tensor's adjoint (-1: every variable sliced out)
  int64_t adj_bs = 0, adj_es = 1;
  int32_t adj_batched = 0;
  int32_t out = 0;           // column of the set's table in the joint row
  int32_t n_full = 1;        // entries of the table over the whole set
  int32_t v_begin = 0, v_end = 0;
};
void launch_joint(const float *arena, const JointDesc *d, int n, const int32_t *tab, const int32_t *evidence,
                  int n_vars, int batch, int row, double *out, void *stream);

// Argmax readout: steps run level by level (the steps of a level in
// parallel); each reads x at its input labels, fetches an argmax index and
// decodes it into its output labels.
struct BackStep {
  int64_t arg;       // int32 offset of the argmax array in the index arena
  int64_t bs;        // per-instance stride of the argmax array (0 = shared)
  int64_t es;        // element stride of the argmax array
  int32_t in_begin, in_end;    // (var, stride) pairs
  int32_t out_begin, out_end;  // (var, card) pairs, last fastest
};
// Readout chunks: runs of whole levels whose steps (<= kBackChunkSteps) and
// (var, stride / card) pairs (<= kBackChunkPairs, contiguous: the pairs are
// laid out in step order) a workgroup stages in LDS with one round of loads;
// per chunk: first and end level, first and end step, first and end pair.
// A level larger than a chunk is a chunk of its own, read from global memory.
static constexpr int kBackChunkSteps = 128, kBackChunkPairs = 2048, kBackChunkInts = 6;
// lev: n_lev + 1 level boundaries, then n_chunks chunks
void launch_backtrack(const int32_t *iarena, const BackStep *steps, const int32_t *lev, int n_lev, int n_chunks,
                      const int32_t *pairs, int n_vars, int batch, int32_t *assign, void *stream);

// Top-down sampling steps (see tn_sample).
struct SampleStep {
  int64_t A, B;        // float offsets of the two children (B < 0: none)
  int64_t Ar, Br;      // the children summed over their private eliminated
                       // labels (the child itself when it has none): the
                       // weights of the shared eliminated labels
  int32_t node;        // tree node id (Philox counter word 2)
  int32_t aIn_b, aIn_e;    // (var, card, stride in A, stride in Ar) for A's labels already drawn
  int32_t bIn_b, bIn_e;    // (var, card, stride in B, stride in Br)
  int32_t k_b, k_e;        // (var, card, strideA, strideB): shared eliminated
  int32_t kr_b, kr_e;      // (var, card, strideAr, strideBr): the same labels in Ar, Br
  int32_t pa_b, pa_e;      // (var, card, strideA, 0): A-private eliminated
  int32_t pb_b, pb_e;      // (var, card, 0, strideB): B-private eliminated
};
// n samples; sample j uses index ids[j] (ids == nullptr: j) as its Philox
// counter and writes row ids[j] of out
void launch_sample(const float *arena, const SampleStep *steps, int n_steps, const int32_t *meta,
                   int n_vars, int64_t n, uint64_t seed, const int32_t *init, const int64_t *ids,
                   int32_t *out, void *stream);
// Philox4x32-10 uniform in [0, 1) with 53 bits, counter (sample, node, slot),
// key seed: the draws of the sampler, on the host (slice choice)
double sample_uniform(uint64_t sample, uint32_t node, uint32_t slot, uint64_t seed);
static constexpr uint32_t kSliceDrawNode = 0xffffffffu;  // node word of a sample's slice draw

// Staging of the allocation-free sampler: a file-scope device array of
// kScratchInts int32 per GPU (16 MiB).  scratch_ptr(dev) returns that GPU's
// address (looked up once per device, with the device current), or nullptr
// with a message in err.
static constexpr int64_t kScratchInts = int64_t(1) << 22;
int32_t *scratch_ptr(int dev, std::string &err);

void launch_tolog(const float *src, const int32_t *ex, int slot, int64_t n, float *dst,
                  void *stream);

// Accumulate a sliced partial result into an accumulator with exponent
// alignment: acc = acc + src (both raw tables with exponents).
void launch_slice_acc(const float *src, const uint32_t *mx, const int32_t *ex, int slot_src,
                      double *acc, int32_t *acc_ex, int64_t n, int first, void *stream);
void launch_acc_tolog(const double *acc, const int32_t *acc_ex, int64_t n, float *dst, void *stream);

}  // namespace tn
