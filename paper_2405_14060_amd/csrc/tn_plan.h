// Plan structures of libtn (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "tn_internal.h"

namespace tn {

// A tensor resident in the float arena.  Values are row-major over the
// sorted labels (last label fastest); batched tensors hold one copy per
// instance, instance outermost (element e of instance b at b * size + e) or,
// in interleaved plans, innermost (at e * max_batch + b).  Sum-product
// tensors carry a scaling slot: value = raw * 2^ex[slot (+ instance)].
struct TensorBuf {
  Labels lab;
  int64_t size = 1;      // elements per instance
  bool batched = false;
  int64_t off = -1;      // float offset in the arena
  int slot = -1;         // first scaling slot, -1 for max-plus tensors
};

struct IntBuf {
  int64_t size = 1;
  bool batched = false;
  int64_t off = -1;      // int32 offset in the index arena
};

// One launch of the generic contraction kernel.
struct Op {
  int semi = SEMI_SUM;
  int X = -1, Y = -1, Z = -1, I = -1;  // tensor ids; I = argmax IntBuf id
  bool split = false;
  int nb = 1;                         // grid rows: instances (interleaved form: groups of 64)
  int inst = 1;                       // instances computed
  ContractArgs a;                     // pointers filled after allocation
  // table offsets into the host table store (-1 = unused)
  int64_t t_rX[2], t_rY[2], t_rZ[2], t_cY[2], t_cZ[2], t_sX[2], t_sY[2];
  int64_t t_gbX[2], t_gbY[2], t_gbZ[2], t_gmX[2], t_gmZ[2];  // dense form
  int64_t t_oX[2], t_oY[2];           // generic form in output order
  double flops = 0, bytes = 0;        // algorithmic, per instance
  int64_t part_off = -1;              // partial-sum region of a split contraction
  ContractArgs *d_a = nullptr;        // device copy of `a`
  // fused chain segment (seg >= 0): 1 carrier forward, 2 carrier reverse,
  // 3 composed map, 4 small operands' adjoints; extra tensors read /
  // written, for scheduling
  int seg = -1, seg_kind = 0;
  std::vector<int> ins, outs;
  int Y2 = -1, Y3 = -1;               // max-plus chain in one pass: the second's and third's Y
  int forms = 0;                      // eligible kernel forms: 1 generic, 2 row, 4 dense, 8 wave,
                                      // 16 interleaved, 256 dense with 128 x 128 tiles, 512 generic
                                      // in output order, 1024 batch-uniform row form
};

// Host description of a fused segment (tables as offsets into the plan's
// int32 table store).
struct SegPlan {
  std::vector<int> ops;               // forward op indices, in order
  int c0 = -1, cL = -1;               // input / output carrier tensors
  int64_t oX[2], oZ[2], inX = 0, outZ = 0;
  uint32_t nO = 1, nOl = 1;
  int32_t n_in0 = 0, n_outL = 0;
  int64_t list_off = 0;               // the steps' CSR lists in the table store
  int32_t in_lo_shift = 5, out_lo_shift = 5;
  std::vector<SegStep> steps;
  int mt = -1;                        // tensor holding the composed map M
  int spt = -1;                       // reverse: tensor holding the partials of S (-1 = none)
  int32_t n_part = 0;                 // reverse: workgroups of the carrier kernel
  int32_t list_len = 0;               // int32 entries of the lists
  int32_t mat_lds = 0, fin_lds = 0;   // floats of LDS of the sweep kernels
  std::vector<int> ybar_tensor;       // reverse: adjoint tensor of each small operand (-1)
  int g = -1, c0bar = -1;             // reverse: adjoint tensors of C_L and C_0
  double bytes_fwd = 0, bytes_bwd = 0, flops = 0;
  Labels loc_in, loc_out, outer;      // local labels of C_0 and C_L; outer labels
  int pair = -1;                      // index of the two-segment pass holding it (-1: none)
};

// Two consecutive segments run as one carrier pass (DSegArgs).
struct DSegPlan {
  int s1 = -1, s2 = -1;               // segments: s1's output carrier is s2's input
  uint32_t nO = 1, nOl = 1;           // common outer labels O
  int64_t oX[2], oZ[2];               // their offset tables in C_0 and C_2
  int32_t nob = 1, nQ = 1, nR = 1, q_fast = 0, r_fast = 0;
  int32_t aug1 = 1, aug2 = 1;         // assignments of the common outer label moved into
                                      // the first (second) map's rows and columns (1: none)
  int32_t in_lo_shift = 5, out_lo_shift = 5;
  int64_t tab = 0;                    // kDSegTab x 32 tables in the table store
  int32_t n_part = 0;                 // workgroups
  double bytes_fwd = 0, bytes_bwd = 0, flops = 0;
};

// One launch of a schedule: a single contraction, or several independent
// contractions of one stage run by the grouped kernel.
struct Launch {
  int semi = SEMI_SUM;
  bool split = false;
  bool gemm = false;                  // dense-form contractions (matrix cores)
  bool inter = false;                 // interleaved-form contractions
  bool mpair = false;                 // pairs of max-plus contractions (kKindMaxPair)
  bool seg = false;                   // fused-segment kernels (carrier kinds alone)
  int seg_kind = 0;
  std::vector<int> ops;               // indices into the op list
  int32_t *d_ids = nullptr;           // segment kinds 3 / 4: device list of segment indices
  int lds = 0;                        // segment kinds 3 / 4: LDS floats
  // grouped launches: device copies of the ops' arguments and block ranges
  ContractArgs *d_args = nullptr;
  tn::GroupBlock *d_blk = nullptr;    // map, or split partials
  uint32_t *d_nblk = nullptr;
  tn::GroupBlock *d_blk2 = nullptr;   // split finish
  uint32_t *d_nblk2 = nullptr;
  uint32_t total = 0, total2 = 0;
};

// Stages of independent contractions.  Forward passes are scheduled as soon
// as possible, the reverse pass as late as possible, so that contractions
// hanging off the critical path collect into few grouped launches.
struct Schedule {
  std::vector<Launch> launches;
  int n_stages = 0;
};

// A contraction tree bound to tensors.
struct TreeExec {
  std::vector<int> leaf_tensor;       // tensor id of every leaf
  std::vector<Pair> pairs;
  Labels out;
  std::vector<Labels> lab;            // node labels (leaves, then pairs)
  std::vector<int> node_tensor;       // tensor id of every node
  int root = -1;                      // tensor holding the result over `out`
  std::vector<Op> ops;
  std::vector<Op> fops;               // forward list with fused segments or max-plus pairs (when fused)
  std::vector<int> chain_prev;        // max-plus chains run in one pass: per op, the chain's
                                      // previous contraction (-1: none)
  std::vector<char> chain_inner;      // 1: a later contraction of its chain follows (the chain's
                                      // last one holds the index of every step)
  bool fused = false;
  std::vector<std::vector<int>> node_ops;  // op indices per pair (reductions, then main)
  int root_op = -1;                   // op reducing the root to `out`, if any
  // max-plus only: readout steps
  std::vector<BackStep> back;
  std::vector<int32_t> back_meta;
  std::vector<int32_t> back_lev;      // readout levels: steps [back_lev[l], back_lev[l + 1]),
                                      // then the chunks (kBackChunkInts each)
  int32_t n_back_lev = 0, n_back_chunks = 0;
};

}  // namespace tn

struct tn_plan_impl {
  tn_plan_opts opts{};
  const tn_net *net_src = nullptr;     // not owned; copied fields below
  int n_vars = 0;
  std::vector<int> card;
  int mode = 0;
  int max_batch = 1;
  bool batched_ev = false;             // instances run as one batch (INDICATOR, or SLICED with max_batch > 1)
  bool inter = false;                  // batched tensors interleaved (instance fastest)
  std::vector<tn::Op> samp_ops;        // sampling: children summed over their private labels
  tn::Schedule sched_samp;
  bool want_sum = false, want_max = false, want_grad = false, is_mmap = false;
  std::vector<int> observed;           // mode SLICED
  std::vector<char> is_obs;

  // leaves of the main tree
  std::vector<tn::Labels> leaf_lab;
  std::vector<int> leaf_kind;          // 0 factor, 1 unity, 2 indicator
  std::vector<int> leaf_var, leaf_factor;
  std::vector<tn::Pair> pairs;
  tn::TreeStats stats;
  int planner_used = 0;
  bool two_front = false;
  std::vector<int> sliced;

  // tensors
  std::vector<tn::TensorBuf> T;
  std::vector<tn::IntBuf> IB;
  int n_slots = 0;
  int reset_begin = 0, reset_end = 0;
  std::vector<int32_t> tabs;           // host copy of offset tables
  std::vector<int32_t> gmap;           // leaf gather maps
  std::vector<int32_t> obs;            // (var, stride) pairs
  std::vector<tn::LeafDesc> leaves_sum, leaves_max;

  // executable pieces
  tn::TreeExec sum_tree, max_tree;
  std::vector<tn::Op> bwd;
  tn::Schedule sched_fwd, sched_bwd, sched_max, sched_q;
  // fused variants of the sum-product passes (log Z / marginals)
  bool fused = false;
  std::vector<tn::SegPlan> segs;
  std::vector<tn::Op> ffwd, fbwd;
  tn::Schedule sched_ffwd, sched_fbwd;
  tn::SegArgs *d_seg_fwd = nullptr, *d_seg_bwd = nullptr;
  std::vector<tn::SegArgs> seg_fwd_h, seg_bwd_h;
  std::vector<tn::DSegPlan> dsegs;    // two-segment carrier passes
  std::vector<tn::DSegArgs> dseg_fwd_h, dseg_bwd_h;
  std::vector<tn::Schedule> sched_groups;
  int seed_tensor = -1;                // adjoint of the root (ones)
  std::vector<int> adj_tensor;         // per node of sum_tree, -1 = none
  std::vector<tn::MargDesc> marg;
  std::vector<tn::GradDesc> grads;
  std::vector<tn::SampleStep> samp;
  std::vector<int32_t> samp_meta;
  std::vector<int> marg_col;           // column offset of each variable
  int marg_row = 0;
  // joint marginals: variable sets (sorted), their unity tensors' tables
  std::vector<std::vector<int>> joint_sets;
  std::vector<tn::JointDesc> joint;
  std::vector<int32_t> joint_tab;      // (var, card, stride in the unity tensor or -1) per set variable
  int joint_row = 0;

  // MMAP
  std::vector<tn::TreeExec> groups;    // sum phase, one tree per group
  std::vector<std::vector<tn::LeafDesc>> group_leaves;
  std::vector<int> group_log;          // tensor id of the log-domain copy of each group root
  tn::TreeExec qtree;                  // max phase over the query variables
  std::vector<tn::LeafDesc> qleaves;
  std::vector<int> query;              // sorted
  double mmap_const = 0.0;             // log of summed variables in no factor
  std::vector<int> group_sliced_vars;  // per group: sliced variables (flattened)
  std::vector<int> group_sliced_ptr;

  // device
  hipStream_t stream = nullptr;
  bool own_stream = false;
  float *arena = nullptr;
  int32_t *iarena = nullptr;
  uint32_t *mx = nullptr;
  int32_t *ex = nullptr;
  int32_t *d_tabs = nullptr, *d_gmap = nullptr, *d_obs = nullptr;
  int32_t *d_evidence = nullptr;       // [max_batch][n_vars]
  int32_t *d_slice_rows = nullptr;     // sliced plans: evidence rows of a chunk of slices
  double *d_slice_lz = nullptr;        // and their log Z_s
  int32_t *d_assign = nullptr;         // [max_batch][n_vars]
  double *d_out = nullptr;             // logz [max_batch]
  double *d_marg = nullptr;            // [max_batch][marg_row]
  double *d_joint = nullptr;           // [max_batch][joint_row]
  tn::JointDesc *d_joint_desc = nullptr;
  int32_t *d_joint_tab = nullptr;
  double *d_fmarg = nullptr;           // [max_batch][n_values] (plans with factor adjoints)
  tn::LeafDesc *d_leaves_sum = nullptr, *d_leaves_max = nullptr, *d_qleaves = nullptr;
  std::vector<tn::LeafDesc *> d_group_leaves;
  tn::MargDesc *d_marg_desc = nullptr;
  tn::GradDesc *d_grad_desc = nullptr;
  tn::BackStep *d_back = nullptr, *d_qback = nullptr;
  int32_t *d_back_meta = nullptr, *d_qback_meta = nullptr;
  int32_t *d_back_lev = nullptr, *d_qback_lev = nullptr;
  tn::SampleStep *d_samp = nullptr;
  int32_t *d_samp_meta = nullptr;
  int32_t *d_samp_out = nullptr;
  int64_t samp_cap = 0;
  float *d_part = nullptr;
  int32_t *d_parti = nullptr;
  double *d_acc = nullptr;             // MMAP slice accumulator
  int64_t arena_floats = 0, iarena_ints = 0, part_floats = 0;
  int64_t device_bytes = 0;
  std::vector<void *> allocs;

  int device = 0;                      // GPU the plan's memory lives on
  bool eager = false;                  // launch directly even with use_graph (allocation-free calls)
  std::map<std::string, hipGraphExec_t> graphs;
  ~tn_plan_impl();
};
