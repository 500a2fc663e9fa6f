// HIP kernels of libtn for gfx950 (CDNA4, 64-wide wavefronts).
//
// One generic pairwise-contraction kernel family carries every tree node
// (paper: eq. contraction-definition applied to two tensors; eq. tropical
// for the max-plus algebra) and every adjoint contraction of the reverse
// pass (eq. einback).  A contraction is described by index classes of the
// output Z relative to the larger operand X and the smaller Y:
//   rows    labels of Z held by X          (offsets in X, Y, Z)
//   columns labels of Z not held by X      (offsets in Y, Z; broadcast when
//                                           Y lacks them too)
//   summed  labels of X or Y not in Z      (offsets in X, Y)
// Each class owns split offset tables, offset(i) = hi[i / nlo] + lo[i % nlo],
// so any interleaving of labels in the operands' layouts is a gather and no
// separate transpose pass is needed; the row order follows the canonical
// (sorted-label) layout so consecutive lanes touch consecutive addresses of
// the operand that owns the fastest label.
//   k_map    one lane per output element, summed labels looped in order;
//   k_split  outputs few, summed set large: each workgroup reduces one chunk
//            of the summed index for every output, k_split_finish combines
//            the chunks in a fixed order (deterministic, no atomics on data).
// Sum-product operands are rescaled on load by 2^-k with k the exponent of
// the operand's recorded maximum; each launch records the maximum of its
// output (atomicMax on the IEEE bits of non-negative floats) and its
// exponent, so the value of a tensor is raw * 2^ex (per instance).
// Max-plus keeps the first maximiser in canonical order of the summed
// labels, and every candidate is exactly one FP32 addition.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>

#include "tn_internal.h"

namespace tn {

static constexpr int kBlock = 256;

// Global-address-space views of device pointers: loads and stores through
// them compile to global (not flat) memory instructions, which address with
// a scalar base plus a 32-bit lane offset and wait only on the vector memory
// counter.
typedef __attribute__((address_space(1))) const int32_t gint;
typedef __attribute__((address_space(1))) const uint32_t gu32;
typedef __attribute__((address_space(1))) const float gcfloat;
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) int32_t gint_w;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const f32x4 gcf32x4;
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const f32x2 gcf32x2;
typedef __attribute__((address_space(1))) f32x4 gf32x4;
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (operands are finite)
__device__ __forceinline__ short bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
// One 16 x 16 x 16 matrix-core step with operands rounded to BF16 (PREC 1)
// or FP16 (PREC 2), FP32 accumulation: lane l supplies A[l % 16][4 (l / 16) + j]
// and B[4 (l / 16) + j][l % 16], j = 0..3.
template <int PREC>
__device__ __forceinline__ f32x4 mfma16_lp(const float (&a)[4], const float (&b)[4], f32x4 c) {
  if (PREC == 1) {
    const bf16x4 av = {bf16_rne(a[0]), bf16_rne(a[1]), bf16_rne(a[2]), bf16_rne(a[3])};
    const bf16x4 bv = {bf16_rne(b[0]), bf16_rne(b[1]), bf16_rne(b[2]), bf16_rne(b[3])};
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, c, 0, 0, 0);
  } else {
    const f16x4 av = {(_Float16)a[0], (_Float16)a[1], (_Float16)a[2], (_Float16)a[3]};
    const f16x4 bv = {(_Float16)b[0], (_Float16)b[1], (_Float16)b[2], (_Float16)b[3]};
    return __builtin_amdgcn_mfma_f32_16x16x16f16(av, bv, c, 0, 0, 0);
  }
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// exponent k of the recorded maximum m (m = f * 2^k, f in [0.5, 1)),
// clamped so that 2^-k is a normal float
// Dense-form tile q of tm x tn tiles per batch -> (batch, row tile, column
// tile): column tile fastest, then row tile, then batch, except that the
// nBlo batches whose labels are faster than the tiles' labels vary fastest
// of all (their tiles read the same cache lines).
__device__ __forceinline__ void dense_tile(uint32_t q, uint32_t tm, uint32_t tn, uint32_t nBlo, uint32_t &bt,
                                           uint32_t &mt, uint32_t &nt) {
  const uint32_t blo = q % nBlo;
  q /= nBlo;
  nt = q % tn;
  q /= tn;
  mt = q % tm;
  bt = (q / tm) * nBlo + blo;
}

__device__ __forceinline__ int max_exponent(uint32_t bits) {
  float m = __uint_as_float(bits);
  if (!(m > 0.f)) return 0;
  int k;
  frexpf(m, &k);
  return k < -126 ? -126 : (k > 126 ? 126 : k);
}

// Maxima live in kMaxSub sub-slots per tensor, sub-slot-major
// (mx[sub * stride + slot]) so that the sub-slots of one tensor sit on
// different cache lines: the workgroups of a launch spread their atomics
// over them instead of serialising on one address.  A reader takes the
// maximum over the sub-slots with one wave-wide load.
static constexpr int kMaxSub = kMaxSubSlots;

__device__ __forceinline__ uint32_t read_max(const uint32_t *mx, int stride, int slot) {
  const uint32_t v = ((gu32 *)mx)[(threadIdx.x & 63) * stride + slot];
  return __float_as_uint(wave_max(__uint_as_float(v)));
}

// Record the block's maximum in *slot.  One candidate per block; the atomic
// is skipped when the stored value is already larger (maxima only grow
// within a launch, so a stale read only costs an unneeded atomic).
// GUARD = false skips the read (one memory round trip less at the end of a
// launch) where few workgroups share a sub-slot.
template <int NT = kBlock, bool GUARD = true>
__device__ __forceinline__ void block_record_max(float v, uint32_t *slot) {
  __shared__ float red[NT / 64];
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = red[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) m = fmaxf(m, red[w]);
    if (m > 0.f && (!GUARD || __uint_as_float(*(volatile uint32_t *)slot) < m))
      atomicMax(slot, __float_as_uint(m));
  }
}

__device__ __forceinline__ int32_t tab_off(const Tab2 &t, uint32_t i, uint32_t nlo) {
  uint32_t h = i / nlo;
  return ((gint *)t.hi)[h] + ((gint *)t.lo)[i - h * nlo];
}

// Workgroup x of n (ids counted from the first of a segment or launch) -> its
// tile.  Workgroups go to the XCDs in turn (id modulo 8); the tiles are dealt
// so that each XCD takes a run of consecutive tiles, whose pieces of an
// operand share cache lines when a tile's runs are shorter than a line (the
// other pieces of the line are then read from that XCD's L2 instead of again
// from HBM).
__device__ __forceinline__ uint32_t xcd_tile(uint32_t x, uint32_t n) {
  const uint32_t k = x & 7u;
  return k * (n >> 3) + min(k, n & 7u) + (x >> 3);
}

// --------------------------------------------------------------------------
// generic contraction, one lane per output element
// --------------------------------------------------------------------------
static constexpr int kMapU = 4;  // outputs per lane and pass of the generic form

template <int SEMI, bool HASY>
__device__ __forceinline__ void map_body(const ContractArgs &a, const int b, const uint32_t blk,
                                         const uint32_t nblk) {
  gcfloat *__restrict__ X = (gcfloat *)(a.X + (int64_t)b * a.bsX);
  gcfloat *__restrict__ Y = HASY ? (gcfloat *)(a.Y + (int64_t)b * a.bsY) : nullptr;
  gfloat *__restrict__ Z = (gfloat *)(a.Z + (int64_t)b * a.bsZ);
  gint_w *__restrict__ I = SEMI == SEMI_MAX ? (gint_w *)(a.I + (int64_t)b * a.bsZ) : nullptr;
  float sx = 1.f, sy = 1.f;
  int kx = 0, ky = 0;
  if (SEMI == SEMI_SUM) {
    kx = max_exponent(read_max(a.mx, a.mx_stride, a.slotX + (a.batX ? b : 0)));
    sx = ldexpf(1.f, -kx);
    if (HASY) {
      ky = max_exponent(read_max(a.mx, a.mx_stride, a.slotY + (a.batY ? b : 0)));
      sy = ldexpf(1.f, -ky);
    }
  }
  const uint32_t nR = a.nR, nC = a.nC, nRl = a.nRl, nCl = a.nCl, nSl = a.nSl;
  const uint32_t n_out = nR * nC;
  const uint32_t nSh = a.nS / nSl;
  const bool colf = a.col_fastest != 0;
  const Tab2 rX = a.rX, rY = a.rY, rZ = a.rZ, cY = a.cY, cZ = a.cZ, sXt = a.sX, sYt = a.sY;
  // output order (tile 1): output o is Z[o]; X and Y offsets from tables
  // over Z's labels
  const bool oord = a.tile == 1;
  const Tab2 oX = a.oX, oY = a.oY;
  const uint32_t nOl = a.nOl;
  const int osh = (nOl & (nOl - 1)) == 0 ? __builtin_ctz(nOl) : -1;
  // kMapU outputs per lane and pass, kMapU grid strides apart (each of them
  // coalesced across the wave), their operand loads issued together so that
  // several are in flight per lane; lanes past the end clamp to the last
  // output (loads stay in range) and store nothing
  auto offsets = [&](uint32_t o, int32_t &xo, int32_t &yo, int32_t &zo) {
    if (oord) {
      const uint32_t oh = osh >= 0 ? o >> osh : o / nOl, ol = o - oh * nOl;
      xo = oX.hi[oh] + oX.lo[ol];
      yo = HASY ? oY.hi[oh] + oY.lo[ol] : 0;
      zo = (int32_t)o;
    } else {
      uint32_t r, c;
      if (colf) {
        r = o / nC;
        c = o - r * nC;
      } else {
        c = o / nR;
        r = o - c * nR;
      }
      const uint32_t rh = r / nRl, rl = r - rh * nRl;
      xo = rX.hi[rh] + rX.lo[rl];
      zo = rZ.hi[rh] + rZ.lo[rl];
      yo = HASY ? rY.hi[rh] + rY.lo[rl] : 0;
      if (nC > 1) {
        const uint32_t ch = c / nCl, cl = c - ch * nCl;
        zo += cZ.hi[ch] + cZ.lo[cl];
        if (HASY) yo += cY.hi[ch] + cY.lo[cl];
      }
    }
  };
  float lmax = 0.f;
  const uint32_t step = nblk * kBlock;
  for (uint32_t o0 = blk * kBlock + threadIdx.x; o0 < n_out; o0 += kMapU * step) {
    int32_t xo[kMapU], yo[kMapU], zo[kMapU];
    bool live[kMapU];
#pragma unroll
    for (int u = 0; u < kMapU; ++u) {
      const uint32_t o = o0 + u * step;
      live[u] = o < n_out;
      offsets(live[u] ? o : n_out - 1, xo[u], yo[u], zo[u]);
    }
    if (SEMI == SEMI_SUM) {
      float acc[kMapU];
#pragma unroll
      for (int u = 0; u < kMapU; ++u) acc[u] = 0.f;
      for (uint32_t sh = 0; sh < nSh; ++sh) {
        const int32_t xs = sXt.hi[sh];
        const int32_t ys = HASY ? sYt.hi[sh] : 0;
        for (uint32_t sl = 0; sl < nSl; ++sl) {
          const int32_t xl = xs + sXt.lo[sl], yl = HASY ? ys + sYt.lo[sl] : 0;
          float xv[kMapU], yv[kMapU];
#pragma unroll
          for (int u = 0; u < kMapU; ++u) {
            xv[u] = X[xo[u] + xl];
            if (HASY) yv[u] = Y[yo[u] + yl];
          }
#pragma unroll
          for (int u = 0; u < kMapU; ++u) {
            if (HASY)
              acc[u] = fmaf(xv[u] * sx, yv[u] * sy, acc[u]);
            else
              acc[u] += xv[u] * sx;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kMapU; ++u)
        if (live[u]) {
          Z[zo[u]] = acc[u];
          lmax = fmaxf(lmax, acc[u]);
        }
    } else {
      float best[kMapU];
      int32_t bi[kMapU];
#pragma unroll
      for (int u = 0; u < kMapU; ++u) {
        best[u] = -INFINITY;
        bi[u] = 0;
      }
      uint32_t s = 0;
      for (uint32_t sh = 0; sh < nSh; ++sh) {
        const int32_t xs = sXt.hi[sh];
        const int32_t ys = HASY ? sYt.hi[sh] : 0;
        for (uint32_t sl = 0; sl < nSl; ++sl, ++s) {
          const int32_t xl = xs + sXt.lo[sl], yl = HASY ? ys + sYt.lo[sl] : 0;
          float v[kMapU];
#pragma unroll
          for (int u = 0; u < kMapU; ++u) {
            v[u] = X[xo[u] + xl];
            if (HASY) v[u] = v[u] + Y[yo[u] + yl];
          }
#pragma unroll
          for (int u = 0; u < kMapU; ++u)
            if (s == 0 || v[u] > best[u]) {
              best[u] = v[u];
              bi[u] = (int32_t)s;
            }
        }
      }
#pragma unroll
      for (int u = 0; u < kMapU; ++u)
        if (live[u]) {
          Z[zo[u]] = best[u];
          I[zo[u]] = bi[u];
        }
    }
  }
  if (SEMI == SEMI_SUM) {
    block_record_max(lmax, a.mx + (blk % kMaxSub) * a.mx_stride + a.slotZ + (a.batZ ? b : 0));
    if (blk == 0 && threadIdx.x == 0) {
      int e = a.ex[a.slotX + (a.batX ? b : 0)] + kx;
      if (HASY) e += a.ex[a.slotY + (a.batY ? b : 0)] + ky;
      a.ex[a.slotZ + (a.batZ ? b : 0)] = e;
    }
  }
}

// --------------------------------------------------------------------------
// generic contraction, summed index split across workgroups
// --------------------------------------------------------------------------
// Outputs are processed in groups of kSplitOuts kept in registers, so that
// each lane streams its share of the summed index once per group and every
// element of the operands is read once per group.
static constexpr int kSplitOuts = 16;

template <int SEMI, bool HASY>
__device__ __forceinline__ void split_body(const ContractArgs &a, const int b, const uint32_t chunk) {
  gcfloat *__restrict__ X = (gcfloat *)(a.X + (int64_t)b * a.bsX);
  gcfloat *__restrict__ Y = HASY ? (gcfloat *)(a.Y + (int64_t)b * a.bsY) : nullptr;
  float sx = 1.f, sy = 1.f;
  if (SEMI == SEMI_SUM) {
    sx = ldexpf(1.f, -max_exponent(read_max(a.mx, a.mx_stride, a.slotX + (a.batX ? b : 0))));
    if (HASY) sy = ldexpf(1.f, -max_exponent(read_max(a.mx, a.mx_stride, a.slotY + (a.batY ? b : 0))));
  }
  const uint32_t nSh = a.nS / a.nSl;
  const uint32_t per = (nSh + a.n_chunks - 1) / a.n_chunks;
  const uint32_t h0 = chunk * per, h1 = min(nSh, h0 + per);
  const uint32_t n_out = a.nR * a.nC;
  __shared__ float sv[kBlock / 64][kSplitOuts];
  __shared__ int32_t si[kBlock / 64][kSplitOuts];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (uint32_t o0 = 0; o0 < n_out; o0 += kSplitOuts) {
    const int no = (int)min((uint32_t)kSplitOuts, n_out - o0);
    int32_t xo[kSplitOuts], yo[kSplitOuts];
    float acc[kSplitOuts];
    int32_t arg[kSplitOuts];
#pragma unroll
    for (int j = 0; j < kSplitOuts; ++j) {
      xo[j] = 0;
      yo[j] = 0;
      acc[j] = SEMI == SEMI_SUM ? 0.f : -INFINITY;
      arg[j] = -1;
      if (j < no) {
        const uint32_t o = o0 + j;
        uint32_t r, c;
        if (a.col_fastest) {
          r = o / a.nC;
          c = o - r * a.nC;
        } else {
          c = o / a.nR;
          r = o - c * a.nR;
        }
        xo[j] = tab_off(a.rX, r, a.nRl);
        if (HASY) {
          yo[j] = tab_off(a.rY, r, a.nRl);
          if (a.nC > 1) yo[j] += tab_off(a.cY, c, a.nCl);
        }
      }
    }
    for (uint32_t sh = h0; sh < h1; ++sh) {
      const int32_t xs0 = a.sX.hi[sh];
      const int32_t ys0 = HASY ? a.sY.hi[sh] : 0;
      for (uint32_t sl = threadIdx.x; sl < a.nSl; sl += kBlock) {
        const int32_t xs = xs0 + a.sX.lo[sl];
        const int32_t ys = HASY ? ys0 + a.sY.lo[sl] : 0;
        const int32_t sidx = (int32_t)(sh * a.nSl + sl);
#pragma unroll
        for (int j = 0; j < kSplitOuts; ++j) {
          if (j >= no) continue;
          if (SEMI == SEMI_SUM) {
            const float xv = X[xo[j] + xs] * sx;
            acc[j] = HASY ? fmaf(xv, Y[yo[j] + ys] * sy, acc[j]) : acc[j] + xv;
          } else {
            float v = X[xo[j] + xs];
            if (HASY) v = v + Y[yo[j] + ys];
            if (arg[j] < 0 || v > acc[j]) {
              acc[j] = v;
              arg[j] = sidx;
            }
          }
        }
      }
    }
    // reduce every output over the block, fixed shape
#pragma unroll
    for (int j = 0; j < kSplitOuts; ++j) {
      if (j >= no) continue;
      float v = acc[j];
      int32_t i = arg[j];
      if (SEMI == SEMI_SUM) {
        v = wave_sum(v);
      } else {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const float ov = __shfl_xor(v, off, 64);
          const int32_t oi = __shfl_xor(i, off, 64);
          if (oi >= 0 && (i < 0 || ov > v || (ov == v && oi < i))) {
            v = ov;
            i = oi;
          }
        }
      }
      if (lane == 0) {
        sv[wid][j] = v;
        si[wid][j] = i;
      }
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)no) {
      const int j = threadIdx.x;
      const size_t pidx = ((size_t)b * a.n_chunks + chunk) * n_out + o0 + j;
      if (SEMI == SEMI_SUM) {
        float t = 0.f;
        for (int w = 0; w < kBlock / 64; ++w) t += sv[w][j];
        a.part[pidx] = t;
      } else {
        float v = sv[0][j];
        int32_t i = si[0][j];
        for (int w = 1; w < kBlock / 64; ++w)
          if (si[w][j] >= 0 && (i < 0 || sv[w][j] > v || (sv[w][j] == v && si[w][j] < i))) {
            v = sv[w][j];
            i = si[w][j];
          }
        a.part[pidx] = v;
        a.parti[pidx] = i;
      }
    }
    __syncthreads();
  }
}

template <int SEMI, bool HASY>
__device__ __forceinline__ void finish_body(const ContractArgs &a, const int b, const uint32_t o) {
  // one block per output element: lanes stride over the chunks, then a
  // fixed-shape tree reduction (deterministic)
  gfloat *__restrict__ Z = (gfloat *)(a.Z + (int64_t)b * a.bsZ);
  const uint32_t n_out = a.nR * a.nC;
  uint32_t r, c;
  if (a.col_fastest) {
    r = o / a.nC;
    c = o - r * a.nC;
  } else {
    c = o / a.nR;
    r = o - c * a.nR;
  }
  int32_t zo = tab_off(a.rZ, r, a.nRl);
  if (a.nC > 1) zo += tab_off(a.cZ, c, a.nCl);
  const size_t base = (size_t)b * a.n_chunks * n_out + o;
  __shared__ float sv[kBlock / 64];
  __shared__ int32_t si[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int kx = 0, ky = 0;
  if (SEMI == SEMI_SUM && o == 0) {  // whole-block branch: every wave reads
    kx = max_exponent(read_max(a.mx, a.mx_stride, a.slotX + (a.batX ? b : 0)));
    if (HASY) ky = max_exponent(read_max(a.mx, a.mx_stride, a.slotY + (a.batY ? b : 0)));
  }
  if (SEMI == SEMI_SUM) {
    float acc = 0.f;
    for (uint32_t ch = threadIdx.x; ch < a.n_chunks; ch += kBlock) acc += a.part[base + (size_t)ch * n_out];
    acc = wave_sum(acc);
    if (lane == 0) sv[wid] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      float t = 0.f;
      for (int w = 0; w < kBlock / 64; ++w) t += sv[w];
      Z[zo] = t;
      if (t > 0.f) atomicMax(a.mx + (o % kMaxSub) * a.mx_stride + a.slotZ + (a.batZ ? b : 0), __float_as_uint(t));
      if (o == 0) {
        int e = a.ex[a.slotX + (a.batX ? b : 0)] + kx;
        if (HASY) e += a.ex[a.slotY + (a.batY ? b : 0)] + ky;
        a.ex[a.slotZ + (a.batZ ? b : 0)] = e;
      }
    }
  } else {
    gint_w *__restrict__ I = (gint_w *)(a.I + (int64_t)b * a.bsZ);
    float bv = -INFINITY;
    int32_t bj = -1;
    for (uint32_t ch = threadIdx.x; ch < a.n_chunks; ch += kBlock) {
      const float v = a.part[base + (size_t)ch * n_out];
      const int32_t i = a.parti[base + (size_t)ch * n_out];
      if (i >= 0 && (bj < 0 || v > bv || (v == bv && i < bj))) {
        bv = v;
        bj = i;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const float ov = __shfl_xor(bv, off, 64);
      const int32_t oi = __shfl_xor(bj, off, 64);
      if (oi >= 0 && (bj < 0 || ov > bv || (ov == bv && oi < bj))) {
        bv = ov;
        bj = oi;
      }
    }
    if (lane == 0) {
      sv[wid] = bv;
      si[wid] = bj;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      float v = sv[0];
      int32_t j = si[0];
      for (int w = 1; w < kBlock / 64; ++w)
        if (si[w] >= 0 && (j < 0 || sv[w] > v || (sv[w] == v && si[w] < j))) {
          v = sv[w];
          j = si[w];
        }
      Z[zo] = v;
      I[zo] = j < 0 ? 0 : j;
    }
  }
}

// --------------------------------------------------------------------------
// row form: one lane per row of the output; the summed entries (<= B) are
// loaded once into registers and every column (<= B) is produced from them
// --------------------------------------------------------------------------
template <int SEMI, bool HASY, int B>
__device__ __forceinline__ void rows_body(const ContractArgs &a, const int b, const uint32_t blk,
                                          const uint32_t nblk) {
  // every argument is copied to registers before the loop: the arguments
  // live in device memory and stores to Z would otherwise force reloads
  gcfloat *__restrict__ X = (gcfloat *)(a.X + (int64_t)b * a.bsX);
  gcfloat *__restrict__ Y = HASY ? (gcfloat *)(a.Y + (int64_t)b * a.bsY) : nullptr;
  gfloat *__restrict__ Z = (gfloat *)(a.Z + (int64_t)b * a.bsZ);
  gint_w *__restrict__ I = SEMI == SEMI_MAX ? (gint_w *)(a.I + (int64_t)b * a.bsZ) : nullptr;
  const int32_t *__restrict__ rXh = a.rX.hi, *__restrict__ rXl = a.rX.lo;
  const int32_t *__restrict__ rZh = a.rZ.hi, *__restrict__ rZl = a.rZ.lo;
  const int32_t *__restrict__ rYh = a.rY.hi, *__restrict__ rYl = a.rY.lo;
  const uint32_t nR = a.nR, nRl = a.nRl;
  const int rls = a.rl_shift;
  const int ns = a.ns, nc = a.nc;
  int32_t sx[B], sy[B], cy[B], cz[B];
#pragma unroll
  for (int k = 0; k < B; ++k) {
    sx[k] = k < ns ? a.sx[k] : 0;
    sy[k] = k < ns ? a.sy[k] : 0;
    cy[k] = k < nc ? a.cy[k] : 0;
    cz[k] = k < nc ? a.cz[k] : 0;
  }
  float fx = 1.f, fy = 1.f;
  int kx = 0, ky = 0;
  if (SEMI == SEMI_SUM) {
    kx = max_exponent(read_max(a.mx, a.mx_stride, a.slotX + (a.batX ? b : 0)));
    fx = ldexpf(1.f, -kx);
    if (HASY) {
      ky = max_exponent(read_max(a.mx, a.mx_stride, a.slotY + (a.batY ? b : 0)));
      fy = ldexpf(1.f, -ky);
    }
  }
  float lmax = 0.f;
  // U rows per lane per pass (U = 4 for the small sum-product variant): all
  // their offsets and operand loads are issued before the first product;
  // rows past nR repeat row 0's addresses and are not stored
  constexpr int U = (B <= 4 && SEMI == SEMI_SUM) ? 4 : 1;
  const uint32_t stride = nblk * kBlock;
  // With low tables of a power of two >= 64 entries the 64 rows of a wave
  // (64-aligned, consecutive) share one high entry, and with a grid stride
  // that is a multiple of the low table every row of a lane has the same low
  // entry: the lane reads its low offsets once, and the high ones are one
  // wave-uniform read per row group.
  const bool fixed_lo = rls >= 6 && (stride & (nRl - 1)) == 0;
  int32_t xl = 0, zl = 0, yl = 0;
  if (fixed_lo) {
    const uint32_t rl = (blk * kBlock + threadIdx.x) & (nRl - 1);
    xl = ((gint *)rXl)[rl];
    zl = ((gint *)rZl)[rl];
    yl = HASY ? ((gint *)rYl)[rl] : 0;
  }
  for (uint32_t r0 = blk * kBlock + threadIdx.x; r0 < nR; r0 += U * stride) {
    int32_t xo[U], zo[U], yo[U];
    bool live[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t r = r0 + u * stride;
      live[u] = r < nR;
      const uint32_t rr = live[u] ? r : 0u;
      if (fixed_lo) {  // nR is a multiple of nRl >= 64: live is wave-uniform, so is rh
        const uint32_t rh = __builtin_amdgcn_readfirstlane(rr >> rls);
        xo[u] = ((gint *)rXh)[rh] + xl;
        zo[u] = ((gint *)rZh)[rh] + zl;
        yo[u] = HASY ? ((gint *)rYh)[rh] + yl : 0;
        continue;
      }
      uint32_t rh, rl;
      if (rls >= 0) {
        rh = rr >> rls;
        rl = rr & (nRl - 1);
      } else {
        rh = rr / nRl;
        rl = rr - rh * nRl;
      }
      xo[u] = ((gint *)rXh)[rh] + ((gint *)rXl)[rl];
      zo[u] = ((gint *)rZh)[rh] + ((gint *)rZl)[rl];
      yo[u] = HASY ? ((gint *)rYh)[rh] + ((gint *)rYl)[rl] : 0;
    }
    float xv[U][B];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < B; ++k)
        if (k < ns) xv[u][k] = SEMI == SEMI_SUM ? X[xo[u] + sx[k]] * fx : X[xo[u] + sx[k]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int c = 0; c < B; ++c) {
        if (c >= nc) continue;
        const int32_t yc = yo[u] + cy[c];
        if (SEMI == SEMI_SUM) {
          float acc = 0.f;
#pragma unroll
          for (int k = 0; k < B; ++k)
            if (k < ns) acc = HASY ? fmaf(xv[u][k], Y[yc + sy[k]] * fy, acc) : acc + xv[u][k];
          if (live[u]) {
            Z[zo[u] + cz[c]] = acc;
            lmax = fmaxf(lmax, acc);
          }
        } else {
          float best = -INFINITY;
          int32_t bi = 0;
#pragma unroll
          for (int k = 0; k < B; ++k)
            if (k < ns) {
              float v = xv[u][k];
              if (HASY) v = v + Y[yc + sy[k]];
              if (k == 0 || v > best) {
                best = v;
                bi = k;
              }
            }
          if (live[u]) {
            Z[zo[u] + cz[c]] = best;
            I[zo[u] + cz[c]] = bi;
          }
        }
      }
    }
  }
  if (SEMI == SEMI_SUM) {
    block_record_max(lmax, a.mx + (blk % kMaxSub) * a.mx_stride + a.slotZ + (a.batZ ? b : 0));
    if (blk == 0 && threadIdx.x == 0) {
      int e = a.ex[a.slotX + (a.batX ? b : 0)] + kx;
      if (HASY) e += a.ex[a.slotY + (a.batY ? b : 0)] + ky;
      a.ex[a.slotZ + (a.batZ ? b : 0)] = e;
    }
  }
}

// --------------------------------------------------------------------------
// wave form (kind 3): one wavefront per output element, the lanes striding
// over the summed index (consecutive lanes on consecutive summed entries,
// so the stride-1 summed label of X is read coalesced), combined with
// wavefront shuffles.  Max-plus keeps (value, index) pairs: the larger
// value wins, equal values keep the smaller index, so the result is the
// first maximiser in canonical order whatever the lane that found it.
// --------------------------------------------------------------------------
static constexpr int kWaveOuts = kBlock / 64;  // outputs per workgroup pass

template <int SEMI, bool HASY>
__device__ __forceinline__ void wave_body(const ContractArgs &a, const int b, const uint32_t blk,
                                          const uint32_t nblk) {
  gcfloat *__restrict__ X = (gcfloat *)(a.X + (int64_t)b * a.bsX);
  gcfloat *__restrict__ Y = HASY ? (gcfloat *)(a.Y + (int64_t)b * a.bsY) : nullptr;
  gfloat *__restrict__ Z = (gfloat *)(a.Z + (int64_t)b * a.bsZ);
  gint_w *__restrict__ I = SEMI == SEMI_MAX ? (gint_w *)(a.I + (int64_t)b * a.bsZ) : nullptr;
  float sx = 1.f, sy = 1.f;
  int kx = 0, ky = 0;
  if (SEMI == SEMI_SUM) {
    kx = max_exponent(read_max(a.mx, a.mx_stride, a.slotX + (a.batX ? b : 0)));
    sx = ldexpf(1.f, -kx);
    if (HASY) {
      ky = max_exponent(read_max(a.mx, a.mx_stride, a.slotY + (a.batY ? b : 0)));
      sy = ldexpf(1.f, -ky);
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t n_out = a.nR * a.nC, nS = a.nS, nSl = a.nSl;
  float lmax = 0.f;
  for (uint32_t o = blk * kWaveOuts + wid; o < n_out; o += nblk * kWaveOuts) {
    uint32_t r, c;
    if (a.col_fastest) {
      r = o / a.nC;
      c = o - r * a.nC;
    } else {
      c = o / a.nR;
      r = o - c * a.nR;
    }
    const int32_t xo = tab_off(a.rX, r, a.nRl);
    int32_t zo = tab_off(a.rZ, r, a.nRl);
    int32_t yo = HASY ? tab_off(a.rY, r, a.nRl) : 0;
    if (a.nC > 1) {
      zo += tab_off(a.cZ, c, a.nCl);
      if (HASY) yo += tab_off(a.cY, c, a.nCl);
    }
    if (SEMI == SEMI_SUM) {
      float acc = 0.f;
      for (uint32_t sidx = lane; sidx < nS; sidx += 64) {
        const uint32_t sh = sidx / nSl, sl = sidx - sh * nSl;
        const float xv = X[xo + a.sX.hi[sh] + a.sX.lo[sl]] * sx;
        acc = HASY ? fmaf(xv, Y[yo + a.sY.hi[sh] + a.sY.lo[sl]] * sy, acc) : acc + xv;
      }
      acc = wave_sum(acc);
      if (lane == 0) {
        Z[zo] = acc;
        lmax = fmaxf(lmax, acc);
      }
    } else {
      float best = -INFINITY;
      int32_t bi = 0x7fffffff;
      for (uint32_t sidx = lane; sidx < nS; sidx += 64) {
        const uint32_t sh = sidx / nSl, sl = sidx - sh * nSl;
        float v = X[xo + a.sX.hi[sh] + a.sX.lo[sl]];
        if (HASY) v = v + Y[yo + a.sY.hi[sh] + a.sY.lo[sl]];
        if (bi == 0x7fffffff || v > best) {  // first candidate of the lane, or strictly larger
          best = v;
          bi = (int32_t)sidx;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const float ov = __shfl_xor(best, off, 64);
        const int32_t oi = __shfl_xor(bi, off, 64);
        if (oi != 0x7fffffff && (bi == 0x7fffffff || ov > best || (ov == best && oi < bi))) {
          best = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        Z[zo] = best;
        I[zo] = bi;
      }
    }
  }
  if (SEMI == SEMI_SUM) {
    block_record_max(lmax, a.mx + (blk % kMaxSub) * a.mx_stride + a.slotZ + (a.batZ ? b : 0));
    if (blk == 0 && threadIdx.x == 0) {
      int e = a.ex[a.slotX + (a.batX ? b : 0)] + kx;
      if (HASY) e += a.ex[a.slotY + (a.batY ? b : 0)] + ky;
      a.ex[a.slotZ + (a.batZ ? b : 0)] = e;
    }
  }
}

// --------------------------------------------------------------------------
// batch-uniform row form (kind 1, tile 1; sum-product with Y): the rows are
// (batch assignment g of the labels Y holds too, M assignment m of the
// others).  A wavefront takes 64 consecutive m of one g, so the block
// Y[g][s][c] (ns x nc <= BS x BC <= 128 entries) is the same for all its
// lanes: it is read once per wavefront, two entries per lane, into LDS,
// and every product reads its entry there (one address for all lanes).  A
// lane keeps its row of X (ns entries) and its row of Z (nc entries) in
// registers: X and Z are read and written once, Y once per wavefront.
// Each output sums its products in canonical summed order, as the row form.
// --------------------------------------------------------------------------
template <int BS, int BC>
__device__ __forceinline__ void rowsb_body(const ContractArgs &a, const int b, const uint32_t blk,
                                           const uint32_t nblk) {
  static_assert(BS * BC <= kRowBlock && BC % 4 == 0, "at most two block entries per lane, columns in fours");
  constexpr int kWaves = kBlock / 64;
  __shared__ float4 yblk[kWaves][kRowBlock / 4];  // each wavefront's block of Y, rows of BC entries
  gcfloat *__restrict__ X = (gcfloat *)(a.X + (int64_t)b * a.bsX);
  gcfloat *__restrict__ Y = (gcfloat *)(a.Y + (int64_t)b * a.bsY);
  gfloat *__restrict__ Z = (gfloat *)(a.Z + (int64_t)b * a.bsZ);
  const int ns = a.ns, nc = a.nc;
  int32_t sx[BS], cz[BC];
#pragma unroll
  for (int k = 0; k < BS; ++k) sx[k] = k < ns ? a.sx[k] : 0;
#pragma unroll
  for (int k = 0; k < BC; ++k) cz[k] = k < nc ? a.cz[k] : 0;
  const int kx = max_exponent(read_max(a.mx, a.mx_stride, a.slotX + (a.batX ? b : 0)));
  const int ky = max_exponent(read_max(a.mx, a.mx_stride, a.slotY + (a.batY ? b : 0)));
  const float fx = ldexpf(1.f, -kx), fy = ldexpf(1.f, -ky);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float *const yw = (float *)yblk[wv];
  // the lane's two entries of the block: index s * BC + c
  int32_t yoff[2];
  bool yok[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int idx = lane + 64 * h, s = idx / BC, c = idx % BC;
    yok[h] = s < ns && c < nc;
    yoff[h] = yok[h] ? a.sy[s] + a.cy[c] : 0;
  }
  // wavefront w takes batch assignment w % nB and M assignments 64 (w / nB)
  // on: consecutive wavefronts run the batch assignments of one run of M
  // assignments, which share the cache lines of X and Z where batch labels
  // are faster than M labels (consecutive workgroups run on one XCD)
  const uint32_t nM = a.nM, nB = a.nB, wpg = (nM + 63) / 64;  // wavefronts per batch assignment
  const uint32_t n_waves = nB * wpg;
  float lmax = 0.f;
  // every wavefront of the workgroup runs every pass (the barriers), a pass
  // past the last wavefront computes nothing it stores
  for (uint32_t w0 = blk * kWaves; w0 < n_waves; w0 += nblk * kWaves) {
    const uint32_t w = w0 + wv < n_waves ? w0 + wv : n_waves - 1;
    const uint32_t mb = w / nB, g = w - mb * nB, m = mb * 64 + lane;
    const bool live = w0 + wv < n_waves && m < nM;
    const uint32_t mc = m < nM ? m : 0u;
    const int32_t yg = tab_off(a.gbY, g, a.nBl);
    const int32_t xo = tab_off(a.gbX, g, a.nBl) + tab_off(a.gmX, mc, a.nMl);
    const int32_t zo = tab_off(a.gbZ, g, a.nBl) + tab_off(a.gmZ, mc, a.nMl);
    float xv[BS];
#pragma unroll
    for (int h = 0; h < 2; ++h) yw[lane + 64 * h] = yok[h] ? Y[yg + yoff[h]] * fy : 0.f;
    if (BS >= 4 && a.row_vx == 1) {  // summed entries in aligned runs of four
#pragma unroll
      for (int k = 0; k < BS; k += 4)
        if (k < ns) {
          const f32x4 v = *(gcf32x4 *)(X + xo + sx[k]);
          xv[k] = v[0] * fx;
          xv[k + 1] = v[1] * fx;
          xv[k + 2] = v[2] * fx;
          xv[k + 3] = v[3] * fx;
        } else {
          xv[k] = xv[k + 1] = xv[k + 2] = xv[k + 3] = 0.f;
        }
    } else if (BS >= 2 && a.row_vx == 2) {  // in aligned pairs
#pragma unroll
      for (int k = 0; k < BS; k += 2)
        if (k < ns) {
          const f32x2 v = *(gcf32x2 *)(X + xo + sx[k]);
          xv[k] = v[0] * fx;
          xv[k + 1] = v[1] * fx;
        } else {
          xv[k] = xv[k + 1] = 0.f;
        }
    } else {
#pragma unroll
      for (int k = 0; k < BS; ++k) xv[k] = k < ns ? X[xo + sx[k]] * fx : 0.f;
    }
    __syncthreads();
    float acc[BC];
#pragma unroll
    for (int c = 0; c < BC; ++c) acc[c] = 0.f;
#pragma unroll
    for (int k = 0; k < BS; ++k) {
      if (k >= ns) break;
#pragma unroll
      for (int c4 = 0; c4 < BC / 4; ++c4) {
        const float4 y = yblk[wv][k * (BC / 4) + c4];  // the same address on every lane
        acc[4 * c4] = fmaf(xv[k], y.x, acc[4 * c4]);
        acc[4 * c4 + 1] = fmaf(xv[k], y.y, acc[4 * c4 + 1]);
        acc[4 * c4 + 2] = fmaf(xv[k], y.z, acc[4 * c4 + 2]);
        acc[4 * c4 + 3] = fmaf(xv[k], y.w, acc[4 * c4 + 3]);
      }
    }
    if (live && a.row_vz) {  // columns in aligned runs of four
#pragma unroll
      for (int c = 0; c < BC; c += 4)
        if (c < nc) {
          const f32x4 v = {acc[c], acc[c + 1], acc[c + 2], acc[c + 3]};
          *(gf32x4 *)(Z + zo + cz[c]) = v;
          lmax = fmaxf(lmax, fmaxf(fmaxf(acc[c], acc[c + 1]), fmaxf(acc[c + 2], acc[c + 3])));
        }
    } else if (live) {
#pragma unroll
      for (int c = 0; c < BC; ++c)
        if (c < nc) {
          Z[zo + cz[c]] = acc[c];
          lmax = fmaxf(lmax, acc[c]);
        }
    }
    __syncthreads();  // the next pass rewrites the blocks
  }
  block_record_max(lmax, a.mx + (blk % kMaxSub) * a.mx_stride + a.slotZ + (a.batZ ? b : 0));
  if (blk == 0 && threadIdx.x == 0)
    a.ex[a.slotZ + (a.batZ ? b : 0)] = a.ex[a.slotX + (a.batX ? b : 0)] + kx + a.ex[a.slotY + (a.batY ? b : 0)] + ky;
}

// --------------------------------------------------------------------------
// two consecutive max-plus contractions in one pass (kind kKindMaxPair; the
// arguments' layout is described with ContractArgs): a lane takes one
// assignment r of R2, forms the first step's outputs (r, s2) for every s2
// in registers with their argmax s1, then the second step's outputs (r, c);
// its index array gets both choices as one index, s1 * ns2 + s2 (the
// readout assigns both steps' variables from it).  Values are one FP32 add
// per candidate and the first maximiser in canonical order wins, exactly as
// in the other max-plus forms.
// --------------------------------------------------------------------------
// three steps, each summing at most two assignments (steps = 3)
__device__ __forceinline__ void mtriple_body(const ContractArgs &a, const uint32_t blk, const uint32_t nblk) {
  gcfloat *__restrict__ X = (gcfloat *)a.X;
  gcfloat *__restrict__ Y1 = (gcfloat *)a.Y;
  gcfloat *__restrict__ Y2 = (gcfloat *)a.Y2;
  gcfloat *__restrict__ Y3 = (gcfloat *)a.Y3;
  gfloat *__restrict__ Z = (gfloat *)a.Z;
  gint_w *__restrict__ I = (gint_w *)a.I;
  const int n1 = a.ns, n2 = a.ns2, n3 = a.ns3, nc = a.nc;
  constexpr int K = kTripleMax;
  int32_t sx[K * K * K], sy[K * K * K], y2[K * K], y3[K * K], zc[K];
#pragma unroll
  for (int k = 0; k < K * K * K; ++k) {
    const bool in = k / (K * K) < n3 && (k / K) % K < n2 && k % K < n1;
    sx[k] = in ? a.sx[k] : 0;
    sy[k] = in ? a.sy[k] : 0;
  }
#pragma unroll
  for (int k = 0; k < K * K; ++k) {
    y2[k] = (k / K < n3 && k % K < n2) ? a.cy[k] : 0;
    y3[k] = (k / K < nc && k % K < n3) ? a.cz[k] : 0;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) zc[k] = k < nc ? a.cz[kPairZ + k] : 0;
  const uint32_t nR = a.nR, nRl = a.nRl;
  const int rls = a.rl_shift;
  for (uint32_t r = blk * kBlock + threadIdx.x; r < nR; r += nblk * kBlock) {
    uint32_t rh, rl;
    if (rls >= 0) {
      rh = r >> rls;
      rl = r & (nRl - 1);
    } else {
      rh = r / nRl;
      rl = r - rh * nRl;
    }
    const int32_t xo = ((gint *)a.rX.hi)[rh] + ((gint *)a.rX.lo)[rl];
    const int32_t y1o = ((gint *)a.rY.hi)[rh] + ((gint *)a.rY.lo)[rl];
    const int32_t y2o = ((gint *)a.gbY.hi)[rh] + ((gint *)a.gbY.lo)[rl];
    const int32_t y3o = ((gint *)a.gmX.hi)[rh] + ((gint *)a.gmX.lo)[rl];
    const int32_t zo = ((gint *)a.rZ.hi)[rh] + ((gint *)a.rZ.lo)[rl];
    float xv[K * K * K];
    if (a.row_vx) {  // the eight entries adjacent: two 16-byte loads
      const f32x4 lo = *(gcf32x4 *)(X + xo + sx[0]), hi = *(gcf32x4 *)(X + xo + sx[0] + 4);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        xv[k] = lo[k] + Y1[y1o + sy[k]];
        xv[k + 4] = hi[k] + Y1[y1o + sy[k + 4]];
      }
    } else {
#pragma unroll
      for (int k = 0; k < K * K * K; ++k)
        if (k / (K * K) < n3 && (k / K) % K < n2 && k % K < n1) xv[k] = X[xo + sx[k]] + Y1[y1o + sy[k]];
    }
    // first step: outputs (r, s3, s2) and their first maximiser s1
    float v1[K * K];
    int32_t i1[K * K];
#pragma unroll
    for (int q = 0; q < K * K; ++q) {
      v1[q] = -INFINITY;
      i1[q] = 0;
      if (q / K < n3 && q % K < n2) {
#pragma unroll
        for (int w = 0; w < K; ++w)
          if (w < n1 && (w == 0 || xv[K * q + w] > v1[q])) {
            v1[q] = xv[K * q + w];
            i1[q] = w;
          }
      }
    }
    // second step: outputs (r, s3); the index over (s1, s2) of its choice
    float v2[K];
    int32_t i2[K];
#pragma unroll
    for (int u3 = 0; u3 < K; ++u3) {
      v2[u3] = -INFINITY;
      i2[u3] = 0;
      if (u3 < n3) {
#pragma unroll
        for (int u2 = 0; u2 < K; ++u2)
          if (u2 < n2) {
            const float v = v1[K * u3 + u2] + Y2[y2o + y2[K * u3 + u2]];
            if (u2 == 0 || v > v2[u3]) {
              v2[u3] = v;
              i2[u3] = i1[K * u3 + u2] * n2 + u2;
            }
          }
      }
    }
    // third step: the outputs (r, c) and the index over (s1, s2, s3)
#pragma unroll
    for (int c = 0; c < K; ++c) {
      if (c >= nc) break;
      float best = -INFINITY;
      int32_t bi = 0;
#pragma unroll
      for (int u3 = 0; u3 < K; ++u3)
        if (u3 < n3) {
          const float v = v2[u3] + Y3[y3o + y3[K * c + u3]];
          if (u3 == 0 || v > best) {
            best = v;
            bi = i2[u3] * n3 + u3;
          }
        }
      Z[zo + zc[c]] = best;
      I[zo + zc[c]] = bi;
    }
  }
}

__device__ __forceinline__ void mpair_body(const ContractArgs &a, const uint32_t blk, const uint32_t nblk) {
  if (a.steps == 3) {
    mtriple_body(a, blk, nblk);
    return;
  }
  gcfloat *__restrict__ X = (gcfloat *)a.X;
  gcfloat *__restrict__ Y1 = (gcfloat *)a.Y;
  gcfloat *__restrict__ Y2 = (gcfloat *)a.Y2;
  gfloat *__restrict__ Z = (gfloat *)a.Z;
  gint_w *__restrict__ I2 = (gint_w *)a.I;
  const int n1 = a.ns, n2 = a.ns2, nc = a.nc;
  constexpr int K = kPairMax;
  int32_t sx[K * K], sy[K * K], y2[K * K], z2[K];
#pragma unroll
  for (int k = 0; k < K * K; ++k) {
    const bool in1 = (k / K) < n2 && (k % K) < n1, in2 = (k / K) < nc && (k % K) < n2;
    sx[k] = in1 ? a.sx[k] : 0;
    sy[k] = in1 ? a.sy[k] : 0;
    y2[k] = in2 ? a.cy[k] : 0;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) z2[k] = k < nc ? a.cz[kPairZ + k] : 0;
  const uint32_t nR = a.nR, nRl = a.nRl;
  const int rls = a.rl_shift;
  for (uint32_t r = blk * kBlock + threadIdx.x; r < nR; r += nblk * kBlock) {
    uint32_t rh, rl;
    if (rls >= 0) {
      rh = r >> rls;
      rl = r & (nRl - 1);
    } else {
      rh = r / nRl;
      rl = r - rh * nRl;
    }
    const int32_t xo = ((gint *)a.rX.hi)[rh] + ((gint *)a.rX.lo)[rl];
    const int32_t y1o = ((gint *)a.rY.hi)[rh] + ((gint *)a.rY.lo)[rl];
    const int32_t zo = ((gint *)a.rZ.hi)[rh] + ((gint *)a.rZ.lo)[rl];
    const int32_t y2o = ((gint *)a.gbY.hi)[rh] + ((gint *)a.gbY.lo)[rl];
    float xv[K * K], v1[K];
    int32_t i1[K];
    if (a.row_vx) {  // two steps of two summed assignments, the four entries adjacent: one 16-byte load
      const f32x4 x4 = *(gcf32x4 *)(X + xo + sx[0]);
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int w = 0; w < 2; ++w) xv[K * u + w] = x4[2 * u + w] + Y1[y1o + sy[K * u + w]];
    } else {
#pragma unroll
      for (int k = 0; k < K * K; ++k)
        if ((k / K) < n2 && (k % K) < n1) xv[k] = X[xo + sx[k]] + Y1[y1o + sy[k]];
    }
#pragma unroll
    for (int u = 0; u < K; ++u) {
      if (u >= n2) break;
      float best = -INFINITY;
      int32_t bi = 0;
#pragma unroll
      for (int w = 0; w < K; ++w)
        if (w < n1 && (w == 0 || xv[K * u + w] > best)) {
          best = xv[K * u + w];
          bi = w;
        }
      v1[u] = best;
      i1[u] = bi;
    }
#pragma unroll
    for (int c = 0; c < K; ++c) {
      if (c >= nc) break;
      float best = -INFINITY;
      int32_t bi = 0, b1 = i1[0];
#pragma unroll
      for (int u = 0; u < K; ++u)
        if (u < n2) {
          const float v = v1[u] + Y2[y2o + y2[K * c + u]];
          if (u == 0 || v > best) {
            best = v;
            bi = u;
            b1 = i1[u];
          }
        }
      Z[zo + z2[c]] = best;
      I2[zo + z2[c]] = b1 * n2 + bi;
    }
  }
}

template <int SEMI, bool HASY>
__device__ __forceinline__ void any_map_body(const ContractArgs &a, const int b, const uint32_t blk,
                                             const uint32_t nblk) {
  if (a.kind == 1) {
    if (a.ns <= 4 && a.nc <= 4) rows_body<SEMI, HASY, 4>(a, b, blk, nblk);
    else rows_body<SEMI, HASY, kRowFormMax>(a, b, blk, nblk);
  } else if (a.kind == 3) {
    wave_body<SEMI, HASY>(a, b, blk, nblk);
  } else {
    map_body<SEMI, HASY>(a, b, blk, nblk);
  }
}

// --------------------------------------------------------------------------
// dense form on the matrix cores (sum-product): for one batch assignment,
// a 64 x 64 tile of Z[M, N] = sum_S X[M, S] Y[S, N], FP32 operands on
// v_mfma_f32_16x16x4_f32 (lane l holds A[l % 16][l / 16], B[l / 16][l % 16],
// D[4 (l / 16) + r][l % 16]).  Operands are gathered through the offset
// tables into LDS chunks of 16 summed entries (consecutive threads on the
// operand's stride-1 label), scaled on load; each wave owns a 32 x 32
// quarter of the tile (2 x 2 MFMA tiles); the tile leaves through LDS with
// consecutive threads on Z's stride-1 label.
// --------------------------------------------------------------------------
static constexpr int kGT = kGemmTile;   // 64
static constexpr int kGK = 16;          // summed entries per chunk
static constexpr int kGKP = kGT + 16;   // chunk row pitch: conflict-free MFMA operand reads
static constexpr int kGCP = kGT + 1;    // epilogue tile pitch

// Summed entries per chunk of the sum-product dense form, and the largest
// summed set whose offsets are staged in LDS once per workgroup (larger sets
// look their offsets up per element).
static constexpr int kDK = 32;
static constexpr int kDSOff = 2048;

template <int PREC>
__device__ __forceinline__ void gemm_body(const ContractArgs &a, const int b, const uint32_t blk) {
  __shared__ int32_t oMX[kGT], oMZ[kGT], oNY[kGT], oNZ[kGT];
  __shared__ int32_t sOX[kDSOff], sOY[kDSOff];
  __shared__ float AB[2 * kDK * kGKP];
  __shared__ int ksh[2];
  float *As = AB, *Bs = AB + kDK * kGKP;
  float *Cs = AB;  // the epilogue tile reuses the operand chunks (64 x 65 <= 2 x 32 x 80 floats)
  static_assert(kGT * kGCP <= 2 * kDK * kGKP, "epilogue tile fits the operand chunks");
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const uint32_t tm = (a.nM + kGT - 1) / kGT, tn = (a.nC + kGT - 1) / kGT;
  uint32_t bt, mt, nt;
  dense_tile(blk, tm, tn, a.nBlo, bt, mt, nt);
  const uint32_t m0 = mt * kGT, n0 = nt * kGT;
  const int32_t xb = tab_off(a.gbX, bt, a.nBl), yb = tab_off(a.gbY, bt, a.nBl), zb = tab_off(a.gbZ, bt, a.nBl);
  gcfloat *__restrict__ X = (gcfloat *)(a.X + (int64_t)b * a.bsX + xb);
  gcfloat *__restrict__ Y = (gcfloat *)(a.Y + (int64_t)b * a.bsY + yb);
  gfloat *__restrict__ Z = (gfloat *)(a.Z + (int64_t)b * a.bsZ + zb);
  const uint32_t nS = a.nS;
  const bool staged = nS <= (uint32_t)kDSOff;
  // prologue: row / column offsets, the operands' exponents and (small
  // summed sets) every summed entry's offsets, one read each
  if (w == 0) {
    const uint32_t m = m0 + l;
    oMX[l] = m < a.nM ? tab_off(a.gmX, m, a.nMl) : -1;
    oMZ[l] = m < a.nM ? tab_off(a.gmZ, m, a.nMl) : -1;
  } else if (w == 1) {
    const uint32_t n = n0 + l;
    oNY[l] = n < a.nC ? (a.nC > 1 ? tab_off(a.cY, n, a.nCl) : 0) : -1;
    oNZ[l] = n < a.nC ? (a.nC > 1 ? tab_off(a.cZ, n, a.nCl) : 0) : -1;
  } else {
    const int slot = w == 2 ? a.slotX + (a.batX ? b : 0) : a.slotY + (a.batY ? b : 0);
    const int k = max_exponent(read_max(a.mx, a.mx_stride, slot));
    if (l == 0) ksh[w - 2] = k;
  }
  if (staged)
    for (uint32_t s = t; s < nS; s += kBlock) {
      sOX[s] = tab_off(a.sX, s, a.nSl);
      sOY[s] = tab_off(a.sY, s, a.nSl);
    }
  __syncthreads();
  const int kx = ksh[0], ky = ksh[1];
  const float sx = ldexpf(1.f, -kx), sy = ldexpf(1.f, -ky);
  // per thread: 8 entries of each operand per chunk; entry q of A is
  // (row mA[q], summed kA[q]) and of B (summed kB[q], column nB[q]), with
  // consecutive threads on the operand's stride-1 label
  constexpr int NQ = kGT * kDK / kBlock;
  int32_t oa[NQ], ob[NQ];
  int kA[NQ], kB[NQ], dA[NQ], dB[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = t + q * kBlock;
    int m, k;
    if (a.x_s_fast) { k = e % kDK; m = e / kDK; } else { m = e % kGT; k = e / kGT; }
    oa[q] = oMX[m];
    kA[q] = k;
    dA[q] = k * kGKP + m;
    int n, k2;
    if (a.y_n_fast) { n = e % kGT; k2 = e / kGT; } else { k2 = e % kDK; n = e / kDK; }
    ob[q] = oNY[n];
    kB[q] = k2;
    dB[q] = k2 * kGKP + n;
  }
  // loads of one chunk: every address in bounds (rows past the tile and
  // summed entries past nS read entry 0 of the operand), masked afterwards
  auto load_chunk = [&](uint32_t s0, float (&va)[NQ], float (&vb)[NQ]) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const uint32_t s = s0 + kA[q], s2 = s0 + kB[q];
      const uint32_t sc = s < nS ? s : 0u, sc2 = s2 < nS ? s2 : 0u;
      const int32_t ox = staged ? sOX[sc] : tab_off(a.sX, sc, a.nSl);
      const int32_t oy = staged ? sOY[sc2] : tab_off(a.sY, sc2, a.nSl);
      const float x = X[(oa[q] >= 0 ? oa[q] : 0) + ox];
      const float y = Y[(ob[q] >= 0 ? ob[q] : 0) + oy];
      va[q] = (oa[q] >= 0 && s < nS) ? x * sx : 0.f;
      vb[q] = (ob[q] >= 0 && s2 < nS) ? y * sy : 0.f;
    }
  };
  f32x4 acc[2][2] = {};
  const int wm = w & 1, wn = w >> 1;
  float va[NQ], vb[NQ], na[NQ], nb[NQ];
  load_chunk(0, va, vb);
  for (uint32_t s0 = 0; s0 < nS; s0 += kDK) {
    const bool more = s0 + kDK < nS;
    if (more) load_chunk(s0 + kDK, na, nb);  // next chunk in flight during this one's products
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      As[dA[q]] = va[q];
      Bs[dB[q]] = vb[q];
    }
    __syncthreads();
    if (PREC == 0) {
#pragma unroll
      for (int kk = 0; kk < kDK; kk += 4) {
        const int r = (kk + (l >> 4)) * kGKP + (l & 15);
        const float a0 = As[r + 32 * wm], a1 = As[r + 32 * wm + 16];
        const float b0 = Bs[r + 32 * wn], b1 = Bs[r + 32 * wn + 16];
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
      }
    } else {  // 16 summed entries per low-precision step
#pragma unroll
      for (int kk = 0; kk < kDK; kk += 16) {
        float a0[4], a1[4], b0[4], b1[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = (kk + 4 * (l >> 4) + j) * kGKP + (l & 15);
          a0[j] = As[r + 32 * wm];
          a1[j] = As[r + 32 * wm + 16];
          b0[j] = Bs[r + 32 * wn];
          b1[j] = Bs[r + 32 * wn + 16];
        }
        acc[0][0] = mfma16_lp<PREC>(a0, b0, acc[0][0]);
        acc[0][1] = mfma16_lp<PREC>(a0, b1, acc[0][1]);
        acc[1][0] = mfma16_lp<PREC>(a1, b0, acc[1][0]);
        acc[1][1] = mfma16_lp<PREC>(a1, b1, acc[1][1]);
      }
    }
    __syncthreads();
    if (more) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        va[q] = na[q];
        vb[q] = nb[q];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        Cs[(32 * wm + 16 * i + 4 * (l >> 4) + r) * kGCP + 32 * wn + 16 * j + (l & 15)] = acc[i][j][r];
  __syncthreads();
  float lmax = 0.f;
#pragma unroll 4
  for (int q = 0; q < kGT * kGT / kBlock; ++q) {
    const int e = t + q * kBlock;
    int m, n;
    if (a.z_n_fast) { n = e % kGT; m = e / kGT; } else { m = e % kGT; n = e / kGT; }
    const int32_t om = oMZ[m], on = oNZ[n];
    if (om >= 0 && on >= 0) {
      const float v = Cs[m * kGCP + n];
      Z[om + on] = v;
      lmax = fmaxf(lmax, v);
    }
  }
  block_record_max(lmax, a.mx + (blk % kMaxSub) * a.mx_stride + a.slotZ + (a.batZ ? b : 0));
  if (blk == 0 && threadIdx.x == 0)
    a.ex[a.slotZ + (a.batZ ? b : 0)] = a.ex[a.slotX + (a.batX ? b : 0)] + kx + a.ex[a.slotY + (a.batY ? b : 0)] + ky;
}

// --------------------------------------------------------------------------
// dense form of a max-plus node on the vector ALUs: a 64 x 64 tile of
// Z[M, N] = max_S (X[M, S] + Y[S, N]) with the argmax index over S.  Chunks
// of 16 summed entries are gathered into LDS as in the sum-product form
// (entries past nS read as -inf, so they never win); every thread keeps a
// 4 x 4 block of (value, index) pairs in registers and scans the chunk in
// canonical order with a strict comparison, so the first maximiser is kept
// (every candidate one FP32 addition).  The next chunk's loads are in flight
// (registers) during this chunk's candidates, and the summed entries'
// offsets of small summed sets are staged in LDS once.
// --------------------------------------------------------------------------
static constexpr int kMSOff = 1024;  // largest summed set whose offsets are staged in LDS

__device__ __forceinline__ void gemm_max_body(const ContractArgs &a, const int b, const uint32_t blk) {
  __shared__ int32_t oMX[kGT], oMZ[kGT], oNY[kGT], oNZ[kGT];
  __shared__ float As[kGK * kGKP], Bs[kGK * kGKP];
  __shared__ int32_t Ci[kGT * kGCP];
  __shared__ float U[kGT * kGCP];  // the staged summed offsets during the scan, the value tile after it
  static_assert(2 * kMSOff <= kGT * kGCP, "staged offsets fit the epilogue tile");
  int32_t *sOX = reinterpret_cast<int32_t *>(U), *sOY = sOX + kMSOff;
  float *Cs = U;
  const int t = threadIdx.x;
  const int l = t & 63, w = t >> 6;
  const uint32_t tm = (a.nM + kGT - 1) / kGT, tn = (a.nC + kGT - 1) / kGT;
  uint32_t bt, mt, nt;
  dense_tile(blk, tm, tn, a.nBlo, bt, mt, nt);
  const uint32_t m0 = mt * kGT, n0 = nt * kGT;
  const int32_t xb = tab_off(a.gbX, bt, a.nBl), yb = tab_off(a.gbY, bt, a.nBl), zb = tab_off(a.gbZ, bt, a.nBl);
  gcfloat *__restrict__ X = (gcfloat *)(a.X + (int64_t)b * a.bsX + xb);
  gcfloat *__restrict__ Y = (gcfloat *)(a.Y + (int64_t)b * a.bsY + yb);
  gfloat *__restrict__ Z = (gfloat *)(a.Z + (int64_t)b * a.bsZ + zb);
  gint_w *__restrict__ I = (gint_w *)(a.I + (int64_t)b * a.bsZ + zb);
  const uint32_t nS = a.nS;
  const bool staged = nS <= (uint32_t)kMSOff;
  if (w == 0) {
    const uint32_t m = m0 + l;
    oMX[l] = m < a.nM ? tab_off(a.gmX, m, a.nMl) : -1;
    oMZ[l] = m < a.nM ? tab_off(a.gmZ, m, a.nMl) : -1;
  } else if (w == 1) {
    const uint32_t n = n0 + l;
    oNY[l] = n < a.nC ? (a.nC > 1 ? tab_off(a.cY, n, a.nCl) : 0) : -1;
    oNZ[l] = n < a.nC ? (a.nC > 1 ? tab_off(a.cZ, n, a.nCl) : 0) : -1;
  }
  if (staged)
    for (uint32_t s = t; s < nS; s += kBlock) {
      sOX[s] = tab_off(a.sX, s, a.nSl);
      sOY[s] = tab_off(a.sY, s, a.nSl);
    }
  __syncthreads();
  // per thread: 4 entries of each operand per chunk, consecutive threads on
  // the operand's stride-1 label
  constexpr int NQ = kGT * kGK / kBlock;
  int32_t oa[NQ], ob[NQ];
  int kA[NQ], kB[NQ], dA[NQ], dB[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = t + q * kBlock;
    int m, k;
    if (a.x_s_fast) { k = e % kGK; m = e / kGK; } else { m = e % kGT; k = e / kGT; }
    oa[q] = oMX[m];
    kA[q] = k;
    dA[q] = k * kGKP + m;
    int n, k2;
    if (a.y_n_fast) { n = e % kGT; k2 = e / kGT; } else { k2 = e % kGK; n = e / kGK; }
    ob[q] = oNY[n];
    kB[q] = k2;
    dB[q] = k2 * kGKP + n;
  }
  // every address in bounds (rows past the tile and summed entries past nS
  // read entry 0), masked to -inf afterwards
  auto load_chunk = [&](uint32_t s0, float (&va)[NQ], float (&vb)[NQ]) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const uint32_t s = s0 + kA[q], s2 = s0 + kB[q];
      const uint32_t sc = s < nS ? s : 0u, sc2 = s2 < nS ? s2 : 0u;
      const int32_t ox = staged ? sOX[sc] : tab_off(a.sX, sc, a.nSl);
      const int32_t oy = staged ? sOY[sc2] : tab_off(a.sY, sc2, a.nSl);
      const float x = X[(oa[q] >= 0 ? oa[q] : 0) + ox];
      const float y = Y[(ob[q] >= 0 ? ob[q] : 0) + oy];
      va[q] = (oa[q] >= 0 && s < nS) ? x : -INFINITY;
      vb[q] = (ob[q] >= 0 && s2 < nS) ? y : -INFINITY;
    }
  };
  // thread (ty, tx) owns rows ty + 16 i and columns tx + 16 j, i, j < 4
  const int ty = t >> 4, tx = t & 15;
  float best[4][4];
  int32_t arg[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      best[i][j] = -INFINITY;
      arg[i][j] = 0;
    }
  float va[NQ], vb[NQ], na[NQ], nb[NQ];
  if (nS > 0) load_chunk(0, va, vb);
  for (uint32_t s0 = 0; s0 < nS; s0 += kGK) {
    const bool more = s0 + kGK < nS;
    if (more) load_chunk(s0 + kGK, na, nb);  // next chunk in flight during this one's candidates
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      As[dA[q]] = va[q];
      Bs[dB[q]] = vb[q];
    }
    __syncthreads();
    const int kn = (int)min((uint32_t)kGK, nS - s0);
    for (int k = 0; k < kn; ++k) {
      float av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        av[i] = As[k * kGKP + ty + 16 * i];
        bv[i] = Bs[k * kGKP + tx + 16 * i];
      }
      const int32_t sidx = (int32_t)(s0 + k);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float v = av[i] + bv[j];
          if (v > best[i][j]) {
            best[i][j] = v;
            arg[i][j] = sidx;
          }
        }
    }
    __syncthreads();
    if (more) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        va[q] = na[q];
        vb[q] = nb[q];
      }
    }
  }
  // the value tile reuses the staged offsets (the last chunk's loads are done)
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Cs[(ty + 16 * i) * kGCP + tx + 16 * j] = best[i][j];
      Ci[(ty + 16 * i) * kGCP + tx + 16 * j] = arg[i][j];
    }
  __syncthreads();
#pragma unroll 4
  for (int q = 0; q < kGT * kGT / kBlock; ++q) {
    const int e = t + q * kBlock;
    int m, n;
    if (a.z_n_fast) { n = e % kGT; m = e / kGT; } else { m = e % kGT; n = e / kGT; }
    const int32_t om = oMZ[m], on = oNZ[n];
    if (om >= 0 && on >= 0) {
      Z[om + on] = Cs[m * kGCP + n];
      I[om + on] = Ci[m * kGCP + n];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_gemm_max(const ContractArgs *__restrict__ ap) {
  gemm_max_body(*ap, blockIdx.y, blockIdx.x);
}

// one kernel per operand precision (a runtime switch inside one kernel would
// size its registers for the largest variant)
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_gemm(const ContractArgs *__restrict__ ap) {
  gemm_body<PREC>(*ap, blockIdx.y, blockIdx.x);
}

// --------------------------------------------------------------------------
// dense form with large tiles (FP32 sum-product, wide row and column sets):
// a 128 x 128 tile of Z[M, N] = sum_S X[M, S] Y[S, N] per workgroup, each
// wave a 64 x 64 quarter as 4 x 4 v_mfma_f32_16x16x4_f32 tiles.  A chunk of
// 16 summed entries sits in LDS summed-fastest (rows of A and columns of B,
// pitch 20 floats), so one 128-bit LDS read gives a lane its operand for four
// MFMA steps: in step j the lanes of group g = l / 16 supply summed entry
// 4 g + j of both operands, which covers the chunk once.  Two LDS buffers
// and two register sets: the global loads of the chunk after next are in
// flight during this chunk's products, and one barrier per chunk separates
// the reuse of an LDS buffer.  The tile leaves
// through LDS in two halves of 64 rows with consecutive threads on Z's
// stride-1 label.  Workgroup ids are remapped so that the workgroups one XCD
// receives (every eighth id) take consecutive tiles, which share operand
// rows and columns in that XCD's L2.
// --------------------------------------------------------------------------
static constexpr int kBT = 2 * kGemmTile;  // 128
static constexpr int kBK = 16;             // summed entries per chunk
static constexpr int kBKP = 20;            // LDS pitch of a row (column) of a chunk, floats
static constexpr int kBCP = kBT + 1;       // epilogue pitch
static constexpr int kBBuf = 2 * kBT * kBKP;  // floats of one buffer (A rows, then B columns)
static constexpr int kBSOff = 1024;        // largest summed set whose offsets are staged in LDS

__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void *base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)0xffffffff, 0x00020000);
}

// one FP32 word per lane at byte offset row + lane (the builtin returns the raw bits)
__device__ __forceinline__ float ld_row(__amdgpu_buffer_rsrc_t r, int lane_off, int row_off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, lane_off, row_off, 0));
}

// P2 (X and Y summed-fast, their stride-1 summed label of two values):
// each thread reads an adjacent pair of summed entries with one 8-byte load
// (row or column (t >> 3) + 32 q, summed entries 2 (t % 8) and the next)
template <bool XS, bool YN, bool ST, bool P2 = false>
__device__ __forceinline__ void gemm_big_body(const ContractArgs &a, const int b, const uint32_t blk,
                                              const uint32_t nblk) {
  static_assert(!P2 || (XS && !YN && ST), "pair loads: both operands summed-fast, offsets staged");
  __shared__ int32_t oMX[kBT], oMZ[kBT], oNY[kBT], oNZ[kBT];
  __shared__ int32_t sOX[ST ? kBSOff : 1], sOY[ST ? kBSOff : 1];
  __shared__ __align__(16) float AB[2 * kBBuf];
  __shared__ int ksh[2];
  static_assert(64 * kBCP <= 2 * kBBuf, "half of the epilogue tile fits the operand buffers");
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const uint32_t tile = (nblk & 7u) == 0 ? (blk & 7u) * (nblk >> 3) + (blk >> 3) : blk;
  const uint32_t tm = (a.nM + kBT - 1) / kBT, tn = (a.nC + kBT - 1) / kBT;
  uint32_t bt, mt, nt;
  dense_tile(tile, tm, tn, a.nBlo, bt, mt, nt);
  const uint32_t m0 = mt * kBT, n0 = nt * kBT;
  const int32_t xb = tab_off(a.gbX, bt, a.nBl), yb = tab_off(a.gbY, bt, a.nBl), zb = tab_off(a.gbZ, bt, a.nBl);
  // operands through buffer resources (each operand below 2^30 entries:
  // 32-bit byte offsets)
  const __amdgpu_buffer_rsrc_t rX = raw_rsrc(a.X + (int64_t)b * a.bsX + xb);
  const __amdgpu_buffer_rsrc_t rY = raw_rsrc(a.Y + (int64_t)b * a.bsY + yb);
  gfloat *__restrict__ Z = (gfloat *)(a.Z + (int64_t)b * a.bsZ + zb);
  const uint32_t nS = a.nS;
  // prologue: row offsets (waves 0, 1), column offsets and the operands'
  // exponents (waves 2, 3), the summed entries' offsets (all)
  if (t < kBT) {
    const uint32_t m = m0 + t;
    oMX[t] = m < a.nM ? tab_off(a.gmX, m, a.nMl) : -1;
    oMZ[t] = m < a.nM ? tab_off(a.gmZ, m, a.nMl) : -1;
  } else {
    const uint32_t n = n0 + (t - kBT);
    oNY[t - kBT] = n < a.nC ? tab_off(a.cY, n, a.nCl) : -1;
    oNZ[t - kBT] = n < a.nC ? tab_off(a.cZ, n, a.nCl) : -1;
    const int slot = w == 2 ? a.slotX + (a.batX ? b : 0) : a.slotY + (a.batY ? b : 0);
    const int k = max_exponent(read_max(a.mx, a.mx_stride, slot));
    if (l == 0) ksh[w - 2] = k;
  }
  if (ST)
    for (uint32_t s = t; s < nS; s += kBlock) {
      sOX[s] = tab_off(a.sX, s, a.nSl) * 4;
      sOY[s] = tab_off(a.sY, s, a.nSl) * 4;
    }
  __syncthreads();
  const int kx = ksh[0], ky = ksh[1];
  const float sx = ldexpf(1.f, -kx), sy = ldexpf(1.f, -ky);
  // 8 entries of each operand per thread and chunk, consecutive threads on
  // the operand's stride-1 label: summed-fast A takes (row t / 16 + 16 q,
  // summed t % 16), row-fast A (row t % 128, summed t / 128 + 2 q); B alike.
  // Row (column) byte offsets are fixed per thread; rows past the operand
  // read its entry 0 and are masked at the LDS store.
  constexpr int NQ = kBT * kBK / kBlock;
  constexpr int NL = P2 ? NQ / 2 : NQ;  // loads per operand and chunk
  const int kA0 = XS ? (P2 ? 2 * (t & 7) : (t & 15)) : (t >> 7);
  const int kB0 = YN ? (t >> 7) : (P2 ? 2 * (t & 7) : (t & 15));
  auto rowA = [&](int q) { return XS ? (P2 ? (t >> 3) + 32 * q : (t >> 4) + 16 * q) : (t & 127); };
  auto sumA = [&](int q) { return XS ? kA0 : kA0 + 2 * q; };
  auto colB = [&](int q) { return YN ? (t & 127) : (P2 ? (t >> 3) + 32 * q : (t >> 4) + 16 * q); };
  auto sumB = [&](int q) { return YN ? kB0 + 2 * q : kB0; };
  int32_t oa[XS ? NL : 1], ob[YN ? 1 : NL];
  uint32_t live = 0;  // bit q: A entry q's row exists; bit NQ + q: B entry q's column
#pragma unroll
  for (int q = 0; q < (XS ? NL : 1); ++q) {
    const int32_t o = oMX[rowA(q)];
    oa[q] = o >= 0 ? o * 4 : 0;
  }
#pragma unroll
  for (int q = 0; q < (YN ? 1 : NL); ++q) {
    const int32_t o = oNY[colB(q)];
    ob[q] = o >= 0 ? o * 4 : 0;
  }
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    live |= (oMX[rowA(q)] >= 0 ? 1u : 0u) << q;
    live |= (oNY[colB(q)] >= 0 ? 1u : 0u) << (q + NQ);
  }
  auto sx_off = [&](uint32_t s) { return ST ? sOX[s] : tab_off(a.sX, s, a.nSl) * 4; };
  auto sy_off = [&](uint32_t s) { return ST ? sOY[s] : tab_off(a.sY, s, a.nSl) * 4; };
  // raw values stay untouched until their LDS store, so that the loads of
  // later chunks stay in flight during this chunk's products; summed
  // entries past nS read entry 0 and are masked at the store
  auto load_chunk = [&](uint32_t s0, float (&ra)[NQ], float (&rb)[NQ]) {
    const uint32_t sa = s0 + kA0, sb = s0 + kB0;
    const int32_t oxc = XS ? sx_off(sa < nS ? sa : 0u) : 0, oyc = YN ? 0 : sy_off(sb < nS ? sb : 0u);
    if (P2) {  // entries 2q, 2q + 1: an adjacent pair
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const auto va = __builtin_amdgcn_raw_buffer_load_b64(rX, oa[q] + oxc, 0, 0);
        const auto vb = __builtin_amdgcn_raw_buffer_load_b64(rY, ob[q] + oyc, 0, 0);
        ra[2 * q] = __uint_as_float(va[0]);
        ra[2 * q + 1] = __uint_as_float(va[1]);
        rb[2 * q] = __uint_as_float(vb[0]);
        rb[2 * q + 1] = __uint_as_float(vb[1]);
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const uint32_t s = s0 + sumA(q), s2 = s0 + sumB(q);
      const int32_t ox = XS ? oa[q] + oxc : oa[0] + sx_off(s < nS ? s : 0u);
      const int32_t oy = YN ? ob[0] + sy_off(s2 < nS ? s2 : 0u) : ob[q] + oyc;
      ra[q] = ld_row(rX, ox, 0);
      rb[q] = ld_row(rY, oy, 0);
    }
  };
  f32x4 acc[4][4] = {};
  const int wm = w & 1, wn = w >> 1, g = l >> 4, li = l & 15;
  const bool full_rows = P2 || live == (1u << (2 * NQ)) - 1u;
  // chunk c: its raw values (loaded two chunks ahead, register set c % 2)
  // go to LDS buffer c % 2, then the loads of chunk c + 2 are issued, then
  // the products of chunk c run
  auto step = [&](uint32_t s0, uint32_t c, float (&ra)[NQ], float (&rb)[NQ]) {
    float *As = AB + (c & 1u) * kBBuf, *Bs = As + kBT * kBKP;
    if (P2) {
      const bool in = s0 + kA0 < nS;  // the pair (nS even)
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const bool va = (live >> q & 1u) && in, vb = (live >> (q + NQ) & 1u) && in;
        As[rowA(q) * kBKP + kA0] = va ? ra[2 * q] * sx : 0.f;
        As[rowA(q) * kBKP + kA0 + 1] = va ? ra[2 * q + 1] * sx : 0.f;
        Bs[colB(q) * kBKP + kB0] = vb ? rb[2 * q] * sy : 0.f;
        Bs[colB(q) * kBKP + kB0 + 1] = vb ? rb[2 * q + 1] * sy : 0.f;
      }
    } else if (full_rows && s0 + kBK <= nS) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        As[rowA(q) * kBKP + sumA(q)] = ra[q] * sx;
        Bs[colB(q) * kBKP + sumB(q)] = rb[q] * sy;
      }
    } else {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const bool va = (live >> q & 1u) && s0 + sumA(q) < nS, vb = (live >> (q + NQ) & 1u) && s0 + sumB(q) < nS;
        As[rowA(q) * kBKP + sumA(q)] = va ? ra[q] * sx : 0.f;
        Bs[colB(q) * kBKP + sumB(q)] = vb ? rb[q] * sy : 0.f;
      }
    }
    __syncthreads();
    if (s0 + 2 * kBK < nS) load_chunk(s0 + 2 * kBK, ra, rb);
    f32x4 av[4], bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      av[i] = *(const f32x4 *)&As[(64 * wm + 16 * i + li) * kBKP + 4 * g];
      bv[i] = *(const f32x4 *)&Bs[(64 * wn + 16 * i + li) * kBKP + 4 * g];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i][j], bv[jj][j], acc[i][jj], 0, 0, 0);
  };
  float ra0[NQ], rb0[NQ], ra1[NQ], rb1[NQ];
  load_chunk(0, ra0, rb0);
  if (kBK < nS) load_chunk(kBK, ra1, rb1);
  for (uint32_t s0 = 0, c = 0; s0 < nS; s0 += 2 * kBK, c += 2) {
    step(s0, c, ra0, rb0);
    if (s0 + kBK < nS) step(s0 + kBK, c + 1, ra1, rb1);
  }
  // epilogue: two halves of 64 rows through LDS
  float lmax = 0.f;
  float *Cs = AB;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __syncthreads();  // the operand buffers (or the previous half) are no longer read
    if (wm == h) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            Cs[(16 * i + 4 * g + r) * kBCP + 64 * wn + 16 * jj + li] = acc[i][jj][r];
    }
    __syncthreads();
#pragma unroll 4
    for (int q = 0; q < 64 * kBT / kBlock; ++q) {
      const int e = t + q * kBlock;
      int m, n;
      if (a.z_n_fast) { n = e % kBT; m = e / kBT; } else { m = e % 64; n = e / 64; }
      const int32_t om = oMZ[64 * h + m], on = oNZ[n];
      if (om >= 0 && on >= 0) {
        const float v = Cs[m * kBCP + n];
        Z[om + on] = v;
        lmax = fmaxf(lmax, v);
      }
    }
  }
  block_record_max(lmax, a.mx + (blk % kMaxSub) * a.mx_stride + a.slotZ + (a.batZ ? b : 0));
  if (blk == 0 && threadIdx.x == 0)
    a.ex[a.slotZ + (a.batZ ? b : 0)] = a.ex[a.slotX + (a.batX ? b : 0)] + kx + a.ex[a.slotY + (a.batY ? b : 0)] + ky;
}

// three workgroups per CU (LDS holds three; registers capped to match)
template <bool XS, bool YN, bool ST, bool P2 = false>
__global__ __launch_bounds__(kBlock, 3) void k_gemm_big(const ContractArgs *__restrict__ ap) {
  gemm_big_body<XS, YN, ST, P2>(*ap, blockIdx.y, blockIdx.x, gridDim.x);
}

// --------------------------------------------------------------------------
// interleaved-instance form (batched evidence).  Element e of instance b of
// a batched tensor sits at e * es + b, so one wavefront computes the same
// output elements for 64 consecutive instances (lane = instance): every
// offset is uniform across the wave and lives in scalar registers, every
// operand load and output store is one contiguous 256-byte row, and each lane
// carries its own instance's scale.  A wave owns tiles of TM rows (M labels)
// x TN columns within one batch-label assignment: per summed entry it loads
// TM rows of X and TN rows of Y and does TM x TN multiply-adds (or max-plus
// candidates).  Operand rows are read with buffer loads: the row's byte
// offset is a scalar operand and the lane's offset a constant vector
// register, so addressing costs no vector instructions.  The summed entries'
// offsets are fetched 64 at a time, one per lane, and broadcast with
// readlane; tile offsets likewise.  Edge tiles repeat their last row /
// column (loads stay in bounds, the copies are never stored), so the inner
// loop has no branches; it is software-pipelined (the rows of the next one
// or two summed entries are loaded while the current ones are multiplied).  Tile variants (a.tile): 0 = 4 x 4, 1 = 8 x 8, 2 = 16 x 1.  With
// ksplit = 4 (4 x 4 tiles) the four waves of a workgroup share one tile and
// split the summed range in four consecutive parts, folded in wave order
// through LDS (deterministic; for max-plus the earlier part wins ties, which
// keeps the first maximiser).
// --------------------------------------------------------------------------
static constexpr int kIT = kInterTile;

__device__ __forceinline__ int32_t bcast(int32_t v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// raw buffer over a tensor (no range limit: every offset is in bounds by
// construction); word 3 as for all gfx9 parts

template <int TM, int TN>
struct InterShared {
  float v[kBlock / 64 - 1][TM * TN][64];
  int32_t i[kBlock / 64 - 1][TM * TN][64];
};

template <int SEMI, bool HASY, int TM, int TN0, bool SPLIT>
__device__ __forceinline__ void inter_tiles(const ContractArgs &a, const int slab, const uint32_t blk,
                                            const uint32_t nblk) {
  constexpr int TN = HASY ? TN0 : 1;  // without Y there are no column labels
  constexpr int NW = kBlock / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = slab * kInterLanes + lane;
  // uniform bases at this group's first instance; the lane offset is a constant
  const __amdgpu_buffer_rsrc_t rX = raw_rsrc(a.X + (int64_t)slab * kInterLanes * a.bsX);
  const __amdgpu_buffer_rsrc_t rY = raw_rsrc(HASY ? a.Y + (int64_t)slab * kInterLanes * a.bsY : a.X);
  const int vx = lane * 4 * (int)a.bsX, vy = HASY ? lane * 4 * (int)a.bsY : 0;
  const int esX = a.esX * 4, esY = HASY ? a.esY * 4 : 0;  // bytes per element
  gfloat *__restrict__ Zp = (gfloat *)a.Z;
  gint_w *__restrict__ Ip = (gint_w *)a.I;
  const int64_t esZ = a.esZ;
  // operand maxima (one word per lane for batched operands) and, for the
  // wave that writes the output exponent, the operands' exponents: issued
  // here, first used after the first tile's offset loads are in flight
  uint32_t mxX = 0, mxY = 0;
  int exX = 0, exY = 0;
  const bool ex_writer = SEMI == SEMI_SUM && blk == 0 && w == 0;
  if (SEMI == SEMI_SUM) {
    mxX = a.batX ? ((gu32 *)a.mx)[a.slotX + b] : read_max(a.mx, a.mx_stride, a.slotX);
    if (HASY) mxY = a.batY ? ((gu32 *)a.mx)[a.slotY + b] : read_max(a.mx, a.mx_stride, a.slotY);
    if (ex_writer) {
      exX = ((gint *)a.ex)[a.slotX + (a.batX ? b : 0)];
      if (HASY) exY = ((gint *)a.ex)[a.slotY + (a.batY ? b : 0)];
    }
  }
  float sx = 1.f, sy = 1.f;
  int kx = 0, ky = 0;
  bool scaled = false;
  const uint32_t nM = a.nM, nC = a.nC, nS = a.nS, nSl = a.nSl;
  const uint32_t tm = (nM + TM - 1) / TM, tn = (nC + TN - 1) / TN;
  const uint32_t ntiles = a.nB * tm * tn;
  const bool split = SPLIT && a.ksplit > 1;
  uint32_t sb = 0, se = nS;
  if (split) {
    const uint32_t per = (nS + NW - 1) / NW;
    sb = min(nS, w * per);
    se = min(nS, sb + per);
  }
  const uint32_t t0 = split ? blk : blk * NW + w, tstep = split ? nblk : nblk * NW;
  float lmax = 0.f;
  for (uint32_t t = t0; t < ntiles; t += tstep) {
    const uint32_t bt = t / (tm * tn), rem = t - bt * tm * tn;
    const uint32_t mt = rem / tn, nt = rem - mt * tn;
    const uint32_t m0 = mt * TM, n0 = nt * TN;
    const int mi = (int)min((uint32_t)TM, nM - m0), nj = (int)min((uint32_t)TN, nC - n0);
    // tile offsets: lanes 0..TM-1 rows, 32..32+TN-1 columns, 63 the batch labels
    int32_t v0 = 0, v1 = 0, v2 = 0;
    if (lane < mi) {
      v0 = tab_off(a.gmX, m0 + lane, a.nMl);
      v1 = tab_off(a.gmZ, m0 + lane, a.nMl);
    } else if (lane >= 32 && lane < 32 + nj) {
      v0 = HASY ? tab_off(a.cY, n0 + lane - 32, a.nCl) : 0;
      v1 = tab_off(a.cZ, n0 + lane - 32, a.nCl);
    } else if (lane == 63) {
      v0 = tab_off(a.gbX, bt, a.nBl);
      v1 = HASY ? tab_off(a.gbY, bt, a.nBl) : 0;
      v2 = tab_off(a.gbZ, bt, a.nBl);
    }
    if (SEMI == SEMI_SUM && !scaled) {
      kx = max_exponent(mxX);
      sx = ldexpf(1.f, -kx);
      if (HASY) {
        ky = max_exponent(mxY);
        sy = ldexpf(1.f, -ky);
      }
      scaled = true;
    }
    const int32_t xb = bcast(v0, 63), yb = bcast(v1, 63), zb = bcast(v2, 63);
    int32_t xm[TM], zm[TM], yn[TN], zn[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int ii = i < mi ? i : mi - 1;
      xm[i] = xb + bcast(v0, ii);
      zm[i] = zb + bcast(v1, ii);
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int jj = j < nj ? j : nj - 1;
      yn[j] = yb + bcast(v0, 32 + jj);
      zn[j] = bcast(v1, 32 + jj);
    }
    float acc[TM][TN];
    int32_t arg[SEMI == SEMI_MAX ? TM : 1][SEMI == SEMI_MAX ? TN : 1];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        acc[i][j] = SEMI == SEMI_SUM ? 0.f : -INFINITY;
        if (SEMI == SEMI_MAX) arg[i][j] = 0;
      }
    auto step = [&](int32_t xs, int32_t ys, int32_t s) {
      float xv[TM], yv[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) xv[i] = ld_row(rX, vx, (xm[i] + xs) * esX);
#pragma unroll
      for (int j = 0; j < TN; ++j) yv[j] = HASY ? ld_row(rY, vy, (yn[j] + ys) * esY) : 0.f;
      if (SEMI == SEMI_SUM) {
#pragma unroll
        for (int i = 0; i < TM; ++i) xv[i] *= sx;
#pragma unroll
        for (int j = 0; j < TN; ++j) yv[j] *= sy;
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          if (SEMI == SEMI_SUM) {
            if (HASY) acc[i][j] = fmaf(xv[i], yv[j], acc[i][j]);
            else acc[i][j] += xv[i];
          } else {
            const float v = HASY ? xv[i] + yv[j] : xv[i];
            if (s == 0 || v > acc[i][j]) {
              acc[i][j] = v;
              arg[i][j] = s;
            }
          }
        }
    };
    for (uint32_t s0 = sb; s0 < se; s0 += 64) {
      int32_t ox = 0, oy = 0;
      if (s0 + lane < se) {
        ox = tab_off(a.sX, s0 + lane, nSl);
        if (HASY) oy = tab_off(a.sY, s0 + lane, nSl);
      }
      const int cnt = (int)min(64u, se - s0);
      // software pipeline over groups of G summed entries: the rows of the
      // next group are in flight while the current group is multiplied
      constexpr int G = TM * TN >= 64 ? 1 : 2;
      float xa[G][TM], ya[G][TN], xb2[G][TM], yb2[G][TN];
      auto load = [&](float (&xv)[G][TM], float (&yv)[G][TN], int k) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int32_t xs = bcast(ox, k + g), ys = HASY ? bcast(oy, k + g) : 0;
#pragma unroll
          for (int i = 0; i < TM; ++i) xv[g][i] = ld_row(rX, vx, (xm[i] + xs) * esX);
#pragma unroll
          for (int j = 0; j < TN; ++j) yv[g][j] = HASY ? ld_row(rY, vy, (yn[j] + ys) * esY) : 0.f;
        }
      };
      auto compute = [&](float (&xv)[G][TM], float (&yv)[G][TN], int32_t s) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          if (SEMI == SEMI_SUM) {
#pragma unroll
            for (int i = 0; i < TM; ++i) xv[g][i] *= sx;
#pragma unroll
            for (int j = 0; j < TN; ++j) yv[g][j] *= sy;
          }
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
              if (SEMI == SEMI_SUM) {
                if (HASY) acc[i][j] = fmaf(xv[g][i], yv[g][j], acc[i][j]);
                else acc[i][j] += xv[g][i];
              } else {
                const float v = HASY ? xv[g][i] + yv[g][j] : xv[g][i];
                if (s + g == 0 || v > acc[i][j]) {
                  acc[i][j] = v;
                  arg[i][j] = s + g;
                }
              }
            }
        }
      };
      const int ng = cnt / G;
      if (ng > 0) {
        load(xa, ya, 0);
        int q = 0;
        for (; q + 2 <= ng; q += 2) {
          load(xb2, yb2, (q + 1) * G);
          compute(xa, ya, (int32_t)(s0 + q * G));
          if (q + 2 < ng) load(xa, ya, (q + 2) * G);
          compute(xb2, yb2, (int32_t)(s0 + (q + 1) * G));
        }
        if (q < ng) compute(xa, ya, (int32_t)(s0 + q * G));
      }
      for (int k = ng * G; k < cnt; ++k) step(bcast(ox, k), HASY ? bcast(oy, k) : 0, (int32_t)(s0 + k));
    }
    if (SPLIT && split) {
      __shared__ InterShared<TM, TN> red;
      if (w > 0) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            red.v[w - 1][i * TN + j][lane] = acc[i][j];
            if (SEMI == SEMI_MAX) red.i[w - 1][i * TN + j][lane] = arg[i][j];
          }
      }
      __syncthreads();
      if (w == 0) {
        for (int q = 0; q < NW - 1; ++q)
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
              const float v = red.v[q][i * TN + j][lane];
              if (SEMI == SEMI_SUM) {
                acc[i][j] += v;
              } else if (v > acc[i][j]) {
                acc[i][j] = v;
                arg[i][j] = red.i[q][i * TN + j][lane];
              }
            }
      }
      __syncthreads();
      if (w > 0) continue;
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        if (i < mi && j < nj) {
          const int64_t zo = (int64_t)(zm[i] + zn[j]) * esZ;
          Zp[zo + b] = acc[i][j];
          if (SEMI == SEMI_SUM) lmax = fmaxf(lmax, acc[i][j]);
          else Ip[zo + b] = arg[i][j];
        }
  }
  if (SEMI == SEMI_SUM) {
    // this wave's maximum per instance, recorded in sub-slot 0 of the
    // instance's slot; with many waves per group of instances the atomic is
    // skipped where the stored maximum is already larger (maxima only grow
    // within a launch)
    uint32_t *slot = a.mx + a.slotZ + b;
    const bool guard = tstep > 16;
    if (lmax > 0.f && (!guard || __uint_as_float(*(volatile uint32_t *)slot) < lmax))
      atomicMax(slot, __float_as_uint(lmax));
    if (ex_writer) {
      if (!scaled) {
        kx = max_exponent(mxX);
        ky = HASY ? max_exponent(mxY) : 0;
      }
      ((gint_w *)a.ex)[a.slotZ + b] = exX + kx + (HASY ? exY + ky : 0);
    }
  }
}

template <int SEMI, bool HASY>
__device__ __forceinline__ void inter_body(const ContractArgs &a, const int slab, const uint32_t blk,
                                           const uint32_t nblk) {
  if (SEMI == SEMI_SUM && a.tile == 1) inter_tiles<SEMI, HASY, 8, 8, false>(a, slab, blk, nblk);
  else if (SEMI == SEMI_SUM && a.tile == 2) inter_tiles<SEMI, HASY, 16, 1, false>(a, slab, blk, nblk);
  else inter_tiles<SEMI, HASY, kIT, kIT, true>(a, slab, blk, nblk);
}

// Workgroups of a launch go to the XCDs in turn (workgroup id modulo 8), so
// the id is decoded group-of-instances fastest: with 8 (or a multiple of 8)
// groups every workgroup of one group of 64 instances lands on the same XCD
// and the tiles that share operand rows share that XCD's L2.
template <int SEMI, bool HASY>
__global__ __launch_bounds__(kBlock) void k_inter(const ContractArgs *__restrict__ ap) {
  const ContractArgs &a = *ap;
  const uint32_t ns = (uint32_t)a.nslab;
  inter_body<SEMI, HASY>(a, (int)(blockIdx.x % ns), blockIdx.x / ns, gridDim.x / ns);
}

// Arguments live in device memory (a pointer is the only kernel argument):
// large by-value argument blocks cost microseconds per launch.
template <int SEMI, bool HASY>
__global__ __launch_bounds__(kBlock) void k_map(const ContractArgs *__restrict__ ap) {
  any_map_body<SEMI, HASY>(*ap, blockIdx.y, blockIdx.x, gridDim.x);
}
// the batch-uniform row form runs in launches of its own (its registers
// would lower the occupancy of the other map forms)
template <int BS, int BC>
__global__ __launch_bounds__(kBlock) void k_rowsb(const ContractArgs *__restrict__ ap) {
  rowsb_body<BS, BC>(*ap, blockIdx.y, xcd_tile(blockIdx.x, gridDim.x), gridDim.x);
}
__global__ __launch_bounds__(kBlock) void k_mpair(const ContractArgs *__restrict__ ap) {
  mpair_body(*ap, blockIdx.x, gridDim.x);
}
template <int SEMI, bool HASY>
__global__ __launch_bounds__(kBlock) void k_split(const ContractArgs *__restrict__ ap) {
  split_body<SEMI, HASY>(*ap, blockIdx.y, blockIdx.x);
}
template <int SEMI, bool HASY>
__global__ __launch_bounds__(kBlock) void k_split_finish(const ContractArgs *__restrict__ ap) {
  finish_body<SEMI, HASY>(*ap, blockIdx.y, blockIdx.x);
}

// Several independent contractions in one launch (one stage of the tree
// schedule).  Workgroup x runs contraction tab[x].op, its workgroup
// tab[x].local, split as instance-major (b, blk) with nblk[op] workgroups per
// instance: one read of a table built at plan time (a search over the ops'
// block ranges cost a chain of dependent loads, up to 12 on a launch of
// 760 leaf products).

template <int SEMI, int PHASE>
__global__ __launch_bounds__(kBlock) void k_group(const ContractArgs *__restrict__ ops,
                                                  const GroupBlock *__restrict__ tab,
                                                  const uint32_t *__restrict__ nblk, int n) {
  const GroupBlock e = tab[blockIdx.x];
  const int i = (int)e.op;
  const ContractArgs &a = ops[i];
  const uint32_t local = e.local;
  const uint32_t per = nblk[i];
  const bool hy = a.Y != nullptr;
  if (PHASE == 6) {  // interleaved form: group of 64 instances fastest (see k_inter)
    const uint32_t ns = (uint32_t)a.nslab;
    if (hy) inter_body<SEMI, true>(a, (int)(local % ns), local / ns, per);
    else inter_body<SEMI, false>(a, (int)(local % ns), local / ns, per);
    return;
  }
  const int b = (int)(local / per);
  const uint32_t blk = local - (uint32_t)b * per;
  if (PHASE == 7) {  // pairs of max-plus contractions (one instance)
    mpair_body(a, blk, per);
    return;
  }
  if (PHASE == 0) {
    if (hy) any_map_body<SEMI, true>(a, b, blk, per);
    else any_map_body<SEMI, false>(a, b, blk, per);
  } else if (PHASE == 1) {
    if (hy) split_body<SEMI, true>(a, b, blk);
    else split_body<SEMI, false>(a, b, blk);
  } else if (PHASE >= 3 && PHASE <= 5) {  // dense form (sum-product: operand precision PHASE - 3)
    if (SEMI == SEMI_MAX) gemm_max_body(a, b, blk);
    else gemm_body<PHASE - 3>(a, b, blk);
  } else {
    if (hy) finish_body<SEMI, true>(a, b, blk);
    else finish_body<SEMI, false>(a, b, blk);
  }
}

void launch_group(int semi, int phase, const ContractArgs *ops, const GroupBlock *start, const uint32_t *nblk,
                  int n, uint32_t total_blocks, void *stream) {
  if (n <= 0 || total_blocks == 0) return;
  hipStream_t s = (hipStream_t)stream;
  dim3 g(total_blocks);
  if (phase == 6) {
    if (semi == SEMI_SUM) k_group<SEMI_SUM, 6><<<g, kBlock, 0, s>>>(ops, start, nblk, n);
    else k_group<SEMI_MAX, 6><<<g, kBlock, 0, s>>>(ops, start, nblk, n);
    return;
  }
  if (phase == 7) {  // pairs of max-plus contractions
    k_group<SEMI_MAX, 7><<<g, kBlock, 0, s>>>(ops, start, nblk, n);
    return;
  }
  if (phase >= 3 && semi == SEMI_MAX) {  // dense max-plus form
    k_group<SEMI_MAX, 3><<<g, kBlock, 0, s>>>(ops, start, nblk, n);
    return;
  }
  if (phase >= 3) {  // dense form (sum-product), operand precision phase - 3
    if (phase == 4) k_group<SEMI_SUM, 4><<<g, kBlock, 0, s>>>(ops, start, nblk, n);
    else if (phase == 5) k_group<SEMI_SUM, 5><<<g, kBlock, 0, s>>>(ops, start, nblk, n);
    else k_group<SEMI_SUM, 3><<<g, kBlock, 0, s>>>(ops, start, nblk, n);
    return;
  }
  if (semi == SEMI_SUM) {
    if (phase == 0) k_group<SEMI_SUM, 0><<<g, kBlock, 0, s>>>(ops, start, nblk, n);
    else if (phase == 1) k_group<SEMI_SUM, 1><<<g, kBlock, 0, s>>>(ops, start, nblk, n);
    else k_group<SEMI_SUM, 2><<<g, kBlock, 0, s>>>(ops, start, nblk, n);
  } else {
    if (phase == 0) k_group<SEMI_MAX, 0><<<g, kBlock, 0, s>>>(ops, start, nblk, n);
    else if (phase == 1) k_group<SEMI_MAX, 1><<<g, kBlock, 0, s>>>(ops, start, nblk, n);
    else k_group<SEMI_MAX, 2><<<g, kBlock, 0, s>>>(ops, start, nblk, n);
  }
}

uint32_t map_blocks(const ContractArgs &a) {
  if (a.kind == 4) {  // one tile per wave (split: per workgroup), grid-stride beyond 256 workgroups
    const uint32_t TM = a.tile == 1 ? 8 : (a.tile == 2 ? 16 : kIT), TN = a.tile == 1 ? 8 : (a.tile == 2 ? 1 : kIT);
    const uint32_t tn = a.Y ? (a.nC + TN - 1) / TN : 1;
    const uint32_t tiles = a.nB * ((a.nM + TM - 1) / TM) * tn;
    const uint32_t blocks = a.ksplit > 1 ? tiles : (tiles + kBlock / 64 - 1) / (kBlock / 64);
    return blocks > 256u ? 256u : blocks;
  }
  if (a.kind == 2 && a.tile == 1)  // one 128 x 128 tile per workgroup
    return a.nB * ((a.nM + kBT - 1) / kBT) * ((a.nC + kBT - 1) / kBT);
  if (a.kind == 2)  // one 64 x 64 tile per workgroup
    return a.nB * ((a.nM + kGT - 1) / kGT) * ((a.nC + kGT - 1) / kGT);
  if (a.kind == kKindMaxPair) {  // one lane per row
    const uint32_t blocks = (a.nR + kBlock - 1) / kBlock;
    return blocks > 65536u ? 65536u : blocks;
  }
  if (a.kind == 1 && a.tile == 1) {  // one pass per wavefront of 64 M assignments of one batch assignment
    const uint64_t waves = (uint64_t)a.nB * ((a.nM + 63) / 64);
    const uint64_t blocks = (waves + kBlock / 64 - 1) / (kBlock / 64);
    return blocks > (1u << 20) ? (1u << 20) : (uint32_t)blocks;
  }
  const uint32_t n_out = a.kind == 1 ? a.nR : a.nR * a.nC;
  if (a.kind == 3) {  // kWaveOuts outputs per workgroup pass
    const uint32_t blocks = (n_out + kWaveOuts - 1) / kWaveOuts;
    return blocks > 4096u ? 4096u : blocks;
  }
  uint32_t blocks = (n_out + kBlock - 1) / kBlock;
  // Grid-stride launches of about 8 workgroups per CU, except over many
  // outputs (>= 2^22), where one pass per lane (four rows per lane in the
  // row form, four outputs per lane in the generic form) leaves the overlap
  // of memory latency to the hardware's wave dispatch: measured on
  // 2^24..2^27-row contractions, a long grid-stride loop per wave ran at
  // 1.3-1.6 TB/s, one pass per lane 1.7-2.2 TB/s.
  if (n_out >= (1u << 22)) return (blocks + 3) / 4;  // the row form's rows, the generic form's kMapU outputs
  return blocks > 2048u ? 2048u : blocks;
}

void launch_contract(int semi, bool has_y, bool split, const ContractArgs &a, const ContractArgs *d_a, int nb,
                     void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const uint32_t n_out = a.nR * a.nC;
  if (a.kind == 4) {  // nb: groups of 64 instances
    const dim3 g(map_blocks(a) * nb);
    if (semi == SEMI_SUM) {
      if (has_y) k_inter<SEMI_SUM, true><<<g, kBlock, 0, s>>>(d_a);
      else k_inter<SEMI_SUM, false><<<g, kBlock, 0, s>>>(d_a);
    } else {
      if (has_y) k_inter<SEMI_MAX, true><<<g, kBlock, 0, s>>>(d_a);
      else k_inter<SEMI_MAX, false><<<g, kBlock, 0, s>>>(d_a);
    }
    return;
  }
  if (a.kind == 2 && a.tile == 1) {  // large tiles: FP32 sum-product only
    const dim3 g(map_blocks(a), nb);
    const bool st = a.nS <= (uint32_t)kBSOff;  // summed offsets staged in LDS
    if (a.x_s_fast && a.y_n_fast) {
      if (st) k_gemm_big<true, true, true><<<g, kBlock, 0, s>>>(d_a);
      else k_gemm_big<true, true, false><<<g, kBlock, 0, s>>>(d_a);
    } else if (a.x_s_fast) {
      if (st && a.s_pair) k_gemm_big<true, false, true, true><<<g, kBlock, 0, s>>>(d_a);
      else if (st) k_gemm_big<true, false, true><<<g, kBlock, 0, s>>>(d_a);
      else k_gemm_big<true, false, false><<<g, kBlock, 0, s>>>(d_a);
    } else if (a.y_n_fast) {
      if (st) k_gemm_big<false, true, true><<<g, kBlock, 0, s>>>(d_a);
      else k_gemm_big<false, true, false><<<g, kBlock, 0, s>>>(d_a);
    } else {
      if (st) k_gemm_big<false, false, true><<<g, kBlock, 0, s>>>(d_a);
      else k_gemm_big<false, false, false><<<g, kBlock, 0, s>>>(d_a);
    }
    return;
  }
  if (a.kind == 2) {
    const dim3 g(map_blocks(a), nb);
    if (semi == SEMI_MAX) k_gemm_max<<<g, kBlock, 0, s>>>(d_a);
    else if (a.prec == 1) k_gemm<1><<<g, kBlock, 0, s>>>(d_a);
    else if (a.prec == 2) k_gemm<2><<<g, kBlock, 0, s>>>(d_a);
    else k_gemm<0><<<g, kBlock, 0, s>>>(d_a);
    return;
  }
  if (a.kind == kKindMaxPair) {
    k_mpair<<<map_blocks(a), kBlock, 0, s>>>(d_a);
    return;
  }
  if (a.kind == 1 && a.tile == 1) {  // batch-uniform row form: sum-product with Y
    const dim3 g(map_blocks(a), nb);
    if (a.ns <= 4 && a.nc <= 8) k_rowsb<4, 8><<<g, kBlock, 0, s>>>(d_a);
    else if (a.ns <= 4 && a.nc <= 16) k_rowsb<4, 16><<<g, kBlock, 0, s>>>(d_a);
    else if (a.ns <= 4) k_rowsb<4, 32><<<g, kBlock, 0, s>>>(d_a);
    else if (a.ns <= 8 && a.nc <= 8) k_rowsb<8, 8><<<g, kBlock, 0, s>>>(d_a);
    else if (a.ns <= 8) k_rowsb<8, 16><<<g, kBlock, 0, s>>>(d_a);
    else if (a.ns <= 16) k_rowsb<16, 8><<<g, kBlock, 0, s>>>(d_a);
    else k_rowsb<32, 4><<<g, kBlock, 0, s>>>(d_a);
    return;
  }
  if (!split) {
    dim3 g(map_blocks(a), nb);  // grid-stride: at most about 8 blocks per CU
    if (semi == SEMI_SUM) {
      if (has_y) k_map<SEMI_SUM, true><<<g, kBlock, 0, s>>>(d_a);
      else k_map<SEMI_SUM, false><<<g, kBlock, 0, s>>>(d_a);
    } else {
      if (has_y) k_map<SEMI_MAX, true><<<g, kBlock, 0, s>>>(d_a);
      else k_map<SEMI_MAX, false><<<g, kBlock, 0, s>>>(d_a);
    }
    return;
  }
  dim3 g(a.n_chunks, nb);
  dim3 gf(n_out, nb);
  if (semi == SEMI_SUM) {
    if (has_y) {
      k_split<SEMI_SUM, true><<<g, kBlock, 0, s>>>(d_a);
      k_split_finish<SEMI_SUM, true><<<gf, kBlock, 0, s>>>(d_a);
    } else {
      k_split<SEMI_SUM, false><<<g, kBlock, 0, s>>>(d_a);
      k_split_finish<SEMI_SUM, false><<<gf, kBlock, 0, s>>>(d_a);
    }
  } else {
    if (has_y) {
      k_split<SEMI_MAX, true><<<g, kBlock, 0, s>>>(d_a);
      k_split_finish<SEMI_MAX, true><<<gf, kBlock, 0, s>>>(d_a);
    } else {
      k_split<SEMI_MAX, false><<<g, kBlock, 0, s>>>(d_a);
      k_split_finish<SEMI_MAX, false><<<gf, kBlock, 0, s>>>(d_a);
    }
  }
}


// --------------------------------------------------------------------------
// fused chain segments
// --------------------------------------------------------------------------

static constexpr int kSegThreads = 1024;          // 16 waves: enough in flight per CU to cover latency
static constexpr int kSweepThreads = 256;         // sweep kernels (one workgroup per segment)
static constexpr int kFinThreads = 1024;          // the adjoint sweep: its per-step loops span up to 32 x 32 entries
static constexpr int kSegOB = kSegOuterBlock;     // outer assignments per workgroup (32 per wave)
static constexpr int kSegRow = kSegOB + 1;        // padded LDS tile row: conflict-free in both directions

unsigned seg_blocks(const SegArgs &a) { return (a.nO + kSegOB - 1) / kSegOB; }

__device__ __forceinline__ int32_t outer_off(const Tab2 &t, uint32_t o, uint32_t nlo) {
  const uint32_t h = o / nlo;
  return t.hi[h] + t.lo[o - h * nlo];
}
__device__ __forceinline__ int32_t seg_outer(const SegArgs &a, const Tab2 &ot, uint32_t og) {
  if (a.ol_shift >= 0) return ot.hi[og >> a.ol_shift] + ot.lo[og & (a.nOl - 1)];
  return outer_off(ot, og, a.nOl);
}

// Offsets of the workgroup's outer assignments in the input and output
// carriers (-1 past nO) and of the local entries, staged in LDS once so that
// every element move below is a single independent global access.
static_assert(kSegThreads >= 2 * kSegOB, "one thread per outer offset of each carrier");
// Per-workgroup constants of a carrier kernel, staged in LDS by a prologue
// in which every thread makes at most two global reads and no location is
// read by more than one wave of the workgroup (a location read by every wave
// of every workgroup would serialise in one L2 channel): outer offsets of
// both carriers, local offsets, the composed map M (zero-padded to 32 x 32)
// and the exponents of the operands' maxima.
struct SegShared {
  int32_t offX[kSegOB], offZ[kSegOB], locX[kSegMaxLocal], locZ[kSegMaxLocal];
  float m[kSegMaxLocal * (kSegMaxLocal + 1)];
  int32_t kx, kg;
  int32_t exX, exG, exM;  // workgroup 0: the operands' exponents (for the output's exponent)
};

// M into LDS (zero-padded to 32 x 32), one entry per thread
__device__ __forceinline__ void seg_stage_m(const SegArgs &a, SegShared &sh) {
  const int t = threadIdx.x;
  const int r = t >> 5, c = t & 31;
  const float x = ((gcfloat *)(a.arena + a.M))[min(r, a.n_outL - 1) * a.n_in0 + min(c, a.n_in0 - 1)];
  sh.m[r * (kSegMaxLocal + 1) + c] = (r < a.n_outL && c < a.n_in0) ? x : 0.f;
}
static_assert(kSegThreads == kSegMaxLocal * kSegMaxLocal, "one M entry per thread");

// The rest of the prologue, by eight waves (wave index wv in 0..7 within
// them): outer offsets, local offsets, operand maxima, exponents.
__device__ __forceinline__ void seg_roles(const SegArgs &a, uint32_t blk, bool want_g, SegShared &sh, int wv) {
  const uint32_t o0 = blk * kSegOB;
  const int t = threadIdx.x;
  const int l = t & 63;
  if (wv < 4) {  // outer offsets: waves 0-1 the input carrier, 2-3 the output carrier
    const bool in = wv < 2;
    const int tt = t & (kSegOB - 1);
    const uint32_t og = o0 + tt, oc = min(og, a.nO - 1);
    gint *hi = (gint *)(in ? a.oX.hi : a.oZ.hi), *lo = (gint *)(in ? a.oX.lo : a.oZ.lo);
    int32_t oo;
    if (a.ol_shift >= 0) oo = hi[oc >> a.ol_shift] + lo[oc & (a.nOl - 1)];
    else oo = hi[oc / a.nOl] + lo[oc % a.nOl];
    (in ? sh.offX : sh.offZ)[tt] = og < a.nO ? oo : -1;
  } else if (wv == 4) {  // local offsets: lanes 0-31 input, 32-63 output
    const int j = l & 31;
    if (l < 32) {
      const int32_t v = ((gint *)a.inX)[min(j, a.n_in0 - 1)];
      if (j < a.n_in0) sh.locX[j] = v;
    } else {
      const int32_t v = ((gint *)a.outZ)[min(j, a.n_outL - 1)];
      if (j < a.n_outL) sh.locZ[j] = v;
    }
  } else if (wv == 5 || (wv == 6 && want_g)) {  // maxima of the operands (64 sub-slots)
    const int slot = wv == 5 ? a.slotX : a.slotG;
    const uint32_t v = ((gu32 *)a.mx)[l * a.mx_stride + slot];
    const int k = max_exponent(__float_as_uint(wave_max(__uint_as_float(v))));
    if (l == 0) (wv == 5 ? sh.kx : sh.kg) = k;
  } else if (wv == 7 && blk == 0 && l == 0) {  // read here, not after the stores
    sh.exX = a.ex[a.slotX];
    sh.exM = a.ex[a.slotM];
    if (want_g) sh.exG = a.ex[a.slotG];
  }
}

__device__ __forceinline__ void seg_prologue(const SegArgs &a, uint32_t blk, bool want_g, SegShared &sh) {
  seg_stage_m(a, sh);
  const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x) >> 6;  // wave index, uniform
  if (wv < 8) seg_roles(a, blk, want_g, sh, wv);
}

// Move a tile (kSegMaxLocal entries x kSegOB outer assignments) between a
// carrier in global memory and LDS.  Consecutive threads take consecutive
// addresses of the carrier: outer-fastest when the carrier's stride-1 label
// is an outer label, entry-fastest otherwise.  Every thread issues all of
// its kSegIter accesses before using them.  Loads fill entries past n and
// outer assignments past nO with zeros; stores return the largest value
// written by the thread.
static constexpr int kSegIter = kSegMaxLocal * kSegOB / kSegThreads;


// (entry, outer assignment) of task t.  The carrier's labels below its
// fastest outer label (2^ls local entries, the fastest ones of the local
// index) vary fastest, then the outer assignment, then the other local
// entries: consecutive threads then take consecutive addresses of the
// carrier (runs of 2^ls x kSegOB floats when the block's outer labels are
// the carrier's next-fastest ones).
__device__ __forceinline__ int2 seg_task(int t, int ls) {
  const int l = t & ((1 << ls) - 1);
  const int o = (t >> ls) & (kSegOB - 1);
  const int h = t >> (ls + 7);
  return make_int2((h << ls) | l, o);
}
static_assert(kSegOB == 128, "seg_task decodes 7 bits of outer assignment");

// global -> registers (entries past n and outer assignments past nO read 0)
__device__ __forceinline__ void seg_fetch(const float *src, const int32_t *off, const int32_t *loc, int n, int ls,
                                          float (&v)[kSegIter]) {
  const gfloat *g = (const gfloat *)src;
#pragma unroll
  for (int k = 0; k < kSegIter; ++k) {
    const int2 jo = seg_task(threadIdx.x + k * kSegThreads, ls);
    const int32_t oo = off[jo.y];
    v[k] = (jo.x < n && oo >= 0) ? g[(uint32_t)(oo + loc[jo.x])] : 0.f;
  }
}
// registers -> LDS tile, scaled
__device__ __forceinline__ void seg_stash(const float (&v)[kSegIter], int ls, float *tile, float scale) {
#pragma unroll
  for (int k = 0; k < kSegIter; ++k) {
    const int2 jo = seg_task(threadIdx.x + k * kSegThreads, ls);
    tile[jo.x * kSegRow + jo.y] = v[k] * scale;
  }
}
__device__ __forceinline__ void seg_load(const float *src, const int32_t *off, const int32_t *loc, int n, int ls,
                                         float *tile, float scale) {
  float v[kSegIter];
  seg_fetch(src, off, loc, n, ls, v);
  seg_stash(v, ls, tile, scale);
}

__device__ __forceinline__ float seg_store(float *dst, const int32_t *off, const int32_t *loc, int n, int ls,
                                           const float *tile) {
  gfloat *g = (gfloat *)dst;
  float lmax = 0.f;
#pragma unroll
  for (int k = 0; k < kSegIter; ++k) {
    const int2 jo = seg_task(threadIdx.x + k * kSegThreads, ls);
    const int32_t oo = off[jo.y];
    if (jo.x < n && oo >= 0) {
      const float x = tile[jo.x * kSegRow + jo.y];
      g[(uint32_t)(oo + loc[jo.x])] = x;
      lmax = fmaxf(lmax, x);
    }
  }
  return lmax;
}

// Matrix-core tiles: v_mfma_f32_16x16x4_f32, D (16 x 16) += A (16 x 4) B (4 x 16)
// with lane l holding A[l % 16][l / 16], B[l / 16][l % 16] and
// D[4 (l / 16) + r][l % 16] in register r.  A workgroup's 32 x kSegOB output
// is 2 x 8 tiles, one per wave: rows 16 (w % 2), columns 16 (w / 2).

// D tile of the wave = A (its 16 rows x 32) * B (32 x its 16 columns of `b`);
// the A operand comes from the staged M (transposed when TRANS)
template <int PREC, bool TRANS>
__device__ __forceinline__ f32x4 seg_mfma(const SegShared &sh, const float *b) {
  f32x4 acc = {};
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = 16 * (w & 1) + (l & 15);
  const float *bp = b + 16 * (w >> 1) + (l & 15);
  auto A = [&](int k) { return TRANS ? sh.m[k * (kSegMaxLocal + 1) + i] : sh.m[i * (kSegMaxLocal + 1) + k]; };
  if (PREC == 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = 4 * q + (l >> 4);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A(k), bp[k * kSegRow], acc, 0, 0, 0);
    }
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float av[4], bv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 16 * h + 4 * (l >> 4) + j;
        av[j] = A(k);
        bv[j] = bp[k * kSegRow];
      }
      acc = mfma16_lp<PREC>(av, bv, acc);
    }
  }
  return acc;
}
// write the wave's D tile into rows < n of a tile
__device__ __forceinline__ void seg_put(const f32x4 &d, int n, float *tile) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * (w & 1) + 4 * (l >> 4) + r;
    if (row < n) tile[row * kSegRow + 16 * (w >> 1) + (l & 15)] = d[r];
  }
}

// Forward: C_L[:, o] = M C_0[:, o] for the workgroup's kSegOB outer
// assignments (one 32-wide column block per wave).  The arguments are passed
// by value: the kernel's first reads then come from the argument block
// itself, one dependent round trip fewer than through a pointer to them
// (measured on the 20 x 20 grid: 7.4 -> 6.6 us forward, 9.6 -> 9.1 us reverse).
template <int PREC>
__device__ __forceinline__ void seg_fwd_body(const SegArgs &a, const uint32_t blk) {
  __shared__ float tile[kSegMaxLocal * kSegRow];
  __shared__ SegShared sh;
  const int n_in = a.n_in0, n_out = a.n_outL;
  seg_prologue(a, blk, false, sh);
  __syncthreads();
  const int kx = sh.kx;
  seg_load(a.arena + a.X, sh.offX, sh.locX, n_in, a.in_lo_shift, tile, ldexpf(1.f, -kx));
  __syncthreads();
  const f32x4 d = seg_mfma<PREC, false>(sh, tile);
  __syncthreads();
  seg_put(d, n_out, tile);
  __syncthreads();
  const float lmax = seg_store(a.arena + a.Z, sh.offZ, sh.locZ, n_out, a.out_lo_shift, tile);
  block_record_max<kSegThreads, false>(lmax, a.mx + (blk % kMaxSub) * a.mx_stride + a.slotZ);
  if (blk == 0 && threadIdx.x == 0) a.ex[a.slotZ] = sh.exX + kx + sh.exM;
}

template <int PREC>
__global__ __launch_bounds__(kSegThreads) void k_seg_fwd(const SegArgs a) {
  seg_fwd_body<PREC>(a, xcd_tile(blockIdx.x, gridDim.x));
}

// Two independent segments of one stage in one launch: workgroups
// [0, split) run the first, the rest the second.  (Measured on the 20 x 20
// grid: one workgroup per tile of each segment; a workgroup taking the same
// tile of both segments, with both tiles' loads in flight together, ran
// slower, 11.2 vs 10.4 us forward and 15.4 vs 14.2 us reverse per pair.)
template <int PREC>
__global__ __launch_bounds__(kSegThreads) void k_seg_fwd2(const SegPair g) {
  const uint32_t second = blockIdx.x >= g.split ? 1u : 0u;
  seg_fwd_body<PREC>(g.a[second], xcd_tile(blockIdx.x - second * g.split, second ? gridDim.x - g.split : g.split));
}

// Reverse: Cbar_0[:, o] = M^T Gbar[:, o], and the workgroup's partial of
// S = sum_o Gbar[:, o] C_0[:, o]^T: wave w computes the 16 x 16 quadrant
// w % 4 of S over the outer quarter w / 4; quarters are added in order.
// After the loads: the tiles into LDS, Cbar_0 tile = M^T Gbar tile, the S
// partial, the stores, the maximum.  vg: Gbar tile, vx: C_0 tile (when the
// segment needs S).
template <int PREC>
__device__ __forceinline__ void seg_bwd_finish(const SegArgs &a, const uint32_t blk, const SegShared &sh,
                                               const float (&vg)[kSegIter], const float (&vx)[kSegIter],
                                               float *tg, float *tx) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n_in = a.n_in0, n_out = a.n_outL;
  const bool want_s = a.n_part > 0;
  const int kx = sh.kx, kg = sh.kg;
  seg_stash(vg, a.out_lo_shift, tg, ldexpf(1.f, -kg));
  if (want_s) seg_stash(vx, a.in_lo_shift, tx, ldexpf(1.f, -kx));
  __syncthreads();
  const f32x4 xb = seg_mfma<PREC, true>(sh, tg);  // A = M^T
  f32x4 s = {};
  if (want_s) {
    // S quadrant (rows 16 qr of Gbar's entries, columns 16 qc of C_0's) over
    // the outer quarter kq: A = Gbar (16 x 32 outer), B = C_0^T (32 outer x 16)
    const int qr = w & 1, qc = (w >> 1) & 1, kq = w >> 2;
    const float *ga = tg + (16 * qr + (l & 15)) * kSegRow + 32 * kq;
    const float *xa = tx + (16 * qc + (l & 15)) * kSegRow + 32 * kq;
    if (PREC == 0) {
#pragma unroll
      for (int q = 0; q < 8; ++q)
        s = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[4 * q + (l >> 4)], xa[4 * q + (l >> 4)], s, 0, 0, 0);
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float av[4], bv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          av[j] = ga[16 * h + 4 * (l >> 4) + j];
          bv[j] = xa[16 * h + 4 * (l >> 4) + j];
        }
        s = mfma16_lp<PREC>(av, bv, s);
      }
    }
  }
  __syncthreads();
  seg_put(xb, n_in, tx);
  if (want_s && w >= 4) {
#pragma unroll
    for (int r = 0; r < 4; ++r) tg[(w - 4) * 256 + r * 64 + l] = s[r];
  }
  __syncthreads();
  const float lmax = seg_store(a.arena + a.Z, sh.offX, sh.locX, n_in, a.in_lo_shift, tx);
  if (want_s && w < 4) {
    const int nS = n_out * n_in;
    float *part = a.arena + a.Sp + (size_t)blk * nS;
    const int qr = w & 1, qc = w >> 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float v = ((s[r] + tg[w * 256 + r * 64 + l]) + tg[(w + 4) * 256 + r * 64 + l]) +
                      tg[(w + 8) * 256 + r * 64 + l];
      const int j = 16 * qr + 4 * (l >> 4) + r, i = 16 * qc + (l & 15);
      if (j < n_out && i < n_in) part[j * n_in + i] = v;
    }
  }
  block_record_max<kSegThreads, false>(lmax, a.mx + (blk % kMaxSub) * a.mx_stride + a.slotZ);
  if (blk == 0 && threadIdx.x == 0) {
    a.ex[a.slotZ] = sh.exG + kg + sh.exM;
    if (want_s) a.ex[a.slotSp] = (sh.exG + kg) + (sh.exX + kx);
  }
}

template <int PREC>
__device__ __forceinline__ void seg_bwd_body(const SegArgs &a, const uint32_t blk) {
  __shared__ float tg[kSegMaxLocal * kSegRow];  // output adjoint; later the waves' S partials
  __shared__ float tx[kSegMaxLocal * kSegRow];  // input carrier; later its adjoint
  __shared__ SegShared sh;
  seg_prologue(a, blk, true, sh);
  __syncthreads();
  float vg[kSegIter], vx[kSegIter];
  seg_fetch(a.arena + a.G, sh.offZ, sh.locZ, a.n_outL, a.out_lo_shift, vg);
  if (a.n_part > 0) seg_fetch(a.arena + a.X, sh.offX, sh.locX, a.n_in0, a.in_lo_shift, vx);
  seg_bwd_finish<PREC>(a, blk, sh, vg, vx, tg, tx);
}

template <int PREC>
__global__ __launch_bounds__(kSegThreads) void k_seg_bwd(const SegArgs a) {
  seg_bwd_body<PREC>(a, xcd_tile(blockIdx.x, gridDim.x));
}

// Two independent segments' reverse steps in one launch, as k_seg_fwd2.
template <int PREC>
__global__ __launch_bounds__(kSegThreads) void k_seg_bwd2(const SegPair g) {
  const uint32_t second = blockIdx.x >= g.split ? 1u : 0u;
  seg_bwd_body<PREC>(g.a[second], xcd_tile(blockIdx.x - second * g.split, second ? gridDim.x - g.split : g.split));
}

// --- sweeps over the steps (one workgroup per segment) ---------------------
// (red: NT / 64 floats)
template <int NT = kSweepThreads>
__device__ __forceinline__ float seg_block_max(float v, float *red) {
  v = wave_max(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float m = red[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) m = fmaxf(m, red[w]);
  return m;
}

// Scale v[0, n) so that its maximum lies in [0.5, 1); returns the exponent
// taken out (values are non-negative).
template <int NT = kSweepThreads>
__device__ int seg_normalize(float *v, int n, float *red) {
  float m = 0.f;
  for (int t = threadIdx.x; t < n; t += NT) m = fmaxf(m, v[t]);
  m = seg_block_max<NT>(m, red);
  const int k = max_exponent(__float_as_uint(m));
  if (k != 0) {
    const float sc = ldexpf(1.f, -k);
    for (int t = threadIdx.x; t < n; t += NT) v[t] *= sc;
  }
  __syncthreads();
  return k;
}

// The sweep kernels stage the segment's step descriptors, the exponents of
// its small operands, its index lists and the small operands in LDS first,
// so that every step below reads LDS only.  Each thread issues a batch of
// loads before it stores any of them: a load followed at once by its LDS
// store costs one memory round trip per loop pass.
struct SegStepsLds {
  SegStep st[kSegMaxSteps];
  int32_t ey[kSegMaxSteps];  // exponent of each step's small operand
};
static constexpr int kStageBatch = 8;
static_assert(kSegMaxSteps * 64 % kSweepThreads == 0 && kSegMaxSteps * 64 % kFinThreads == 0,
              "whole (step, entry) pairs per thread");

// descriptors and exponents (one thread per step), then the lists; the
// caller synchronises before seg_stage_operands
template <int NT = kSweepThreads>
__device__ __forceinline__ void seg_stage_lists(const SegArgs &a, SegStepsLds &ss, int32_t *li) {
  if ((int)threadIdx.x < a.n_steps) {  // word by word (a struct copy goes through private memory)
    const int32_t *src = (const int32_t *)(a.steps + threadIdx.x);
    int32_t *dst = (int32_t *)&ss.st[threadIdx.x];
    int32_t w[sizeof(SegStep) / 4];
#pragma unroll
    for (int j = 0; j < (int)(sizeof(SegStep) / 4); ++j) w[j] = src[j];
    ss.ey[threadIdx.x] = a.ex[a.steps[threadIdx.x].yslot];
#pragma unroll
    for (int j = 0; j < (int)(sizeof(SegStep) / 4); ++j) dst[j] = w[j];
  }
  for (int t0 = 0; t0 < a.list_len; t0 += kStageBatch * NT) {
    int32_t v[kStageBatch];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) {
      const int t = t0 + u * NT + (int)threadIdx.x;
      v[u] = t < a.list_len ? a.lists[t] : 0;
    }
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) {
      const int t = t0 + u * NT + (int)threadIdx.x;
      if (t < a.list_len) li[t] = v[u];
    }
  }
}
// small operands, 64 entries per step (needs the staged descriptors)
template <int NT = kSweepThreads>
__device__ __forceinline__ void seg_stage_operands(const SegArgs &a, const SegStepsLds &ss, float *yv) {
  constexpr int kPer = kSegMaxSteps * 64 / NT;
  float v[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int p = (int)threadIdx.x + u * NT, k = p >> 6, i = p & 63;
    v[u] = (k < a.n_steps && i < ss.st[k].ny) ? a.arena[ss.st[k].y + i] : 0.f;
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int p = (int)threadIdx.x + u * NT, k = p >> 6, i = p & 63;
    if (k < a.n_steps && i < ss.st[k].ny) yv[k * 64 + i] = v[u];
  }
}

// out = (step's map) in, column by column: out[j][c] = sum over the triples
// of output entry j of in[i][c] * y[s]; rows of nc columns.
template <int NT = kSweepThreads>
__device__ void seg_step_fwd(const SegStep &st, const int32_t *li, const float *y, const float *in, float *out,
                             int nc) {
  const int32_t *ptr = li + st.fo_ptr, *xi = li + st.fo_in, *xs = li + st.fo_s;
  for (int t = threadIdx.x; t < st.n_out * nc; t += NT) {
    const int j = t / nc, c = t - j * nc;
    float acc = 0.f;
    for (int e = ptr[j]; e < ptr[j + 1]; ++e) acc = fmaf(in[xi[e] * nc + c], y[xs[e]], acc);
    out[t] = acc;
  }
}

// out = (step's map)^T in: out[i][c] = sum over the triples of input entry i
// of in[j][c] * y[s].
template <int NT = kSweepThreads>
__device__ void seg_step_bwd(const SegStep &st, const int32_t *li, const float *y, const float *in, float *out,
                             int nc) {
  const int32_t *ptr = li + st.bi_ptr, *xo = li + st.bi_out, *xs = li + st.bi_s;
  for (int t = threadIdx.x; t < st.n_in * nc; t += NT) {
    const int i = t / nc, c = t - i * nc;
    float acc = 0.f;
    for (int e = ptr[i]; e < ptr[i + 1]; ++e) acc = fmaf(in[xo[e] * nc + c], y[xs[e]], acc);
    out[t] = acc;
  }
}

// M = (last step's map) ... (first step's map), applied to the identity,
// renormalised after every step.  LDS: two 32 x 32 work areas, the lists,
// 64 floats of small operand per step.
__global__ __launch_bounds__(kSweepThreads) void k_seg_mat(const SegArgs *__restrict__ base,
                                                           const int32_t *__restrict__ ids) {
  const SegArgs &a = base[ids[blockIdx.x]];
  extern __shared__ float lds[];
  __shared__ float red[4];
  __shared__ __align__(16) unsigned char ss_mem[sizeof(SegStepsLds)];  // SegStep has initialisers
  SegStepsLds &ss = *reinterpret_cast<SegStepsLds *>(ss_mem);
  const int nc = a.n_in0;
  float *A = lds, *B = lds + 1024, *yv = lds + 2048;
  int32_t *li = (int32_t *)(yv + 64 * a.n_steps);
  seg_stage_lists(a, ss, li);
  for (int t = threadIdx.x; t < nc * nc; t += kSweepThreads) A[t] = (t / nc == t % nc) ? 1.f : 0.f;
  __syncthreads();
  seg_stage_operands(a, ss, yv);
  __syncthreads();
  int e = 0;
  for (int k = 0; k < a.n_steps; ++k) {
    const SegStep &st = ss.st[k];
    seg_step_fwd(st, li, yv + 64 * k, A, B, nc);
    __syncthreads();
    e += ss.ey[k] + seg_normalize(B, st.n_out * nc, red);
    float *tmp = A;
    A = B;
    B = tmp;
  }
  for (int t = threadIdx.x; t < a.n_outL * nc; t += kSweepThreads) a.arena[a.M + t] = A[t];
  if (threadIdx.x == 0) a.ex[a.slotM] = e;
}

// Adjoints of the small operands.  With P_k the map of the first k steps
// (P_0 = I) and G_k = (steps k..L-1)^T S (G_L = S), the adjoint of step k's
// map is W_k = G_{k+1} P_k^T (eq. einback summed over the outer labels), and
// the small operand's adjoint entry s sums W_k over the triples of s.
// LDS: three 32 x 32 work areas, the lists, the small operands, P_0 .. P_{L-1}.
__global__ __launch_bounds__(kFinThreads) void k_seg_fin(const SegArgs *__restrict__ base,
                                                           const int32_t *__restrict__ ids) {
  const SegArgs &a = base[ids[blockIdx.x]];
  extern __shared__ float lds[];
  __shared__ float red[kFinThreads / 64];
  __shared__ int eP[kSegMaxSteps], poff[kSegMaxSteps + 1];
  __shared__ __align__(16) unsigned char ss_mem[sizeof(SegStepsLds)];  // SegStep has initialisers
  SegStepsLds &ss = *reinterpret_cast<SegStepsLds *>(ss_mem);
  __shared__ int eS;
  const int nc = a.n_in0, L = a.n_steps, nS = a.n_outL * nc;
  float *G0 = lds, *G1 = lds + 1024, *W = lds + 2048;
  int32_t *li = (int32_t *)(lds + 3072);
  float *yv = (float *)(li + a.list_len), *P = yv + 64 * L;
  seg_stage_lists<kFinThreads>(a, ss, li);
  // S (summed by k_seg_sred into the first partial) and its exponent
  {
    static_assert(kSegMaxLocal * kSegMaxLocal == kFinThreads, "one entry of S per thread");
    const int t = (int)threadIdx.x;
    const float v = t < nS ? a.arena[a.Sp + t] : 0.f;
    if (threadIdx.x == 0) eS = a.ex[a.slotSp];
    if (t < nS) G0[t] = v;
  }
  for (int t = threadIdx.x; t < nc * nc; t += kFinThreads) P[t] = (t / nc == t % nc) ? 1.f : 0.f;
  __syncthreads();
  if (threadIdx.x == 0) {
    int off = 0;
    for (int k = 0; k < L; ++k) {
      poff[k] = off;
      off += ss.st[k].n_in * nc;
    }
    poff[L] = off;
    eP[0] = 0;
  }
  seg_stage_operands<kFinThreads>(a, ss, yv);
  __syncthreads();
  for (int k = 0; k + 1 < L; ++k) {
    const SegStep &st = ss.st[k];
    float *nxt = P + poff[k + 1];
    seg_step_fwd<kFinThreads>(st, li, yv + 64 * k, P + poff[k], nxt, nc);
    __syncthreads();
    const int sh = seg_normalize<kFinThreads>(nxt, st.n_out * nc, red);
    if (threadIdx.x == 0) eP[k + 1] = eP[k] + ss.ey[k] + sh;
  }
  int eG = eS + seg_normalize<kFinThreads>(G0, nS, red);
  for (int k = L - 1; k >= 0; --k) {
    const SegStep &st = ss.st[k];
    if (st.ybar >= 0) {
      const float *Pk = P + poff[k];
      // lanes of one wave take consecutive i: rows of Pk nc floats apart, so
      // each lane starts its sum at column i (mod nc) — otherwise the 32
      // lanes of a row of W read one LDS bank in every step (nc = 32)
      for (int t = threadIdx.x; t < st.n_out * st.n_in; t += kFinThreads) {
        const int j = t / st.n_in, i = t - j * st.n_in;
        const float *gj = G0 + j * nc, *pi = Pk + i * nc;
        int c = i % nc;
        float acc = 0.f;
        for (int u = 0; u < nc; ++u) {
          acc = fmaf(gj[c], pi[c], acc);
          c = c + 1 == nc ? 0 : c + 1;
        }
        W[t] = acc;
      }
      __syncthreads();
      const int32_t *ptr = li + st.bs_ptr, *xi = li + st.bs_in, *xo = li + st.bs_out;
      float m = 0.f;
      for (int sidx = threadIdx.x; sidx < st.ny; sidx += kFinThreads) {
        float acc = 0.f;
        for (int e = ptr[sidx]; e < ptr[sidx + 1]; ++e) acc += W[xo[e] * st.n_in + xi[e]];
        a.arena[st.ybar + sidx] = acc;
        m = fmaxf(m, acc);
      }
      m = seg_block_max<kFinThreads>(m, red);
      if (threadIdx.x == 0) {
        a.mx[st.ybar_slot] = __float_as_uint(m);
        a.ex[st.ybar_slot] = eG + eP[k];
      }
    }
    if (k > 0) {
      seg_step_bwd<kFinThreads>(st, li, yv + 64 * k, G0, G1, nc);
      __syncthreads();
      eG += ss.ey[k] + seg_normalize<kFinThreads>(G1, st.n_in * nc, red);
      float *tmp = G0;
      G0 = G1;
      G1 = tmp;
    }
  }
}

// S = sum of the carrier kernel's partials, in a fixed order, written over
// the first partial.  Workgroup (segment, chunk) owns kSredEntries entries;
// four lanes per entry take every fourth partial, combined in lane order.
static constexpr int kSredEntries = 64;
static constexpr int kSredChunks = kSegMaxLocal * kSegMaxLocal / kSredEntries;

__global__ __launch_bounds__(kSweepThreads) void k_seg_sred(const SegArgs *__restrict__ base,
                                                          const int32_t *__restrict__ ids) {
  const SegArgs &a = base[ids[blockIdx.x / kSredChunks]];
  __shared__ float red[kSweepThreads];
  const int nS = a.n_outL * a.n_in0;
  const int e = (blockIdx.x % kSredChunks) * kSredEntries + (threadIdx.x & (kSredEntries - 1));
  const int g = threadIdx.x / kSredEntries;
  float *part = a.arena + a.Sp;
  float acc = 0.f;
  if (e < nS) {
#pragma unroll 8
    for (int b = g; b < a.n_part; b += kSweepThreads / kSredEntries) acc += part[(size_t)b * nS + e];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (g == 0 && e < nS) {
    float t = red[threadIdx.x];
    for (int q = 1; q < kSweepThreads / kSredEntries; ++q) t += red[q * kSredEntries + threadIdx.x];
    part[e] = t;
  }
}

void launch_seg_fwd(const SegArgs &a, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  if (a.prec == 1) k_seg_fwd<1><<<seg_blocks(a), kSegThreads, 0, s>>>(a);
  else if (a.prec == 2) k_seg_fwd<2><<<seg_blocks(a), kSegThreads, 0, s>>>(a);
  else k_seg_fwd<0><<<seg_blocks(a), kSegThreads, 0, s>>>(a);
}
void launch_seg_bwd(const SegArgs &a, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  if (a.prec == 1) k_seg_bwd<1><<<seg_blocks(a), kSegThreads, 0, s>>>(a);
  else if (a.prec == 2) k_seg_bwd<2><<<seg_blocks(a), kSegThreads, 0, s>>>(a);
  else k_seg_bwd<0><<<seg_blocks(a), kSegThreads, 0, s>>>(a);
}
void launch_seg_fwd2(const SegArgs &a, const SegArgs &b, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  SegPair g;
  g.a[0] = a;
  g.a[1] = b;
  g.split = seg_blocks(a);
  const unsigned nb = g.split + seg_blocks(b);
  if (a.prec == 1) k_seg_fwd2<1><<<nb, kSegThreads, 0, s>>>(g);
  else if (a.prec == 2) k_seg_fwd2<2><<<nb, kSegThreads, 0, s>>>(g);
  else k_seg_fwd2<0><<<nb, kSegThreads, 0, s>>>(g);
}
void launch_seg_bwd2(const SegArgs &a, const SegArgs &b, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  SegPair g;
  g.a[0] = a;
  g.a[1] = b;
  g.split = seg_blocks(a);
  const unsigned nb = g.split + seg_blocks(b);
  if (a.prec == 1) k_seg_bwd2<1><<<nb, kSegThreads, 0, s>>>(g);
  else if (a.prec == 2) k_seg_bwd2<2><<<nb, kSegThreads, 0, s>>>(g);
  else k_seg_bwd2<0><<<nb, kSegThreads, 0, s>>>(g);
}
void launch_seg_mat(const SegArgs *d_base, const int32_t *d_ids, int n, int lds_floats, void *stream) {
  k_seg_mat<<<n, kSweepThreads, (size_t)lds_floats * sizeof(float), (hipStream_t)stream>>>(d_base, d_ids);
}
void launch_seg_fin(const SegArgs *d_base, const int32_t *d_ids, int n, int lds_floats, void *stream) {
  k_seg_sred<<<n * kSredChunks, kSweepThreads, 0, (hipStream_t)stream>>>(d_base, d_ids);
  k_seg_fin<<<n, kFinThreads, (size_t)lds_floats * sizeof(float), (hipStream_t)stream>>>(d_base, d_ids);
}

// --------------------------------------------------------------------------
// two consecutive segments in one carrier pass
// --------------------------------------------------------------------------
// A workgroup takes nob assignments of the common outer labels O.  Its X
// tile is C_0 over A (rows) x (Q, o) (columns), its Z tile C_2 over D x
// (R, o); the column order follows the carriers' memory order (q_fast,
// r_fast).  Y = M1 X is C_1 over B x (Q, o).  Column (r, o) of the second
// map's operand, row c = (p, q), is Y[P part of c + R part of r][column of
// (q, o)]: per c the tables give the P part (pb) and the Q column part (qc),
// per Z column the R part (yr, -1: no such column) and the o part (yc).

unsigned dseg_blocks(const DSegArgs &a) { return (a.nO + (uint32_t)a.nob - 1) / (uint32_t)a.nob; }

struct DSegShared {
  int32_t colX[kSegOB], colZ[kSegOB];  // column offsets in C_0 / C_2 (-1: none)
  int32_t yr[kSegOB], yc[kSegOB];      // per Z column: row and column parts in Y
  int32_t locA[kSegMaxLocal], locD[kSegMaxLocal], pb[kSegMaxLocal], qc[kSegMaxLocal];
  float m1[kSegMaxLocal * (kSegMaxLocal + 1)], m2[kSegMaxLocal * (kSegMaxLocal + 1)];
  int32_t kx, kg;
  int32_t exX, exG, exM1, exM2;
};

// D (16 x 16) += sum over k < 32 of A(i, k) B(k, j) for the lane's row i
// and column j (both l % 16, bound by the caller): fa(k), fb(k) give the
// lane's operands; register r of the result is row 4 (l / 16) + r.
template <int PREC, class FA, class FB>
__device__ __forceinline__ f32x4 mfma_k32(FA fa, FB fb) {
  const int l = threadIdx.x & 63;
  f32x4 acc = {};
  if (PREC == 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = 4 * q + (l >> 4);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fa(k), fb(k), acc, 0, 0, 0);
    }
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float av[4], bv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 16 * h + 4 * (l >> 4) + j;
        av[j] = fa(k);
        bv[j] = fb(k);
      }
      acc = mfma16_lp<PREC>(av, bv, acc);
    }
  }
  return acc;
}

// Entry (r, c) of a map M (x) I_aug over rows (o, i) and columns (o', j),
// M row-major (nr / aug) x (nc / aug): M[i][j] when o == o', else zero; zero
// past nr rows or nc columns.
__device__ __forceinline__ float dseg_map_entry(const gcfloat *m, int nr, int nc, int aug, int r, int c) {
  int nr0 = nr, nc0 = nc, r0 = r, c0 = c;
  bool diag = true;
  if (aug > 1) {
    nr0 = nr / aug;
    nc0 = nc / aug;
    r0 = r % nr0;
    c0 = c % nc0;
    diag = r / nr0 == c / nc0;
  }
  const float x = m[min(r0, nr0 - 1) * nc0 + min(c0, nc0 - 1)];
  return (r < nr && c < nc && diag) ? x : 0.f;
}

// Prologue: both maps (one entry of each per thread), then by waves 0-10:
// column offsets of both tiles, local offsets, the gather tables, operand
// maxima and (workgroup 0) exponents.  Every global read is independent.
__device__ __forceinline__ void dseg_prologue(const DSegArgs &a, uint32_t blk, bool want_g, DSegShared &sh) {
  const int t = threadIdx.x, l = t & 63;
  {
    const int r = t >> 5, c = t & 31;
    sh.m1[r * (kSegMaxLocal + 1) + c] = dseg_map_entry((gcfloat *)(a.arena + a.M1), a.nB, a.nA, a.aug1, r, c);
    sh.m2[r * (kSegMaxLocal + 1) + c] = dseg_map_entry((gcfloat *)(a.arena + a.M2), a.nD, a.nC, a.aug2, r, c);
  }
  const int wv = __builtin_amdgcn_readfirstlane(t) >> 6;
  gint *tab = (gint *)a.tab;
  if (wv < 4) {  // column offsets: waves 0-1 the X tile (A x (Q, o)), 2-3 the Z tile (D x (R, o))
    const bool in = wv < 2;
    const int c = t & (kSegOB - 1);
    const int nq = in ? a.nQ : a.nR, fast = in ? a.q_fast : a.r_fast;
    const int q = fast ? c % nq : c / a.nob, ol = fast ? c / nq : (c & (a.nob - 1));
    const uint32_t o = blk * (uint32_t)a.nob + (uint32_t)ol, oc = min(o, a.nO - 1);
    gint *hi = (gint *)(in ? a.oX.hi : a.oZ.hi), *lo = (gint *)(in ? a.oX.lo : a.oZ.lo);
    int32_t oo;
    if (a.ol_shift >= 0) oo = hi[oc >> a.ol_shift] + lo[oc & (a.nOl - 1)];
    else oo = hi[oc / a.nOl] + lo[oc % a.nOl];
    const int32_t qo = tab[(in ? 2 : 3) * kSegMaxLocal + min(q, nq - 1)];
    (in ? sh.colX : sh.colZ)[c] = (q < nq && ol < a.nob && o < a.nO) ? oo + qo : -1;
  } else if (wv == 4) {  // local offsets: lanes 0-31 A in C_0, 32-63 D in C_2
    const int j = l & 31;
    const int32_t v = tab[(l < 32 ? 0 : 1) * kSegMaxLocal + j];
    (l < 32 ? sh.locA : sh.locD)[j] = v;
  } else if (wv == 5) {  // per c: P part of the row in Y (lanes 0-31), Q column part (32-63)
    const int j = l & 31;
    const int32_t v = tab[(l < 32 ? 4 : 5) * kSegMaxLocal + j];
    if (l < 32) sh.pb[j] = v;
    else sh.qc[j] = a.q_fast ? v : v * a.nob;
  } else if (wv == 6 || wv == 7) {  // per Z column: R part of the row in Y, o part of its column
    const int c = t & (kSegOB - 1);
    const int r = a.r_fast ? c % a.nR : c / a.nob, ol = a.r_fast ? c / a.nR : (c & (a.nob - 1));
    const int32_t v = tab[6 * kSegMaxLocal + min(r, a.nR - 1)];
    const bool ok = r < a.nR && ol < a.nob;
    sh.yr[c] = ok ? v : -1;
    sh.yc[c] = a.q_fast ? ol * a.nQ : ol;
  } else if (wv == 8 || (wv == 9 && want_g)) {  // maxima of the operands (64 sub-slots)
    const int slot = wv == 8 ? a.slotX : a.slotG;
    const uint32_t v = ((gu32 *)a.mx)[l * a.mx_stride + slot];
    const int k = max_exponent(__float_as_uint(wave_max(__uint_as_float(v))));
    if (l == 0) (wv == 8 ? sh.kx : sh.kg) = k;
  } else if (wv == 10 && blk == 0 && l == 0) {
    sh.exX = a.ex[a.slotX];
    sh.exM1 = a.ex[a.slotM1];
    sh.exM2 = a.ex[a.slotM2];
    if (want_g) sh.exG = a.ex[a.slotG];
  }
}

// Operand of the second map: row k (an assignment c of C), column n (an
// assignment (r, o) of the Z tile), read from the Y tile.
__device__ __forceinline__ float dseg_b2(const DSegShared &sh, const float *ty, int nC, int k, int n) {
  const int yr = sh.yr[n];
  return (k < nC && yr >= 0) ? ty[(sh.pb[k] + yr) * kSegRow + sh.qc[k] + sh.yc[n]] : 0.f;
}

template <int PREC>
__device__ __forceinline__ void dseg_fwd_body(const DSegArgs &a, const uint32_t blk) {
  __shared__ float tx[kSegMaxLocal * kSegRow];  // C_0 tile, later the C_2 tile
  __shared__ float ty[kSegMaxLocal * kSegRow];  // C_1 tile
  __shared__ DSegShared sh;
  dseg_prologue(a, blk, false, sh);
  __syncthreads();
  const int kx = sh.kx;
  seg_load(a.arena + a.X, sh.colX, sh.locA, a.nA, a.in_lo_shift, tx, ldexpf(1.f, -kx));
  __syncthreads();
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = 16 * (w & 1) + (l & 15), n = 16 * (w >> 1) + (l & 15);
  const f32x4 y = mfma_k32<PREC>([&](int k) { return sh.m1[i * (kSegMaxLocal + 1) + k]; },
                                 [&](int k) { return tx[k * kSegRow + n]; });
  seg_put(y, kSegMaxLocal, ty);
  __syncthreads();
  const int nC = a.nC;
  const f32x4 z = mfma_k32<PREC>([&](int k) { return sh.m2[i * (kSegMaxLocal + 1) + k]; },
                                 [&](int k) { return dseg_b2(sh, ty, nC, k, n); });
  seg_put(z, a.nD, tx);
  __syncthreads();
  const float lmax = seg_store(a.arena + a.Z, sh.colZ, sh.locD, a.nD, a.out_lo_shift, tx);
  block_record_max<kSegThreads, false>(lmax, a.mx + (blk % kMaxSub) * a.mx_stride + a.slotZ);
  if (blk == 0 && threadIdx.x == 0) a.ex[a.slotZ] = sh.exX + kx + sh.exM1 + sh.exM2;
}

template <int PREC>
__global__ __launch_bounds__(kSegThreads) void k_dseg_fwd(const DSegPair g) {
  const uint32_t second = blockIdx.x >= g.split ? 1u : 0u;
  dseg_fwd_body<PREC>(g.a[second], xcd_tile(blockIdx.x - second * g.split, second ? gridDim.x - g.split : g.split));
}

// Wave w's 16 x 16 quadrant (w % 4) of sum over the column quarter w / 4
// of F(row, col) G(row', col): rows of F are the result's rows.
template <int PREC, class F, class G>
__device__ __forceinline__ f32x4 dseg_s_quadrant(F f, G gf) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int qr = w & 1, qc = (w >> 1) & 1, n0 = 32 * (w >> 2);
  const int i = 16 * qr + (l & 15), j = 16 * qc + (l & 15);
  return mfma_k32<PREC>([&](int k) { return f(i, n0 + k); }, [&](int k) { return gf(j, n0 + k); });
}
// The four quarters of a quadrant added in order (waves 4-15 park theirs in
// park[]; waves 0-3 add them after a barrier), then the partial is written.
__device__ __forceinline__ void dseg_s_park(const f32x4 &s, float *park) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (w >= 4) {
#pragma unroll
    for (int r = 0; r < 4; ++r) park[(w - 4) * 256 + r * 64 + l] = s[r];
  }
}
__device__ __forceinline__ void dseg_s_write(const f32x4 &s, const float *park, float *part, int n_rows, int n_cols) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (w >= 4) return;
  const int qr = w & 1, qc = w >> 1;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float v = ((s[r] + park[w * 256 + r * 64 + l]) + park[(w + 4) * 256 + r * 64 + l]) +
                    park[(w + 8) * 256 + r * 64 + l];
    const int row = 16 * qr + 4 * (l >> 4) + r, col = 16 * qc + (l & 15);
    if (row < n_rows && col < n_cols) part[row * n_cols + col] = v;
  }
}

// As dseg_s_write for a map M (x) I_aug: the S of the whole tile (rows
// (o, b), columns (o', a)) goes to LDS after park's twelve quarters, and M's
// partial is the sum of its aug diagonal blocks.  Every thread of the
// workgroup calls it.
__device__ __forceinline__ void dseg_s_fold(const f32x4 &s, float *park, float *part, int nB, int nA, int aug) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  float *full = park + 12 * 256;  // 32 x (kSegMaxLocal + 1)
  if (w < 4) {
    const int qr = w & 1, qc = w >> 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float v = ((s[r] + park[w * 256 + r * 64 + l]) + park[(w + 4) * 256 + r * 64 + l]) +
                      park[(w + 8) * 256 + r * 64 + l];
      full[(16 * qr + 4 * (l >> 4) + r) * (kSegMaxLocal + 1) + 16 * qc + (l & 15)] = v;
    }
  }
  __syncthreads();
  const int nB0 = nB / aug, nA0 = nA / aug, t = threadIdx.x;
  if (t < nB0 * nA0) {
    const int b = t / nA0, c = t - b * nA0;
    float v = 0.f;
    for (int o = 0; o < aug; ++o) v += full[(o * nB0 + b) * (kSegMaxLocal + 1) + o * nA0 + c];
    part[t] = v;
  }
}
static_assert(12 * 256 + kSegMaxLocal * (kSegMaxLocal + 1) <= kSegMaxLocal * kSegRow, "fold area fits the tile");

// Reverse: with G2 = the C_2 tile's adjoint and Y = M1 X recomputed,
//   S2 = sum over columns of G2 B2^T (B2 = the second map's operand),
//   G1 = M2^T G2 placed back into Y's layout (the adjoint of C_1),
//   S1 = sum over columns of G1 X^T, and the adjoint of C_0 = M1^T G1.
template <int PREC>
__device__ __forceinline__ void dseg_bwd_body(const DSegArgs &a, const uint32_t blk) {
  __shared__ float tg[kSegMaxLocal * kSegRow];  // G2 tile; later S2's parked quarters, then S1's
  __shared__ float tx[kSegMaxLocal * kSegRow];  // C_0 tile; later its adjoint
  __shared__ float ty[kSegMaxLocal * kSegRow];  // C_1 tile; later its adjoint
  __shared__ DSegShared sh;
  dseg_prologue(a, blk, true, sh);
  __syncthreads();
  const int kx = sh.kx, kg = sh.kg;
  {
    float vg[kSegIter], vx[kSegIter];
    seg_fetch(a.arena + a.G, sh.colZ, sh.locD, a.nD, a.out_lo_shift, vg);
    seg_fetch(a.arena + a.X, sh.colX, sh.locA, a.nA, a.in_lo_shift, vx);
    seg_stash(vg, a.out_lo_shift, tg, ldexpf(1.f, -kg));
    seg_stash(vx, a.in_lo_shift, tx, ldexpf(1.f, -kx));
  }
  __syncthreads();
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = 16 * (w & 1) + (l & 15), n = 16 * (w >> 1) + (l & 15);
  const int nC = a.nC;
  const f32x4 y = mfma_k32<PREC>([&](int k) { return sh.m1[i * (kSegMaxLocal + 1) + k]; },
                                 [&](int k) { return tx[k * kSegRow + n]; });
  const f32x4 wt = mfma_k32<PREC>([&](int k) { return sh.m2[k * (kSegMaxLocal + 1) + i]; },
                                  [&](int k) { return tg[k * kSegRow + n]; });
  seg_put(y, kSegMaxLocal, ty);  // rows past nB are zero (zero rows of M1)
  __syncthreads();
  const bool want2 = a.slotSp2 >= 0, want1 = a.slotSp1 >= 0;
  f32x4 s2 = {};
  if (want2)
    s2 = dseg_s_quadrant<PREC>([&](int r, int c) { return tg[r * kSegRow + c]; },
                               [&](int r, int c) { return dseg_b2(sh, ty, nC, r, c); });
  __syncthreads();
  // G1 over Y: every entry of a valid (row, column) of Y is written once; the
  // rest of Y is zero
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int c = 16 * (w & 1) + 4 * (l >> 4) + r;
    const int yr = sh.yr[n];
    if (c < nC && yr >= 0) ty[(sh.pb[c] + yr) * kSegRow + sh.qc[c] + sh.yc[n]] = wt[r];
  }
  if (want2) dseg_s_park(s2, tg);
  __syncthreads();
  f32x4 s1 = {};
  if (want1)
    s1 = dseg_s_quadrant<PREC>([&](int r, int c) { return ty[r * kSegRow + c]; },
                               [&](int r, int c) { return tx[r * kSegRow + c]; });
  const f32x4 xb = mfma_k32<PREC>([&](int k) { return sh.m1[k * (kSegMaxLocal + 1) + i]; },
                                  [&](int k) { return ty[k * kSegRow + n]; });
  const int nP2 = (a.nD / a.aug2) * (a.nC / a.aug2), nP1 = (a.nB / a.aug1) * (a.nA / a.aug1);
  if (want2) {
    if (a.aug2 > 1) dseg_s_fold(s2, tg, a.arena + a.Sp2 + (size_t)blk * nP2, a.nD, a.nC, a.aug2);
    else dseg_s_write(s2, tg, a.arena + a.Sp2 + (size_t)blk * nP2, a.nD, a.nC);
  }
  __syncthreads();
  seg_put(xb, a.nA, tx);
  if (want1) dseg_s_park(s1, tg);
  __syncthreads();
  const float lmax = seg_store(a.arena + a.Z, sh.colX, sh.locA, a.nA, a.in_lo_shift, tx);
  if (want1) {
    if (a.aug1 > 1) dseg_s_fold(s1, tg, a.arena + a.Sp1 + (size_t)blk * nP1, a.nB, a.nA, a.aug1);
    else dseg_s_write(s1, tg, a.arena + a.Sp1 + (size_t)blk * nP1, a.nB, a.nA);
  }
  block_record_max<kSegThreads, false>(lmax, a.mx + (blk % kMaxSub) * a.mx_stride + a.slotZ);
  if (blk == 0 && threadIdx.x == 0) {
    const int eg = sh.exG + kg, exx = sh.exX + kx;
    a.ex[a.slotZ] = eg + sh.exM2 + sh.exM1;
    if (want2) a.ex[a.slotSp2] = eg + (exx + sh.exM1);
    if (want1) a.ex[a.slotSp1] = (eg + sh.exM2) + exx;
  }
}

template <int PREC>
__global__ __launch_bounds__(kSegThreads) void k_dseg_bwd(const DSegPair g) {
  const uint32_t second = blockIdx.x >= g.split ? 1u : 0u;
  dseg_bwd_body<PREC>(g.a[second], xcd_tile(blockIdx.x - second * g.split, second ? gridDim.x - g.split : g.split));
}

static DSegPair dseg_pair(const DSegArgs &a, const DSegArgs *b, unsigned &nb) {
  DSegPair g;
  g.a[0] = a;
  g.a[1] = b ? *b : a;
  g.split = dseg_blocks(a);
  nb = g.split + (b ? dseg_blocks(*b) : 0u);
  return g;
}
void launch_dseg_fwd(const DSegArgs &a, const DSegArgs *b, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  unsigned nb = 0;
  const DSegPair g = dseg_pair(a, b, nb);
  if (a.prec == 1) k_dseg_fwd<1><<<nb, kSegThreads, 0, s>>>(g);
  else if (a.prec == 2) k_dseg_fwd<2><<<nb, kSegThreads, 0, s>>>(g);
  else k_dseg_fwd<0><<<nb, kSegThreads, 0, s>>>(g);
}
void launch_dseg_bwd(const DSegArgs &a, const DSegArgs *b, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  unsigned nb = 0;
  const DSegPair g = dseg_pair(a, b, nb);
  if (a.prec == 1) k_dseg_bwd<1><<<nb, kSegThreads, 0, s>>>(g);
  else if (a.prec == 2) k_dseg_bwd<2><<<nb, kSegThreads, 0, s>>>(g);
  else k_dseg_bwd<0><<<nb, kSegThreads, 0, s>>>(g);
}

// --------------------------------------------------------------------------
// leaf preparation: evidence slicing (gather), indicator vectors, maxima;
// extra blocks clear the maxima of the tensors produced in this solve
// --------------------------------------------------------------------------
static constexpr int kPrepBatch = 8;  // loads in flight per thread in a leaf's gather

__global__ __launch_bounds__(kBlock) void k_prepare(PrepareArgs a) {
  const int b = blockIdx.y;
  const int n_lb = a.n_leaves + a.big_blk0[a.n_big];  // workgroups of leaves
  if ((int)blockIdx.x >= n_lb) {
    if (b != 0) return;
    const int n = a.reset_end - a.reset_begin;
    for (int i = (blockIdx.x - n_lb) * kBlock + threadIdx.x; i < n * kMaxSub; i += (gridDim.x - n_lb) * kBlock)
      a.mx[(i / n) * a.mx_stride + a.reset_begin + i % n] = 0u;
    return;
  }
  int li = blockIdx.x, sub = 0;
  if (li >= a.n_leaves) {  // a workgroup of a large leaf
    const int x = li - a.n_leaves;
    int j = 0;
    while (j + 1 < a.n_big && a.big_blk0[j + 1] <= x) ++j;
    li = a.big_leaf[j];
    sub = x - a.big_blk0[j];
  }
  const LeafDesc d = a.leaves[li];
  if (blockIdx.x < (unsigned)a.n_leaves && d.nsub > 1) return;  // prepared by its own workgroups
  const int nsub = d.nsub > 1 ? d.nsub : 1;
  if (!d.batched && b > 0) return;
  if (d.batched && a.interleaved) {
    // one thread per instance: element i of instance bi at i * max_batch + bi
    const int bi = b * kBlock + threadIdx.x;
    if (bi >= a.max_batch) return;
    gfloat *dst = (gfloat *)(a.arena + d.dst) + bi;
    const int64_t es = a.max_batch;
    float m = 1.f;
    if (d.kind == 0) {
      int64_t base = 0;
      for (int o = d.obs_begin; o < d.obs_end; ++o)
        base += (int64_t)a.evidence[(int64_t)bi * a.n_vars + a.obs[2 * o]] * a.obs[2 * o + 1];
      const float *src = a.arena + d.src + base;
      m = 0.f;
      if (d.ident) {
        for (int i = 0; i < d.size; ++i) {
          const float v = src[i];
          dst[i * es] = v;
          m = fmaxf(m, fabsf(v));
        }
      } else {
        for (int i = 0; i < d.size; ++i) {
          const float v = src[a.gmap[d.gmap + i]];
          dst[i * es] = v;
          m = fmaxf(m, fabsf(v));
        }
      }
    } else if (d.kind == 1) {
      const float one = d.maxdom ? 0.f : 1.f;
      for (int i = 0; i < d.size; ++i) dst[i * es] = one;
    } else {
      const float one = d.maxdom ? 0.f : 1.f, zero = d.maxdom ? -INFINITY : 0.f;
      const int e = a.evidence[(int64_t)bi * a.n_vars + d.var];
      for (int i = 0; i < d.size; ++i) dst[i * es] = (e < 0 || e == i) ? one : zero;
    }
    if (d.slot >= 0) {
      a.mx[d.slot + bi] = __float_as_uint(m);
      a.ex[d.slot + bi] = 0;
    }
    return;
  }
  const int row = d.batched ? b : 0;
  // element stride: interleaved batched leaves hold element i of instance b at i * max_batch + b
  float *dst = a.arena + d.dst + (d.batched ? (int64_t)b * d.size : 0);
  const float one = d.maxdom ? 0.f : 1.f;
  const float zero = d.maxdom ? -INFINITY : 0.f;
  float lmax = 0.f;
  const int i0 = sub * kBlock + threadIdx.x, istep = nsub * kBlock;
  if (d.kind == 0) {
    int64_t base = 0;
    for (int o = d.obs_begin; o < d.obs_end; ++o)
      base += (int64_t)a.evidence[(int64_t)row * a.n_vars + a.obs[2 * o]] * a.obs[2 * o + 1];
    const float *__restrict__ src = a.arena + d.src + base;
    const int32_t *__restrict__ gm = a.gmap + d.gmap;
    // a large leaf has at most kMaxSubSlots workgroups (one maximum each), so
    // every thread keeps kPrepBatch loads in flight: the map entries first
    // (none for an identity map), then the values, then the stores
    int i = i0;
    for (; i + (kPrepBatch - 1) * istep < d.size; i += kPrepBatch * istep) {
      int32_t o[kPrepBatch];
#pragma unroll
      for (int k = 0; k < kPrepBatch; ++k) o[k] = d.ident ? i + k * istep : gm[i + k * istep];
      float v[kPrepBatch];
#pragma unroll
      for (int k = 0; k < kPrepBatch; ++k) v[k] = src[o[k]];
#pragma unroll
      for (int k = 0; k < kPrepBatch; ++k) {
        dst[i + k * istep] = v[k];
        lmax = fmaxf(lmax, fabsf(v[k]));
      }
    }
    for (; i < d.size; i += istep) {
      const float v = src[d.ident ? i : gm[i]];
      dst[i] = v;
      lmax = fmaxf(lmax, fabsf(v));
    }
  } else if (d.kind == 1) {
    for (int i = i0; i < d.size; i += istep) dst[i] = one;
    lmax = 1.f;
  } else {
    const int e = a.evidence[(int64_t)row * a.n_vars + d.var];
    for (int i = i0; i < d.size; i += istep) dst[i] = (e < 0 || e == i) ? one : zero;
    lmax = 1.f;
  }
  __shared__ float sm[kBlock / 64];
  lmax = wave_max(lmax);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = lmax;
  __syncthreads();
  if (threadIdx.x == 0 && d.slot >= 0) {
    float m = sm[0];
    for (int w = 1; w < kBlock / 64; ++w) m = fmaxf(m, sm[w]);
    // workgroup sub of a large leaf: sub-slot sub (the same sub-slots on
    // every call, the others stay zero)
    a.mx[sub * a.mx_stride + d.slot + (d.batched ? b : 0)] = __float_as_uint(m);
    if (sub == 0) a.ex[d.slot + (d.batched ? b : 0)] = 0;
  }
}

void launch_prepare(const PrepareArgs &a, void *stream) {
  const int reset_blocks = (a.reset_end - a.reset_begin + kBlock - 1) / kBlock;
  // interleaved batched leaves take one thread per instance
  dim3 g(a.n_leaves + a.big_blk0[a.n_big] + (reset_blocks > 0 ? (reset_blocks > 1024 ? 1024 : reset_blocks) : 0),
         a.interleaved ? (a.batch + kBlock - 1) / kBlock : a.batch);
  if (g.x == 0) return;
  k_prepare<<<g, kBlock, 0, (hipStream_t)stream>>>(a);
}

// --------------------------------------------------------------------------
// log Z per instance, in FP64: ln(root) + ex * ln 2
// --------------------------------------------------------------------------
__global__ void k_logz(const float *root, int64_t bs, const int32_t *ex, int slot, int batched,
                       int batch, double *out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const float z = root[(int64_t)b * bs];
  const int e = ex[slot + (batched ? b : 0)];
  out[b] = z > 0.f ? log((double)z) + (double)e * 0.69314718055994530942 : -INFINITY;
}

void launch_logz(const float *root, int64_t bs, const int32_t *ex, int slot, int batched, int batch,
                 double *out, void *stream) {
  k_logz<<<(batch + 63) / 64, 64, 0, (hipStream_t)stream>>>(root, bs, ex, slot, batched, batch, out);
}

// --------------------------------------------------------------------------
// marginals: p(v = x | e) = adj(x) * lambda(x) / sum (MAR algorithm step 3)
// --------------------------------------------------------------------------
__global__ void k_marg(const float *arena, const MargDesc *d, int n, int batch, int row,
                       double *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= n || b >= batch) return;
  const MargDesc m = d[i];
  const float *adj = arena + m.adj + (m.adj_batched ? (int64_t)b * m.adj_bs : 0);
  const float *lam = arena + m.leaf + (m.leaf_batched ? (int64_t)b * m.leaf_bs : 0);
  double tot = 0.0;
  for (int x = 0; x < m.card; ++x) tot += (double)adj[x * m.adj_es] * (double)lam[x * m.leaf_es];
  for (int x = 0; x < m.card; ++x)
    out[(int64_t)b * row + m.out + x] =
        tot > 0.0 ? (double)adj[x * m.adj_es] * (double)lam[x * m.leaf_es] / tot : 0.0;
}

void launch_marg(const float *arena, const MargDesc *d, int n, int batch, int row, double *out,
                 void *stream) {
  if (n <= 0) return;
  dim3 g((n + 63) / 64, batch);
  k_marg<<<g, 64, 0, (hipStream_t)stream>>>(arena, d, n, batch, row, out);
}

// --------------------------------------------------------------------------
// d logZ / d T_f = adjoint / Z, scattered back through the leaf gather map
// --------------------------------------------------------------------------
__global__ void k_factor_grad(const float *arena, const GradDesc *d, int n, const int32_t *gmap,
                              const int32_t *obs, const int32_t *evidence, const int32_t *ex,
                              const float *root, int root_slot, float *grad) {
  const int f = blockIdx.x;
  if (f >= n) return;
  const GradDesc g = d[f];
  const double z = (double)root[0];
  const int er = ex[root_slot];
  int64_t base = 0;
  for (int o = g.obs_begin; o < g.obs_end; ++o) base += (int64_t)evidence[obs[2 * o]] * obs[2 * o + 1];
  const double sc = ldexp(1.0, ex[g.slot] - er) / z;
  for (int i = threadIdx.x; i < g.size; i += blockDim.x)
    grad[g.dst + base + gmap[g.gmap + i]] = (float)((double)arena[g.adj + i] * sc);
}

void launch_factor_grad(const float *arena, const GradDesc *d, int n, const int32_t *gmap,
                        const int32_t *obs, const int32_t *evidence, const int32_t *ex,
                        const float *root, int root_slot, int64_t n_values, float *grad,
                        void *stream) {
  (void)n_values;
  if (n <= 0) return;
  k_factor_grad<<<n, 256, 0, (hipStream_t)stream>>>(arena, d, n, gmap, obs, evidence, ex, root,
                                                    root_slot, grad);
}

// --------------------------------------------------------------------------
// factor marginals and joint marginals (one workgroup per table and instance)
// --------------------------------------------------------------------------
static constexpr int kMargThreads = 256;

__device__ __forceinline__ double block_sum_f64(double v, double *red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
#pragma unroll
  for (int h = kMargThreads / 2; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kMargThreads) void k_factor_marg(const float *arena, const GradDesc *d, int n,
                                                              const int32_t *gmap, const int32_t *obs,
                                                              const int32_t *evidence, int n_vars,
                                                              int64_t row, double *out) {
  __shared__ double red[kMargThreads];
  const int f = blockIdx.x, b = blockIdx.y;
  if (f >= n) return;
  const GradDesc g = d[f];
  const float *adj = arena + g.adj + (g.adj_batched ? (int64_t)b * g.adj_bs : 0);
  const float *leaf = arena + g.leaf + (g.leaf_batched ? (int64_t)b * g.leaf_bs : 0);
  const int64_t les = g.leaf_batched ? g.leaf_es : 1;
  double part = 0.0;
  for (int i = threadIdx.x; i < g.size; i += kMargThreads)
    part += (double)leaf[i * les] * (double)adj[(int64_t)i * g.adj_es];
  const double tot = block_sum_f64(part, red);
  double *o = out + (int64_t)b * row + g.dst;
  for (int j = threadIdx.x; j < g.full; j += kMargThreads) o[j] = 0.0;
  __syncthreads();  // the zeros before the consistent entries (same workgroup)
  int64_t base = 0;
  for (int k = g.obs_begin; k < g.obs_end; ++k) base += (int64_t)evidence[(int64_t)b * n_vars + obs[2 * k]] * obs[2 * k + 1];
  const double inv = tot > 0.0 ? 1.0 / tot : 0.0;
  for (int i = threadIdx.x; i < g.size; i += kMargThreads)
    o[base + gmap[g.gmap + i]] = (double)leaf[i * les] * (double)adj[(int64_t)i * g.adj_es] * inv;
}

void launch_factor_marg(const float *arena, const GradDesc *d, int n, const int32_t *gmap, const int32_t *obs,
                        const int32_t *evidence, int n_vars, int batch, int64_t row, double *out, void *stream) {
  if (n <= 0 || batch <= 0) return;
  k_factor_marg<<<dim3(n, batch), kMargThreads, 0, (hipStream_t)stream>>>(arena, d, n, gmap, obs, evidence, n_vars,
                                                                          row, out);
}

__global__ __launch_bounds__(kMargThreads) void k_joint(const float *arena, const JointDesc *d, int n,
                                                        const int32_t *tab, const int32_t *evidence, int n_vars,
                                                        int row, double *out) {
  __shared__ double red[kMargThreads];
  const int k = blockIdx.x, b = blockIdx.y;
  if (k >= n) return;
  const JointDesc j = d[k];
  const float *adj = j.adj >= 0 ? arena + j.adj + (j.adj_batched ? (int64_t)b * j.adj_bs : 0) : nullptr;
  const int32_t *ev = evidence + (int64_t)b * n_vars;
  // entry e of the whole table -> the unity tensor's entry (-1: an observed
  // variable takes another value)
  auto free_index = [&](int32_t e) -> int64_t {
    int64_t fi = 0;
    for (int t = j.v_end - 1; t >= j.v_begin; --t) {
      const int32_t var = tab[3 * t], card = tab[3 * t + 1], st = tab[3 * t + 2];
      const int32_t x = e % card;
      e /= card;
      if (st < 0) {
        if (x != ev[var]) return -1;
      } else {
        fi += (int64_t)x * st;
      }
    }
    return fi;
  };
  double part = 0.0;
  for (int32_t e = threadIdx.x; e < j.n_full; e += kMargThreads) {
    const int64_t fi = free_index(e);
    if (fi >= 0) part += adj ? (double)adj[fi * j.adj_es] : 1.0;
  }
  const double tot = block_sum_f64(part, red);
  const double inv = tot > 0.0 ? 1.0 / tot : 0.0;
  double *o = out + (int64_t)b * row + j.out;
  for (int32_t e = threadIdx.x; e < j.n_full; e += kMargThreads) {
    const int64_t fi = free_index(e);
    o[e] = fi >= 0 ? (adj ? (double)adj[fi * j.adj_es] : 1.0) * inv : 0.0;
  }
}

void launch_joint(const float *arena, const JointDesc *d, int n, const int32_t *tab, const int32_t *evidence,
                  int n_vars, int batch, int row, double *out, void *stream) {
  if (n <= 0 || batch <= 0) return;
  k_joint<<<dim3(n, batch), kMargThreads, 0, (hipStream_t)stream>>>(arena, d, n, tab, evidence, n_vars, row, out);
}

// --------------------------------------------------------------------------
// argmax readout (MPE configuration), one lane per instance
// --------------------------------------------------------------------------
// One workgroup per instance; the levels run in order, the steps of a level
// spread over the threads.  The assignment lives in LDS when it fits (else in
// global memory, fenced between levels).  Levels are taken in chunks: a
// chunk's steps, pairs and level boundaries are staged in LDS with one round
// of loads, so that a level costs one dependent global read (the argmax
// entry) instead of three (step, pairs, entry).
static constexpr int kBackLdsVars = 8192;

// pairs: the chunk's (var, stride / card) pairs, pair i at pairs[2 (i - p0)]
__device__ __forceinline__ void back_step(const int32_t *__restrict__ iarena, const BackStep &s,
                                          const int32_t *__restrict__ pairs, int p0, int b, int32_t *x) {
  int64_t off = 0;
  bool ok = true;
  for (int i = s.in_begin; i < s.in_end; ++i) {
    const int32_t xv = x[pairs[2 * (i - p0)]];
    ok = ok && xv >= 0;
    off += (int64_t)xv * pairs[2 * (i - p0) + 1];
  }
  if (!ok) return;  // an input left unassigned: leave this step's outputs unset
  int32_t k = iarena[s.arg + (int64_t)b * s.bs + off * s.es];
  for (int j = s.out_end - 1; j >= s.out_begin; --j) {
    const int c = pairs[2 * (j - p0) + 1];
    x[pairs[2 * (j - p0)]] = k % c;
    k /= c;
  }
}

template <bool LDS_X>
__global__ __launch_bounds__(kBlock) void k_backtrack(const int32_t *iarena, const BackStep *steps, const int32_t *lev,
                                                      int n_lev, int n_chunks, const int32_t *pairs, int n_vars,
                                                      int32_t *assign) {
  extern __shared__ int32_t xs[];
  __shared__ BackStep cs[kBackChunkSteps];
  __shared__ int32_t cp[2 * kBackChunkPairs];
  __shared__ int32_t cl[kBackChunkSteps + 1];
  const int b = blockIdx.x;
  int32_t *xg = assign + (int64_t)b * n_vars;
  int32_t *x = LDS_X ? xs : xg;
  if (LDS_X) {
    for (int i = threadIdx.x; i < n_vars; i += kBlock) xs[i] = xg[i];
    __syncthreads();
  }
  const int32_t *chunk = lev + n_lev + 1;
  for (int c = 0; c < n_chunks; ++c) {
    const int l0 = chunk[kBackChunkInts * c], l1 = chunk[kBackChunkInts * c + 1];
    const int s0 = chunk[kBackChunkInts * c + 2], s1 = chunk[kBackChunkInts * c + 3];
    const int p0 = chunk[kBackChunkInts * c + 4], p1 = chunk[kBackChunkInts * c + 5];
    const bool staged = s1 - s0 <= kBackChunkSteps && p1 - p0 <= kBackChunkPairs && l1 - l0 <= kBackChunkSteps;
    if (staged) {  // the previous chunk's last level ended with a barrier
      for (int i = threadIdx.x; i < s1 - s0; i += kBlock) cs[i] = steps[s0 + i];
      for (int i = threadIdx.x; i < 2 * (p1 - p0); i += kBlock) cp[i] = pairs[2 * p0 + i];
      for (int i = threadIdx.x; i <= l1 - l0; i += kBlock) cl[i] = lev[l0 + i];
      __syncthreads();
      for (int l = 0; l < l1 - l0; ++l) {
        for (int st = cl[l] + threadIdx.x; st < cl[l + 1]; st += kBlock) back_step(iarena, cs[st - s0], cp, p0, b, x);
        if (!LDS_X) __threadfence();
        __syncthreads();
      }
    } else {
      for (int l = l0; l < l1; ++l) {
        for (int st = lev[l] + threadIdx.x; st < lev[l + 1]; st += kBlock) back_step(iarena, steps[st], pairs, 0, b, x);
        if (!LDS_X) __threadfence();
        __syncthreads();
      }
    }
  }
  if (LDS_X)
    for (int i = threadIdx.x; i < n_vars; i += kBlock) xg[i] = xs[i];
}

void launch_backtrack(const int32_t *iarena, const BackStep *steps, const int32_t *lev, int n_lev, int n_chunks,
                      const int32_t *pairs, int n_vars, int batch, int32_t *assign, void *stream) {
  if (n_lev <= 0) return;
  hipStream_t s = (hipStream_t)stream;
  if (n_vars <= kBackLdsVars)
    k_backtrack<true><<<batch, kBlock, (size_t)n_vars * sizeof(int32_t), s>>>(iarena, steps, lev, n_lev, n_chunks,
                                                                                pairs, n_vars, assign);
  else
    k_backtrack<false><<<batch, kBlock, 0, s>>>(iarena, steps, lev, n_lev, n_chunks, pairs, n_vars, assign);
}

// --------------------------------------------------------------------------
// sampling along the tree (eq. sample / eq. condition-prob)
// --------------------------------------------------------------------------

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications with the Weyl-sequence key schedule.
__host__ __device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
  }
}

__host__ __device__ __forceinline__ double uniform53(uint64_t sample, uint32_t node, uint32_t slot,
                                                     uint64_t seed) {
  uint32_t c[4] = {(uint32_t)sample, (uint32_t)(sample >> 32), node, slot};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  return ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6)) * (1.0 / 9007199254740992.0);
}

// meta quadruples (var, card, strideA, strideB)
// k < the labels' assignment count, below 2^31 (a tensor's entries): 32-bit
// division
__device__ __forceinline__ void decode_offsets(int64_t k64, const int32_t *q, int qb, int qe,
                                               int64_t &oa, int64_t &ob) {
  uint32_t k = (uint32_t)k64;
  oa = 0;
  ob = 0;
  for (int j = qe - 1; j >= qb; --j) {
    const uint32_t c = (uint32_t)q[4 * j + 1];
    const uint32_t h = k / c, d = k - h * c;
    k = h;
    oa += (int64_t)d * q[4 * j + 2];
    ob += (int64_t)d * q[4 * j + 3];
  }
}
// assigns the labels' values of index k into the row x; `write`: whether
// this lane writes (one lane for a row in LDS, every lane for a row in
// global memory, whose lanes read back only their own writes)
__device__ __forceinline__ void decode_assign(int64_t k64, const int32_t *q, int qb, int qe, int32_t *x,
                                              bool write = true) {
  uint32_t k = (uint32_t)k64;
  for (int j = qe - 1; j >= qb; --j) {
    const uint32_t c = (uint32_t)q[4 * j + 1];
    const uint32_t h = k / c;
    if (write) x[q[4 * j]] = (int32_t)(k - h * c);
    k = h;
  }
}
__device__ __forceinline__ int64_t count_of(const int32_t *q, int qb, int qe) {
  int64_t n = 1;
  for (int j = qb; j < qe; ++j) n *= q[4 * j + 1];
  return n;
}

double sample_uniform(uint64_t sample, uint32_t node, uint32_t slot, uint64_t seed) {
  return uniform53(sample, node, slot, seed);
}

// One wavefront per sample.  A categorical draw over n entries in canonical
// order: lane l sums the weights of its contiguous chunk, an exclusive scan
// over the lanes gives each chunk's starting cumulative weight, and the lane
// whose chunk holds the target scans it: the first entry with positive
// weight whose cumulative weight exceeds u * total (the last positive entry
// if rounding leaves the target at the end) - the sequential rule, with the
// sum associated chunk-wise.
template <class W>
__device__ __forceinline__ int64_t wave_draw(int64_t n, double u, W weight) {
  const int lane = threadIdx.x & 63;
  const int64_t ch = (n + 63) / 64, b0 = min(n, lane * ch), b1 = min(n, b0 + ch);
  double part = 0.0;
  int64_t lastpos = -1;
  for (int64_t k = b0; k < b1; ++k) {
    const double w = weight(k);
    part += w;
    if (w > 0.0) lastpos = k;
  }
  double incl = part;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  const double total = __shfl(incl, 63, 64);
  const double excl = incl - part;
  const double target = u * total;
  const bool mine = part > 0.0 && incl > target;
  const uint64_t m = __ballot(mine);
  int64_t pick = -1;
  if (m) {
    const int L = __ffsll((unsigned long long)m) - 1;
    if (lane == L) {
      double cum = excl;
      for (int64_t k = b0; k < b1; ++k) {
        const double w = weight(k);
        cum += w;
        if (w > 0.0 && cum > target) {
          pick = k;
          break;
        }
      }
      if (pick < 0) pick = lastpos;
    }
    pick = __shfl(pick, L, 64);
  } else {
    // rounding: the last entry with positive weight (0 if none)
    int64_t lp = lastpos;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lp = max(lp, (int64_t)__shfl_xor(lp, o, 64));
    pick = lp < 0 ? 0 : lp;
  }
  return pick;
}

// Rows of up to kSampleLdsVars variables are built in LDS (one row per
// wavefront, written by lane 0: LDS instructions of a wavefront complete in
// order, so every lane's later read sees them) and copied out at the end;
// longer rows are built in place in global memory, every lane writing every
// value (each lane then reads back only its own writes).
static constexpr int kSampleLdsVars = 2048;

template <bool LDS>
__global__ void k_sample(const float *arena, const SampleStep *steps, int n_steps, const int32_t *q,
                         int n_vars, int64_t n, uint64_t seed, const int32_t *init, const int64_t *ids,
                         int32_t *out) {
  __shared__ int32_t rows[LDS ? 4 * kSampleLdsVars : 1];
  const int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (j >= n) return;  // whole waves (no workgroup barrier below)
  const int lane = threadIdx.x & 63;
  const int64_t s = ids ? ids[j] : j;
  int32_t *x = LDS ? rows + (threadIdx.x >> 6) * kSampleLdsVars : out + s * n_vars;
  const bool w = !LDS || lane == 0;  // lanes that write the row
  if (LDS) {
    for (int v = lane; v < n_vars; v += 64) x[v] = init[v];
    __builtin_amdgcn_wave_barrier();
  } else {
    for (int v = 0; v < n_vars; ++v) x[v] = init[v];
  }
  for (int t = 0; t < n_steps; ++t) {
    const SampleStep st = steps[t];
    const float *A = arena + st.A;
    const float *B = st.B >= 0 ? arena + st.B : nullptr;
    const float *Ar = arena + st.Ar;
    const float *Br = st.Br >= 0 ? arena + st.Br : nullptr;
    // offsets of the labels already drawn, in each child and its reduction
    int64_t oa = 0, ob = 0, oar = 0, obr = 0;
    bool ok = true;
    for (int i = st.aIn_b; i < st.aIn_e; ++i) {
      const int32_t xv = x[q[4 * i]];
      ok = ok && xv >= 0;
      oa += (int64_t)xv * q[4 * i + 2];
      oar += (int64_t)xv * q[4 * i + 3];
    }
    for (int i = st.bIn_b; i < st.bIn_e; ++i) {
      const int32_t xv = x[q[4 * i]];
      ok = ok && xv >= 0;
      ob += (int64_t)xv * q[4 * i + 2];
      obr += (int64_t)xv * q[4 * i + 3];
    }
    if (!ok) continue;  // an input left unassigned: leave this step's outputs unset (uniform)
    // shared eliminated labels: w(k) = Ar[z, k] * Br[z, k]
    if (st.k_e > st.k_b) {
      const int64_t nK = count_of(q, st.k_b, st.k_e);
      const int64_t pick = wave_draw(nK, uniform53((uint64_t)s, (uint32_t)st.node, 0u, seed), [&](int64_t k) {
        int64_t ka, kb;
        decode_offsets(k, q, st.kr_b, st.kr_e, ka, kb);
        return (double)Ar[oar + ka] * (Br ? (double)Br[obr + kb] : 1.0);
      });
      int64_t ka, kb;
      decode_offsets(pick, q, st.k_b, st.k_e, ka, kb);
      decode_assign(pick, q, st.k_b, st.k_e, x, w);
      if (LDS) __builtin_amdgcn_wave_barrier();
      oa += ka;
      ob += kb;
    }
    // private labels of each child, drawn from the child itself
    for (int side = 0; side < 2; ++side) {
      const int pb = side ? st.pb_b : st.pa_b, pe = side ? st.pb_e : st.pa_e;
      if (pe <= pb) continue;
      const float *T = side ? B : A;
      const int64_t base = side ? ob : oa;
      const int64_t nP = count_of(q, pb, pe);
      const int64_t pick = wave_draw(nP, uniform53((uint64_t)s, (uint32_t)st.node, 1u + side, seed), [&](int64_t p) {
        int64_t da, db;
        decode_offsets(p, q, pb, pe, da, db);
        return (double)T[base + (side ? db : da)];
      });
      decode_assign(pick, q, pb, pe, x, w);
      if (LDS) __builtin_amdgcn_wave_barrier();
    }
  }
  if (LDS) {
    int32_t *o = out + s * n_vars;
    for (int v = lane; v < n_vars; v += 64) o[v] = x[v];
  }
}

void launch_sample(const float *arena, const SampleStep *steps, int n_steps, const int32_t *meta,
                   int n_vars, int64_t n, uint64_t seed, const int32_t *init, const int64_t *ids,
                   int32_t *out, void *stream) {
  if (n <= 0) return;
  const int64_t blocks = (n + 3) / 4;  // four samples (waves) per workgroup
  if (n_vars <= kSampleLdsVars)
    k_sample<true><<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(arena, steps, n_steps, meta, n_vars, n,
                                                                     seed, init, ids, out);
  else
    k_sample<false><<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(arena, steps, n_steps, meta, n_vars, n,
                                                                      seed, init, ids, out);
}

// --------------------------------------------------------------------------
// Library-held staging for the allocation-free sampler: one copy of this
// array per GPU, alive until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is a stand-in, not a device
// address): scratch_ptr() looks up each device's address once with
// hipGetSymbolAddress, with that device current, and keeps it.
// --------------------------------------------------------------------------
static __device__ __align__(256) int32_t scratch[kScratchInts];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t *g_scratch_dev[kMaxDevices] = {};
}  // namespace

int32_t *scratch_ptr(int dev, std::string &err) {
  if (dev < 0 || dev >= kMaxDevices) {
    err = "device id out of range";
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[dev]) return g_scratch_dev[dev];
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
  void *ptr = nullptr;
  if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (cur >= 0 && cur != dev) {
    const hipError_t e2 = hipSetDevice(cur);
    if (e == hipSuccess) e = e2;
  }
  if (e != hipSuccess || !ptr) {
    err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return nullptr;
  }
  g_scratch_dev[dev] = (int32_t *)ptr;
  return g_scratch_dev[dev];
}

// --------------------------------------------------------------------------
// domain conversion for the MMAP max phase: log(raw) + ex * ln 2 (FP64 math)
// --------------------------------------------------------------------------
__global__ void k_tolog(const float *src, const int32_t *ex, int slot, int64_t n, float *dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v = src[i];
  dst[i] = v > 0.f ? (float)(log((double)v) + (double)ex[slot] * 0.69314718055994530942) : -INFINITY;
}

void launch_tolog(const float *src, const int32_t *ex, int slot, int64_t n, float *dst, void *stream) {
  if (n <= 0) return;
  k_tolog<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(src, ex, slot, n, dst);
}

// --------------------------------------------------------------------------
// slice accumulation (FP64): acc = sum over slices of raw * 2^ex; the first
// slice fixes the reference exponent acc_ex
// --------------------------------------------------------------------------
__global__ void k_slice_acc(const float *src, const int32_t *ex, int slot, double *acc,
                            int32_t *acc_ex, int64_t n, int first) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int es = ex[slot];
  if (first) {
    if (i == 0) acc_ex[0] = es;
    if (i < n) acc[i] = (double)src[i];
  } else if (i < n) {
    acc[i] += ldexp((double)src[i], es - acc_ex[0]);
  }
}

void launch_slice_acc(const float *src, const uint32_t *mx, const int32_t *ex, int slot_src, double *acc,
                      int32_t *acc_ex, int64_t n, int first, void *stream) {
  (void)mx;
  k_slice_acc<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(src, ex, slot_src, acc, acc_ex, n,
                                                                             first);
}

__global__ void k_acc_tolog(const double *acc, const int32_t *acc_ex, int64_t n, float *dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = acc[i];
  dst[i] = v > 0.0 ? (float)(log(v) + (double)acc_ex[0] * 0.69314718055994530942) : -INFINITY;
}

void launch_acc_tolog(const double *acc, const int32_t *acc_ex, int64_t n, float *dst, void *stream) {
  if (n <= 0) return;
  k_acc_tolog<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(acc, acc_ex, n, dst);
}

}  // namespace tn
