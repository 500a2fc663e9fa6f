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

#include "tn_internal.h"

namespace tn {

static constexpr int kBlock = 256;

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
  const uint32_t v = mx[(threadIdx.x & 63) * stride + slot];
  return __float_as_uint(wave_max(__uint_as_float(v)));
}

// Record the block's maximum in *slot.  One candidate per block; the atomic
// is skipped when the stored value is already larger (maxima only grow
// within a launch, so a stale read only costs an unneeded atomic).
template <int NT = kBlock>
__device__ __forceinline__ void block_record_max(float v, uint32_t *slot) {
  __shared__ float red[NT / 64];
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = red[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) m = fmaxf(m, red[w]);
    if (m > 0.f && __uint_as_float(*(volatile uint32_t *)slot) < m) atomicMax(slot, __float_as_uint(m));
  }
}

__device__ __forceinline__ int32_t tab_off(const Tab2 &t, uint32_t i, uint32_t nlo) {
  uint32_t h = i / nlo;
  return t.hi[h] + t.lo[i - h * nlo];
}

// --------------------------------------------------------------------------
// generic contraction, one lane per output element
// --------------------------------------------------------------------------
template <int SEMI, bool HASY>
__device__ __forceinline__ void map_body(const ContractArgs &a, const int b, const uint32_t blk,
                                         const uint32_t nblk) {
  const float *__restrict__ X = a.X + (int64_t)b * a.bsX;
  const float *__restrict__ Y = HASY ? a.Y + (int64_t)b * a.bsY : nullptr;
  float *__restrict__ Z = a.Z + (int64_t)b * a.bsZ;
  int32_t *__restrict__ I = SEMI == SEMI_MAX ? a.I + (int64_t)b * a.bsZ : nullptr;
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
  float lmax = 0.f;
  for (uint32_t o = blk * kBlock + threadIdx.x; o < n_out; o += nblk * kBlock) {
    uint32_t r, c;
    if (colf) {
      r = o / nC;
      c = o - r * nC;
    } else {
      c = o / nR;
      r = o - c * nR;
    }
    const uint32_t rh = r / nRl, rl = r - rh * nRl;
    const int32_t xo = rX.hi[rh] + rX.lo[rl];
    int32_t zo = rZ.hi[rh] + rZ.lo[rl];
    int32_t yo = HASY ? rY.hi[rh] + rY.lo[rl] : 0;
    if (nC > 1) {
      const uint32_t ch = c / nCl, cl = c - ch * nCl;
      zo += cZ.hi[ch] + cZ.lo[cl];
      if (HASY) yo += cY.hi[ch] + cY.lo[cl];
    }
    if (SEMI == SEMI_SUM) {
      float acc = 0.f;
      for (uint32_t sh = 0; sh < nSh; ++sh) {
        const int32_t xs = xo + sXt.hi[sh];
        const int32_t ys = HASY ? yo + sYt.hi[sh] : 0;
        for (uint32_t sl = 0; sl < nSl; ++sl) {
          const float xv = X[xs + sXt.lo[sl]] * sx;
          if (HASY)
            acc = fmaf(xv, Y[ys + sYt.lo[sl]] * sy, acc);
          else
            acc += xv;
        }
      }
      Z[zo] = acc;
      lmax = fmaxf(lmax, acc);
    } else {
      float best = -INFINITY;
      int32_t bi = 0;
      uint32_t s = 0;
      for (uint32_t sh = 0; sh < nSh; ++sh) {
        const int32_t xs = xo + sXt.hi[sh];
        const int32_t ys = HASY ? yo + sYt.hi[sh] : 0;
        for (uint32_t sl = 0; sl < nSl; ++sl, ++s) {
          float v = X[xs + sXt.lo[sl]];
          if (HASY) v = v + Y[ys + sYt.lo[sl]];
          if (s == 0 || v > best) {
            best = v;
            bi = (int32_t)s;
          }
        }
      }
      Z[zo] = best;
      I[zo] = bi;
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
  const float *__restrict__ X = a.X + (int64_t)b * a.bsX;
  const float *__restrict__ Y = HASY ? a.Y + (int64_t)b * a.bsY : nullptr;
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
  float *__restrict__ Z = a.Z + (int64_t)b * a.bsZ;
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
    int32_t *__restrict__ I = a.I + (int64_t)b * a.bsZ;
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
  const float *__restrict__ X = a.X + (int64_t)b * a.bsX;
  const float *__restrict__ Y = HASY ? a.Y + (int64_t)b * a.bsY : nullptr;
  float *__restrict__ Z = a.Z + (int64_t)b * a.bsZ;
  int32_t *__restrict__ I = SEMI == SEMI_MAX ? a.I + (int64_t)b * a.bsZ : nullptr;
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
  for (uint32_t r = blk * kBlock + threadIdx.x; r < nR; r += nblk * kBlock) {
    uint32_t rh, rl;
    if (rls >= 0) {
      rh = r >> rls;
      rl = r & (nRl - 1);
    } else {
      rh = r / nRl;
      rl = r - rh * nRl;
    }
    const int32_t xo = rXh[rh] + rXl[rl];
    const int32_t zo = rZh[rh] + rZl[rl];
    const int32_t yo = HASY ? rYh[rh] + rYl[rl] : 0;
    float xv[B];
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (k < ns) xv[k] = SEMI == SEMI_SUM ? X[xo + sx[k]] * fx : X[xo + sx[k]];
#pragma unroll
    for (int c = 0; c < B; ++c) {
      if (c >= nc) continue;
      const int32_t yc = yo + cy[c];
      if (SEMI == SEMI_SUM) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < B; ++k)
          if (k < ns) acc = HASY ? fmaf(xv[k], Y[yc + sy[k]] * fy, acc) : acc + xv[k];
        Z[zo + cz[c]] = acc;
        lmax = fmaxf(lmax, acc);
      } else {
        float best = -INFINITY;
        int32_t bi = 0;
#pragma unroll
        for (int k = 0; k < B; ++k)
          if (k < ns) {
            float v = xv[k];
            if (HASY) v = v + Y[yc + sy[k]];
            if (k == 0 || v > best) {
              best = v;
              bi = k;
            }
          }
        Z[zo + cz[c]] = best;
        I[zo + cz[c]] = bi;
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

template <int SEMI, bool HASY>
__device__ __forceinline__ void any_map_body(const ContractArgs &a, const int b, const uint32_t blk,
                                             const uint32_t nblk) {
  if (a.kind == 1) {
    if (a.ns <= 4 && a.nc <= 4) rows_body<SEMI, HASY, 4>(a, b, blk, nblk);
    else rows_body<SEMI, HASY, kRowMax>(a, b, blk, nblk);
  } else {
    map_body<SEMI, HASY>(a, b, blk, nblk);
  }
}

// Arguments live in device memory (a pointer is the only kernel argument):
// large by-value argument blocks cost microseconds per launch.
template <int SEMI, bool HASY>
__global__ __launch_bounds__(kBlock) void k_map(const ContractArgs *__restrict__ ap) {
  any_map_body<SEMI, HASY>(*ap, blockIdx.y, blockIdx.x, gridDim.x);
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
// schedule).  Block ranges: op i owns blocks [start[i], start[i+1]), split
// as instance-major (b, blk) with nblk[i] blocks per instance.
__device__ __forceinline__ int find_op(const uint32_t *start, int n, uint32_t x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int SEMI, int PHASE>
__global__ __launch_bounds__(kBlock) void k_group(const ContractArgs *__restrict__ ops,
                                                  const uint32_t *__restrict__ start,
                                                  const uint32_t *__restrict__ nblk, int n) {
  const int i = find_op(start, n, blockIdx.x);
  const ContractArgs &a = ops[i];
  const uint32_t local = blockIdx.x - start[i];
  const uint32_t per = nblk[i];
  const int b = (int)(local / per);
  const uint32_t blk = local - (uint32_t)b * per;
  const bool hy = a.Y != nullptr;
  if (PHASE == 0) {
    if (hy) any_map_body<SEMI, true>(a, b, blk, per);
    else any_map_body<SEMI, false>(a, b, blk, per);
  } else if (PHASE == 1) {
    if (hy) split_body<SEMI, true>(a, b, blk);
    else split_body<SEMI, false>(a, b, blk);
  } else {
    if (hy) finish_body<SEMI, true>(a, b, blk);
    else finish_body<SEMI, false>(a, b, blk);
  }
}

void launch_group(int semi, int phase, const ContractArgs *ops, const uint32_t *start, const uint32_t *nblk,
                  int n, uint32_t total_blocks, void *stream) {
  if (n <= 0 || total_blocks == 0) return;
  hipStream_t s = (hipStream_t)stream;
  dim3 g(total_blocks);
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
  const uint32_t n_out = a.kind == 1 ? a.nR : a.nR * a.nC;
  uint32_t blocks = (n_out + kBlock - 1) / kBlock;
  return blocks > 2048u ? 2048u : blocks;
}

void launch_contract(int semi, bool has_y, bool split, const ContractArgs &a, const ContractArgs *d_a, int nb,
                     void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const uint32_t n_out = a.nR * a.nC;
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
__device__ __forceinline__ int32_t outer_off(const Tab2 &t, uint32_t o, uint32_t nlo) {
  const uint32_t h = o / nlo;
  return t.hi[h] + t.lo[o - h * nlo];
}

static constexpr int kSegBlock = 256;
static constexpr int kSegOB = 32;       // outer assignments per block (one 128-byte line of floats)
static constexpr int kSegOBP = kSegOB + 1;  // padded tile row (no LDS bank conflicts in either mapping)

// LDS (floats) of a segment launch: index lists, per-triple coefficients,
// then the tiles (entry-major rows of kSegOBP).
size_t seg_fwd_lds(const SegArgs &a) {
  return ((size_t)a.list_len + 64 * a.n_steps + 2 * (size_t)a.te * kSegOBP) * sizeof(float);
}
size_t seg_bwd_lds(const SegArgs &a) {
  return ((size_t)a.list_len + 64 * a.n_steps + (size_t)(a.n_steps + 2) * a.te * kSegOBP + a.n_sb) *
         sizeof(float);
}
// one slab of kSegOB outer assignments per block
static unsigned seg_blocks(const SegArgs &a) { return (a.nO + kSegOB - 1) / kSegOB; }
unsigned seg_grid(const SegArgs &a) { return seg_blocks(a); }

// Stage the segment's constants in LDS in one phase: the index lists and
// the small operands' raw values.  Inside a segment the small operands are
// used unscaled (their exponents add to the output's); only the carrier is
// renormalised.  Returns the sum of the small operands' exponents.
__device__ __forceinline__ int seg_stage(const SegArgs &a, int32_t *li, float *yv) {
  for (int e = threadIdx.x; e < a.list_len; e += kSegBlock) li[e] = a.lists[e];
  int ey = 0;
  for (int i = 0; i < a.n_steps; ++i) {
    const SegStep &st = a.steps[i];
    ey += a.ex[st.yslot];
    for (int e = threadIdx.x; e < st.ny; e += kSegBlock) yv[i * 64 + e] = a.arena[st.y + e];
  }
  __syncthreads();
  return ey;
}

__device__ __forceinline__ int32_t seg_outer(const SegArgs &a, const Tab2 &ot, uint32_t og) {
  if (a.ol_shift >= 0) return ot.hi[og >> a.ol_shift] + ot.lo[og & (a.nOl - 1)];
  return outer_off(ot, og, a.nOl);
}

// Move a slab (n entries x kSegOB outer assignments) between a carrier in
// global memory and an LDS tile.  The thread mapping puts consecutive
// threads on consecutive addresses of the carrier: outer-fastest when the
// carrier's stride-1 label is an outer label, entry-fastest otherwise.
template <bool LOAD>
__device__ __forceinline__ float seg_slab(const SegArgs &a, const float *src, float *dst, const Tab2 &ot,
                                          const int32_t *loc, int n, bool outer_fast, uint32_t o0, float *tile,
                                          float scale) {
  float lmax = 0.f;
  const int tasks = n * kSegOB;
  for (int t = threadIdx.x; t < tasks; t += kSegBlock) {
    int j, o;
    if (outer_fast) {
      j = t / kSegOB;
      o = t - j * kSegOB;
    } else {
      o = t / n;
      j = t - o * n;
    }
    const uint32_t og = o0 + o;
    if (LOAD) {
      tile[j * kSegOBP + o] = og < a.nO ? src[seg_outer(a, ot, og) + loc[j]] * scale : 0.f;
    } else if (og < a.nO) {
      const float v = tile[j * kSegOBP + o];
      dst[seg_outer(a, ot, og) + loc[j]] = v;
      lmax = fmaxf(lmax, v);
    }
  }
  return lmax;
}

// One step on the tiles: out[j][o] = sum over the triples of entry j of
// in[i][o] * coef.  All threads share the (entry, outer) tasks.
__device__ __forceinline__ void seg_apply(const int32_t *pp, const int32_t *ix, const int32_t *sx, const float *yv,
                                          int n_out, const float *tin, float *tout) {
  const int tasks = n_out * kSegOB;
  for (int t = threadIdx.x; t < tasks; t += kSegBlock) {
    const int j = t / kSegOB, o = t - j * kSegOB;
    float acc = 0.f;
    for (int e = pp[j]; e < pp[j + 1]; ++e) acc = fmaf(tin[ix[e] * kSegOBP + o], yv[sx[e]], acc);
    tout[j * kSegOBP + o] = acc;
  }
}

// Forward: input carrier slab -> steps -> output carrier slab, one slab of
// kSegOB outer assignments per block.
__global__ __launch_bounds__(kSegBlock) void k_seg_fwd(const SegArgs *__restrict__ ap) {
  const SegArgs &a = *ap;
  extern __shared__ float lds[];
  int32_t *li = (int32_t *)lds;
  float *yv = lds + a.list_len;
  float *t0 = yv + 64 * a.n_steps;
  float *t1 = t0 + (size_t)a.te * kSegOBP;
  const int kx = max_exponent(read_max(a.mx, a.mx_stride, a.slotX));
  const uint32_t o0 = blockIdx.x * kSegOB;
  seg_slab<true>(a, a.arena + a.X, nullptr, a.oX, a.inX, a.n_in0, a.in_outer_fast, o0, t0, ldexpf(1.f, -kx));
  const int esum = a.ex[a.slotX] + kx + seg_stage(a, li, yv);
  for (int i = 0; i < a.n_steps; ++i) {
    const SegStep &st = a.steps[i];
    seg_apply(li + st.fo_ptr, li + st.fo_in, li + st.fo_s, yv + i * 64, st.n_out, t0, t1);
    __syncthreads();
    float *tmp = t0;
    t0 = t1;
    t1 = tmp;
  }
  const float lmax =
      seg_slab<false>(a, nullptr, a.arena + a.Z, a.oZ, a.outZ, a.n_outL, a.out_outer_fast, o0, t0, 1.f);
  block_record_max<kSegBlock>(lmax, a.mx + (blockIdx.x % kMaxSub) * a.mx_stride + a.slotZ);
  if (blockIdx.x == 0 && threadIdx.x == 0) a.ex[a.slotZ] = esum;
}

// Reverse pass of a segment: recompute the carrier tiles of the slab from
// the input carrier, then run the steps backwards (eq. einback per step).
// The adjoint tile flows to the input carrier's adjoint (triples grouped by
// input entry); every small operand's adjoint entry is a sum over its
// triples (grouped by small entry) and over the slab, written per block to
// `part` and summed in a fixed order by k_seg_bwd_finish.
__global__ __launch_bounds__(kSegBlock) void k_seg_bwd(const SegArgs *__restrict__ ap) {
  const SegArgs &a = *ap;
  extern __shared__ float lds[];
  const int te = a.te, L = a.n_steps;
  int32_t *li = (int32_t *)lds;
  float *yv = lds + a.list_len;
  float *T = yv + 64 * L;                            // L tiles: input tile of every step
  float *g0 = T + (size_t)L * te * kSegOBP;
  float *g1 = g0 + (size_t)te * kSegOBP;
  float *sbw = g1 + (size_t)te * kSegOBP;            // n_sb block totals
  const int kx = max_exponent(read_max(a.mx, a.mx_stride, a.slotX));
  const int kg = max_exponent(read_max(a.mx, a.mx_stride, a.slotG));
  const uint32_t o0 = blockIdx.x * kSegOB;
  seg_slab<true>(a, a.arena + a.X, nullptr, a.oX, a.inX, a.n_in0, a.in_outer_fast, o0, T, ldexpf(1.f, -kx));
  seg_slab<true>(a, a.arena + a.G, nullptr, a.oZ, a.outZ, a.n_outL, a.out_outer_fast, o0, g0, ldexpf(1.f, -kg));
  for (int k = threadIdx.x; k < a.n_sb; k += kSegBlock) sbw[k] = 0.f;
  const int ey = seg_stage(a, li, yv);
  for (int i = 0; i + 1 < L; ++i) {
    const SegStep &st = a.steps[i];
    seg_apply(li + st.fo_ptr, li + st.fo_in, li + st.fo_s, yv + i * 64, st.n_out, T + (size_t)i * te * kSegOBP,
              T + (size_t)(i + 1) * te * kSegOBP);
    __syncthreads();
  }
  for (int i = L - 1; i >= 0; --i) {
    const SegStep &st = a.steps[i];
    const float *tin = T + (size_t)i * te * kSegOBP;
    if (st.sb_off >= 0) {
      // (small entry, outer) tasks; the 32 outer assignments of one entry
      // are 32 consecutive lanes, summed with shuffles
      const int32_t *pp = li + st.bs_ptr, *xi = li + st.bs_in, *xo = li + st.bs_out;
      const int tasks = st.ny * kSegOB;
      for (int t0 = 0; t0 < tasks; t0 += kSegBlock) {
        const int t = t0 + threadIdx.x;
        float acc = 0.f;
        int s2 = 0;
        if (t < tasks) {
          s2 = t / kSegOB;
          const int o = t - s2 * kSegOB;
          for (int e = pp[s2]; e < pp[s2 + 1]; ++e)
            acc = fmaf(g0[xo[e] * kSegOBP + o], tin[xi[e] * kSegOBP + o], acc);
        }
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (t < tasks && (t & (kSegOB - 1)) == 0) sbw[st.sb_off + s2] += acc;
      }
    }
    seg_apply(li + st.bi_ptr, li + st.bi_out, li + st.bi_s, yv + i * 64, st.n_in, g0, g1);
    __syncthreads();
    float *tmp = g0;
    g0 = g1;
    g1 = tmp;
  }
  const float lmax =
      seg_slab<false>(a, nullptr, a.arena + a.Z, a.oX, a.inX, a.n_in0, a.in_outer_fast, o0, g0, 1.f);
  block_record_max<kSegBlock>(lmax, a.mx + (blockIdx.x % kMaxSub) * a.mx_stride + a.slotZ);
  for (int k = threadIdx.x; k < a.n_sb; k += kSegBlock) a.part[(size_t)blockIdx.x * a.n_sb + k] = sbw[k];
  if (blockIdx.x == 0 && threadIdx.x == 0) a.ex[a.slotZ] = a.ex[a.slotG] + kg + ey;
}

// Sum the per-block partials of every small-operand adjoint entry (fixed
// order) and record maxima and exponents.
__global__ __launch_bounds__(256) void k_seg_bwd_finish(const SegArgs *__restrict__ ap, int n_blocks) {
  const SegArgs &a = *ap;
  const int k = blockIdx.x;
  float acc = 0.f;
  for (int w = threadIdx.x; w < n_blocks; w += 256) acc += a.part[(size_t)w * a.n_sb + k];
  __shared__ float red[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  const int kx = max_exponent(read_max(a.mx, a.mx_stride, a.slotX));
  const int kg = max_exponent(read_max(a.mx, a.mx_stride, a.slotG));
  int ey = 0, step = -1, sidx = 0, ei = 0;
  for (int i = 0; i < a.n_steps; ++i) {
    const SegStep &st = a.steps[i];
    const int e = a.ex[st.yslot];
    ey += e;
    if (st.sb_off >= 0 && k >= st.sb_off && k < st.sb_off + st.ny) {
      step = i;
      sidx = k - st.sb_off;
      ei = e;
    }
  }
  if (threadIdx.x == 0 && step >= 0) {
    const SegStep &st = a.steps[step];
    const float t = red[0] + red[1] + red[2] + red[3];
    a.arena[st.ybar + sidx] = t;
    if (t > 0.f) atomicMax(a.mx + (sidx % kMaxSub) * a.mx_stride + st.ybar_slot, __float_as_uint(t));
    if (sidx == 0) a.ex[st.ybar_slot] = (a.ex[a.slotG] + kg) + (a.ex[a.slotX] + kx) + (ey - ei);
  }
}

void launch_seg_fwd(const SegArgs &a, const SegArgs *d_a, void *stream) {
  const unsigned blocks = seg_blocks(a);
  k_seg_fwd<<<blocks, kSegBlock, seg_fwd_lds(a), (hipStream_t)stream>>>(d_a);
}

void launch_seg_bwd(const SegArgs &a, const SegArgs *d_a, void *stream) {
  const unsigned blocks = seg_blocks(a);
  k_seg_bwd<<<blocks, kSegBlock, seg_bwd_lds(a), (hipStream_t)stream>>>(d_a);
  if (a.n_sb > 0) k_seg_bwd_finish<<<a.n_sb, 256, 0, (hipStream_t)stream>>>(d_a, (int)blocks);
}

// --------------------------------------------------------------------------
// leaf preparation: evidence slicing (gather), indicator vectors, maxima;
// extra blocks clear the maxima of the tensors produced in this solve
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_prepare(PrepareArgs a) {
  const int b = blockIdx.y;
  if ((int)blockIdx.x >= a.n_leaves) {
    if (b != 0) return;
    const int n = a.reset_end - a.reset_begin;
    for (int i = (blockIdx.x - a.n_leaves) * kBlock + threadIdx.x; i < n * kMaxSub;
         i += (gridDim.x - a.n_leaves) * kBlock)
      a.mx[(i / n) * a.mx_stride + a.reset_begin + i % n] = 0u;
    return;
  }
  const LeafDesc d = a.leaves[blockIdx.x];
  if (!d.batched && b > 0) return;
  const int row = d.batched ? b : 0;
  float *dst = a.arena + d.dst + (d.batched ? (int64_t)b * d.size : 0);
  const float one = d.maxdom ? 0.f : 1.f;
  const float zero = d.maxdom ? -INFINITY : 0.f;
  float lmax = 0.f;
  if (d.kind == 0) {
    int64_t base = 0;
    for (int o = d.obs_begin; o < d.obs_end; ++o)
      base += (int64_t)a.evidence[(int64_t)row * a.n_vars + a.obs[2 * o]] * a.obs[2 * o + 1];
    const float *src = a.arena + d.src + base;
    for (int i = threadIdx.x; i < d.size; i += kBlock) {
      const float v = src[a.gmap[d.gmap + i]];
      dst[i] = v;
      lmax = fmaxf(lmax, fabsf(v));
    }
  } else if (d.kind == 1) {
    for (int i = threadIdx.x; i < d.size; i += kBlock) dst[i] = one;
    lmax = 1.f;
  } else {
    const int e = a.evidence[(int64_t)row * a.n_vars + d.var];
    for (int i = threadIdx.x; i < d.size; i += kBlock) dst[i] = (e < 0 || e == i) ? one : zero;
    lmax = 1.f;
  }
  __shared__ float sm[kBlock / 64];
  lmax = wave_max(lmax);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = lmax;
  __syncthreads();
  if (threadIdx.x == 0 && d.slot >= 0) {
    float m = sm[0];
    for (int w = 1; w < kBlock / 64; ++w) m = fmaxf(m, sm[w]);
    a.mx[d.slot + (d.batched ? b : 0)] = __float_as_uint(m);
    a.ex[d.slot + (d.batched ? b : 0)] = 0;
  }
}

void launch_prepare(const PrepareArgs &a, void *stream) {
  const int reset_blocks = (a.reset_end - a.reset_begin + kBlock - 1) / kBlock;
  dim3 g(a.n_leaves + (reset_blocks > 0 ? (reset_blocks > 1024 ? 1024 : reset_blocks) : 0),
         a.batch);
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
  for (int x = 0; x < m.card; ++x) tot += (double)adj[x] * (double)lam[x];
  for (int x = 0; x < m.card; ++x)
    out[(int64_t)b * row + m.out + x] = tot > 0.0 ? (double)adj[x] * (double)lam[x] / tot : 0.0;
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
// argmax readout (MPE configuration), one lane per instance
// --------------------------------------------------------------------------
__global__ void k_backtrack(const int32_t *iarena, const BackStep *steps, int n_steps,
                            const int32_t *pairs, int n_vars, int batch, int32_t *assign) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  int32_t *x = assign + (int64_t)b * n_vars;
  for (int st = 0; st < n_steps; ++st) {
    const BackStep s = steps[st];
    int64_t off = 0;
    bool ok = true;
    for (int i = s.in_begin; i < s.in_end; ++i) {
      const int32_t xv = x[pairs[2 * i]];
      ok = ok && xv >= 0;
      off += (int64_t)xv * pairs[2 * i + 1];
    }
    if (!ok) continue;  // an input left unassigned: leave this step's outputs unset
    int32_t k = iarena[s.arg + (int64_t)b * s.bs + off];
    for (int j = s.out_end - 1; j >= s.out_begin; --j) {
      const int c = pairs[2 * j + 1];
      x[pairs[2 * j]] = k % c;
      k /= c;
    }
  }
}

void launch_backtrack(const int32_t *iarena, const BackStep *steps, int n_steps, const int32_t *pairs,
                      int n_vars, int batch, int32_t *assign, void *stream) {
  k_backtrack<<<(batch + 63) / 64, 64, 0, (hipStream_t)stream>>>(iarena, steps, n_steps, pairs,
                                                                 n_vars, batch, assign);
}

// --------------------------------------------------------------------------
// sampling along the tree (eq. sample / eq. condition-prob)
// --------------------------------------------------------------------------

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications with the Weyl-sequence key schedule.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
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

__device__ __forceinline__ double uniform53(uint64_t sample, uint32_t node, uint32_t slot,
                                            uint64_t seed) {
  uint32_t c[4] = {(uint32_t)sample, (uint32_t)(sample >> 32), node, slot};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  return ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6)) * (1.0 / 9007199254740992.0);
}

// meta quadruples (var, card, strideA, strideB)
__device__ __forceinline__ void decode_offsets(int64_t k, const int32_t *q, int qb, int qe,
                                               int64_t &oa, int64_t &ob) {
  oa = 0;
  ob = 0;
  for (int j = qe - 1; j >= qb; --j) {
    const int c = q[4 * j + 1];
    const int64_t d = k % c;
    k /= c;
    oa += d * q[4 * j + 2];
    ob += d * q[4 * j + 3];
  }
}
__device__ __forceinline__ void decode_assign(int64_t k, const int32_t *q, int qb, int qe, int32_t *x) {
  for (int j = qe - 1; j >= qb; --j) {
    const int c = q[4 * j + 1];
    x[q[4 * j]] = (int32_t)(k % c);
    k /= c;
  }
}
__device__ __forceinline__ int64_t count_of(const int32_t *q, int qb, int qe) {
  int64_t n = 1;
  for (int j = qb; j < qe; ++j) n *= q[4 * j + 1];
  return n;
}

__global__ void k_sample(const float *arena, const SampleStep *steps, int n_steps, const int32_t *q,
                         int n_vars, int64_t n, uint64_t seed, const int32_t *init, int32_t *out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  int32_t *x = out + s * n_vars;
  for (int v = 0; v < n_vars; ++v) x[v] = init[v];
  for (int t = 0; t < n_steps; ++t) {
    const SampleStep st = steps[t];
    const float *A = arena + st.A;
    const float *B = st.B >= 0 ? arena + st.B : nullptr;
    int64_t oa = 0, ob = 0;
    bool ok = true;
    for (int i = st.aIn_b; i < st.aIn_e; ++i) {
      ok = ok && x[q[4 * i]] >= 0;
      oa += (int64_t)x[q[4 * i]] * q[4 * i + 2];
    }
    for (int i = st.bIn_b; i < st.bIn_e; ++i) {
      ok = ok && x[q[4 * i]] >= 0;
      ob += (int64_t)x[q[4 * i]] * q[4 * i + 3];
    }
    if (!ok) continue;  // an input left unassigned: leave this step's outputs unset
    // shared eliminated labels: w(k) = (sum_pa A) * (sum_pb B)
    if (st.k_e > st.k_b) {
      const int64_t nK = count_of(q, st.k_b, st.k_e);
      const int64_t nPa = count_of(q, st.pa_b, st.pa_e), nPb = count_of(q, st.pb_b, st.pb_e);
      auto weight = [&](int64_t k) {
        int64_t ka, kb;
        decode_offsets(k, q, st.k_b, st.k_e, ka, kb);
        double wa = 0.0, wb = 0.0;
        for (int64_t p = 0; p < nPa; ++p) {
          int64_t pa, dummy;
          decode_offsets(p, q, st.pa_b, st.pa_e, pa, dummy);
          wa += (double)A[oa + ka + pa];
        }
        if (B) {
          for (int64_t p = 0; p < nPb; ++p) {
            int64_t dummy, pb;
            decode_offsets(p, q, st.pb_b, st.pb_e, dummy, pb);
            wb += (double)B[ob + kb + pb];
          }
        } else {
          wb = 1.0;
        }
        return wa * wb;
      };
      double tot = 0.0;
      for (int64_t k = 0; k < nK; ++k) tot += weight(k);
      const double target = uniform53((uint64_t)s, (uint32_t)st.node, 0u, seed) * tot;
      double cum = 0.0;
      int64_t pick = -1, last = 0;
      for (int64_t k = 0; k < nK; ++k) {
        const double w = weight(k);
        if (w > 0.0) last = k;
        cum += w;
        if (w > 0.0 && cum > target) {
          pick = k;
          break;
        }
      }
      if (pick < 0) pick = last;
      int64_t ka, kb;
      decode_offsets(pick, q, st.k_b, st.k_e, ka, kb);
      decode_assign(pick, q, st.k_b, st.k_e, x);
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
      double tot = 0.0;
      for (int64_t p = 0; p < nP; ++p) {
        int64_t da, db;
        decode_offsets(p, q, pb, pe, da, db);
        tot += (double)T[base + (side ? db : da)];
      }
      const double target = uniform53((uint64_t)s, (uint32_t)st.node, 1u + side, seed) * tot;
      double cum = 0.0;
      int64_t pick = -1, last = 0;
      for (int64_t p = 0; p < nP; ++p) {
        int64_t da, db;
        decode_offsets(p, q, pb, pe, da, db);
        const double w = (double)T[base + (side ? db : da)];
        if (w > 0.0) last = p;
        cum += w;
        if (w > 0.0 && cum > target) {
          pick = p;
          break;
        }
      }
      if (pick < 0) pick = last;
      decode_assign(pick, q, pb, pe, x);
    }
  }
}

void launch_sample(const float *arena, const SampleStep *steps, int n_steps, const int32_t *meta,
                   int n_vars, int64_t n, uint64_t seed, const int32_t *init, int32_t *out,
                   void *stream) {
  if (n <= 0) return;
  const int64_t blocks = (n + 63) / 64;
  k_sample<<<(unsigned)blocks, 64, 0, (hipStream_t)stream>>>(arena, steps, n_steps, meta, n_vars, n,
                                                            seed, init, out);
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
