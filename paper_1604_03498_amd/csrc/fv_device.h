// Device building blocks shared by the gfx950 Fisher-vector kernels.
//
// Layout conventions (v_mfma_f32_32x32x2_f32 on a 64-lane wavefront):
//   lane l = 32*h + j  (h = half of the wave, j = 0..31)
//   A operand: lane supplies A[i = j][k = h];  B operand: lane supplies B[k = h][j]
//   C/D: register r of lane l holds C[row = 8*(r/4) + 4*h + r%4][col = j]
// E-step: rows = the 32 descriptors of a tile, cols = the wave's 32 components.
// Statistics: rows = 32 features of a block, cols = components, reduction over descriptors;
// gamma is consumed straight from the E-step result registers as the B operand, so the
// descriptor order inside each 2-deep MFMA step is the C-layout row order (a permutation of
// the tile rows, harmless for a sum).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fv_internal.h"

namespace fv {
namespace dev {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Lane permutations within a row of 16 lanes (DPP), compile-time controls.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

struct MaxOp {
  __device__ __forceinline__ float operator()(float a, float b) const { return fmaxf(a, b); }
};
struct AddOp {
  __device__ __forceinline__ float operator()(float a, float b) const { return a + b; }
};

// All-reduce over the 32 lanes of a half-wave (lanes 0-31 and 32-63 reduce separately).
// Every step combines symmetric partners, so all 32 lanes end with bit-identical results.
template <class Op>
__device__ __forceinline__ float allreduce32(float v, Op op) {
  v = op(v, dpp<0xB1>(v));   // quad_perm [1,0,3,2]: lane ^ 1
  v = op(v, dpp<0x4E>(v));   // quad_perm [2,3,0,1]: lane ^ 2
  v = op(v, dpp<0x141>(v));  // row_half_mirror: combine the two quads of each 8 lanes
  v = op(v, dpp<0x140>(v));  // row_mirror: combine the two halves of each 16 lanes
  auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return op(__uint_as_float(p[0]), __uint_as_float(p[1]));  // rows 0<->1, 2<->3
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

__device__ __forceinline__ float select_f(bool c, float a, float b) { return c ? a : b; }

// Orders LDS writes of this wave before its later LDS reads (no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Reduce-scatter of the 16 C-layout registers over the 32 lanes of a half-wave: lane j ends
// with the reduction (over all 32 lanes) of register j >> 1, i.e. of row crow(j >> 1, h);
// lanes 2r and 2r+1 hold the same, bit-identical value.  Five exchange stages halve the
// register count each time (38 VALU instructions for all 16 rows, against 16 separate
// all-reduces of 6 each):
//   stage 1  lanes j ^ 16  v_permlane16_swap of register pairs (r, r+8)
//   stage 2  lanes j ^ 8   DPP row_ror:8,          pairs (r, r+4)
//   stage 3  lanes j ^ 7   DPP row_half_mirror,    pairs (r, r+2)
//   stage 4  lanes j ^ 2   DPP quad_perm [2,3,0,1], pairs (r, r+1)
//   stage 5  lanes j ^ 1   DPP quad_perm [1,0,3,2]
// A lane keeps the half of each pair selected by its own lane bit, sends the other half, and
// combines what it keeps with what its partner sent.  The partner sets of successive stages
// are disjoint, so every register is combined over all 32 lanes exactly once.
template <class Op>
__device__ __forceinline__ float reduce_scatter16(const float (&v)[16], int j, Op op) {
  float a[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[r]), __float_as_uint(v[r + 8]),
                                              false, false);
    a[r] = op(__uint_as_float(p[0]), __uint_as_float(p[1]));  // bit 4 = 0: reg r, else r + 8
  }
  const bool b3 = (j >> 3) & 1, b2 = (j >> 2) & 1, b1 = (j >> 1) & 1;
  float b[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float keep = select_f(b3, a[r + 4], a[r]);
    const float send = select_f(b3, a[r], a[r + 4]);
    b[r] = op(keep, dpp<0x128>(send));  // row_ror:8
  }
  float c[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const float keep = select_f(b2, b[r + 2], b[r]);
    const float send = select_f(b2, b[r], b[r + 2]);
    c[r] = op(keep, dpp<0x141>(send));  // row_half_mirror
  }
  const float keep = select_f(b1, c[1], c[0]);
  const float send = select_f(b1, c[0], c[1]);
  float d = op(keep, dpp<0x4E>(send));  // quad_perm [2,3,0,1]
  return op(d, dpp<0xB1>(d));           // quad_perm [1,0,3,2]
}

// Row of the 32-row tile held in register r of a lane in half h.
__device__ __forceinline__ constexpr int crow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

// Soft assignment, wave-local part: for the tile's 32 rows and this wave's 32 components,
// e = exp2((hi - m_w) + lo) with m_w the wave's row maximum.  The row maxima and the row sums
// of e are published for the cross-wave combine at xm[row * W + w], xs[row * W + w]; `loc`
// (32 floats, private to this wave) carries the maxima back to every lane of the wave.
template <int W>
__device__ __forceinline__ void softmax_wave(const f32x16& hi, const f32x16& lo, f32x16& e,
                                             float* xm, float* xs, float* loc, int w, int j,
                                             int h) {
  float v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = hi[r];
  const float mrow = reduce_scatter16(v, j, MaxOp());
  const int myrow = crow(j >> 1, h);
  if (!(j & 1)) {
    loc[myrow] = mrow;
    xm[myrow * W + w] = mrow;
  }
  wave_sync();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const f32x4 m = *reinterpret_cast<const f32x4*>(loc + 8 * q + 4 * h);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int r = 4 * q + p;
      e[r] = fast_exp2((hi[r] - m[p]) + lo[r]);
      v[r] = e[r];
    }
  }
  const float srow = reduce_scatter16(v, j, AddOp());
  if (!(j & 1)) xs[myrow * W + w] = srow;
}

// Cross-wave combine, after a workgroup barrier: the lane pair that owns row crow(j>>1, h)
// reads the W published (max, sum) pairs of its row and forms M = max_v m_v and
// Z = sum_v s_v 2^(m_v - M).  Returns the scale of this wave's e for that row,
// 2^(m_w - M) / Z (0 for rows past `valid`), and M and log2 Z through the references.
template <int W>
__device__ __forceinline__ float softmax_combine(const float* xm, const float* xs, int w, int j,
                                                 int h, int valid, float& M, float& L2Z) {
  const int row = crow(j >> 1, h);
  float m[W], sv[W];
#pragma unroll
  for (int v = 0; v < W; ++v) {
    m[v] = xm[row * W + v];
    sv[v] = xs[row * W + v];
  }
  M = m[0];
#pragma unroll
  for (int v = 1; v < W; ++v) M = fmaxf(M, m[v]);
  float Z = 0.f, mine = 0.f;
#pragma unroll
  for (int v = 0; v < W; ++v) {
    const float sc = fast_exp2(m[v] - M);
    Z += sv[v] * sc;
    if (v == w) mine = sc;
  }
  L2Z = log2f(Z);
  return row < valid ? mine / Z : 0.f;
}

// ---- two-pass normaliser -----------------------------------------------------------------
// The first pass leaves (row max m_g, log2 of the row sum s_g) per group g of up to 256
// components at lse[g * stride + row].  fetch_lse loads them (ok: row inside the tile);
// merge_lse forms M = max_g m_g and log2 Z, Z = sum_g s_g 2^(m_g - M), in group order.
constexpr int kMaxLseGroups = kMaxK / (kMaxWaves * kCompsPerWave);

__device__ __forceinline__ void fetch_lse(float2 (&l)[kMaxLseGroups], const float2* __restrict__ lse,
                                          int G, int64_t stride, int64_t row, bool ok) {
#pragma unroll
  for (int g = 0; g < kMaxLseGroups; ++g)
    if (ok && g < G) l[g] = lse[(size_t)g * stride + row];
}

__device__ __forceinline__ void merge_lse(const float2 (&l)[kMaxLseGroups], int G, float& M,
                                          float& L2Z) {
  M = l[0].x;
  if (G == 1) {
    L2Z = l[0].y;
    return;
  }
  float Z = exp2f(l[0].y);
#pragma unroll
  for (int g = 1; g < kMaxLseGroups; ++g) {
    if (g < G) {
      const float Mn = fmaxf(M, l[g].x);
      Z = Z * fast_exp2(M - Mn) + exp2f(l[g].y) * fast_exp2(l[g].x - Mn);
      M = Mn;
    }
  }
  L2Z = log2f(Z);
}

// ---- descriptor tile staging ------------------------------------------------------------
// Every kernel works on centred descriptors x - m0, where m0 is one per-model vector (the
// weighted mean of the component means, rounded to float; zero past D) whose subtraction the
// model constants already account for: the encoding is invariant under translating the
// descriptors and the means together, and centring keeps x, x^2 and the raw moments small
// when the data sit far from the origin.  stage_centre copies m0 into LDS once per workgroup
// (and waits for it); the tile loaders subtract it as they write a tile.
template <int DP, int NT>
__device__ __forceinline__ void stage_centre(float* cs, const float* __restrict__ cen, int tid) {
  for (int i = tid; i < DP; i += NT) cs[i] = cen[i];
  __syncthreads();
}

// Tile = 32 rows x DP features, fetched as float4 slots into registers by NT threads (thread
// index `tid`), then written to LDS as [x (DP) | x^2 (DP) | pad 4] per row, or as [x (DP) |
// pad 4] when SQ is false (the consumer squares on the fly; x * x is rounded the same way),
// x being the centred value.  Rows past `valid` and features past D are fetched as zero (a
// row past `valid` is staged as -m0 and always gets a zero posterior).
template <int DP, int NT, bool SQ = true>
struct TileIO {
  static constexpr int kSlotsPerRow = DP / 4;
  static constexpr int kSlots = kTile * kSlotsPerRow;
  static constexpr int kPer = (kSlots + NT - 1) / NT;
  static constexpr int XS = SQ ? 2 * DP + 4 : DP + 4;

  __device__ __forceinline__ static void fetch(f32x4 (&pre)[kPer], const float* __restrict__ X,
                                               int D, bool vec_ok, int64_t row0, int valid,
                                               int tid) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int idx = tid + q * NT;
      f32x4 v = {0.f, 0.f, 0.f, 0.f};
      if (idx < kSlots) {
        const int row = idx / kSlotsPerRow;
        const int c4 = (idx % kSlotsPerRow) * 4;
        if (row < valid) {
          const float* src = X + (row0 + row) * (int64_t)D + c4;
          if (vec_ok) {
            if (c4 < D) v = *reinterpret_cast<const f32x4*>(src);
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (c4 + e < D) v[e] = src[e];
          }
        }
      }
      pre[q] = v;
    }
  }

  // cen: the model centre in LDS (stage_centre); the tile holds x - centre
  __device__ __forceinline__ static void store(float* xs, const f32x4 (&pre)[kPer],
                                               const float* cen, int tid) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int idx = tid + q * NT;
      if (idx < kSlots) {
        const int row = idx / kSlotsPerRow;
        const int c4 = (idx % kSlotsPerRow) * 4;
        const f32x4 v = pre[q] - *reinterpret_cast<const f32x4*>(cen + c4);
        *reinterpret_cast<f32x4*>(xs + row * XS + c4) = v;
        if (SQ) *reinterpret_cast<f32x4*>(xs + row * XS + DP + c4) = v * v;
      }
    }
  }
};

// ---- E-step on FP32 MFMA --------------------------------------------------------------------
// Logits (log2 units) of the tile's 32 rows for 32 components: c + [x, x^2] . A, where lane
// (h, j) supplies areg[s] = A[s + DP*h][component j] and xr points at row j, column DP*h of
// the LDS tile.  The 2*DP products are accumulated in chains of 16 MFMA steps and the chain
// sums are added with TwoSum, so the logit is the unevaluated pair hi + lo: downstream code
// evaluates (hi - reference) + lo, accurate to the size of the difference rather than of the
// logit itself (which reaches a few hundred).  The offset c joins the first chain's sum once
// (not as its initial value), so no chain accumulates at the offset's magnitude.
template <int DP>
__device__ __forceinline__ void estep_f32(const float* __restrict__ xr, const float (&areg)[DP],
                                          float cval, f32x16& hi, f32x16& lo) {
  constexpr int CH = 16;  // MFMA steps per accumulation chain
#pragma unroll
  for (int ch = 0; ch < DP / CH; ++ch) {
    f32x16 a;
#pragma unroll
    for (int r = 0; r < 16; ++r) a[r] = 0.f;
#pragma unroll
    for (int s = CH * ch; s < CH * ch + CH; s += 4) {
      const f32x4 xv = *reinterpret_cast<const f32x4*>(xr + s);
      a = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[0], areg[s + 0], a, 0, 0, 0);
      a = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[1], areg[s + 1], a, 0, 0, 0);
      a = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[2], areg[s + 2], a, 0, 0, 0);
      a = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[3], areg[s + 3], a, 0, 0, 0);
    }
    if (ch == 0) {
      // the offset joins after the first chain: the chain's partial sums stay small
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        hi[r] = a[r] + cval;
        lo[r] = 0.f;
      }
      // the adds complete before the next chain starts (FP32 MFMAs do not overlap VALU anyway),
      // so the chain sum and the logit never need registers at the same time
      __builtin_amdgcn_sched_barrier(0);
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float t = hi[r] + a[r];
        const float bp = t - hi[r];
        const float err = (hi[r] - (t - bp)) + (a[r] - bp);
        hi[r] = t;
        lo[r] += err;
      }
    }
  }
}

// Same E-step with the operand slice in LDS instead of registers: ar points at this lane's
// row of the wave's slice, laid out [component j][2*DP (+ pad)] and offset by DP*h, and xr at
// row j of an x-only tile; lanes of the upper half (h = 1) square x on the fly.  Operands and
// accumulation order are those of estep_f32, so the logits are bitwise the same.
template <int DP>
__device__ __forceinline__ void estep_f32_lds(const float* __restrict__ xr,
                                              const float* __restrict__ ar, int h, float cval,
                                              f32x16& hi, f32x16& lo) {
  constexpr int CH = 16;
  // Operands of the next 4 steps are read while the current 4 MFMAs issue; the scheduling
  // fences keep the compiler from hoisting all 2*DP operand reads (which would spill).
  f32x4 xn = *reinterpret_cast<const f32x4*>(xr);
  f32x4 an = *reinterpret_cast<const f32x4*>(ar);
#pragma unroll
  for (int ch = 0; ch < DP / CH; ++ch) {
    f32x16 a;
#pragma unroll
    for (int r = 0; r < 16; ++r) a[r] = 0.f;
#pragma unroll
    for (int s = CH * ch; s < CH * ch + CH; s += 4) {
      f32x4 xv = xn;
      const f32x4 av = an;
      if (s + 4 < DP) {
        xn = *reinterpret_cast<const f32x4*>(xr + s + 4);
        an = *reinterpret_cast<const f32x4*>(ar + s + 4);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) xv[e] = h ? xv[e] * xv[e] : xv[e];
      a = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[0], av[0], a, 0, 0, 0);
      a = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[1], av[1], a, 0, 0, 0);
      a = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[2], av[2], a, 0, 0, 0);
      a = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[3], av[3], a, 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (ch == 0) {
      // the offset joins after the first chain: the chain's partial sums stay small
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        hi[r] = a[r] + cval;
        lo[r] = 0.f;
      }
      // the adds complete before the next chain starts (FP32 MFMAs do not overlap VALU anyway),
      // so the chain sum and the logit never need registers at the same time
      __builtin_amdgcn_sched_barrier(0);
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float t = hi[r] + a[r];
        const float bp = t - hi[r];
        const float err = (hi[r] - (t - bp)) + (a[r] - bp);
        hi[r] = t;
        lo[r] += err;
      }
    }
  }
}

// This lane's E-step operand values for component block cb from the fragment-ordered A32:
// areg[s] = A[s + DP*h][32cb + j], sixteen-byte loads, 1 KB contiguous per wave load.
template <int DP>
__device__ __forceinline__ void load_areg(float (&areg)[DP], const float* __restrict__ A32,
                                          int cb, int lane) {
  const f32x4* src = reinterpret_cast<const f32x4*>(A32) + (size_t)cb * (DP / 4) * 64 + lane;
#pragma unroll
  for (int g = 0; g < DP / 4; ++g) {
    const f32x4 v = src[g * 64];
#pragma unroll
    for (int e = 0; e < 4; ++e) areg[4 * g + e] = v[e];
  }
}

// Copy of one wave's operand slice (component block cb) into LDS as [j][k] with row stride
// AS: lane (h, j) writes A[DP*h .. DP*h + DP)[32cb + j] in sixteen-byte pieces.
template <int DP>
__device__ __forceinline__ void load_a_lds(float* __restrict__ as, const float* __restrict__ A32,
                                           int cb, int lane, int AS) {
  const f32x4* src = reinterpret_cast<const f32x4*>(A32) + (size_t)cb * (DP / 4) * 64 + lane;
  float* dst = as + (lane & 31) * AS + DP * (lane >> 5);
#pragma unroll 4
  for (int g = 0; g < DP / 4; ++g) *reinterpret_cast<f32x4*>(dst + 4 * g) = src[g * 64];
}

// ---- the paper's posterior threshold --------------------------------------------------------
// gamma <= thr contributes nothing (thr < 0: every term contributes).  thr is uniform, so the
// test is a scalar branch.
__device__ __forceinline__ void apply_threshold(f32x16& g, float thr) {
  if (thr >= 0.f) {
#pragma unroll
    for (int r = 0; r < 16; ++r) g[r] = g[r] > thr ? g[r] : 0.f;
  }
}

// True when no lane of the wave has a nonzero value in v (a wave-uniform answer).
__device__ __forceinline__ bool wave_all_zero(bool nonzero) {
  return __builtin_amdgcn_ballot_w64(nonzero) == 0;
}

// Bit s set when gamma register s is nonzero in some lane (all bits set without SKIP).  The
// mask is taken before the contraction so that its steps stay one straight block each.
template <bool SKIP>
__device__ __forceinline__ uint32_t live_steps(const f32x16& gam) {
  uint32_t live = 0xffffu;
  if (SKIP) {
    live = 0;
#pragma unroll
    for (int s = 0; s < 16; ++s) live |= wave_all_zero(gam[s] != 0.f) ? 0u : (1u << s);
  }
  return live;
}

// ---- statistics on FP32 MFMA -----------------------------------------------------------------
// acc[b] (rows = features 32b..32b+31 of [x, x^2], cols = the wave's components) +=
// sum over the tile's rows of Xa[row][f] * gamma[row][comp].  gam is in E-step C layout.
// With SKIP, a step whose gamma is zero in every lane is left out (its MFMAs would add exact
// zeros for finite descriptors): the paper's early termination, per 2-row step.
template <int DP, bool SKIP = false>
__device__ __forceinline__ void stats_f32(const float* __restrict__ xb, int h, int j,
                                          const f32x16& gam, f32x16 (&acc)[2 * DP / 32]) {
  constexpr int XS = 2 * DP + 4;
  constexpr int NB = 2 * DP / 32;
  const uint32_t live = live_steps<SKIP>(gam);
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    if (SKIP && !(live & (1u << s))) continue;
    const float* xrow = xb + crow(s, h) * XS + j;
#pragma unroll
    for (int b = 0; b < NB; ++b)
      acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(xrow[32 * b], gam[s], acc[b], 0, 0, 0);
  }
}

// Same contraction from an x-only tile (row stride DP + 4): feature f < DP is x[f], feature
// f >= DP is x[f - DP]^2, squared on the fly.
template <int DP, bool SKIP = false>
__device__ __forceinline__ void stats_f32_x(const float* __restrict__ xb, int h, int j,
                                            const f32x16& gam, f32x16 (&acc)[2 * DP / 32]) {
  constexpr int XS = DP + 4;
  constexpr int NB = 2 * DP / 32;
  auto fetch = [&](int s, float (&v)[NB]) {
    const float* xrow = xb + crow(s, h) * XS;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int f = 32 * b + j;
      if (32 * (b + 1) <= DP)
        v[b] = xrow[f];
      else if (32 * b >= DP)
        v[b] = xrow[f - DP];
      else
        v[b] = xrow[f < DP ? f : f - DP];
    }
  };
  const uint32_t live = live_steps<SKIP>(gam);
  float vn[NB];
  fetch(0, vn);
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    float v[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) v[b] = vn[b];
    if (s + 1 < 16) fetch(s + 1, vn);
    if (SKIP && !(live & (1u << s))) continue;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int f = 32 * b + j;
      float u = v[b];
      if (32 * (b + 1) <= DP) {
      } else if (32 * b >= DP) {
        u = u * u;
      } else {
        u = f < DP ? u : u * u;
      }
      acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(u, gam[s], acc[b], 0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}

}  // namespace dev
}  // namespace fv
