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

// Row of the 32-row tile held in register r of a lane in half h.
__device__ __forceinline__ constexpr int crow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

// ---- descriptor tile staging ------------------------------------------------------------
// Tile = 32 rows x DP features, fetched as float4 slots into registers by NT threads (thread
// index `tid`), then written to LDS as [x (DP) | x^2 (DP) | pad 4] per row.  Rows past
// `valid` and features past D are zero.
template <int DP, int NT>
struct TileIO {
  static constexpr int kSlotsPerRow = DP / 4;
  static constexpr int kSlots = kTile * kSlotsPerRow;
  static constexpr int kPer = (kSlots + NT - 1) / NT;
  static constexpr int XS = 2 * DP + 4;

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

  __device__ __forceinline__ static void store(float* xs, const f32x4 (&pre)[kPer], int tid) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int idx = tid + q * NT;
      if (idx < kSlots) {
        const int row = idx / kSlotsPerRow;
        const int c4 = (idx % kSlotsPerRow) * 4;
        const f32x4 v = pre[q];
        *reinterpret_cast<f32x4*>(xs + row * XS + c4) = v;
        *reinterpret_cast<f32x4*>(xs + row * XS + DP + c4) = v * v;
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
// logit itself (which reaches a few hundred).
template <int DP>
__device__ __forceinline__ void estep_f32(const float* __restrict__ xr, const float (&areg)[DP],
                                          float cval, f32x16& hi, f32x16& lo) {
#pragma unroll
  for (int ch = 0; ch < DP / 16; ++ch) {
    f32x16 a;
#pragma unroll
    for (int r = 0; r < 16; ++r) a[r] = (ch == 0) ? cval : 0.f;
#pragma unroll
    for (int s = 16 * ch; s < 16 * ch + 16; s += 4) {
      const f32x4 xv = *reinterpret_cast<const f32x4*>(xr + s);
      a = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[0], areg[s + 0], a, 0, 0, 0);
      a = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[1], areg[s + 1], a, 0, 0, 0);
      a = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[2], areg[s + 2], a, 0, 0, 0);
      a = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[3], areg[s + 3], a, 0, 0, 0);
    }
    if (ch == 0) {
      hi = a;
#pragma unroll
      for (int r = 0; r < 16; ++r) lo[r] = 0.f;
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

// ---- statistics on FP32 MFMA -----------------------------------------------------------------
// acc[b] (rows = features 32b..32b+31 of [x, x^2], cols = the wave's components) +=
// sum over the tile's rows of Xa[row][f] * gamma[row][comp].  gam is in E-step C layout.
template <int DP>
__device__ __forceinline__ void stats_f32(const float* __restrict__ xb, int h, int j,
                                          const f32x16& gam, f32x16 (&acc)[2 * DP / 32]) {
  constexpr int XS = 2 * DP + 4;
  constexpr int NB = 2 * DP / 32;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const float* xrow = xb + crow(s, h) * XS + j;
#pragma unroll
    for (int b = 0; b < NB; ++b)
      acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(xrow[32 * b], gam[s], acc[b], 0, 0, 0);
  }
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}

}  // namespace dev
}  // namespace fv
