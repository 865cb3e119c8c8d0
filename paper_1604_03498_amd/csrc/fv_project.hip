// Projection prologue: y = A (x - m) for every descriptor, the dimension reduction the paper
// applies to its dense-SIFT descriptors before encoding (PCA of the 128 SIFT values to m
// dimensions, plus the normalised image coordinates passed through, Sec. 3.1).  A is any
// [D x Din] matrix, so pass-through coordinates are identity rows of A.
//
// One FP32 MFMA contraction (32x32x2): a workgroup has one wave per 32 output columns; each
// wave keeps its 32 rows of A in registers, in operand order (lane l = 32h + j holds
// A[32w + j][2s + h] for step s), takes the other operand from a 32-descriptor tile staged in
// LDS and starts every accumulator at -A m.  The result tile is written row-major (lane j
// writes column 32w + j of its rows).
#include "fv_internal.h"

#include <stdint.h>

namespace fv {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

template <int V> struct VecT;
template <> struct VecT<1> { using type = float; };
template <> struct VecT<2> { using type = f32x2; };
template <> struct VecT<4> { using type = f32x4; };

__device__ __forceinline__ int prow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

// S: the MFMA steps (Din rounded up, halved; operand rows past Din are zero).  NC: waves per
// row block (one per 32 output columns, Dp = 32 NC).  A workgroup has 4 waves, RB = 4 / NC row
// blocks of 32 descriptors (one when NC = 3: the fourth wave only helps to load), so a tile is
// RB * 32 rows.  The rows of a tile are one contiguous block of floats, copied to LDS in the
// same row-major layout with coalesced loads of V floats (V = 4 when X is 16-byte aligned and
// 4 | Din, 2 when 8-byte aligned and 2 | Din); several workgroups per CU overlap one tile's
// loads with another's MFMAs: the register budget is held to two waves per SIMD up to S = 112
// (above that the operand fragments alone need more, and one wave per SIMD beats spilling).
template <int S, int NC, int V>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(S <= 112 ? 2 : 1)))
void project_kernel(
    const float* __restrict__ X, int64_t N, int Din, const float* __restrict__ frag,
    const float* __restrict__ bias, int Dp, int D, float* __restrict__ Y,
    const Counts* __restrict__ cnt) {
  constexpr int RB = NC == 3 ? 1 : 4 / NC;
  constexpr int TR = 32 * RB;
  constexpr int kMaxF = TR * 2 * S;
  __shared__ __attribute__((aligned(16))) float xs[kMaxF];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int h = lane >> 5;
  const int j = lane & 31;
  const int cb = w % NC;  // column block
  const int rb = w / NC;  // row block (rb >= RB: load-only wave)
  const int col = 32 * cb + j;

  float b[S];
#pragma unroll
  for (int s = 0; s < S; ++s) b[s] = frag[(size_t)(2 * s + h) * Dp + col];
  const float c0 = bias[col];

  // A tile is copied to LDS in rounds of 8 loads per thread, all in flight together (indices
  // clamped in bounds, values past the tile's end replaced by zeros), so that only 8 loads'
  // registers are live; at two workgroups per CU the other workgroup's MFMAs cover the loads.
  using VT = typename VecT<V>::type;
  N = live_rows(cnt, N);  // a batched sequence's row count (device side), else the argument
  const int64_t ntiles = (N + TR - 1) / TR;
  auto rows_of = [&](int64_t t) { return N - t * TR < TR ? (int)(N - t * TR) : TR; };
  auto copy_tile = [&](int64_t t) {
    const float* src = X + t * TR * (int64_t)Din;
    const int nf = rows_of(t) * Din;  // a multiple of V
    for (int i0 = V * tid; i0 < nf; i0 += 8 * V * 256) {
      VT v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int i = i0 + q * V * 256;
        v[q] = *reinterpret_cast<const VT*>(src + (i < nf ? i : nf - V));
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int i = i0 + q * V * 256;
        if (i < nf) *reinterpret_cast<VT*>(&xs[i]) = v[q];
      }
    }
  };
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t row0 = t * TR;
    const int rows = rows_of(t);
    copy_tile(t);
    __syncthreads();
    if (rb < RB) {
      f32x16 acc;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = c0;
      // rows past the tile's end read stale LDS; their outputs are not stored
      const float* xr = xs + (32 * rb + j) * Din;
      // groups of 8 steps; the fence keeps the compiler from hoisting every operand read
#pragma unroll
      for (int s0 = 0; s0 < S; s0 += 8) {
        if (2 * s0 >= Din) continue;  // uniform; keeps the loop fully unrolled
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = 2 * (s0 + e) + h;
          v[e] = k < Din ? xr[k] : 0.f;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e)
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(v[e], b[s0 + e], acc, 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (col < D) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int orow = 32 * rb + prow(r, h);
          if (orow < rows) Y[(row0 + orow) * D + col] = acc[r];
        }
      }
    }
    __syncthreads();
  }
}

// Split-bf16 form of the same contraction, for the 16-bit encoder forms: every product
// A[c][k] x_k is formed as hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16 (the encoder's
// split, FP32 accumulation), 16 input features per MFMA step instead of 2.  A's hi/lo
// fragments sit in registers in the 32x32x16 B-operand order (lane (j, h) holds
// A[32 cb + j][16 s + 8 h .. + 7] for step s); the A operand of each step, 8 consecutive input
// features of the lane's row, is read from the same FP32 LDS tile and split in registers.
// NS: steps held (Din rounded up to 16, then to a multiple of 4 steps); steps past Din are
// skipped at run time.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_pair(float v0, float v1, uint32_t& hi, uint32_t& lo) {
  hi = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){v0, v1}, bf16x2));
  const float d0 = v0 - __uint_as_float(hi << 16), d1 = v1 - __uint_as_float(hi & 0xffff0000u);
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){d0, d1}, bf16x2));
}

template <int NS, int NC, int V>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void project16_kernel(
    const float* __restrict__ X, int64_t N, int Din, const uint16_t* __restrict__ fhi,
    const uint16_t* __restrict__ flo, const float* __restrict__ bias, int Dp, int D,
    float* __restrict__ Y, const Counts* __restrict__ cnt) {
  constexpr int RB = NC == 3 ? 1 : 4 / NC;
  constexpr int TR = 32 * RB;
  constexpr int kMaxF = TR * 16 * NS;
  // The tile (TR rows, one contiguous block of floats) is fetched as V-float vectors into
  // registers one tile ahead: the loads of tile t + gridDim.x are in flight while tile t is
  // contracted, and are written to LDS after the tile's second barrier.
  constexpr int KL = (kMaxF / V + 255) / 256;  // vectors per thread, at most
  // (when that many registers would not fit beside the fragments, the tile is copied without
  // the look-ahead, in rounds of 8 loads)
  constexpr bool PF = KL * V <= (V == 4 ? 48 : 24) && !(NS == 16 && NC == 3);
  __shared__ __attribute__((aligned(16))) float xs[kMaxF];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int h = lane >> 5;
  const int j = lane & 31;
  const int cb = w % NC;
  const int rb = w / NC;
  const int col = 32 * cb + j;
  const int nsteps = (Din + 15) / 16;

  bf16x8 ah[NS], al[NS];
#pragma unroll
  for (int st = 0; st < NS; ++st) {
    const size_t o = ((size_t)(2 * st + h) * Dp + col) * 8;
    ah[st] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(fhi + o));
    al[st] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(flo + o));
  }
  const float c0 = bias[col];

  using VT = typename VecT<V>::type;
  N = live_rows(cnt, N);
  const int64_t ntiles = (N + TR - 1) / TR;
  auto rows_of = [&](int64_t t) { return N - t * TR < TR ? (int)(N - t * TR) : TR; };
  VT pre[PF ? KL : 1];
  auto fetch = [&](int64_t t) {
    const float* src = X + t * TR * (int64_t)Din;
    const int nf = rows_of(t) * Din;
#pragma unroll
    for (int q = 0; q < (PF ? KL : 0); ++q) {
      const int i = V * (tid + 256 * q);
      if (i + V <= nf) {
        pre[q] = *reinterpret_cast<const VT*>(src + i);
      } else if (V > 1 && i < nf) {  // the tail tile's last partial vector
        float tmp[V];
#pragma unroll
        for (int e = 0; e < V; ++e) tmp[e] = i + e < nf ? src[i + e] : 0.f;
        pre[q] = *reinterpret_cast<const VT*>(tmp);
      }
    }
  };
  auto stage = [&](int64_t t) {
    const int nf = rows_of(t) * Din;
#pragma unroll
    for (int q = 0; q < (PF ? KL : 0); ++q) {
      const int i = V * (tid + 256 * q);
      if (i < nf) *reinterpret_cast<VT*>(&xs[i]) = pre[q];
    }
  };
  auto copy_tile = [&](int64_t t) {  // without look-ahead
    const float* src = X + t * TR * (int64_t)Din;
    const int nf = rows_of(t) * Din;
    for (int i0 = tid; i0 < nf; i0 += 8 * 256) {
      float v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int i = i0 + q * 256;
        v[q] = src[i < nf ? i : nf - 1];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int i = i0 + q * 256;
        if (i < nf) xs[i] = v[q];
      }
    }
  };
  if (PF && (int64_t)blockIdx.x < ntiles) fetch(blockIdx.x);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t row0 = t * TR;
    const int rows = rows_of(t);
    if constexpr (PF) stage(t);
    else copy_tile(t);
    __syncthreads();
    if (PF && t + gridDim.x < ntiles) fetch(t + gridDim.x);
    if (rb < RB) {
      f32x16 acc;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = c0;
      // rows past the tile's end read stale LDS; their outputs are not stored
      const float* xr = xs + (32 * rb + j) * Din;
#pragma unroll
      for (int st = 0; st < NS; ++st) {
        if (st >= nsteps) continue;  // uniform
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = 16 * st + 8 * h + e;
          v[e] = k < Din ? xr[k] : 0.f;
        }
        uint32_t xh[4], xl[4];
#pragma unroll
        for (int pr = 0; pr < 4; ++pr) split_pair(v[2 * pr], v[2 * pr + 1], xh[pr], xl[pr]);
        const bf16x8 xhv = __builtin_bit_cast(bf16x8, xh), xlv = __builtin_bit_cast(bf16x8, xl);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xhv, ah[st], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xhv, al[st], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xlv, ah[st], acc, 0, 0, 0);
        if (st & 1) __builtin_amdgcn_sched_barrier(0);
      }
      if (col < D) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int orow = 32 * rb + prow(r, h);
          if (orow < rows) Y[(row0 + orow) * D + col] = acc[r];
        }
      }
    }
    __syncthreads();
  }
}

template <int NS, int NC>
hipError_t launch16_snc(const ProjConsts& p, const float* X, int64_t N, int vec, float* Y,
                        int grid, hipStream_t stream, const Counts* cnt) {
  if (vec == 4)
    hipLaunchKernelGGL((project16_kernel<NS, NC, 4>), dim3(grid), dim3(256), 0, stream, X, N,
                       p.Din, p.f16hi, p.f16lo, p.bias, p.Dp, p.D, Y, cnt);
  else
    hipLaunchKernelGGL((project16_kernel<NS, NC, 1>), dim3(grid), dim3(256), 0, stream, X, N,
                       p.Din, p.f16hi, p.f16lo, p.bias, p.Dp, p.D, Y, cnt);
  return hipGetLastError();
}

template <int NS>
hipError_t launch16_s(const ProjConsts& p, const float* X, int64_t N, int vec, float* Y,
                      int grid, hipStream_t stream, const Counts* cnt) {
  switch (p.Dp / 32) {
    case 1: return launch16_snc<NS, 1>(p, X, N, vec, Y, grid, stream, cnt);
    case 2: return launch16_snc<NS, 2>(p, X, N, vec, Y, grid, stream, cnt);
    case 3: return launch16_snc<NS, 3>(p, X, N, vec, Y, grid, stream, cnt);
    default: return hipErrorInvalidValue;
  }
}

template <int S, int NC>
hipError_t launch_snc(const ProjConsts& p, const float* X, int64_t N, int vec, float* Y,
                      int grid, hipStream_t stream, const Counts* cnt) {
  if (vec == 4)
    hipLaunchKernelGGL((project_kernel<S, NC, 4>), dim3(grid), dim3(256), 0, stream, X, N, p.Din,
                       p.frag, p.bias, p.Dp, p.D, Y, cnt);
  else if (vec == 2)
    hipLaunchKernelGGL((project_kernel<S, NC, 2>), dim3(grid), dim3(256), 0, stream, X, N, p.Din,
                       p.frag, p.bias, p.Dp, p.D, Y, cnt);
  else
    hipLaunchKernelGGL((project_kernel<S, NC, 1>), dim3(grid), dim3(256), 0, stream, X, N, p.Din,
                       p.frag, p.bias, p.Dp, p.D, Y, cnt);
  return hipGetLastError();
}

template <int S>
hipError_t launch_s(const ProjConsts& p, const float* X, int64_t N, int vec, float* Y,
                    int grid, hipStream_t stream, const Counts* cnt) {
  switch (p.Dp / 32) {
    case 1: return launch_snc<S, 1>(p, X, N, vec, Y, grid, stream, cnt);
    case 2: return launch_snc<S, 2>(p, X, N, vec, Y, grid, stream, cnt);
    case 3: return launch_snc<S, 3>(p, X, N, vec, Y, grid, stream, cnt);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_project(const ProjConsts& p, const float* X, int64_t N, float* Y, int grid,
                          hipStream_t stream, const Counts* cnt, bool split16) {
  if (N <= 0) return hipSuccess;
  // widest load the row layout and X's alignment allow (tiles start at multiples of Din)
  const uintptr_t a = reinterpret_cast<uintptr_t>(X);
  const int vec = (a % 16 == 0 && p.Din % 4 == 0) ? 4 : (a % 8 == 0 && p.Din % 2 == 0) ? 2 : 1;
  if (split16) {
    // a tile is TR * Din floats with TR a multiple of 32, so every tile starts 16-byte aligned
    // when X does: float4 vectors over the flat tile, whatever Din
    const int v16 = (a % 16 == 0) ? 4 : 1;
    switch ((p.Din + 63) / 64) {
      case 1: return launch16_s<4>(p, X, N, v16, Y, grid, stream, cnt);
      case 2: return launch16_s<8>(p, X, N, v16, Y, grid, stream, cnt);
      case 3: return launch16_s<12>(p, X, N, v16, Y, grid, stream, cnt);
      case 4: return launch16_s<16>(p, X, N, v16, Y, grid, stream, cnt);
      default: return hipErrorInvalidValue;
    }
  }
  switch (p.S / 16) {
    case 1: return launch_s<16>(p, X, N, vec, Y, grid, stream, cnt);
    case 2: return launch_s<32>(p, X, N, vec, Y, grid, stream, cnt);
    case 3: return launch_s<48>(p, X, N, vec, Y, grid, stream, cnt);
    case 4: return launch_s<64>(p, X, N, vec, Y, grid, stream, cnt);
    case 5: return launch_s<80>(p, X, N, vec, Y, grid, stream, cnt);
    case 6: return launch_s<96>(p, X, N, vec, Y, grid, stream, cnt);
    case 7: return launch_s<112>(p, X, N, vec, Y, grid, stream, cnt);
    case 8: return launch_s<128>(p, X, N, vec, Y, grid, stream, cnt);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fv
