// gfx950 (CDNA4) kernels for Fisher-vector encoding against a diagonal GMM.
//
// Statistics kernel (fused E-step + soft assignment + moment accumulation, Sec. 2.1 /
// Algorithm 1 of the GPU-FV paper, re-designed for MFMA):
//   * A workgroup of W wavefronts owns all Kp = 32*W components; wave w owns components
//     [32w, 32w+32).  Its slice of the E-step operand A = [mu/sigma^2 ; -1/(2 sigma^2)]
//     (log2(e)-scaled) lives in registers for the whole launch.
//   * Descriptors stream through LDS in tiles of 32 rows as [x, x^2].
//   * E-step: L[32 x 32] = [x, x^2] A + c on v_mfma_f32_32x32x2_f32 (log-joint up to a
//     constant, base 2).  This replaces the paper's per-dimension distance + tree reduction.
//   * Soft assignment: per-row max and sum over the wave's 32 components with DPP/permlane
//     all-reduces, then one exchange of (max, sum) between the W waves through LDS.  This is
//     the paper's maxPost / exp / sum / divide sequence for one descriptor.
//   * Statistics: S^T[2DP x 32] += [x, x^2]^T gamma, again on 32x32x2 MFMA, with gamma taken
//     straight from the E-step result registers as the B operand (the descriptor order inside
//     the contraction is permuted to match the MFMA result layout -- the sum is order-free).
//     S0 = sum gamma is a per-lane VALU sum.  No posterior threshold is applied.
//   * Each work item (a chunk of consecutive rows) writes raw moments to its own partial
//     slot, the analogue of the paper's per-block private U/V copies.
// Finalize kernels: sum a frame's slots in chunk order in double precision, turn raw moments
// into u and v (the paper's reduction kernel plus the improved-FV normalisation).
#include <math.h>

#include "fv_internal.h"

namespace fv {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr unsigned kFlagNoPower = 4u;
constexpr unsigned kFlagNoL2 = 8u;

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

// ---- descriptor tile staging ------------------------------------------------------------
// Tile = 32 rows x DP features, fetched as float4 slots into registers, then written to LDS
// as [x (DP) | x^2 (DP) | pad 4] per row.  Rows past the chunk and features past D are zero.
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

// ---- statistics kernel, FP32 MFMA ---------------------------------------------------------
template <int DP, int W>
__global__ __launch_bounds__(64 * W) void stats_f32_kernel(
    const float* __restrict__ X, int D, int vec_ok, int64_t N, int P,
    const Item* __restrict__ items, int n_items, const float* __restrict__ A32,
    const float* __restrict__ c32, int Kp, float* __restrict__ partials) {
  constexpr int NT = 64 * W;
  constexpr int NB = 2 * DP / 32;  // 32-feature output blocks of the statistics contraction
  using IO = TileIO<DP, NT>;
  constexpr int XS = IO::XS;

  __shared__ __attribute__((aligned(16))) float xs[2][kTile * XS];
  __shared__ __attribute__((aligned(16))) float red_m[W][kTile];
  __shared__ __attribute__((aligned(16))) float red_s[W][kTile];
  __shared__ __attribute__((aligned(16))) float fac[W][kTile];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int h = lane >> 5;  // which half of the wave: selects k = 0/1 in the 32x32x2 operands
  const int j = lane & 31;
  const int comp = w * kCompsPerWave + j;

  // E-step B operand: lane (h, j) supplies A[s + DP*h][comp] at step s.
  float areg[DP];
#pragma unroll
  for (int s = 0; s < DP; ++s) areg[s] = A32[(size_t)(s + DP * h) * Kp + comp];
  const float cval = c32[comp];
  const size_t slot = (size_t)(2 * DP + 1) * Kp;

  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    int64_t row0;
    int nrows;
    if (items != nullptr) {
      const Item t = items[it];
      row0 = t.row0;
      nrows = t.nrows;
    } else {
      row0 = (int64_t)it * P;
      const int64_t rem = N - row0;
      nrows = (int)(rem < (int64_t)P ? rem : (int64_t)P);
    }
    const int ntiles = (nrows + kTile - 1) / kTile;

    f32x16 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[b][r] = 0.f;
    float s0 = 0.f;

    f32x4 pre[IO::kPer];
    IO::fetch(pre, X, D, vec_ok != 0, row0, nrows < kTile ? nrows : kTile, tid);
    IO::store(xs[0], pre, tid);
    __syncthreads();

    for (int t = 0; t < ntiles; ++t) {
      const int buf = t & 1;
      const int valid = (nrows - t * kTile) < kTile ? (nrows - t * kTile) : kTile;
      const bool has_next = (t + 1) < ntiles;
      if (has_next) {
        const int nvalid = (nrows - (t + 1) * kTile) < kTile ? (nrows - (t + 1) * kTile) : kTile;
        IO::fetch(pre, X, D, vec_ok != 0, row0 + (int64_t)(t + 1) * kTile, nvalid, tid);
      }
      const float* xb = xs[buf];

      // ---- E-step: logits of the 32 rows for this wave's 32 components (log2 units).
      // The 2*DP products per logit are accumulated in chains of 16 MFMA steps; the chain
      // sums are added with an error-free transformation (TwoSum), keeping the logit as an
      // unevaluated pair hi + lo.  exp2 later sees (hi - max) + lo, which is accurate to the
      // size of the difference rather than of the logit (|logit| reaches a few hundred).
      f32x16 hi, lo;
      const float* xr = xb + j * XS + DP * h;
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
      f32x16 L;  // becomes exp2(logit - rowmax), then gamma, in place

      // ---- soft assignment.  Register r holds row 8*(r/4) + 4*h + r%4, component `comp`.
      // Per row: this wave's max and sum of exp2(L - max) over its 32 components; lane j == 0
      // of each half publishes them for the cross-wave combine.  L is overwritten with e.
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r >> 2) + 4 * h + (r & 3);
        const float m = allreduce32(hi[r], MaxOp());
        L[r] = fast_exp2((hi[r] - m) + lo[r]);
        const float sum = allreduce32(L[r], AddOp());
        if (j == 0) {
          red_m[w][row] = m;
          red_s[w][row] = sum;
        }
      }
      __syncthreads();
      if (tid < kTile) {  // one thread per row combines the W partial (max, sum) pairs
        const int row = tid;
        float M = red_m[0][row];
#pragma unroll
        for (int v = 1; v < W; ++v) M = fmaxf(M, red_m[v][row]);
        float sc[W];
        float Z = 0.f;
#pragma unroll
        for (int v = 0; v < W; ++v) {
          sc[v] = fast_exp2(red_m[v][row] - M);
          Z += red_s[v][row] * sc[v];
        }
        const float inv = (row < valid) ? 1.0f / Z : 0.0f;
#pragma unroll
        for (int v = 0; v < W; ++v) fac[v][row] = sc[v] * inv;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 f = *reinterpret_cast<const f32x4*>(&fac[w][8 * q + 4 * h]);
#pragma unroll
        for (int p = 0; p < 4; ++p) L[4 * q + p] *= f[p];  // gamma, in place
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) s0 += L[r];

      // ---- statistics: S^T[f][comp] += sum_rows Xa[row][f] * gamma[row][comp]
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const int row = 8 * (s >> 2) + 4 * h + (s & 3);
        const float* xrow = xb + row * XS + j;
#pragma unroll
        for (int b = 0; b < NB; ++b)
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(xrow[32 * b], L[s], acc[b], 0, 0, 0);
      }

      if (has_next) IO::store(xs[buf ^ 1], pre, tid);
      __syncthreads();
    }

    // ---- write this item's raw moments: rows f = 0..2DP-1 (x, x^2 features), then S0.
    // Buffer stores: a per-item resource (bounds = one slot), lane offset comp*4 and a uniform
    // row offset, so no per-store 64-bit addresses are kept live.
    __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        partials + (size_t)it * slot, 0, (int)(slot * sizeof(float)), 0x00020000);
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int f = 32 * b + 8 * (r >> 2) + 4 * h + (r & 3);
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc[b][r]), rs, comp * 4,
                                              f * Kp * 4, 0);
      }
    auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(s0), __float_as_uint(s0), false, false);
    const float s0_total = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    if (h == 0)
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(s0_total), rs, comp * 4,
                                            2 * DP * Kp * 4, 0);
  }
}

// ---- finalize ------------------------------------------------------------------------------
constexpr int kFinThreads = 256;

__global__ __launch_bounds__(kFinThreads) void finalize_reduce_kernel(
    const float* __restrict__ partials, const Frame* __restrict__ frames, Frame single, int K,
    int D, int DP, int Kp, const double* __restrict__ mu64, const double* __restrict__ isd64,
    const double* __restrict__ ivar64, const double* __restrict__ cu64,
    const double* __restrict__ cv64, unsigned flags, float* __restrict__ out,
    double* __restrict__ normpart) {
  __shared__ double red[kFinThreads];
  const int b = blockIdx.y;
  const Frame fr = frames != nullptr ? frames[b] : single;
  const int KD = K * D;
  const int idx = blockIdx.x * kFinThreads + threadIdx.x;
  const size_t slot = (size_t)(2 * DP + 1) * Kp;
  double ss = 0.0;
  if (idx < KD) {
    const int k = idx % K;  // consecutive threads read consecutive components
    const int d = idx / K;
    double S0 = 0.0, S1 = 0.0, S2 = 0.0;
    const float* p = partials + (size_t)fr.item0 * slot;
    for (int c = 0; c < fr.nitems; ++c, p += slot) {
      S0 += (double)p[(size_t)(2 * DP) * Kp + k];
      S1 += (double)p[(size_t)d * Kp + k];
      S2 += (double)p[(size_t)(DP + d) * Kp + k];
    }
    double u = 0.0, v = 0.0;
    if (fr.nrows > 0) {
      const int kd = k * D + d;
      const double m = mu64[kd];
      const double C1 = S1 - m * S0;                      // sum gamma (x - mu)
      const double C2 = S2 - m * (2.0 * S1 - m * S0);     // sum gamma (x - mu)^2
      const double invN = 1.0 / (double)fr.nrows;
      u = C1 * isd64[kd] * cu64[k] * invN;
      v = (C2 * ivar64[kd] - S0) * cv64[k] * invN;
      if (!(flags & kFlagNoPower)) {
        u = (u > 0.0) ? sqrt(u) : ((u < 0.0) ? -sqrt(-u) : 0.0);
        v = (v > 0.0) ? sqrt(v) : ((v < 0.0) ? -sqrt(-v) : 0.0);
      }
    }
    float* o = out + (size_t)b * 2 * KD;
    o[k * D + d] = (float)u;
    o[KD + k * D + d] = (float)v;
    ss = u * u + v * v;
  }
  red[threadIdx.x] = ss;
  __syncthreads();
  for (int s = kFinThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) normpart[(size_t)b * gridDim.x + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kFinThreads) void finalize_l2_kernel(float* __restrict__ out,
                                                                  const double* __restrict__ normpart,
                                                                  int nblk, int len) {
  __shared__ double inv;
  const int b = blockIdx.x;
  if (threadIdx.x == 0) {
    double ss = 0.0;
    for (int i = 0; i < nblk; ++i) ss += normpart[(size_t)b * nblk + i];
    inv = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
  }
  __syncthreads();
  if (inv == 0.0) return;
  float* o = out + (size_t)b * len;
  for (int i = threadIdx.x; i < len; i += kFinThreads) o[i] = (float)((double)o[i] * inv);
}

template <int DP, int W>
hipError_t launch_f32(const Consts& c, const float* X, bool vec_ok, int64_t N, int P,
                      const Item* items, int n_items, int grid, float* partials,
                      hipStream_t stream) {
  hipLaunchKernelGGL((stats_f32_kernel<DP, W>), dim3(grid), dim3(64 * W), 0, stream, X, c.D,
                     vec_ok ? 1 : 0, N, P, items, n_items, c.A32, c.c32, c.Kp, partials);
  return hipGetLastError();
}

template <int W>
hipError_t dispatch_dp_f32(const Consts& c, const float* X, bool vec_ok, int64_t N, int P,
                           const Item* items, int n_items, int grid, float* partials,
                           hipStream_t stream) {
  switch (c.DP) {
    case 16: return launch_f32<16, W>(c, X, vec_ok, N, P, items, n_items, grid, partials, stream);
    case 32: return launch_f32<32, W>(c, X, vec_ok, N, P, items, n_items, grid, partials, stream);
    case 48: return launch_f32<48, W>(c, X, vec_ok, N, P, items, n_items, grid, partials, stream);
    case 64: return launch_f32<64, W>(c, X, vec_ok, N, P, items, n_items, grid, partials, stream);
    case 80: return launch_f32<80, W>(c, X, vec_ok, N, P, items, n_items, grid, partials, stream);
    case 96: return launch_f32<96, W>(c, X, vec_ok, N, P, items, n_items, grid, partials, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_stats(const Consts& c, int precision, const float* X, bool vec_ok, int64_t N,
                        int P, const Item* items, int n_items, int grid, float* partials,
                        hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  if (precision != 0) return hipErrorNotSupported;
  switch (c.W) {
    case 1: return dispatch_dp_f32<1>(c, X, vec_ok, N, P, items, n_items, grid, partials, stream);
    case 2: return dispatch_dp_f32<2>(c, X, vec_ok, N, P, items, n_items, grid, partials, stream);
    case 4: return dispatch_dp_f32<4>(c, X, vec_ok, N, P, items, n_items, grid, partials, stream);
    case 8: return dispatch_dp_f32<8>(c, X, vec_ok, N, P, items, n_items, grid, partials, stream);
    default: return hipErrorInvalidValue;
  }
}

int finalize_blocks(const Consts& c) { return (c.K * c.D + kFinThreads - 1) / kFinThreads; }

hipError_t launch_finalize(const Consts& c, const float* partials, const Frame* frames,
                           Frame single, int B, unsigned flags, float* out, double* normpart,
                           hipStream_t stream) {
  if (B <= 0) return hipSuccess;
  const int nblk = finalize_blocks(c);
  hipLaunchKernelGGL(finalize_reduce_kernel, dim3(nblk, B), dim3(kFinThreads), 0, stream,
                     partials, frames, single, c.K, c.D, c.DP, c.Kp, c.mu64, c.isd64, c.ivar64,
                     c.cu64, c.cv64, flags, out, normpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!(flags & kFlagNoL2)) {
    hipLaunchKernelGGL(finalize_l2_kernel, dim3(B), dim3(kFinThreads), 0, stream, out, normpart,
                       nblk, 2 * c.K * c.D);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace fv
