// gfx950 (CDNA4) statistics kernels for Fisher-vector encoding against a diagonal GMM.
//
// Fused kernel (E-step + soft assignment + moment accumulation in one pass; Sec. 3.1 and
// Algorithm 1 of the GPU-FV paper, its two GPU phases re-designed for MFMA):
//   * A workgroup of W wavefronts owns a group of 32*W components; wave w owns 32 of them
//     and keeps its slice of the E-step operand A = [mu/sigma^2 ; -1/(2 sigma^2)]
//     (log2(e)-scaled) in registers for the whole launch.
//   * Descriptors stream through LDS in tiles of 32 rows, stored as [x, x^2].
//   * E-step: the tile's logits on v_mfma_f32_32x32x2_f32 (the paper computes a distance per
//     dimension and reduces it with a tree in shared memory; here it is one contraction).
//   * Soft assignment: per-row max and sum over the wave's components with DPP/permlane
//     all-reduces, one exchange of (max, sum) between the waves through LDS, and the final
//     scale per (row, wave) -- the paper's maxPost / exp / sum / divide for each descriptor.
//   * Statistics: S^T[2DP x 32] += [x, x^2]^T gamma on the same MFMA shape, gamma taken from
//     the E-step result registers; S0 = sum gamma per lane on the VALU.  No posterior
//     threshold is applied.
//   * Each work item (a chunk of consecutive rows) writes its raw moments to a partial slot
//     of its own -- the analogue of the paper's per-block private U/V copies.
// LSE mode of the same kernel (first pass of the two-pass path): only the E-step and the row
// log-sum-exp over the workgroup's component group; writes (row max, log2 of the row sum).
#include <math.h>

#include "fv_device.h"

namespace fv {
namespace {

using namespace dev;

// GOUT (first pass of one component group only): the posterior factors are also written for
// a second pass that reads them instead of recomputing the E-step: component-major
// e[k * gstride + row] = 2^((logit - m_w) + lo) (m_w: the row maximum over the wave's 32
// components) before the workgroup barrier, then the row scales
// f[(Kp + w) * gstride + row] = 2^(m_w - M) / Z (0 for rows past the frame), so that
// gamma = e * f, the statistics mode's own product.  gstride is a multiple of 32 rows.
template <int DP, int W, bool LSE, bool TH, bool GOUT = false>
__global__ __launch_bounds__(64 * W) void fused_f32_kernel(
    const float* __restrict__ X, int D, int vec_ok, int64_t N, int P,
    const Item* __restrict__ items, int n_items, const float* __restrict__ A32,
    const float* __restrict__ c32, const float* __restrict__ cen, int Kp,
    float* __restrict__ partials, float2* __restrict__ lse, int64_t lse_stride,
    float* __restrict__ gout, int64_t gstride, const Counts* __restrict__ cnt, ItemQueue iqueue) {
  constexpr int NT = 64 * W;
  constexpr int NB = 2 * DP / 32;  // 32-feature output blocks of the statistics contraction
  // At 8 waves (two per SIMD, 256 registers each) the statistics kernel cannot also hold its
  // operand slice in registers without spilling; it keeps the slice in LDS and stages x only.
  constexpr bool ALDS = !LSE && W == 8 && DP == 64;
  constexpr int AS = 2 * DP + 4;  // LDS row stride of the operand slice
  using IO = TileIO<DP, NT, !ALDS>;
  constexpr int XS = IO::XS;

  __shared__ __attribute__((aligned(16))) float xs[2][kTile * XS];
  __shared__ __attribute__((aligned(16))) float as[ALDS ? W * kCompsPerWave * AS : 4];
  __shared__ __attribute__((aligned(16))) float xm[kTile * W];   // [row][wave] maxima
  __shared__ __attribute__((aligned(16))) float xsum[kTile * W]; // [row][wave] sums
  __shared__ __attribute__((aligned(16))) float loc[W][kTile];   // wave-private scratch
  __shared__ __attribute__((aligned(16))) float cs[DP];          // model centre

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int h = lane >> 5;
  const int j = lane & 31;
  const int group = blockIdx.y;  // component group (LSE mode); 0 for the fused statistics
  const int comp = group * (W * kCompsPerWave) + w * kCompsPerWave + j;

  float areg[ALDS ? 1 : DP];
  if constexpr (ALDS)
    load_a_lds<DP>(as + w * kCompsPerWave * AS, A32, comp / kCompsPerWave, lane, AS);
  else
    load_areg<DP>(areg, A32, comp / kCompsPerWave, lane);
  const float cval = c32[comp];
  const size_t slot = (size_t)(2 * DP + 1) * Kp;
  stage_centre<DP, NT>(cs, cen, tid);

  const int n_it = live_items(cnt, items, n_items);
  const int64_t n_rows = live_rows(cnt, N);
  __shared__ int s_it;
  const ItemQueue iq = items != nullptr ? iqueue : ItemQueue{nullptr, nullptr};
  for (int it = item_first(iq, n_it, &s_it); it < n_it; it = item_next(iq, n_it, &s_it, it)) {
    int64_t row0;
    int nrows;
    if (items != nullptr) {
      const Item t = items[it];
      row0 = t.row0;
      nrows = t.nrows;
    } else {
      row0 = (int64_t)it * P;
      const int64_t rem = n_rows - row0;
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
    IO::store(xs[0], pre, cs, tid);
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

      f32x16 hi, lo;
      if constexpr (ALDS)
        estep_f32_lds<DP>(xb + j * XS, as + (w * kCompsPerWave + j) * AS + DP * h, h, cval, hi, lo);
      else
        estep_f32<DP>(xb + j * XS + DP * h, areg, cval, hi, lo);

      // Per row: this wave's max and sum of exp2(logit - max) over its 32 components,
      // published for the cross-wave combine.
      f32x16 e;
      softmax_wave<W>(hi, lo, e, xm, xsum, loc[w], w, j, h);
      if constexpr (LSE && GOUT) {
        // rows crow(4g + p, h) = 8g + 4h + p of component `comp`: four 16-byte stores
        float* ge = gout + (size_t)comp * gstride + row0 + (int64_t)t * kTile + 4 * h;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const f32x4 v = {e[4 * g], e[4 * g + 1], e[4 * g + 2], e[4 * g + 3]};
          __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(ge + 8 * g));
        }
      }
      __syncthreads();
      {
        float M, L2Z;
        const float f = softmax_combine<W>(xm, xsum, w, j, h, valid, M, L2Z);
        if (LSE) {
          const int row = crow(j >> 1, h);
          if (w == 0 && !(j & 1) && row < valid)
            lse[(size_t)group * lse_stride + row0 + (int64_t)t * kTile + row] = make_float2(M, L2Z);
          if constexpr (GOUT) {
            if (!(j & 1))
              gout[(size_t)(Kp + w) * gstride + row0 + (int64_t)t * kTile + row] = f;
          }
        } else {
          if (!(j & 1)) loc[w][crow(j >> 1, h)] = f;
          wave_sync();
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const f32x4 fq = *reinterpret_cast<const f32x4*>(&loc[w][8 * q + 4 * h]);
#pragma unroll
            for (int p = 0; p < 4; ++p) e[4 * q + p] *= fq[p];  // gamma, in place
          }
        }
      }
      if (!LSE) {
        if (TH) apply_threshold(e, kTau);
#pragma unroll
        for (int r = 0; r < 16; ++r) s0 += e[r];
        if constexpr (ALDS)
          stats_f32_x<DP, TH>(xb, h, j, e, acc);
        else
          stats_f32<DP, TH>(xb, h, j, e, acc);
      }

      if (has_next) IO::store(xs[buf ^ 1], pre, cs, tid);
      __syncthreads();
    }

    if (!LSE) {
      // Raw moments of this item: rows f = 0..2DP-1 (x, x^2 features), then S0.  Buffer
      // stores: per-item resource bounded to one slot, per-lane offset (component and half),
      // wave-uniform row offset.
      __amdgpu_buffer_rsrc_t rs = make_rsrc(partials + (size_t)it * slot,
                                            (uint32_t)(slot * sizeof(float)));
      // the lane's half selects rows 4h..4h+3 of each 8-row group: per-lane offset, so the
      // scalar offset stays uniform across the wave
      const int vrow = comp * 4 + 4 * h * Kp * 4;
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc[b][r]), rs, vrow,
                                                (32 * b + crow(r, 0)) * Kp * 4, 0);
      auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(s0), __float_as_uint(s0), false,
                                                false);
      const float s0_total = __uint_as_float(p[0]) + __uint_as_float(p[1]);
      if (h == 0)
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(s0_total), rs, comp * 4,
                                              2 * DP * Kp * 4, 0);
    }
  }
}

// Second pass over whole component groups (see normext16_kernel): the fused kernel's layout
// (W waves x 32 components, a shared double-buffered tile), gamma from the first pass's
// per-row normalisers, one barrier per tile.
template <int DP, int W, bool TH>
__global__ __launch_bounds__(64 * W) void normext_f32_kernel(
    const float* __restrict__ X, int D, int vec_ok, int64_t N, int P,
    const Item* __restrict__ items, int n_items, const float2* __restrict__ lse, int G,
    int64_t lse_stride, const float* __restrict__ A32, const float* __restrict__ c32,
    const float* __restrict__ cen, int Kp, float* __restrict__ partials,
    const Counts* __restrict__ cnt, ItemQueue iqueue) {
  constexpr int NT = 64 * W;
  constexpr int NB = 2 * DP / 32;
  using IO = TileIO<DP, NT>;
  constexpr int XS = IO::XS;

  __shared__ __attribute__((aligned(16))) float xs[2][kTile * XS];
  __shared__ __attribute__((aligned(16))) float nrm[2][2 * kTile];  // per row: M, log2 Z
  __shared__ __attribute__((aligned(16))) float cs[DP];             // model centre

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int h = lane >> 5;
  const int j = lane & 31;
  const int comp = blockIdx.y * (W * kCompsPerWave) + w * kCompsPerWave + j;

  float areg[DP];
  load_areg<DP>(areg, A32, comp / kCompsPerWave, lane);
  const float cval = c32[comp];
  const size_t slot = (size_t)(2 * DP + 1) * Kp;
  stage_centre<DP, NT>(cs, cen, tid);

  const int n_it = live_items(cnt, items, n_items);
  const int64_t n_rows = live_rows(cnt, N);
  __shared__ int s_it;
  const ItemQueue iq = items != nullptr ? iqueue : ItemQueue{nullptr, nullptr};
  for (int it = item_first(iq, n_it, &s_it); it < n_it; it = item_next(iq, n_it, &s_it, it)) {
    int64_t row0;
    int nrows;
    if (items != nullptr) {
      const Item t = items[it];
      row0 = t.row0;
      nrows = t.nrows;
    } else {
      row0 = (int64_t)it * P;
      const int64_t rem = n_rows - row0;
      nrows = (int)(rem < (int64_t)P ? rem : (int64_t)P);
    }
    const int ntiles = (nrows + kTile - 1) / kTile;
    auto valid_of = [&](int t) {
      const int v = nrows - t * kTile;
      return v < kTile ? v : kTile;
    };

    f32x16 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[b][r] = 0.f;
    float s0 = 0.f;

    f32x4 pre[IO::kPer];
    float2 lv[kMaxLseGroups];
    auto fetch = [&](int t) {
      IO::fetch(pre, X, D, vec_ok != 0, row0 + (int64_t)t * kTile, valid_of(t), tid);
      if (tid < kTile) fetch_lse(lv, lse, G, lse_stride, row0 + (int64_t)t * kTile + tid, tid < valid_of(t));
    };
    auto stage = [&](int buf, int t) {
      IO::store(xs[buf], pre, cs, tid);
      if (tid < kTile) {
        float M = 0.f, L2Z = INFINITY;  // rows past the tile end get gamma = 0
        if (tid < valid_of(t)) merge_lse(lv, G, M, L2Z);
        nrm[buf][2 * tid] = M;
        nrm[buf][2 * tid + 1] = L2Z;
      }
    };
    fetch(0);
    stage(0, 0);
    __syncthreads();

    for (int t = 0; t < ntiles; ++t) {
      const int buf = t & 1;
      const bool has_next = (t + 1) < ntiles;
      if (has_next) fetch(t + 1);
      const float* xb = xs[buf];

      f32x16 hi, lo;
      estep_f32<DP>(xb + j * XS + DP * h, areg, cval, hi, lo);
      f32x16 gam;
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const f32x4 a = *reinterpret_cast<const f32x4*>(&nrm[buf][2 * (8 * qq + 4 * h)]);
        const f32x4 b = *reinterpret_cast<const f32x4*>(&nrm[buf][2 * (8 * qq + 4 * h) + 4]);
        const float Ms[4] = {a[0], a[2], b[0], b[2]};
        const float Ls[4] = {a[1], a[3], b[1], b[3]};
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int r = 4 * qq + p;
          gam[r] = fast_exp2(((hi[r] - Ms[p]) + lo[r]) - Ls[p]);
        }
      }
      if (TH) apply_threshold(gam, kTau);
#pragma unroll
      for (int r = 0; r < 16; ++r) s0 += gam[r];
      stats_f32<DP, TH>(xb, h, j, gam, acc);

      if (has_next) stage(buf ^ 1, t + 1);
      __syncthreads();
    }

    __amdgpu_buffer_rsrc_t rs = make_rsrc(partials + (size_t)it * slot,
                                          (uint32_t)(slot * sizeof(float)));
    const int vrow = comp * 4 + 4 * h * Kp * 4;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r)
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc[b][r]), rs, vrow,
                                              (32 * b + crow(r, 0)) * Kp * 4, 0);
    auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(s0), __float_as_uint(s0), false,
                                              false);
    const float s0_total = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    if (h == 0)
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(s0_total), rs, comp * 4,
                                            2 * DP * Kp * 4, 0);
  }
}

template <int DP, int W>
hipError_t launch_normext_dp(const Consts& c, const float* X, bool vec_ok, int64_t N, int P,
                             const Item* items, int n_items, int grid, const float2* lse,
                             int64_t lse_stride, float* partials, hipStream_t stream) {
  const dim3 grd(grid, c.Kp / (kCompsPerWave * W));
  if (c.thresh)
    hipLaunchKernelGGL((normext_f32_kernel<DP, W, true>), grd, dim3(64 * W), 0, stream, X, c.D,
                       vec_ok ? 1 : 0, N, P, items, n_items, lse, lse_groups(c), lse_stride,
                       c.A32, c.c32, c.cen, c.Kp, partials, c.cnt, c.queue);
  else
    hipLaunchKernelGGL((normext_f32_kernel<DP, W, false>), grd, dim3(64 * W), 0, stream, X, c.D,
                       vec_ok ? 1 : 0, N, P, items, n_items, lse, lse_groups(c), lse_stride,
                       c.A32, c.c32, c.cen, c.Kp, partials, c.cnt, c.queue);
  return hipGetLastError();
}

template <int W>
hipError_t normext_dp(const Consts& c, const float* X, bool vec_ok, int64_t N, int P,
                      const Item* items, int n_items, int grid, const float2* lse,
                      int64_t lse_stride, float* partials, hipStream_t stream) {
  switch (c.DP) {
    case 16: return launch_normext_dp<16, W>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, partials, stream);
    case 32: return launch_normext_dp<32, W>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, partials, stream);
    case 48: return launch_normext_dp<48, W>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, partials, stream);
    case 64: return launch_normext_dp<64, W>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, partials, stream);
    case 80: return launch_normext_dp<80, W>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, partials, stream);
    case 96: return launch_normext_dp<96, W>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, partials, stream);
    default: return hipErrorInvalidValue;
  }
}

template <int DP, int W, bool LSE>
hipError_t launch_fused(const Consts& c, const float* X, bool vec_ok, int64_t N, int P,
                        const Item* items, int n_items, int grid, int groups, float* partials,
                        float2* lse, int64_t lse_stride, float* gout, int64_t gstride,
                        hipStream_t stream) {
  if constexpr (!LSE) {
    if (c.thresh) {
      hipLaunchKernelGGL((fused_f32_kernel<DP, W, false, true>), dim3(grid, groups), dim3(64 * W),
                         0, stream, X, c.D, vec_ok ? 1 : 0, N, P, items, n_items, c.A32, c.c32,
                         c.cen, c.Kp, partials, lse, lse_stride, nullptr, 0, c.cnt, c.queue);
      return hipGetLastError();
    }
  } else {
    if (gout != nullptr) {
      // posterior output up to DP = 64 only (the 8-wave variant would spill above)
      if constexpr (DP <= 64) {
        if (groups != 1) return hipErrorInvalidValue;
        hipLaunchKernelGGL((fused_f32_kernel<DP, W, true, false, true>), dim3(grid, 1),
                           dim3(64 * W), 0, stream, X, c.D, vec_ok ? 1 : 0, N, P, items, n_items,
                           c.A32, c.c32, c.cen, c.Kp, partials, lse, lse_stride, gout, gstride,
                           c.cnt, c.queue);
        return hipGetLastError();
      } else {
        return hipErrorInvalidValue;
      }
    }
  }
  hipLaunchKernelGGL((fused_f32_kernel<DP, W, LSE, false>), dim3(grid, groups), dim3(64 * W), 0,
                     stream, X, c.D, vec_ok ? 1 : 0, N, P, items, n_items, c.A32, c.c32, c.cen,
                     c.Kp, partials, lse, lse_stride, nullptr, 0, c.cnt, c.queue);
  return hipGetLastError();
}

template <int W, bool LSE>
hipError_t dispatch_dp(const Consts& c, const float* X, bool vec_ok, int64_t N, int P,
                       const Item* items, int n_items, int grid, int groups, float* partials,
                       float2* lse, int64_t lse_stride, float* gout, int64_t gstride,
                       hipStream_t stream) {
#define FV_CASE(DPV)                                                                   \
  case DPV:                                                                            \
    return launch_fused<DPV, W, LSE>(c, X, vec_ok, N, P, items, n_items, grid, groups, \
                                     partials, lse, lse_stride, gout, gstride, stream);
  switch (c.DP) {
    FV_CASE(16)
    FV_CASE(32)
    FV_CASE(48)
    FV_CASE(64)
    FV_CASE(80)
    FV_CASE(96)
    default: return hipErrorInvalidValue;
  }
#undef FV_CASE
}

template <bool LSE>
hipError_t dispatch_w(int W, const Consts& c, const float* X, bool vec_ok, int64_t N, int P,
                      const Item* items, int n_items, int grid, int groups, float* partials,
                      float2* lse, int64_t lse_stride, float* gout, int64_t gstride,
                      hipStream_t stream) {
  switch (W) {
    case 1: return dispatch_dp<1, LSE>(c, X, vec_ok, N, P, items, n_items, grid, groups, partials, lse, lse_stride, gout, gstride, stream);
    case 2: return dispatch_dp<2, LSE>(c, X, vec_ok, N, P, items, n_items, grid, groups, partials, lse, lse_stride, gout, gstride, stream);
    case 4: return dispatch_dp<4, LSE>(c, X, vec_ok, N, P, items, n_items, grid, groups, partials, lse, lse_stride, gout, gstride, stream);
    case 8: return dispatch_dp<8, LSE>(c, X, vec_ok, N, P, items, n_items, grid, groups, partials, lse, lse_stride, gout, gstride, stream);
    default: return hipErrorNotSupported;
  }
}

}  // namespace

hipError_t launch_stats(const Consts& c, int precision, const float* X, bool vec_ok, int64_t N,
                        int P, const Item* items, int n_items, int grid, float* partials,
                        hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  if (precision != 0 || c.Kp > kMaxWaves * kCompsPerWave) return hipErrorNotSupported;
  return dispatch_w<false>(c.Wg, c, X, vec_ok, N, P, items, n_items, grid, 1, partials, nullptr,
                           0, nullptr, 0, stream);
}

hipError_t launch_lse(const Consts& c, int precision, const float* X, bool vec_ok, int64_t N,
                      const Item* items, int n_items, int grid, float2* lse, int64_t lse_stride,
                      hipStream_t stream, float* gout, int64_t gstride) {
  if (n_items <= 0) return hipSuccess;
  if (precision != 0) return hipErrorNotSupported;
  if (gout != nullptr && (items != nullptr || gstride < N || gstride % kTile != 0))
    return hipErrorInvalidValue;
  return dispatch_w<true>(c.Wg, c, X, vec_ok, N, kTile, items, n_items, grid, lse_groups(c),
                          nullptr, lse, lse_stride, gout, gstride, stream);
}

hipError_t launch_normext(const Consts& c, const float* X, bool vec_ok, int64_t N, int P,
                          const Item* items, int n_items, int grid, const float2* lse,
                          int64_t lse_stride, float* partials, hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  // above DP = 64 an 8-wave workgroup (two waves per SIMD) runs out of registers: use 4 waves
  // (128 components per workgroup, Kp / 128 of them per chunk)
  switch (c.DP > 64 && c.Wg == 8 ? 4 : c.Wg) {
    case 1: return normext_dp<1>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, partials, stream);
    case 2: return normext_dp<2>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, partials, stream);
    case 4: return normext_dp<4>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, partials, stream);
    case 8: return normext_dp<8>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, partials, stream);
    default: return hipErrorNotSupported;
  }
}

}  // namespace fv
