// Second pass of the two-pass path: statistics sliced by component.
//
// The first pass (LSE mode of the fused kernel) leaves, for every descriptor and every group
// of up to 256 components, the row maximum m_g and log2 of the row sum s_g of the base-2
// posteriors.  Here a workgroup owns one chunk of descriptors and one slice of 32
// components: it recomputes those 32 logits per descriptor with the same E-step code (so the
// logits are bit-identical to the first pass), forms the soft assignment directly as
//     gamma = exp2((logit - M) - log2 Z),   M = max_g m_g,  Z = sum_g s_g 2^(m_g - M),
// and accumulates the statistics for its slice.  No cross-lane or cross-wave reduction is
// needed inside the tile loop, so the waves of a workgroup run independent tiles with
// wave-private LDS staging and no workgroup barrier until the end of the chunk, where their
// accumulators are summed (fixed order) and written to the chunk's partial slot.  A workgroup
// has eight waves up to DP = 64 (wave-private tiles of 137 KB of LDS in all; two waves per
// SIMD, so one wave's loads overlap the other's MFMAs) and four beyond.
//
// GIN: with one component group the first pass can also write the posterior factors (e,
// component-major [Kp][gstride], and the row scales f, [Kp / 32][gstride]); the workgroup then
// forms gamma = e * f for its slice instead of recomputing the E-step.
//
// Without GIN this path costs one extra E-step (the logits are computed twice); either way it
// gives a single frame many more independent workgroups and smaller partial traffic than the
// fused kernel, and it is the only path for more than 256 components.
#include <math.h>

#include "fv_device.h"

namespace fv {
namespace {

using namespace dev;

// Waves per workgroup of the second pass (their LDS tiles must fit together).
constexpr int slice_waves(int DP) { return DP <= 64 ? 8 : 4; }

template <int DP, int NW, bool TH, bool GIN>
__global__ __launch_bounds__(64 * NW, 2) void sliced_f32_kernel(
    const float* __restrict__ X, int D, int vec_ok, int64_t N, int P,
    const Item* __restrict__ items, int n_items, const float2* __restrict__ lse, int G,
    int64_t lse_stride, const float* __restrict__ A32, const float* __restrict__ c32,
    const float* __restrict__ cen, int Kp, const float* __restrict__ gin, int64_t gstride,
    float* __restrict__ partials) {
  constexpr int NB = 2 * DP / 32;
  using IO = TileIO<DP, 64>;
  constexpr int XS = IO::XS;

  __shared__ __attribute__((aligned(16))) float xs[NW][kTile * XS];
  __shared__ __attribute__((aligned(16))) float ls[NW][kTile * 2];
  __shared__ __attribute__((aligned(16))) float cs[DP];  // model centre

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int h = lane >> 5;
  const int j = lane & 31;
  const int q = blockIdx.y;  // component slice
  const int comp = q * kCompsPerWave + j;

  float areg[GIN ? 1 : DP];
  float cval = 0.f;
  if constexpr (!GIN) {
    load_areg<DP>(areg, A32, q, lane);
    cval = c32[comp];
  }
  const size_t slot = (size_t)(2 * DP + 1) * Kp;
  float* xw = xs[w];
  float* lw = ls[w];
  stage_centre<DP, 64 * NW>(cs, cen, tid);

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

    for (int t = w; t < ntiles; t += NW) {
      const int valid = (nrows - t * kTile) < kTile ? (nrows - t * kTile) : kTile;
      const int64_t trow = row0 + (int64_t)t * kTile;
      f32x4 pre[IO::kPer];
      IO::fetch(pre, X, D, vec_ok != 0, trow, valid, lane);
      f32x16 gam;
      if constexpr (GIN) {
        // register 4g + p holds row crow(4g + p, h) = 8g + 4h + p: four 16-byte loads each of
        // e (this lane's component) and of the row scales (this slice); rows past the frame
        // have scale 0
        const float* ge = gin + (size_t)comp * gstride + trow + 4 * h;
        const float* gf = gin + (size_t)(Kp + q) * gstride + trow + 4 * h;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const f32x4 ev = *reinterpret_cast<const f32x4*>(ge + 8 * g);
          const f32x4 fv = *reinterpret_cast<const f32x4*>(gf + 8 * g);
#pragma unroll
          for (int p = 0; p < 4; ++p) gam[4 * g + p] = ev[p] * fv[p];
        }
      }
      // per-row normaliser from the first pass, merged over component groups (the same
      // arithmetic as merge_lse, one group at a time to save registers)
      if (!GIN && lane < kTile) {
        float M = 0.f, L2Z = INFINITY;  // rows past the tile end get gamma = 0
        if (lane < valid) {
          float2 v = lse[trow + lane];
          M = v.x;
          float Z = exp2f(v.y);
          for (int g = 1; g < G; ++g) {
            const float2 u = lse[(size_t)g * lse_stride + trow + lane];
            const float Mn = fmaxf(M, u.x);
            Z = Z * fast_exp2(M - Mn) + exp2f(u.y) * fast_exp2(u.x - Mn);
            M = Mn;
          }
          L2Z = (G == 1) ? v.y : log2f(Z);
        }
        lw[2 * lane] = M;
        lw[2 * lane + 1] = L2Z;
      }
      IO::store(xw, pre, cs, lane);
      wave_sync();

      if constexpr (!GIN) {
        f32x16 hi, lo;
        estep_f32<DP>(xw + j * XS + DP * h, areg, cval, hi, lo);
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const f32x4 a = *reinterpret_cast<const f32x4*>(lw + 2 * (8 * qq + 4 * h));
          const f32x4 b = *reinterpret_cast<const f32x4*>(lw + 2 * (8 * qq + 4 * h) + 4);
          const float Ms[4] = {a[0], a[2], b[0], b[2]};
          const float Ls[4] = {a[1], a[3], b[1], b[3]};
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            const int r = 4 * qq + p;
            gam[r] = fast_exp2(((hi[r] - Ms[p]) + lo[r]) - Ls[p]);
          }
        }
      }
      if (TH) apply_threshold(gam, kTau);
#pragma unroll
      for (int r = 0; r < 16; ++r) s0 += gam[r];
      stats_f32<DP, TH>(xw, h, j, gam, acc);
      wave_sync();
    }

    // ---- sum the waves' accumulators in fixed order and write this slice of the slot
    __syncthreads();
    float* red = &xs[0][0];  // [wave][f][32] then S0 [wave][32]
    constexpr int RW = 2 * DP * kCompsPerWave;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) red[w * RW + (32 * b + crow(r, h)) * kCompsPerWave + j] = acc[b][r];
    auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(s0), __float_as_uint(s0), false, false);
    if (h == 0) red[NW * RW + w * kCompsPerWave + j] = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    __syncthreads();
    float* dst = partials + (size_t)it * slot + (size_t)q * kCompsPerWave;
    for (int e = tid; e < (2 * DP + 1) * kCompsPerWave; e += 64 * NW) {
      const int f = e / kCompsPerWave;
      const int jj = e % kCompsPerWave;
      float v;
      if (f < 2 * DP) {
        v = red[f * kCompsPerWave + jj];
#pragma unroll
        for (int ww = 1; ww < NW; ++ww) v += red[ww * RW + f * kCompsPerWave + jj];
      } else {
        v = red[NW * RW + jj];
#pragma unroll
        for (int ww = 1; ww < NW; ++ww) v += red[NW * RW + ww * kCompsPerWave + jj];
      }
      __builtin_nontemporal_store(v, &dst[(size_t)f * Kp + jj]);  // read by another kernel
    }
    __syncthreads();
  }
}

template <int DP, bool TH, bool GIN>
void launch_sliced_k(const Consts& c, const float* X, bool vec_ok, int64_t N, int P,
                     const Item* items, int n_items, int grid, const float2* lse,
                     int64_t lse_stride, const float* gin, int64_t gstride, float* partials,
                     hipStream_t stream) {
  constexpr int NW = slice_waves(DP);
  hipLaunchKernelGGL((sliced_f32_kernel<DP, NW, TH, GIN>), dim3(grid, c.Kp / kCompsPerWave),
                     dim3(64 * NW), 0, stream, X, c.D, vec_ok ? 1 : 0, N, P, items, n_items, lse,
                     lse_groups(c), lse_stride, c.A32, c.c32, c.cen, c.Kp, gin, gstride, partials);
}

template <int DP>
hipError_t launch_sliced_dp(const Consts& c, const float* X, bool vec_ok, int64_t N, int P,
                            const Item* items, int n_items, int grid, const float2* lse,
                            int64_t lse_stride, const float* gin, int64_t gstride,
                            float* partials, hipStream_t stream) {
  if (gin != nullptr && (lse_groups(c) != 1 || items != nullptr || P % kTile != 0 ||
                         gstride < N || gstride % kTile != 0))
    return hipErrorInvalidValue;
  if (gin != nullptr) {
    if constexpr (DP <= 64) {  // the first pass writes posterior factors up to DP = 64
      if (c.thresh)
        launch_sliced_k<DP, true, true>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, gin, gstride, partials, stream);
      else
        launch_sliced_k<DP, false, true>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, gin, gstride, partials, stream);
    } else {
      return hipErrorInvalidValue;
    }
  } else {
    if (c.thresh)
      launch_sliced_k<DP, true, false>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, nullptr, 0, partials, stream);
    else
      launch_sliced_k<DP, false, false>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, nullptr, 0, partials, stream);
  }
  return hipGetLastError();
}

}  // namespace

int sliced_rows_per_wave_round(int DP) { return kTile * slice_waves(DP); }

hipError_t launch_sliced(const Consts& c, int precision, const float* X, bool vec_ok, int64_t N,
                         int P, const Item* items, int n_items, int grid, const float2* lse,
                         int64_t lse_stride, float* partials, hipStream_t stream,
                         const float* gin, int64_t gstride) {
  if (n_items <= 0) return hipSuccess;
  if (precision != 0) return hipErrorNotSupported;
  switch (c.DP) {
    case 16: return launch_sliced_dp<16>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, gin, gstride, partials, stream);
    case 32: return launch_sliced_dp<32>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, gin, gstride, partials, stream);
    case 48: return launch_sliced_dp<48>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, gin, gstride, partials, stream);
    case 64: return launch_sliced_dp<64>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, gin, gstride, partials, stream);
    case 80: return launch_sliced_dp<80>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, gin, gstride, partials, stream);
    case 96: return launch_sliced_dp<96>(c, X, vec_ok, N, P, items, n_items, grid, lse, lse_stride, gin, gstride, partials, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fv
