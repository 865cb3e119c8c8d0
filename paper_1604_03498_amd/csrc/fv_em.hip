// EM step kernels: the GMM the encoder uses is trained beforehand (Sec. 3.1); one EM
// iteration needs exactly the quantities the encoder already computes -- the posteriors'
// per-row normalisers (the first pass) and the per-component sums S0 = sum gamma,
// S1 = gamma^T X, S2 = gamma^T X^2 (the statistics pass) -- so the training step reuses those
// kernels and adds two small ones:
//
//   em_mstep   one thread per (d, k): S0, S1[d], S2[d] summed over the chunk partials in
//              double, in chunk order; then w = S0 / N, mu = S1 / S0,
//              var = max(S2 / S0 - mu^2, floor) (a component with S0 = 0 gets w = 0, mu = 0,
//              var = floor); S1 and S2 are moments of the centred descriptors x - m0, so the
//              mean returned is S1 / S0 + m0
//   em_loglik  per row, log2 of sum_k exp2(logit) = M + log2 Z from the first pass's group
//              normalisers; summed in double per workgroup in a fixed order (grid-stride
//              rows, then a tree over the workgroup); the caller adds the workgroup sums in
//              order, scales by ln 2 and subtracts N (D/2) ln(2 pi)
#include <math.h>

#include "fv_device.h"

namespace fv {
namespace {

constexpr int kEmThreads = 256;

__global__ __launch_bounds__(kEmThreads) void em_mstep_kernel(
    const float* __restrict__ partials, int n_items, int K, int D, int DP, int Kp, double n_rows,
    float var_floor, const float* __restrict__ cen, float* __restrict__ w_out,
    float* __restrict__ mu_out, float* __restrict__ var_out) {
  const int idx = blockIdx.x * kEmThreads + threadIdx.x;
  if (idx >= K * D) return;
  const int k = idx % K;  // consecutive threads: consecutive components (coalesced rows)
  const int d = idx / K;
  const size_t slot = (size_t)(2 * DP + 1) * Kp;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int it = 0; it < n_items; ++it) {
    const float* p = partials + (size_t)it * slot;
    s0 += (double)p[(size_t)2 * DP * Kp + k];
    s1 += (double)p[(size_t)d * Kp + k];
    s2 += (double)p[(size_t)(DP + d) * Kp + k];
  }
  double mu = 0.0, var = (double)var_floor;
  if (s0 > 0.0) {
    mu = s1 / s0;
    var = s2 / s0 - mu * mu;
    if (!(var >= (double)var_floor)) var = (double)var_floor;
  }
  // the statistics are of the centred descriptors x - m0; the mean goes back by m0 (a
  // component with S0 = 0 keeps mu = 0)
  mu_out[(size_t)k * D + d] = (float)(s0 > 0.0 ? mu + (double)cen[d] : 0.0);
  var_out[(size_t)k * D + d] = (float)var;
  if (d == 0) w_out[k] = (float)(s0 / n_rows);
}

__global__ __launch_bounds__(kEmThreads) void em_loglik_kernel(const float2* __restrict__ lse,
                                                                int G, int64_t stride,
                                                                int64_t N,
                                                                double* __restrict__ part) {
  __shared__ double red[kEmThreads];
  double acc = 0.0;
  for (int64_t row = (int64_t)blockIdx.x * kEmThreads + threadIdx.x; row < N;
       row += (int64_t)gridDim.x * kEmThreads) {
    float2 l[dev::kMaxLseGroups];
    dev::fetch_lse(l, lse, G, stride, row, true);
    float M, L2Z;
    dev::merge_lse(l, G, M, L2Z);
    acc += (double)M + (double)L2Z;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kEmThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

}  // namespace

int em_loglik_blocks(int64_t N) {
  const int64_t b = (N + kEmThreads - 1) / kEmThreads;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

hipError_t launch_em(const Consts& c, const float* partials, int n_items, int64_t N,
                     float var_floor, const float2* lse, int64_t lse_stride, float* w_out,
                     float* mu_out, float* var_out, double* ll_part, hipStream_t stream) {
  const int KD = c.K * c.D;
  hipLaunchKernelGGL(em_mstep_kernel, dim3((KD + kEmThreads - 1) / kEmThreads), dim3(kEmThreads),
                     0, stream, partials, n_items, c.K, c.D, c.DP, c.Kp, (double)N, var_floor,
                     c.cen, w_out, mu_out, var_out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(em_loglik_kernel, dim3(em_loglik_blocks(N)), dim3(kEmThreads), 0, stream,
                     lse, lse_groups(c), lse_stride, N, ll_part);
  return hipGetLastError();
}

}  // namespace fv
