// Finalize kernels: the reduction of per-chunk partial statistics (the analogue of the
// paper's second Phase-2 kernel that sums the per-block U/V copies, Sec. 3.2, Algorithm 3),
// followed by the improved-FV assembly and normalisation (Fisher-information scaling,
// signed square root, L2).
//
//   group_reduce   gbuf[g][e] = sum over the group's slots (index order, double) of
//                  partials[slot][e], for every element e of the [2DP+1][Kp] slot layout
//   assemble       per frame and (k, d): S0, S1, S2 = sum of the frame's group rows (in
//                  order); C1 = S1 - mu S0; C2 = S2 - 2 mu S1 + mu^2 S0;
//                  u = C1 / sigma / (N sqrt w); v = (C2 / sigma^2 - S0) / (N sqrt(2 w));
//                  optional signed square root; block sums of squares for the norm
//   l2             phi /= ||phi||_2 (skipped when the norm is 0)
// Every sum has a fixed order that depends only on the frame's own chunking, so a frame's
// result is bitwise independent of the other frames in a batch.
#include <math.h>

#include "fv_internal.h"

namespace fv {
namespace {

constexpr unsigned kFlagNoPower = 4u;
constexpr unsigned kFlagNoL2 = 8u;
constexpr int kThreads = 256;
constexpr int kL2PerThread = 4;

__global__ __launch_bounds__(kThreads) void group_reduce_kernel(
    const float* __restrict__ partials, const Group* __restrict__ groups, int n_items_single,
    int slot, double* __restrict__ gbuf) {
  const int g = blockIdx.y;
  int item0, nitems;
  if (groups != nullptr) {
    const Group gr = groups[g];
    item0 = gr.item0;
    nitems = gr.nitems;
  } else {
    item0 = g * kGroupItems;
    nitems = n_items_single - item0 < kGroupItems ? n_items_single - item0 : kGroupItems;
  }
  const int e = blockIdx.x * kThreads + threadIdx.x;
  if (e >= slot) return;
  const float* p = partials + (size_t)item0 * slot + e;
  double acc = 0.0;
  for (int i = 0; i < nitems; ++i) acc += (double)p[(size_t)i * slot];
  gbuf[(size_t)g * slot + e] = acc;
}

__global__ __launch_bounds__(kThreads) void assemble_kernel(
    const double* __restrict__ gbuf, const Frame* __restrict__ frames, Frame single, int K, int D,
    int DP, int Kp, const double* __restrict__ mu64, const double* __restrict__ isd64,
    const double* __restrict__ ivar64, const double* __restrict__ cu64,
    const double* __restrict__ cv64, unsigned flags, float* __restrict__ out,
    double* __restrict__ normpart) {
  __shared__ double red[kThreads];
  const int b = blockIdx.y;
  const Frame fr = frames != nullptr ? frames[b] : single;
  const int KD = K * D;
  const int idx = blockIdx.x * kThreads + threadIdx.x;
  const size_t slot = (size_t)(2 * DP + 1) * Kp;
  double ss = 0.0;
  if (idx < KD) {
    const int k = idx % K;  // consecutive threads read consecutive components
    const int d = idx / K;
    double S0 = 0.0, S1 = 0.0, S2 = 0.0;
    const double* p = gbuf + (size_t)fr.group0 * slot;
    for (int g = 0; g < fr.ngroups; ++g, p += slot) {
      S0 += p[(size_t)(2 * DP) * Kp + k];
      S1 += p[(size_t)d * Kp + k];
      S2 += p[(size_t)(DP + d) * Kp + k];
    }
    double u = 0.0, v = 0.0;
    if (fr.nrows > 0) {
      const int kd = k * D + d;
      const double m = mu64[kd];
      const double C1 = S1 - m * S0;                   // sum gamma (x - mu)
      const double C2 = S2 - m * (2.0 * S1 - m * S0);  // sum gamma (x - mu)^2
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
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) normpart[(size_t)b * gridDim.x + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kThreads) void l2_kernel(float* __restrict__ out,
                                                      const double* __restrict__ normpart,
                                                      int nblk, int len) {
  __shared__ double red[kThreads];
  const int b = blockIdx.y;
  // fixed-order sum of the frame's block sums: strided per thread, then a tree
  double ss = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kThreads) ss += normpart[(size_t)b * nblk + i];
  red[threadIdx.x] = ss;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double inv = red[0] > 0.0 ? 1.0 / sqrt(red[0]) : 0.0;
  if (inv == 0.0) return;
  float* o = out + (size_t)b * len;
  const int base = blockIdx.x * kThreads * kL2PerThread + threadIdx.x;
#pragma unroll
  for (int q = 0; q < kL2PerThread; ++q) {
    const int i = base + q * kThreads;
    if (i < len) o[i] = (float)((double)o[i] * inv);
  }
}

}  // namespace

int finalize_blocks(const Consts& c) { return (c.K * c.D + kThreads - 1) / kThreads; }

hipError_t launch_finalize(const Consts& c, const float* partials, const Frame* frames,
                           Frame single, int B, const Group* groups, int n_groups, unsigned flags,
                           float* out, double* gbuf, double* normpart, hipStream_t stream) {
  if (B <= 0) return hipSuccess;
  const int slot = (int)slot_floats(c);
  if (n_groups > 0) {
    hipLaunchKernelGGL(group_reduce_kernel, dim3((slot + kThreads - 1) / kThreads, n_groups),
                       dim3(kThreads), 0, stream, partials, groups, single.nitems, slot, gbuf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int nblk = finalize_blocks(c);
  hipLaunchKernelGGL(assemble_kernel, dim3(nblk, B), dim3(kThreads), 0, stream, gbuf, frames,
                     single, c.K, c.D, c.DP, c.Kp, c.mu64, c.isd64, c.ivar64, c.cu64, c.cv64,
                     flags, out, normpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!(flags & kFlagNoL2)) {
    const int len = 2 * c.K * c.D;
    const int per_blk = kThreads * kL2PerThread;
    hipLaunchKernelGGL(l2_kernel, dim3((len + per_blk - 1) / per_blk, B), dim3(kThreads), 0,
                       stream, out, normpart, nblk, len);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace fv
