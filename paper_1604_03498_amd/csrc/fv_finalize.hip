// Finalize kernels: the reduction of per-chunk partial statistics (the analogue of the
// paper's second Phase-2 kernel that sums the per-block U/V copies, Sec. 3.2, Algorithm 3),
// followed by the improved-FV assembly and normalisation (Fisher-information scaling,
// signed square root, L2).
//
//   reduce_assemble  one workgroup per (64-component block, dimension d) of a frame; its three
//                    waves sum the S1[d], S2[d] and S0 rows of the frame's slots in double:
//                    within a chunk group (at most 16 consecutive slots) in index order, then
//                    the group sums in order.  Then C1 = S1 - mu S0; C2 = S2 - 2 mu S1 +
//                    mu^2 S0; u = C1 / sigma / (N sqrt w); v = (C2 / sigma^2 - S0) /
//                    (N sqrt(2 w)); optional signed square root; the block's sum of squares
//   l2               phi /= ||phi||_2 (skipped when the norm is 0)
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
constexpr int kCompBlock = 64;   // components per reduce_assemble workgroup (one per lane)
constexpr int kRedThreads = 192; // three waves: S1 row, S2 row, S0 row

// Loads of one group's slots for one (row, component), unconditional so that all of them are
// in flight together: slot indices are clamped to [0, nclamp) (nclamp >= 1 valid slots from p)
// and values past n (or for a padded component) are replaced by +0.0, which leaves the
// index-order double sum unchanged (the sum never holds -0.0).
__device__ inline void load_group(const float* __restrict__ p, int nclamp, int n, size_t slot,
                                  bool ok, float (&v)[kGroupItems]) {
#pragma unroll
  for (int i = 0; i < kGroupItems; ++i) v[i] = p[(size_t)min(i, nclamp - 1) * slot];
#pragma unroll
  for (int i = 0; i < kGroupItems; ++i) v[i] = (ok && i < n) ? v[i] : 0.f;
}

__device__ inline double sum_group(const float (&v)[kGroupItems]) {
  double a = 0.0;
#pragma unroll
  for (int i = 0; i < kGroupItems; ++i) a += (double)v[i];
  return a;
}

__global__ __launch_bounds__(kRedThreads) void reduce_assemble_kernel(
    const float* __restrict__ partials, const Frame* __restrict__ frames, Frame single,
    const Group* __restrict__ groups, int K, int D, int DP, int Kp, int nkb,
    const double* __restrict__ mu64, const double* __restrict__ isd64,
    const double* __restrict__ ivar64, const double* __restrict__ cu64,
    const double* __restrict__ cv64, unsigned flags, float* __restrict__ out,
    double* __restrict__ normpart, const Counts* __restrict__ cnt) {
  __shared__ double sv[3][kCompBlock];
  const int b = blockIdx.y;
  if (cnt && b >= cnt->B) return;  // a frame slot past the batch (grid sized to a capacity)
  const Frame fr = frames != nullptr ? frames[b] : single;
  const int kb = blockIdx.x % nkb;
  const int d = blockIdx.x / nkb;
  const int wv = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int k = kb * kCompBlock + lane;
  const bool kok = k < K;
  const size_t slot = (size_t)(2 * DP + 1) * Kp;
  const int row = wv == 0 ? d : (wv == 1 ? DP + d : 2 * DP);
  const float* base = partials + (size_t)row * Kp + (kok ? k : 0);
  // the finalize constants of (k, d), loaded up front so that their latency overlaps the sums
  const int kd = (kok ? k : 0) * D + d;
  double mu = 0.0, isd = 0.0, ivar = 0.0, cu = 0.0, cv = 0.0;
  if (wv == 0) {
    mu = mu64[kd];
    isd = isd64[kd];
    ivar = ivar64[kd];
    cu = cu64[kok ? k : 0];
    cv = cv64[kok ? k : 0];
  }

  double tot = 0.0;
  for (int g = 0; g < fr.ngroups; g += 2) {
    int i0a, na, i0b = 0, nb = 0;
    if (groups != nullptr) {
      const Group ga = groups[fr.group0 + g];
      i0a = ga.item0;
      na = ga.nitems;
      if (g + 1 < fr.ngroups) {
        const Group gb = groups[fr.group0 + g + 1];
        i0b = gb.item0;
        nb = gb.nitems;
      }
    } else {
      i0a = fr.item0 + g * kGroupItems;
      na = min(kGroupItems, fr.item0 + fr.nitems - i0a);
      if (g + 1 < fr.ngroups) {
        i0b = i0a + kGroupItems;
        nb = min(kGroupItems, fr.item0 + fr.nitems - i0b);
      }
    }
    float va[kGroupItems], vb[kGroupItems];
    load_group(base + (size_t)i0a * slot, na, na, slot, kok, va);
    if (nb > 0)
      load_group(base + (size_t)i0b * slot, nb, nb, slot, kok, vb);
    else
      load_group(base + (size_t)i0a * slot, na, 0, slot, kok, vb);
    tot += sum_group(va);
    if (g + 1 < fr.ngroups) tot += sum_group(vb);
  }
  sv[wv][lane] = tot;
  __syncthreads();
  if (wv != 0) return;

  double ss = 0.0;
  if (kok) {
    const double S0 = sv[2][lane], S1 = sv[0][lane], S2 = sv[1][lane];
    double u = 0.0, v = 0.0;
    if (fr.nrows > 0) {
      const double C1 = S1 - mu * S0;                    // sum gamma (x - mu)
      const double C2 = S2 - mu * (2.0 * S1 - mu * S0);  // sum gamma (x - mu)^2
      const double invN = 1.0 / (double)fr.nrows;
      u = C1 * isd * cu * invN;
      v = (C2 * ivar - S0) * cv * invN;
      if (!(flags & kFlagNoPower)) {
        u = (u > 0.0) ? sqrt(u) : ((u < 0.0) ? -sqrt(-u) : 0.0);
        v = (v > 0.0) ? sqrt(v) : ((v < 0.0) ? -sqrt(-v) : 0.0);
      }
    }
    const int KD = K * D;
    float* o = out + (size_t)b * 2 * KD;
    o[k * D + d] = (float)u;
    o[KD + k * D + d] = (float)v;
    ss = u * u + v * v;
  }
  // fixed-order butterfly over the wave
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) ss += __shfl_xor(ss, m);
  if (lane == 0) normpart[(size_t)b * gridDim.x + blockIdx.x] = ss;
}

__global__ __launch_bounds__(kThreads) void l2_kernel(float* __restrict__ out,
                                                      const double* __restrict__ normpart,
                                                      int nblk, int len,
                                                      const Counts* __restrict__ cnt) {
  __shared__ double red[kThreads];
  const int b = blockIdx.y;
  if (cnt && b >= cnt->B) return;
  // this thread's output values are loaded first, so their latency overlaps the norm's sum
  float* o = out + (size_t)b * len;
  const int base = blockIdx.x * kThreads * kL2PerThread + threadIdx.x;
  float v[kL2PerThread];
#pragma unroll
  for (int q = 0; q < kL2PerThread; ++q) {
    const int i = base + q * kThreads;
    v[q] = i < len ? o[i] : 0.f;
  }
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
#pragma unroll
  for (int q = 0; q < kL2PerThread; ++q) {
    const int i = base + q * kThreads;
    if (i < len) o[i] = (float)((double)v[q] * inv);
  }
}

}  // namespace

int finalize_blocks(const Consts& c) { return ((c.K + kCompBlock - 1) / kCompBlock) * c.D; }

hipError_t launch_finalize(const Consts& c, const float* partials, const Frame* frames,
                           Frame single, int B, const Group* groups, unsigned flags, float* out,
                           double* normpart, hipStream_t stream) {
  if (B <= 0) return hipSuccess;
  const int nblk = finalize_blocks(c);
  const int nkb = (c.K + kCompBlock - 1) / kCompBlock;
  hipLaunchKernelGGL(reduce_assemble_kernel, dim3(nblk, B), dim3(kRedThreads), 0, stream, partials,
                     frames, single, groups, c.K, c.D, c.DP, c.Kp, nkb, c.mu64, c.isd64, c.ivar64,
                     c.cu64, c.cv64, flags, out, normpart, c.cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!(flags & kFlagNoL2)) {
    const int len = 2 * c.K * c.D;
    const int per_blk = kThreads * kL2PerThread;
    hipLaunchKernelGGL(l2_kernel, dim3((len + per_blk - 1) / per_blk, B), dim3(kThreads), 0,
                       stream, out, normpart, nblk, len, c.cnt);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace fv
