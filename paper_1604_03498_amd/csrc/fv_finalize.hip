// Finalize kernels: the reduction of per-chunk partial statistics (the analogue of the
// paper's second Phase-2 kernel that sums the per-block U/V copies, Sec. 3.2, Algorithm 3),
// followed by the improved-FV assembly and normalisation (Fisher-information scaling,
// signed square root, L2).
//
//   reduce_assemble  one workgroup per (DB dimensions, KC components) of a frame, in two
//                    shapes: DB = 4 and KC = 256 (nine waves, one per S1/S2/S0 row) when the
//                    launch has enough such tiles, else DB = 1 and KC = 64 (three waves).
//                    Each thread reads one row's column of 4 components (wide) or 1 (narrow)
//                    from the frame's slots (all loads of a chunk group, two groups in the
//                    narrow shape, in flight together) and sums it in double:
//                    within a chunk group (at most 16 consecutive slots) in index order, then
//                    the group sums in order.  A batch's frames come longest first.  Then,
//                    one thread per component, C1 = S1 - mu S0; C2 = S2 - 2 mu S1 + mu^2 S0;
//                    u = C1 / sigma / (N sqrt w); v = (C2 / sigma^2 - S0) / (N sqrt(2 w));
//                    optional signed square root; per dimension, a wave's sum of squares over
//                    its 64 components.  Both shapes give the same bits.
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
// A thread's column of CPL consecutive components (CPL = 4: 16 bytes, or 1) in one slot.  The
// slot base address is uniform over the workgroup and the thread's byte offset into the slot
// is 32-bit: a buffer load with a scalar resource per slot and a 32-bit vector offset.
template <int CPL> struct Col;
template <> struct Col<4> {
  typedef unsigned int T __attribute__((ext_vector_type(4)));
  static __device__ inline T load(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
  }
  static __device__ inline float at(const T& v, int q) { return __uint_as_float(v[q]); }
};
template <> struct Col<1> {
  typedef unsigned int T;
  static __device__ inline T load(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0);
  }
  static __device__ inline float at(const T& v, int) { return __uint_as_float(v); }
};

template <int CPL>
__device__ inline typename Col<CPL>::T load_col(const float* __restrict__ partials, int idx,
                                                size_t slot, uint32_t lbytes) {
  const float* sp = partials + (size_t)idx * slot;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(sp), 0, (int)(slot * 4), 0x00020000);
  return Col<CPL>::load(rs, lbytes);
}

// Index-order double sums of one chunk group's n (1..16) slots, with U >= n loads issued
// together: unconditional, slot index clamped to the group, and values of slots past the group
// (or of a row that is not read, ok false) replaced by +0.0, which leaves the sum unchanged (it
// never holds -0.0).  The loads must not sit behind per-slot branches, which would serialise
// them.
template <int U, int CPL>
__device__ inline void sum_group(const float* __restrict__ partials, uint32_t lbytes, int i0,
                                 int n, size_t slot, bool ok, double (&a)[CPL]) {
  typename Col<CPL>::T v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) v[u] = load_col<CPL>(partials, i0 + min(u, n - 1), slot, lbytes);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const bool in = ok && u < n;
#pragma unroll
    for (int q = 0; q < CPL; ++q) a[q] += in ? (double)Col<CPL>::at(v[u], q) : 0.0;
  }
}

// Two consecutive chunk groups (na in 1..16 and nb in 0..16 slots) with all 32 loads issued
// together, then each group's index-order sum added to tot in order: the same sums as
// sum_group on each group in turn.  (Without a second group, nb = 0: its sum is +0.0 and adding
// it changes nothing; there is no branch, so that all loads stay ahead of the sums.)
template <int CPL>
__device__ inline void sum_two_groups(const float* __restrict__ partials, uint32_t lbytes,
                                      Group ga, Group gb, size_t slot, bool ok,
                                      double (&tot)[CPL]) {
  typename Col<CPL>::T v[2 * kGroupItems];
#pragma unroll
  for (int u = 0; u < 2 * kGroupItems; ++u) {
    const int idx = u < kGroupItems ? ga.item0 + min(u, ga.nitems - 1)
                                    : (gb.nitems > 0 ? gb.item0 + min(u - kGroupItems, gb.nitems - 1)
                                                     : ga.item0);
    v[u] = load_col<CPL>(partials, idx, slot, lbytes);
  }
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int n = half == 0 ? ga.nitems : gb.nitems;
    double a[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) a[q] = 0.0;
#pragma unroll
    for (int u = 0; u < kGroupItems; ++u) {
      const bool in = ok && u < n;
#pragma unroll
      for (int q = 0; q < CPL; ++q)
        a[q] += in ? (double)Col<CPL>::at(v[half * kGroupItems + u], q) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < CPL; ++q) tot[q] += a[q];
  }
}

// Waves of a reduce_assemble workgroup: 2 DB + 1 rows of KC / CPL columns, 64 columns a wave.
constexpr int red_waves(int DB, int KC, int CPL) {
  return (2 * DB + 1 + 64 / (KC / CPL) - 1) / (64 / (KC / CPL));
}

template <int DB, int KC, int CPL>
__global__ __launch_bounds__(64 * red_waves(DB, KC, CPL))
__attribute__((amdgpu_waves_per_eu(DB == 1 ? 1 : 5))) void reduce_assemble_kernel(
    const float* __restrict__ partials, const Frame* __restrict__ frames, Frame single,
    int K, int D, int DP, int Kp, int nkc, int nkb,
    const double* __restrict__ mu64, const double* __restrict__ isd64,
    const double* __restrict__ ivar64, const double* __restrict__ cu64,
    const double* __restrict__ cv64, unsigned flags, float* __restrict__ out,
    double* __restrict__ normpart, const Counts* __restrict__ cnt) {
  constexpr int R = 2 * DB + 1;     // rows: S1[d0 + i], S2[d0 + i], S0
  constexpr int NC = KC / CPL;      // columns per row
  __shared__ double sv[R][KC];
  if (cnt && (int)blockIdx.y >= cnt->B) return;  // past the batch (grid sized to a capacity)
  const Frame fr = frames != nullptr ? frames[blockIdx.y] : single;
  const int b = frames != nullptr ? fr.index : 0;  // the frame's output row and norm parts
  const int kc = blockIdx.x % nkc;
  const int d0 = (blockIdx.x / nkc) * DB;
  const int t = threadIdx.x;
  const int col = t % NC;
  const int r = t / NC;             // this thread's row
  const int i = r < DB ? r : r - DB;
  const int kcol = kc * KC + CPL * col;
  const bool rok = r < R && kcol < Kp && (r == 2 * DB || d0 + i < D);
  const int prow = r == 2 * DB ? 2 * DP : (r < DB ? d0 + r : DP + d0 + i);
  const uint32_t lbytes = rok ? (uint32_t)(prow * Kp + kcol) * 4u : 0u;  // bytes into a slot
  const size_t slot = (size_t)(2 * DP + 1) * Kp;

  // a chunk group's (first slot, slot count)
  auto group_at = [&](int g) -> Group {
    const int i0 = fr.item0 + g * kGroupItems;
    return Group{i0, min(kGroupItems, fr.item0 + fr.nitems - i0)};
  };
  // the narrow shape (single frames, latency-bound) also loads its constants up front
  const int kq = kc * KC + t;
  const bool pre = DB == 1 && t < KC && kq < K && d0 < D;
  double mu_p = 0.0, isd_p = 0.0, ivar_p = 0.0, cu_p = 0.0, cv_p = 0.0;
  if (pre) {
    const int kd = kq * D + d0;
    mu_p = mu64[kd];
    isd_p = isd64[kd];
    ivar_p = ivar64[kd];
    cu_p = cu64[kq];
    cv_p = cv64[kq];
  }

  double tot[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) tot[q] = 0.0;
  if constexpr (DB == 1) {
    // the narrow shape: two groups' slots in flight at a time (registers are plentiful at one
    // wave per workgroup)
    for (int g = 0; g < fr.ngroups; g += 2) {
      Group ga = group_at(g);
      Group gb = g + 1 < fr.ngroups ? group_at(g + 1) : Group{0, 0};
      ga.item0 = __builtin_amdgcn_readfirstlane(ga.item0);
      ga.nitems = __builtin_amdgcn_readfirstlane(ga.nitems);
      gb.item0 = __builtin_amdgcn_readfirstlane(gb.item0);
      gb.nitems = __builtin_amdgcn_readfirstlane(gb.nitems);
      if (ga.nitems > 0) sum_two_groups<CPL>(partials, lbytes, ga, gb, slot, rok, tot);
    }
  } else {
    Group cur = fr.ngroups > 0 ? group_at(0) : Group{0, 0};
    for (int g = 0; g < fr.ngroups; ++g) {
      const Group nxt = g + 1 < fr.ngroups ? group_at(g + 1) : cur;
      // uniform over the workgroup: scalar registers, so the slot bases are scalar too
      const int i0 = __builtin_amdgcn_readfirstlane(cur.item0);
      const int n = __builtin_amdgcn_readfirstlane(cur.nitems);
      double a[CPL];
#pragma unroll
      for (int q = 0; q < CPL; ++q) a[q] = 0.0;
      if (n > 8)
        sum_group<16, CPL>(partials, lbytes, i0, n, slot, rok, a);
      else if (n > 4)
        sum_group<8, CPL>(partials, lbytes, i0, n, slot, rok, a);
      else if (n > 0)
        sum_group<4, CPL>(partials, lbytes, i0, n, slot, rok, a);
#pragma unroll
      for (int q = 0; q < CPL; ++q) tot[q] += a[q];
      cur = nxt;
    }
  }
  if (r < R)
#pragma unroll
    for (int q = 0; q < CPL; ++q) sv[r][CPL * col + q] = tot[q];
  __syncthreads();

  // one thread per component (the first KC / 64 waves): u and v of the DB dimensions
  if (t >= KC) return;
  const int k = kc * KC + t;
  const bool kok = k < K;
  const int KD = K * D;
  float* o = out + (size_t)b * 2 * KD + (size_t)(kok ? k : 0) * D + d0;
  const double S0 = sv[2 * DB][t];
  const double invN = fr.nrows > 0 ? 1.0 / (double)fr.nrows : 0.0;
  const double cu = DB == 1 ? cu_p : (kok ? cu64[k] : 0.0);
  const double cv = DB == 1 ? cv_p : (kok ? cv64[k] : 0.0);
  float uo[DB], vo[DB];
  double ss[DB];
#pragma unroll
  for (int j = 0; j < DB; ++j) {
    double u = 0.0, v = 0.0;
    if (kok && d0 + j < D && fr.nrows > 0) {
      const int kd = k * D + d0 + j;
      const double mu = DB == 1 ? mu_p : mu64[kd];
      const double isd = DB == 1 ? isd_p : isd64[kd];
      const double ivar = DB == 1 ? ivar_p : ivar64[kd];
      const double S1 = sv[j][t], S2 = sv[DB + j][t];
      const double C1 = S1 - mu * S0;                    // sum gamma (x - mu)
      const double C2 = S2 - mu * (2.0 * S1 - mu * S0);  // sum gamma (x - mu)^2
      u = C1 * isd * cu * invN;
      v = (C2 * ivar - S0) * cv * invN;
      if (!(flags & kFlagNoPower)) {
        u = (u > 0.0) ? sqrt(u) : ((u < 0.0) ? -sqrt(-u) : 0.0);
        v = (v > 0.0) ? sqrt(v) : ((v < 0.0) ? -sqrt(-v) : 0.0);
      }
    }
    uo[j] = (float)u;
    vo[j] = (float)v;
    ss[j] = u * u + v * v;
  }
  if (kok) {
    if (DB == 4 && D % 4 == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
      *reinterpret_cast<float4*>(o) = make_float4(uo[0], uo[1], uo[2], uo[3]);
      *reinterpret_cast<float4*>(o + KD) = make_float4(vo[0], vo[1], vo[2], vo[3]);
    } else {
#pragma unroll
      for (int j = 0; j < DB; ++j)
        if (d0 + j < D) {
          o[j] = uo[j];
          o[KD + j] = vo[j];
        }
    }
  }
  // per dimension, a fixed-order butterfly over the wave's 64 components (the same in both
  // workgroup shapes); lane 0 writes the (dimension, 64-component block) partial of the norm
  const int kb = (kc * KC + (t & ~63)) / 64;
#pragma unroll
  for (int j = 0; j < DB; ++j) {
    double x = ss[j];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) x += __shfl_xor(x, m);
    if ((t & 63) == 0 && kb < nkb && d0 + j < D)
      normpart[((size_t)b * D + d0 + j) * nkb + kb] = x;
  }
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

int finalize_blocks(const Consts& c) { return c.D * ((c.K + 63) / 64); }

hipError_t launch_finalize(const Consts& c, const float* partials, const Frame* frames,
                           Frame single, int B, unsigned flags, float* out, double* normpart,
                           hipStream_t stream) {
  if (B <= 0) return hipSuccess;
  const int nblk = finalize_blocks(c);
  const int nkb = (c.K + 63) / 64;
  // the wide shape when its tiles alone give at least two workgroups per CU, else the narrow one
  const int nkc_w = (c.Kp + 255) / 256, ndb_w = (c.D + 3) / 4;
  if ((int64_t)B * nkc_w * ndb_w >= 512) {
    hipLaunchKernelGGL((reduce_assemble_kernel<4, 256, 4>), dim3(nkc_w * ndb_w, B),
                       dim3(64 * red_waves(4, 256, 4)), 0, stream, partials, frames, single,
                       c.K, c.D, c.DP, c.Kp, nkc_w, nkb, c.mu64, c.isd64, c.ivar64, c.cu64,
                       c.cv64, flags, out, normpart, c.cnt);
  } else {
    const int nkc_n = (c.Kp + 63) / 64;
    hipLaunchKernelGGL((reduce_assemble_kernel<1, 64, 1>), dim3(nkc_n * c.D, B),
                       dim3(64 * red_waves(1, 64, 1)), 0, stream, partials, frames, single,
                       c.K, c.D, c.DP, c.Kp, nkc_n, nkb, c.mu64, c.isd64, c.ivar64, c.cu64,
                       c.cv64, flags, out, normpart, c.cnt);
  }
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
