// Dense-SIFT front end: the flat-window descriptor extraction that feeds the encoder (Sec. 3.1:
// per scale of the image, every pixel's gradient falls into 8 orientation bins, a triangular
// convolution follows, and each descriptor takes the 8 values of 4 x 4 spatial bins, sampled
// with a stride; Sec. 3.2: the triangular filter is applied once per image dimension, as a
// windowed sum per output point instead of the four running scans, and the second
// convolution is computed only where a descriptor samples it; Sec. 4: stride 4, scales from
// sqrt 2 down to 1/8).
//
// The paper's design (one thread block per image column, the column buffered in shared
// memory, every pixel through the first convolution) targets a scan-shaped CPU code.  Here
// both convolutions are pruned to the points the descriptors read: the filtered maps are
// needed only at rows y0 + jB and columns x0 + iB (bin size B, i, j in 0..3), so with the
// stride a multiple of B one row in B and one column in B.
//
//   dsift_filter_kernel  one workgroup of 256 threads per (needed row r, tile of columns) of
//                        one scale of one image: the scaled image's band of rows r - B ..
//                        r + B over the tile's columns (plus halos) is resampled (bilinear)
//                        from the source image into LDS; each thread then takes one column,
//                        computes the gradient at the 2B - 1 rows the triangular window
//                        covers, splits its magnitude between the two nearest of 8
//                        orientation bins and accumulates the window-weighted sums (the
//                        first convolution, along y, at row r only) into LDS; finally the
//                        second convolution (along x) is evaluated at the tile's needed
//                        columns and written as [row][column][orientation] (32 bytes per
//                        sample point).
//   dsift_desc_kernel    32 lanes per descriptor: lane l reads the 4 orientation values
//                        (16 bytes) of half a spatial bin, the 128 values are L2-normalised,
//                        clamped at 0.2 and normalised again (SIFT's normalisation), and the
//                        row of 130 floats (128 values, then the centre's normalised x and y)
//                        is written with 8-byte stores.
//
// All scales of all images run in the same two launches: a scale table maps a workgroup
// (first kernel) or a descriptor (second kernel) to its scale.
#include <math.h>

#include "fv_internal.h"

namespace fv {
namespace {

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

constexpr int kFiltThreads = 256;
constexpr int kBandCols = kFiltThreads + 2;  // y-convolution columns plus the gradient halo
constexpr int kDescThreads = 256;             // 8 descriptors of 32 lanes
constexpr float kTwoPi = 6.28318530717958647692f;

__device__ __forceinline__ int find_scale_blk(const DsiftScale* __restrict__ sc, int nsc, int b) {
  int si = nsc - 1;
  while (si > 0 && b < sc[si].blk0) --si;
  return si;
}

__device__ __forceinline__ int find_scale_desc(const DsiftScale* __restrict__ sc, int nsc,
                                               int64_t g) {
  int si = nsc - 1;
  while (si > 0 && g < sc[si].desc0) --si;
  return si;
}

// Bilinear sample of the source image at the scaled image's pixel (y, x), the sample point
// (y + 1/2) / s - 1/2 (and likewise for x) clamped to the image; coordinates and weights in
// double, the interpolation in float.
__device__ __forceinline__ float resample(const float* __restrict__ img, int H, int W, double s,
                                          int y, int x) {
  if (s == 1.0) return img[(size_t)y * W + x];
  double v = ((double)y + 0.5) / s - 0.5;
  double u = ((double)x + 0.5) / s - 0.5;
  v = fmin(fmax(v, 0.0), (double)(H - 1));
  u = fmin(fmax(u, 0.0), (double)(W - 1));
  const int y0 = (int)floor(v), x0 = (int)floor(u);
  const int y1 = min(y0 + 1, H - 1), x1 = min(x0 + 1, W - 1);
  const float fy = (float)(v - (double)y0), fx = (float)(u - (double)x0);
  const float* r0 = img + (size_t)y0 * W;
  const float* r1 = img + (size_t)y1 * W;
  const float top = r0[x0] * (1.f - fx) + r0[x1] * fx;
  const float bot = r1[x0] * (1.f - fx) + r1[x1] * fx;
  return top * (1.f - fy) + bot * fy;
}

__global__ __launch_bounds__(kFiltThreads) void dsift_filter_kernel(
    const float* __restrict__ images, int H, int W, const DsiftScale* __restrict__ sc, int nsc,
    const int* __restrict__ lists, int B, float* __restrict__ fxy, int64_t fxy_stride) {
  extern __shared__ float smem[];
  const int BR = 2 * B + 1;  // band rows r - B .. r + B
  float* band = smem;                     // [BR][kBandCols]
  float* fy = smem + BR * kBandCols;      // [8][kFiltThreads]

  const int tid = threadIdx.x;
  const int si = find_scale_blk(sc, nsc, blockIdx.x);
  const DsiftScale S = sc[si];
  const int local = blockIdx.x - S.blk0;
  const int ri = local / S.ntx;
  const int xt = local - ri * S.ntx;
  const int* rows = lists + S.row0;
  const int* cols = lists + S.col0;
  const int r = rows[ri];
  const int TW = kFiltThreads - 2 * (B - 1);  // output columns per tile
  const int xb = xt * TW;                      // first output column of the tile
  const int xs0 = xb - (B - 1);                // column of thread 0 in the y-convolution
  const int Hs = S.Hs, Ws = S.Ws;
  const float* img = images + (size_t)blockIdx.y * H * W;

  // the band of the scaled image: rows r - B .. r + B, columns xs0 - 1 .. xs0 + 256
  for (int i = tid; i < BR * kBandCols; i += kFiltThreads) {
    const int br = i / kBandCols;
    const int bc = i - br * kBandCols;
    const int y = r - B + br;
    const int x = xs0 - 1 + bc;
    band[i] = (y >= 0 && y < Hs && x >= 0 && x < Ws) ? resample(img, H, W, S.s, y, x) : 0.f;
  }
  __syncthreads();

  // first convolution (along y) at row r, column x = xs0 + tid; a column outside the image is
  // zero (the convolution's zero padding)
  {
    const int x = xs0 + tid;
    float acc[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) acc[o] = 0.f;
    if (x >= 0 && x < Ws) {
      const int bc = tid + 1;  // band column of x
      const float invB2 = 1.f / (float)(B * B);
      for (int d = -(B - 1); d <= B - 1; ++d) {
        const int y = r + d;
        if (y < 0 || y >= Hs) continue;
        const float* row = band + (d + B) * kBandCols;
        float gx, gy;
        if (Ws == 1) gx = 0.f;
        else if (x == 0) gx = row[bc + 1] - row[bc];
        else if (x == Ws - 1) gx = row[bc] - row[bc - 1];
        else gx = 0.5f * (row[bc + 1] - row[bc - 1]);
        if (Hs == 1) gy = 0.f;
        else if (y == 0) gy = row[kBandCols + bc] - row[bc];
        else if (y == Hs - 1) gy = row[bc] - row[bc - kBandCols];
        else gy = 0.5f * (row[kBandCols + bc] - row[bc - kBandCols]);
        const float m = sqrtf(gx * gx + gy * gy);
        float th = atan2f(gy, gx);
        if (th < 0.f) th += kTwoPi;
        float t = th * (8.f / kTwoPi);
        if (t >= 8.f) t -= 8.f;
        const float fl = floorf(t);
        const float f = t - fl;
        const int b0 = ((int)fl) & 7;
        const int b1 = (b0 + 1) & 7;
        const float w = (float)(B - (d < 0 ? -d : d)) * invB2;  // triangular window weight
        const float m0 = w * ((1.f - f) * m);
        const float m1 = w * (f * m);
#pragma unroll
        for (int o = 0; o < 8; ++o) acc[o] += (o == b0 ? m0 : 0.f) + (o == b1 ? m1 : 0.f);
      }
    }
#pragma unroll
    for (int o = 0; o < 8; ++o) fy[o * kFiltThreads + tid] = acc[o];
  }
  __syncthreads();

  // second convolution (along x) at the needed columns of [xb, xb + TW): the first needed
  // column index at or after xb, by binary search in the sorted list
  int lo = 0, hi = S.nC;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (cols[mid] < xb) lo = mid + 1;
    else hi = mid;
  }
  int cend = lo;
  {
    int l2 = lo, h2 = S.nC;
    while (l2 < h2) {
      const int mid = (l2 + h2) >> 1;
      if (cols[mid] < xb + TW) l2 = mid + 1;
      else h2 = mid;
    }
    cend = l2;
  }
  const int npairs = (cend - lo) * 8;
  const float invB2 = 1.f / (float)(B * B);
  float* dst = fxy + (int64_t)blockIdx.y * fxy_stride + S.fxy0 + (int64_t)ri * S.nC * 8;
  for (int p = tid; p < npairs; p += kFiltThreads) {
    const int ci = lo + (p >> 3);
    const int o = p & 7;
    const int c = cols[ci];
    const float* src = fy + o * kFiltThreads + (c - xs0);
    float v = 0.f;
    for (int d = -(B - 1); d <= B - 1; ++d)
      v += (float)(B - (d < 0 ? -d : d)) * invB2 * src[d];
    dst[(int64_t)ci * 8 + o] = v;
  }
}

__global__ __launch_bounds__(kDescThreads) void dsift_desc_kernel(
    const DsiftScale* __restrict__ sc, int nsc, const int* __restrict__ lists, int B, int S_,
    const float* __restrict__ fxy, int64_t fxy_stride, int64_t ndesc, float* __restrict__ out) {
  const int tid = threadIdx.x;
  const int lane = tid & 31;  // lane within the descriptor's 32
  const int64_t g = (int64_t)blockIdx.x * (kDescThreads / 32) + (tid >> 5);
  const bool live = g < ndesc;
  const int64_t gq = live ? g : ndesc - 1;  // rows past the end compute a copy, store nothing
  const int si = find_scale_desc(sc, nsc, gq);
  const DsiftScale S = sc[si];
  const int64_t local = gq - S.desc0;
  const int by = (int)(local / S.nx);
  const int ax = (int)(local - (int64_t)by * S.nx);
  const int bin = lane >> 1;  // spatial bin 4 j + i
  const int half = lane & 1;  // orientations 0..3 or 4..7
  const int ci = lists[S.cidx0 + ax * 4 + (bin & 3)];
  const int ri = lists[S.ridx0 + by * 4 + (bin >> 2)];
  const float* src = fxy + (int64_t)blockIdx.y * fxy_stride + S.fxy0 +
                     ((int64_t)ri * S.nC + ci) * 8 + half * 4;
  f32x4_t v = *reinterpret_cast<const f32x4_t*>(src);

  // SIFT normalisation: L2, clamp at 0.2, L2 (a zero vector stays zero); the sums over the
  // descriptor's 32 lanes in a fixed butterfly order
  float ss = v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3];
#pragma unroll
  for (int m = 16; m > 0; m >>= 1) ss += __shfl_xor(ss, m, 32);
  if (ss > 0.f) {
    const float n = sqrtf(ss);
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = fminf(v[e] / n, 0.2f);
    float s2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3];
#pragma unroll
    for (int m = 16; m > 0; m >>= 1) s2 += __shfl_xor(s2, m, 32);
    if (s2 > 0.f) {
      const float n2 = sqrtf(s2);
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = v[e] / n2;
    }
  }
  if (!live) return;
  float* row = out + ((int64_t)blockIdx.y * ndesc + g) * kDsiftDim;
  // value index (4 j + i) * 8 + o = 4 * lane + e
  *reinterpret_cast<f32x2_t*>(row + 4 * lane) = f32x2_t{v[0], v[1]};
  *reinterpret_cast<f32x2_t*>(row + 4 * lane + 2) = f32x2_t{v[2], v[3]};
  if (lane == 0) {
    // the descriptor's centre, at its pixel's centre, over the scaled image's size, minus 1/2
    const double cx = ((double)ax * S_ + 1.5 * B + 0.5) / (double)S.Ws - 0.5;
    const double cy = ((double)by * S_ + 1.5 * B + 0.5) / (double)S.Hs - 0.5;
    *reinterpret_cast<f32x2_t*>(row + 128) = f32x2_t{(float)cx, (float)cy};
  }
}

}  // namespace

size_t dsift_filter_lds_bytes(int B) {
  return (size_t)((2 * B + 1) * kBandCols + 8 * kFiltThreads) * sizeof(float);
}

hipError_t launch_dsift(const DsiftPlan& p, const DsiftScale* dscales, const int* dlists,
                        const float* images, int n_images, float* fxy, float* rows,
                        hipStream_t stream) {
  if (n_images <= 0 || p.ndesc == 0) return hipSuccess;
  hipLaunchKernelGGL(dsift_filter_kernel, dim3((unsigned)p.nblk, (unsigned)n_images),
                     dim3(kFiltThreads), dsift_filter_lds_bytes(p.B), stream, images, p.H, p.W,
                     dscales, p.nsc, dlists, p.B, fxy, p.fxy_floats);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t per = kDescThreads / 32;
  hipLaunchKernelGGL(dsift_desc_kernel, dim3((unsigned)((p.ndesc + per - 1) / per),
                                             (unsigned)n_images),
                     dim3(kDescThreads), 0, stream, dscales, p.nsc, dlists, p.B, p.S, fxy,
                     p.fxy_floats, p.ndesc, rows);
  return hipGetLastError();
}

int dsift_filter_tile_cols(int B) { return kFiltThreads - 2 * (B - 1); }

}  // namespace fv
