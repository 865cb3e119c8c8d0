// 16-bit operand forms of the two contractions (bf16 or fp16 on v_mfma_f32_32x32x16_*,
// FP32 accumulation).
//
// Split form: every FP32 operand v is carried as hi = rne16(v), lo = rne16(v - hi) (v - hi is
// exact in FP32) and a product is formed from three MFMAs, hi*hi + hi*lo + lo*hi; the lo*lo
// term is dropped.  Plain form: hi only (one MFMA), kept as an accuracy control.
//
// 32x32x16 operand layout: lane (h, j) supplies 8 consecutive reduction indices 8h..8h+7 of
// row j (A operand) or column j (B operand); C/D layout is the FP32 one.
//
// LDS tile of 32 rows, written once per tile by the loader:
//   RM_hi / RM_lo  [32][2*DP + 8]   row-major [x, x^2]   -> E-step A operand (16 B per lane)
//   XT_hi / XT_lo  [2*DP][40]       transposed, rows permuted by pos() -> statistics A operand
// pos(row) swaps bits 2 and 3 of the row index.  The statistics k-step q of an MFMA consumes
// the E-step result registers 8q..8q+7 of a lane in half h, i.e. rows
// 16q + 8*(e>>2) + 4h + (e&3) for e = 0..7; pos() maps exactly these to 16q + 8h + e, so the
// A operand is one contiguous 16-byte read.
#pragma once

#include "fv_device.h"

namespace fv {
namespace dev {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <class T>
struct P16;

template <>
struct P16<__bf16> {
  typedef bf16x8 v8;
  __device__ __forceinline__ static f32x16 mfma(v8 a, v8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct P16<_Float16> {
  typedef f16x8 v8;
  __device__ __forceinline__ static f32x16 mfma(v8 a, v8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

template <class T>
__device__ __forceinline__ uint16_t bits16(T v) {
  return __builtin_bit_cast(uint16_t, v);
}

// hi/lo split of an FP32 value (round to nearest even in both conversions).  Where v comes
// from a product, instruction selection may fuse the product into v - hi (a mixed-precision
// FMA forms lo from the unrounded product, slightly more accurate); callers that must give
// the same bits as another kernel make v opaque first (an empty asm on it).
template <class T>
__device__ __forceinline__ void split16(float v, T& hi, T& lo) {
  hi = (T)v;
  lo = (T)(v - (float)hi);
}

// hi/lo split of two FP32 values at once, with the same results as split16 on each: one
// packed conversion gives both hi, each is widened back exactly, one packed conversion gives
// both lo.  hi and lo hold the pair as two 16-bit halves (v0 in the low half).
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <class T>
struct Pack16;
template <>
struct Pack16<__bf16> {
  typedef __bf16 v2 __attribute__((ext_vector_type(2)));
  __device__ __forceinline__ static float widen_lo(uint32_t p) { return __uint_as_float(p << 16); }
  __device__ __forceinline__ static float widen_hi(uint32_t p) { return __uint_as_float(p & 0xffff0000u); }
};
template <>
struct Pack16<_Float16> {
  typedef _Float16 v2 __attribute__((ext_vector_type(2)));
  __device__ __forceinline__ static float widen_lo(uint32_t p) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(p & 0xffffu));
  }
  __device__ __forceinline__ static float widen_hi(uint32_t p) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(p >> 16));
  }
};
// The caller makes v0 and v1 opaque where they come from a product (as split16 does for its
// input), so that their rounded values are split.
template <class T>
__device__ __forceinline__ void split16x2(float v0, float v1, uint32_t& hi, uint32_t& lo) {
  using P = Pack16<T>;
  hi = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){v0, v1}, typename P::v2));
  const float d0 = v0 - P::widen_lo(hi), d1 = v1 - P::widen_hi(hi);
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){d0, d1}, typename P::v2));
}

__device__ __forceinline__ constexpr int tpos(int row) {
  return (row & ~12) | ((row & 4) << 1) | ((row & 8) >> 1);
}

template <int DP>
struct Tile16 {
  static constexpr int RS = 2 * DP + 8;   // row-major stride (16-bit elements)
  static constexpr int TS = 40;           // transposed stride (16-bit elements)
  static constexpr int kRM = kTile * RS;  // elements per row-major array
  static constexpr int kXT = 2 * DP * TS;  // elements per transposed array
  static constexpr int kElems = 2 * kRM + 2 * kXT;
  static constexpr int kBlocks = (kTile / 4) * (DP / 4);  // 4x4 (row, feature) blocks of x
  uint16_t* rm_hi;
  uint16_t* rm_lo;
  uint16_t* xt_hi;
  uint16_t* xt_lo;
  __device__ __forceinline__ explicit Tile16(uint16_t* base)
      : rm_hi(base), rm_lo(base + kRM), xt_hi(base + 2 * kRM), xt_lo(base + 2 * kRM + kXT) {}
};

// Loader: NT threads; each 4x4 block of x (4 rows, 4 features) is fetched as four float4 into
// registers (fetch), then converted and written to the four LDS arrays (store) together with
// the matching block of x^2.
template <int DP, int NT>
struct TileIO16 {
  using TL = Tile16<DP>;
  static constexpr int kPer = (TL::kBlocks + NT - 1) / NT;

  __device__ __forceinline__ static void fetch(f32x4 (&pre)[kPer][4], const float* __restrict__ X,
                                               int D, bool vec_ok, int64_t row0, int valid,
                                               int tid) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int blk = tid + q * NT;
      const int rb = blk % (kTile / 4);  // consecutive threads: consecutive row blocks
      const int c4 = (blk / (kTile / 4)) * 4;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        f32x4 v = {0.f, 0.f, 0.f, 0.f};
        const int row = 4 * rb + rr;
        if (blk < TL::kBlocks && row < valid) {
          const float* src = X + (row0 + row) * (int64_t)D + c4;
          if (vec_ok) {
            if (c4 < D) v = *reinterpret_cast<const f32x4*>(src);
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (c4 + e < D) v[e] = src[e];
          }
        }
        pre[q][rr] = v;
      }
    }
  }

  // cen: the model centre in LDS (stage_centre); the tile holds x - centre
  template <class T, bool SPLIT>
  __device__ __forceinline__ static void store(const TL& t, const f32x4 (&pre)[kPer][4],
                                               const float* cen, int tid) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int blk = tid + q * NT;
      if (blk >= TL::kBlocks) continue;
      const int rb = blk % (kTile / 4);
      const int c4 = (blk / (kTile / 4)) * 4;
      const f32x4 cq = *reinterpret_cast<const f32x4*>(cen + c4);
#pragma unroll
      for (int sq = 0; sq < 2; ++sq) {  // sq = 0: x, sq = 1: x^2
        const int f0 = c4 + sq * DP;
        uint16_t hi[4][4], lo[4][4];  // [row][feature]
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float xc = pre[q][rr][e] - cq[e];
            const float v = sq ? xc * xc : xc;
            T h, l;
            split16<T>(v, h, l);
            hi[rr][e] = bits16<T>(h);
            lo[rr][e] = SPLIT ? bits16<T>(l) : (uint16_t)0;
          }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int row = 4 * rb + rr;
          const u32x2 vh = {(unsigned)hi[rr][0] | ((unsigned)hi[rr][1] << 16),
                            (unsigned)hi[rr][2] | ((unsigned)hi[rr][3] << 16)};
          *reinterpret_cast<u32x2*>(t.rm_hi + row * TL::RS + f0) = vh;
          if (SPLIT) {
            const u32x2 vl = {(unsigned)lo[rr][0] | ((unsigned)lo[rr][1] << 16),
                              (unsigned)lo[rr][2] | ((unsigned)lo[rr][3] << 16)};
            *reinterpret_cast<u32x2*>(t.rm_lo + row * TL::RS + f0) = vl;
          }
        }
        const int p0 = tpos(4 * rb);  // four consecutive rows land on four consecutive slots
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const u32x2 vh = {(unsigned)hi[0][e] | ((unsigned)hi[1][e] << 16),
                            (unsigned)hi[2][e] | ((unsigned)hi[3][e] << 16)};
          *reinterpret_cast<u32x2*>(t.xt_hi + (f0 + e) * TL::TS + p0) = vh;
          if (SPLIT) {
            const u32x2 vl = {(unsigned)lo[0][e] | ((unsigned)lo[1][e] << 16),
                              (unsigned)lo[2][e] | ((unsigned)lo[3][e] << 16)};
            *reinterpret_cast<u32x2*>(t.xt_lo + (f0 + e) * TL::TS + p0) = vl;
          }
        }
      }
    }
  }
};

// Loader for many threads (the fused kernel's whole workgroup): thread slot = (row, 4
// features), consecutive threads on consecutive rows, one float4 per slot held in registers
// between fetch and store.  The transposed arrays take 16-bit writes; consecutive rows land on
// consecutive halves, so a wave's writes touch distinct banks.
template <int DP, int NT>
struct TileIO16Rows {
  using TL = Tile16<DP>;
  static constexpr int kSlots = kTile * (DP / 4);
  static constexpr int kPer = (kSlots + NT - 1) / NT;

  __device__ __forceinline__ static void fetch(f32x4 (&pre)[kPer], const float* __restrict__ X,
                                               int D, bool vec_ok, int64_t row0, int valid,
                                               int tid) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int idx = tid + q * NT;
      const int row = idx % kTile;
      const int c4 = (idx / kTile) * 4;
      f32x4 v = {0.f, 0.f, 0.f, 0.f};
      if (idx < kSlots && row < valid) {
        const float* src = X + (row0 + row) * (int64_t)D + c4;
        if (vec_ok) {
          if (c4 < D) v = *reinterpret_cast<const f32x4*>(src);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (c4 + e < D) v[e] = src[e];
        }
      }
      pre[q] = v;
    }
  }

  // cen: the model centre in LDS (stage_centre); the tile holds x - centre
  template <class T, bool SPLIT>
  __device__ __forceinline__ static void store(const TL& t, const f32x4 (&pre)[kPer],
                                               const float* cen, int tid) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int idx = tid + q * NT;
      if (kSlots % NT != 0 && idx >= kSlots) continue;  // (tid < NT: never when NT divides)
      const int row = idx % kTile;
      const int c4 = (idx / kTile) * 4;
      const int p = tpos(row);
      const f32x4 xc = pre[q] - *reinterpret_cast<const f32x4*>(cen + c4);
#pragma unroll
      for (int sq = 0; sq < 2; ++sq) {
        const int f0 = c4 + sq * DP;
        uint16_t hi[4], lo[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float v = sq ? xc[e] * xc[e] : xc[e];
          asm volatile("" : "+v"(v));  // the rounded square, as TileStoreR16 splits it
          T hh, ll;
          split16<T>(v, hh, ll);
          hi[e] = bits16<T>(hh);
          lo[e] = SPLIT ? bits16<T>(ll) : (uint16_t)0;
        }
        const u32x2 vh = {(unsigned)hi[0] | ((unsigned)hi[1] << 16), (unsigned)hi[2] | ((unsigned)hi[3] << 16)};
        *reinterpret_cast<u32x2*>(t.rm_hi + row * TL::RS + f0) = vh;
        if (SPLIT) {
          const u32x2 vl = {(unsigned)lo[0] | ((unsigned)lo[1] << 16), (unsigned)lo[2] | ((unsigned)lo[3] << 16)};
          *reinterpret_cast<u32x2*>(t.rm_lo + row * TL::RS + f0) = vl;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          t.xt_hi[(f0 + e) * TL::TS + p] = hi[e];
          if (SPLIT) t.xt_lo[(f0 + e) * TL::TS + p] = lo[e];
        }
      }
    }
  }
};

// Row-major 16-bit tile without a transposed copy (pipelined fused kernel): kTile rows of
// 2*DP <= 128 features (x - centre, then its square), hi and lo arrays.  Rows are kRowDw = 80
// dwords apart and the 16-byte chunk c of row r is stored at chunk c ^ ((r >> 2) & kSwz), so
// that 16 consecutive rows of one chunk (the E-step's 16-byte reads) and 4 rows of 4 aligned
// chunks (the statistics' transposed 8-byte reads) each fall on distinct banks of 64.  (A
// layout for 32 banks, 72 dwords and swizzle mask 1, measured 3.9 times the bank-conflict
// cycles.)
// A second layout, 72 dwords with mask 1 (18 KB per hi/lo pair instead of 20), lets eight
// wave-private tiles fit in LDS at the cost of 2-way conflicts on those reads.
constexpr int kRowDw = 80;
constexpr int kSwz = 3;
template <int DP, int RDW = kRowDw, int SWZ = kSwz>
struct TileR16 {
  static_assert(2 * DP <= 2 * RDW, "a row holds the 2*DP features");
  static constexpr int RS = 2 * RDW;       // elements per row
  static constexpr int kArr = kTile * RS;  // elements per array
  static constexpr int kSw = SWZ;
  __device__ __forceinline__ static int at(int row, int chunk) {
    return row * RS + (chunk ^ ((row >> 2) & SWZ)) * 8;
  }
};

// Converts the fetched rows (TileIO16Rows::fetch, NT threads) into a TileR16: x - centre and
// its square, each split into hi/lo, 8-byte stores.
template <int DP, int NT, int RDW = kRowDw, int SWZ = kSwz>
struct TileStoreR16 {
  using TR = TileR16<DP, RDW, SWZ>;
  using IO = TileIO16Rows<DP, NT>;
  template <class T, bool SPLIT>
  __device__ __forceinline__ static void store(uint16_t* hi_arr, uint16_t* lo_arr,
                                               const f32x4 (&pre)[IO::kPer], const float* cen,
                                               int tid) {
#pragma unroll
    for (int q = 0; q < IO::kPer; ++q) {
      const int idx = tid + q * NT;
      if (IO::kSlots % NT != 0 && idx >= IO::kSlots) continue;
      const int row = idx % kTile;
      const int c4 = (idx / kTile) * 4;
      const f32x4 xc = pre[q] - *reinterpret_cast<const f32x4*>(cen + c4);
#pragma unroll
      for (int sq = 0; sq < 2; ++sq) {
        const int f0 = c4 + sq * DP;
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          v[e] = sq ? xc[e] * xc[e] : xc[e];
          asm volatile("" : "+v"(v[e]));  // split the rounded square (split16x2)
        }
        uint32_t h0, h1, l0, l1;
        split16x2<T>(v[0], v[1], h0, l0);
        split16x2<T>(v[2], v[3], h1, l1);
        const int off = TR::at(row, f0 >> 3) + (f0 & 7);
        *reinterpret_cast<u32x2*>(hi_arr + off) = u32x2{h0, h1};
        if (SPLIT) *reinterpret_cast<u32x2*>(lo_arr + off) = u32x2{l0, l1};
      }
    }
  }
};

// gfx950 transposed LDS read of 16-bit data (ds_read_b64_tr_b16): within each group of 16
// lanes, lane 4b + c receives element c of the 8-byte chunks addressed by lanes b, b + 4,
// b + 8 and b + 12 of the group, as its values 0..3.
typedef short s16x4 __attribute__((vector_size(8)));
__device__ __forceinline__ s16x4 lds_read_tr16(const uint16_t* p) {
  return __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (__attribute__((address_space(3))) s16x4*)(p));
}

// The statistics' A operand (features x rows) of feature block b and 16-row step q from a
// TileR16 array, in the row order of the posterior operand: lane (j, h) gets feature 32 b + j
// at rows 16 q + 4 h + e and 16 q + 8 + 4 h + e (e = 0..3).  Each lane addresses row
// 16 q + 4 h + (i >> 2) (and + 8), features 32 b + 16 (j >> 4) + 4 (i & 3) .. + 3
// (i = lane & 15); both rows' chunk swizzle is fixed by h, so the offsets are affine in q, b.
template <int RDW = kRowDw, int SWZ = kSwz>
struct TrOffsetsL {
  int o1, o2;  // element offsets of the two reads for q = b = 0
  __device__ __forceinline__ TrOffsetsL(int lane) {
    const int i = lane & 15, j = lane & 31, h = lane >> 5;
    const int cp = 2 * (j >> 4) + ((i & 3) >> 1);  // chunk within the block's four
    const int row = 4 * h + (i >> 2);
    o1 = row * 2 * RDW + (cp ^ (h & SWZ)) * 8 + 4 * (i & 1);
    o2 = (row + 8) * 2 * RDW + (cp ^ ((h + 2) & SWZ)) * 8 + 4 * (i & 1);
  }
};
using TrOffsets = TrOffsetsL<>;

// Per interval: the two read bases of one array as LDS pointers.  The empty asm keeps the
// compiler from hoisting every (q, b) address out of the loop (32 registers held across the
// kernel); each read then costs one add of a constant.
typedef __attribute__((address_space(3))) s16x4 lds_s16x4;
struct TrBase {
  lds_s16x4* p1;
  lds_s16x4* p2;
  template <class O>
  __device__ __forceinline__ TrBase(const uint16_t* arr, const O& o) {
    int o1 = o.o1, o2 = o.o2;
    asm volatile("" : "+v"(o1), "+v"(o2));
    p1 = (lds_s16x4*)(arr + o1);
    p2 = (lds_s16x4*)(arr + o2);
  }
};

template <class V, int RDW = kRowDw>
__device__ __forceinline__ V tr_operand(const TrBase& t, int q, int b) {
  const int d = (16 * q * 2 * RDW + 32 * b) / 4;  // in 8-byte units
  const s16x4 r1 = __builtin_amdgcn_ds_read_tr16_b64_v4i16(t.p1 + d);
  const s16x4 r2 = __builtin_amdgcn_ds_read_tr16_b64_v4i16(t.p2 + d);
  const s16x4 both[2] = {r1, r2};
  return __builtin_bit_cast(V, both);
}

// E-step, 16-bit operands.  bh/bl: per k-step s (16 features), the lane's 8 constants
// A[16s + 8h + e][comp] as hi/lo fragments.  With COMP, chains of two k-steps (32 features)
// are joined with TwoSum exactly as in the FP32 form; without, one chain (lo = 0).
template <int DP, class T, bool SPLIT, bool COMP>
__device__ __forceinline__ void estep16(const Tile16<DP>& t, int j, int h,
                                        const typename P16<T>::v8 (&bh)[2 * DP / 16],
                                        const typename P16<T>::v8 (&bl)[2 * DP / 16], float cval,
                                        f32x16& hi, f32x16& lo) {
  using V = typename P16<T>::v8;
  constexpr int NS = 2 * DP / 16;
  constexpr int CH = COMP ? 2 : NS;  // k-steps per accumulation chain
  const uint16_t* ah = t.rm_hi + j * Tile16<DP>::RS + 8 * h;
  const uint16_t* al = t.rm_lo + j * Tile16<DP>::RS + 8 * h;
#pragma unroll
  for (int ch = 0; ch < NS / CH; ++ch) {
    f32x16 a;
#pragma unroll
    for (int r = 0; r < 16; ++r) a[r] = (ch == 0) ? cval : 0.f;
#pragma unroll
    for (int s = CH * ch; s < CH * ch + CH; ++s) {
      const V xh = __builtin_bit_cast(V, *reinterpret_cast<const u32x4*>(ah + 16 * s));
      a = P16<T>::mfma(xh, bh[s], a);
      if (SPLIT) {
        const V xl = __builtin_bit_cast(V, *reinterpret_cast<const u32x4*>(al + 16 * s));
        a = P16<T>::mfma(xh, bl[s], a);
        a = P16<T>::mfma(xl, bh[s], a);
      }
    }
    if (ch == 0) {
      hi = a;
#pragma unroll
      for (int r = 0; r < 16; ++r) lo[r] = 0.f;
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float tt = hi[r] + a[r];
        const float bp = tt - hi[r];
        const float err = (hi[r] - (tt - bp)) + (a[r] - bp);
        hi[r] = tt;
        lo[r] += err;
      }
    }
  }
}

// Statistics, 16-bit operands: acc[b] += XT[32b + j][rows] . gamma[rows][comp], gamma split
// into hi/lo from the E-step result registers (k-step q uses registers 8q..8q+7).
// With SKIP, a 16-row step whose gamma is zero in every lane is left out.
template <int DP, class T, bool SPLIT, bool SKIP = false>
__device__ __forceinline__ void stats16(const Tile16<DP>& t, int j, int h, const f32x16& gam,
                                        f32x16 (&acc)[2 * DP / 32]) {
  using V = typename P16<T>::v8;
  constexpr int NB = 2 * DP / 32;
  bool live[2] = {true, true};
  if (SKIP) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      bool nz = false;
#pragma unroll
      for (int e = 0; e < 8; ++e) nz |= gam[8 * q + e] != 0.f;
      live[q] = !wave_all_zero(nz);
    }
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    if (SKIP && !live[q]) continue;
    V gh, gl;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      T hh, ll;
      split16<T>(gam[8 * q + e], hh, ll);
      gh[e] = hh;
      gl[e] = SPLIT ? ll : (T)0.f;
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int off = (32 * b + j) * Tile16<DP>::TS + 16 * q + 8 * h;
      const V xh = __builtin_bit_cast(V, *reinterpret_cast<const u32x4*>(t.xt_hi + off));
      acc[b] = P16<T>::mfma(xh, gh, acc[b]);
      if (SPLIT) {
        const V xl = __builtin_bit_cast(V, *reinterpret_cast<const u32x4*>(t.xt_lo + off));
        acc[b] = P16<T>::mfma(xh, gl, acc[b]);
        acc[b] = P16<T>::mfma(xl, gh, acc[b]);
      }
    }
  }
}

// Loads the lane's E-step constant fragments: fragment (s, h, comp) holds A[16s + 8h + e][comp]
// for e = 0..7, stored contiguously at ((s*2 + h) * Kp + comp) * 8.
template <int DP, class T>
__device__ __forceinline__ void load_frags(const uint16_t* __restrict__ fr, int Kp, int comp, int h,
                                           typename P16<T>::v8 (&b)[2 * DP / 16]) {
  using V = typename P16<T>::v8;
#pragma unroll
  for (int s = 0; s < 2 * DP / 16; ++s)
    b[s] = __builtin_bit_cast(V, *reinterpret_cast<const u32x4*>(fr + ((size_t)(s * 2 + h) * Kp + comp) * 8));
}

}  // namespace dev
}  // namespace fv
