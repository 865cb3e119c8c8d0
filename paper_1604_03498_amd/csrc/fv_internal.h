// Internal interface between the host runtime (fv_api.cpp) and the gfx950 kernels
// (fv_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fv {

constexpr int kTile = 32;        // descriptors per tile (one 32x32 MFMA block of rows)
constexpr int kCompsPerWave = 32; // GMM components owned by one wavefront
constexpr int kMaxWaves = 8;      // 8 waves x 32 components = 256 components per workgroup
constexpr int kMaxK = kCompsPerWave * kMaxWaves;
constexpr int kMaxD = 96;

// Device-resident constants of one GMM (all pointers are device memory owned by the handle).
struct Consts {
  int K, D;    // real sizes
  int Kp, DP;  // padded: Kp = 32 * W, DP = D rounded up to a multiple of 16
  int W;       // waves per workgroup (1, 2, 4 or 8)
  // E-step operand, log2(e)-scaled, [2*DP][Kp] f32: rows 0..DP-1 multiply x, rows DP..2DP-1
  // multiply x^2; padded rows and columns are zero.
  const float* A32;
  // hi/lo splits of A32 for the bf16 and fp16 forms: [2*DP][Kp] each (as 16-bit words)
  const uint16_t* Abf_hi;
  const uint16_t* Abf_lo;
  const uint16_t* Ah_hi;
  const uint16_t* Ah_lo;
  // log2(e)-scaled offsets [Kp]; padded components get -1e30 (posterior exactly 0)
  const float* c32;
  // finalize constants, double, [K*D] or [K]
  const double* mu64;
  const double* isd64;   // 1/sigma
  const double* ivar64;  // 1/sigma^2
  const double* cu64;    // 1/sqrt(w)
  const double* cv64;    // 1/sqrt(2 w)
};

// A chunk of consecutive descriptor rows whose statistics go to one partial slot.
struct Item {
  int64_t row0;
  int32_t nrows;
  int32_t pad;
};

// One frame for the finalize step: its descriptor count and its partial slots.
struct Frame {
  int64_t nrows;
  int32_t item0;
  int32_t nitems;
};

inline size_t slot_floats(const Consts& c) { return (size_t)(2 * c.DP + 1) * c.Kp; }

// Statistics kernel: for every item, the raw moments S0 = sum gamma, S1 = gamma^T X,
// S2 = gamma^T X^2 of its rows go to partials[item] laid out [2*DP+1][Kp] (rows: x features,
// x^2 features, then S0).  Items come from `items` (device) when non-null, else item i covers
// rows [i*P, min(N, (i+1)*P)).  `grid` workgroups loop over the items.
hipError_t launch_stats(const Consts& c, int precision, const float* X, bool vec_ok, int64_t N,
                        int P, const Item* items, int n_items, int grid, float* partials,
                        hipStream_t stream);

// Finalize: per frame, sum its partial slots in order (double), form u and v, apply the
// signed square root unless flagged off, write out[frame][2*K*D]; then L2-normalise unless
// flagged off.  `frames` is a device table of B frames, or null with B == 1 and `single`.
hipError_t launch_finalize(const Consts& c, const float* partials, const Frame* frames,
                           Frame single, int B, unsigned flags, float* out, double* normpart,
                           hipStream_t stream);

// Blocks per frame used by launch_finalize (size of normpart per frame).
int finalize_blocks(const Consts& c);

}  // namespace fv
