// Internal interface between the host runtime (fv_api.cpp) and the gfx950 kernels
// (fv_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdlib>
#include <stdint.h>

#include <vector>

#include "fv.h"

struct fv_gmm;

namespace fv {

constexpr int kTile = 32;        // descriptors per tile (one 32x32 MFMA block of rows)
constexpr int kCompsPerWave = 32; // GMM components owned by one wavefront
constexpr int kMaxWaves = 8;      // 8 waves x 32 components = 256 components per workgroup
constexpr int kFusedMaxK = kCompsPerWave * kMaxWaves;  // fused single-pass kernel
constexpr int kMaxK = 1024;                               // two-pass path
constexpr int kMaxD = 96;
// The paper's posterior threshold (Algorithm 1): with it on, a term enters the statistics only
// if its posterior exceeds kTau.
constexpr float kTau = 1e-6f;

// Sizes of one batched launch sequence, read by its kernels from device memory at the head of
// the work table, so that a captured graph serves every batch within its capacities: rows
// (arithmetic 32-row tiles of the first pass run to it), statistics items, 32-row tiles and
// frames.  Kernels given a null pointer use their arguments instead.
struct Counts {
  int64_t rows;
  int32_t n_items;
  int32_t n_tiles;
  int32_t B;
  int32_t next;  // work-item counter of the statistics launch (0 in the table copy)
};

// Dynamic work assignment of a persistent statistics launch over a work table: a workgroup
// draws its next item from the counter, in `order` (the table's items, largest first), so
// that workgroups finishing early take the remaining items.  Null `next`: the static
// assignment blockIdx.x, blockIdx.x + gridDim.x, ...  Every item's partial slot is computed
// by one workgroup in a fixed order, so the result does not depend on the assignment.  Only a
// launch with one row of workgroups (gridDim.y = 1) over the table's items may take a queue,
// once per reset of the counter.
struct ItemQueue {
  int* next;
  const int* order;
};

// First and next item of the calling workgroup (every thread gets the same index; n = the
// item count).  The dynamic form draws with one thread and shares it through *s_it behind
// barriers, so every thread of the workgroup must call these in the same sequence.
__device__ __forceinline__ int item_draw(const ItemQueue& q, int n) {
  const int k = atomicAdd(q.next, 1);
  return k < n ? q.order[k] : n;
}
__device__ __forceinline__ int item_first(const ItemQueue& q, int n, int* s_it) {
  if (!q.next) return blockIdx.x;
  if (threadIdx.x == 0) *s_it = item_draw(q, n);
  __syncthreads();
  return *s_it;
}
__device__ __forceinline__ int item_next(const ItemQueue& q, int n, int* s_it, int it) {
  if (!q.next) return it + gridDim.x;
  __syncthreads();  // every thread has read the previous index
  if (threadIdx.x == 0) *s_it = item_draw(q, n);
  __syncthreads();
  return *s_it;
}

// Loop bound of a grid-stride kernel: work items from the table (statistics chunks, or the
// arithmetic 32-row tiles when there is no item table), else the launch argument.
__device__ __forceinline__ int live_items(const Counts* cnt, const void* items, int n) {
  return cnt ? (items ? cnt->n_items : cnt->n_tiles) : n;
}
__device__ __forceinline__ int64_t live_rows(const Counts* cnt, int64_t n) {
  return cnt ? cnt->rows : n;
}

// Device-resident constants of one GMM (all pointers are device memory owned by the handle).
struct Consts {
  int K, D;    // real sizes
  int Kp, DP;  // padded: Kp = 32 * Wg * groups, DP = D rounded up to a multiple of 16
  int Wg;      // waves per component group (1, 2, 4 or 8); one group when Kp <= 256, else
               // groups of 256 components (Wg = 8)
  // E-step operand A, log2(e)-scaled, [2*DP][Kp] f32 (rows 0..DP-1 multiply x, rows
  // DP..2DP-1 multiply x^2; padded rows and columns zero), stored in MFMA fragment order: for
  // component block cb (32 components), step group g (4 steps) and lane l = 32h + j, the four
  // values A[4g + e + DP*h][32cb + j], e = 0..3, at ((cb * DP/4 + g) * 64 + l) * 4, so a wave
  // reads 1 KB contiguous per 16-byte load.
  const float* A32;
  // hi/lo splits of A32 for the bf16 and fp16 forms, as MFMA operand fragments: fragment
  // (s, h, comp) holds A[16s + 8h + e][comp], e = 0..7, at ((s*2 + h) * Kp + comp) * 8
  const uint16_t* Abf_hi;
  const uint16_t* Abf_lo;
  const uint16_t* Ah_hi;
  const uint16_t* Ah_lo;
  // log2(e)-scaled offsets [Kp]; padded components get -1e30 (posterior exactly 0)
  const float* c32;
  // model centre m0 [DP] f32 (zero past D): the kernels stage every descriptor as x - m0, and
  // every other constant here is computed for the centred means mu - m0 (the encoding is
  // invariant under translating descriptors and means together)
  const float* cen;
  // finalize constants, double, [K*D] or [K]
  const double* mu64;    // centred means mu - m0
  const double* isd64;   // 1/sigma
  const double* ivar64;  // 1/sigma^2
  const double* cu64;    // 1/sqrt(w)
  const double* cv64;    // 1/sqrt(2 w)
  // Per call, not per model: nonzero applies kTau (the API sets it on its own copy)
  int thresh;
  // Per call: the batched sequence's device-side sizes (null: the launch arguments hold them)
  const Counts* cnt;
  // Per call: dynamic item assignment of the batched statistics launch (null next: static)
  ItemQueue queue;
  // Per call: fused 16-bit kernel at 256 components (0 automatic, 1 wave-specialised,
  // 2 single-role)
  int variant16;
};

// A chunk of consecutive descriptor rows whose statistics go to one partial slot.
struct Item {
  int64_t row0;
  int32_t nrows;
  int32_t pad;
};

// One frame for the finalize step: its descriptor count, its partial slots (items), its place
// in the batch (output row and norm parts) and its number of chunk groups: consecutive runs of
// kGroupItems slots from item0 (the last one shorter), each summed (double, in index order)
// before the group sums are added in order.
struct Frame {
  int64_t nrows;
  int32_t item0;
  int32_t nitems;
  int32_t index;
  int32_t ngroups;
};

// A chunk group: slots [item0, item0 + nitems).
struct Group {
  int32_t item0;
  int32_t nitems;
};

constexpr int kGroupItems = 16;

inline size_t slot_floats(const Consts& c) { return (size_t)(2 * c.DP + 1) * c.Kp; }
inline int lse_groups(const Consts& c) { return c.Kp / (kCompsPerWave * c.Wg); }

// The 16-bit forms' group-wise second pass runs the pipelined specialised-wave kernel on groups
// of 256 components (with the first pass's normalisers) when the model has whole groups and
// DP <= 80; FV_NORMEXT16=w keeps the per-wave kernel (measurements).
inline bool normext16_pipelined(const Consts& c) {
  const char* e = std::getenv("FV_NORMEXT16");
  if (e && e[0] == 'w') return false;
  return c.Wg == kMaxWaves && c.DP <= 80 && c.Kp % (kMaxWaves * kCompsPerWave) == 0;
}

// Statistics kernel: for every item, the raw moments S0 = sum gamma, S1 = gamma^T X,
// S2 = gamma^T X^2 of its rows go to partials[item] laid out [2*DP+1][Kp] (rows: x features,
// x^2 features, then S0).  Items come from `items` (device) when non-null, else item i covers
// rows [i*P, min(N, (i+1)*P)).  `grid` workgroups loop over the items.
hipError_t launch_stats(const Consts& c, int precision, const float* X, bool vec_ok, int64_t N,
                        int P, const Item* items, int n_items, int grid, float* partials,
                        hipStream_t stream);

// First pass of the two-pass path: for every row and component group g, (max_k logit,
// log2 sum_k 2^(logit - max)) over the group's components, written to lse[g * lse_stride +
// row].  Items are tiles of 32 rows (`items` device table, or arithmetic over N when null).
// With gout (FP32, one component group, arithmetic tiles only) the posterior factors are also
// written for launch_sliced's gin: e component-major [Kp][gstride], then the row scales
// [Kp / 32][gstride] (gstride >= N, a multiple of 32; (Kp + Kp / 32) * gstride floats).
hipError_t launch_lse(const Consts& c, int precision, const float* X, bool vec_ok, int64_t N,
                      const Item* items, int n_items, int grid, float2* lse, int64_t lse_stride,
                      hipStream_t stream, float* gout = nullptr, int64_t gstride = 0);

// Second pass: statistics per (item, 32-component slice) from the first pass's normalisers,
// written to the item's partial slot (same layout as launch_stats).  Items hold chunks of P
// rows (table or arithmetic); grid = (grid, Kp / 32) workgroups.
// With gin (the first pass's gout, same gstride; P a multiple of 32, arithmetic chunks) gamma
// = e * f is read instead of recomputed.
hipError_t launch_sliced(const Consts& c, int precision, const float* X, bool vec_ok, int64_t N,
                         int P, const Item* items, int n_items, int grid, const float2* lse,
                         int64_t lse_stride, float* partials, hipStream_t stream,
                         const float* gin = nullptr, int64_t gstride = 0);

// Second pass over whole component groups: grid = (grid, Kp / (32 * W)) workgroups of W waves
// (W = Wg, or 4 when Wg = 8 and DP > 64), each owning a chunk of rows (work table or arithmetic,
// as launch_stats) and one group of 32 * W components; gamma from the first pass's
// normalisers.  Writes the group's columns of every item's partial slot.
hipError_t launch_normext(const Consts& c, const float* X, bool vec_ok, int64_t N, int P,
                          const Item* items, int n_items, int grid, const float2* lse,
                          int64_t lse_stride, float* partials, hipStream_t stream);

// Rows one FP32 workgroup of the second pass consumes per round (its waves x 32-row tiles).
int sliced_rows_per_wave_round(int DP);

// Finalize: per frame, the slots of every chunk group are summed in index order in double
// precision and the group sums are added in order; the totals are turned into u and v,
// signed-square-rooted unless flagged off, and written to out[index][2*K*D]; then L2
// normalisation unless flagged off.  `frames` is a device table of B records (in any order:
// the batch path puts the frames with the most slots first), or null for one frame (B == 1,
// `single`).  normpart holds B * finalize_blocks(c) doubles.
hipError_t launch_finalize(const Consts& c, const float* partials, const Frame* frames,
                           Frame single, int B, unsigned flags, float* out, double* normpart,
                           hipStream_t stream);

// Blocks per frame of the assembly step (size of normpart per frame).
int finalize_blocks(const Consts& c);

// fv_encode with every intermediate in the caller's device scratch (scratch_bytes at scratch):
// X and out in device memory (both FV_X_DEVICE and FV_OUT_DEVICE set), no allocation, no
// graph, no timing events; FV_E_UNSUPPORTED (before any launch) when the frame's
// intermediates do not fit.
int encode_on_scratch(const struct ::fv_gmm* gmm, const float* X, int64_t N, float* out,
                      int precision, unsigned flags, void* hip_stream, char* scratch,
                      size_t scratch_bytes);
// hipSetDevice, and a HIP error turned into an FV_E_* code (recorded for fv_last_device_error).
int set_device(int device);
int device_error(hipError_t e);

// Graph captures and replays so far of the launch sequences on (device, stream) (zero for a
// pair never used).
void stream_graph_counts(int device, hipStream_t s, int64_t* captures, int64_t* replays);

// Capacities a stream's batched launch sequence is sized to: frames, statistics chunks, chunk
// groups and rows.  Its grids and buffers depend on these only.
struct BatchCaps {
  int B = 0, items = 0, groups = 0;
  int64_t rows = 0;
  bool operator==(const BatchCaps& o) const {
    return B == o.B && items == o.items && groups == o.groups && rows == o.rows;
  }
};
inline BatchCaps caps_max(const BatchCaps& a, const BatchCaps& b) {
  BatchCaps m;
  m.B = a.B > b.B ? a.B : b.B;
  m.items = a.items > b.items ? a.items : b.items;
  m.groups = a.groups > b.groups ? a.groups : b.groups;
  m.rows = a.rows > b.rows ? a.rows : b.rows;
  return m;
}
// The capacities a batch of frames of these sizes needs (the handle's chunk length).
BatchCaps batch_need(const struct ::fv_gmm* g, const int64_t* sizes, int B);
// Device bytes of a stream's batch workspace with these capacities on the handle's batched
// path for `precision` (X and out in device memory, no projection).
size_t batch_caps_bytes(const struct ::fv_gmm* g, int precision, const BatchCaps& caps);
// Sets (device, stream)'s batch workspace to exactly these capacities and allocates exactly
// what they take (growing or shrinking it); later batches within them allocate nothing.
// *bytes receives the workspace's device bytes.
int batch_reserve(const struct ::fv_gmm* g, int precision, hipStream_t s, const BatchCaps& caps,
                  size_t* bytes);

// ---- 16-bit operand forms (one translation unit per form) --------------------------------
struct Frags16 {
  const uint16_t* hi;
  const uint16_t* lo;
};

#define FV_DECLARE_FORM(sfx)                                                                  \
  hipError_t launch_stats16_##sfx(const Consts& c, const Frags16& fr, const float* X,          \
                                  bool vec_ok, int64_t N, int P, const Item* items,            \
                                  int n_items, int grid, float* partials, hipStream_t stream); \
  hipError_t launch_lse16_##sfx(const Consts& c, const Frags16& fr, const float* X,            \
                                bool vec_ok, int64_t N, const Item* items, int n_items,        \
                                int grid, float2* lse, int64_t lse_stride,                     \
                                hipStream_t stream);                                           \
  hipError_t launch_sliced16_##sfx(const Consts& c, const Frags16& fr, const float* X,         \
                                   bool vec_ok, int64_t N, int P, const Item* items,           \
                                   int n_items, int grid, const float2* lse,                   \
                                   int64_t lse_stride, float* partials, hipStream_t stream);   \
  hipError_t launch_normext16_##sfx(const Consts& c, const Frags16& fr, const float* X,        \
                                    bool vec_ok, int64_t N, int P, const Item* items,          \
                                    int n_items, int grid, const float2* lse,                  \
                                    int64_t lse_stride, float* partials, hipStream_t stream);  \
  int sliced16_waves_##sfx(int DP);
FV_DECLARE_FORM(bf16s)
FV_DECLARE_FORM(f16s)
FV_DECLARE_FORM(bf16)
#undef FV_DECLARE_FORM

// Projection prologue y = A (x - m) (fv_project.hip).
constexpr int kMaxDin = 256;
struct ProjConsts {
  int Din, D;
  int S;   // MFMA steps: Din rounded up to a multiple of 32, halved (operand rows 0..2S-1)
  int Dp;  // D rounded up to a multiple of 32
  const float* frag;  // [2S][Dp], frag[k][c] = A[c][k] (zero for k >= Din or c >= D)
  const float* bias;  // [Dp], -(A m)[c] computed in double (zero for c >= D)
  // bf16 hi/lo fragments of A for the split form, [NS16][2][Dp][8] (NS16 = 16 rounded-up
  // steps of 16 input features, 4 | NS16): element e of (step s, half h, column c) is
  // A[c][16 s + 8 h + e] (zero past Din or D)
  const uint16_t* f16hi;
  const uint16_t* f16lo;
};
// With cnt (a batched sequence) the row count is read from cnt->rows; N is then only the
// capacity the grid was sized for.  split16: the split-bf16 contraction (16-bit encoder forms)
// instead of FP32.
hipError_t launch_project(const ProjConsts& p, const float* X, int64_t N, float* Y, int grid,
                          hipStream_t stream, const Counts* cnt = nullptr, bool split16 = false);

// EM step (fv_em.hip): M-step from the statistics partials, log-likelihood from the first
// pass's row normalisers (ll_part: em_loglik_blocks(N) workgroup sums, log2 units).
int em_loglik_blocks(int64_t N);
hipError_t launch_em(const Consts& c, const float* partials, int n_items, int64_t N,
                     float var_floor, const float2* lse, int64_t lse_stride, float* w_out,
                     float* mu_out, float* var_out, double* ll_part, hipStream_t stream);

// ---- dense-SIFT front end (fv_dsift.hip, fv_dsift_host.cpp) -------------------------------
constexpr int kDsiftDim = 130;  // 128 SIFT values + the centre's normalised x and y
constexpr int kDsiftMaxScales = 16;
constexpr int kDsiftMaxBin = 16;
constexpr int kDsiftMaxSide = 16384;   // source image side
constexpr int kDsiftMaxScaled = 32768; // scaled image side

// One scale of the extraction (scales without descriptors are left out of the table).  The
// filtered maps are evaluated at the nR needed rows and nC needed columns (sorted lists at
// lists[row0..], lists[col0..]); descriptor (a, b) of the nx x ny grid reads spatial bin
// (i, j) at needed column lists[cidx0 + 4a + i] and needed row lists[ridx0 + 4b + j].
struct DsiftScale {
  double s;          // scale factor (1: the source image itself)
  int Hs, Ws;        // scaled image size
  int nx, ny;        // descriptor grid
  int nR, nC;        // needed rows and columns
  int ntx;           // column tiles of the filter kernel
  int blk0;          // first filter workgroup of this scale (per image)
  int row0, col0, ridx0, cidx0;
  int pad;
  int64_t desc0;     // first descriptor of this scale (per image)
  int64_t fxy0;      // first filtered value of this scale (per image): [nR][nC][8] floats
};

struct DsiftPlan {
  int H = 0, W = 0, B = 0, S = 0, nsc = 0;
  int64_t ndesc = 0;       // descriptors per image
  int64_t fxy_floats = 0;  // filtered values per image
  int64_t nblk = 0;        // filter workgroups per image
  std::vector<DsiftScale> scales;
  std::vector<int> lists;
  std::vector<double> factors;  // the requested scale factors (cache key)
};

// LDS bytes of one filter workgroup and its output columns per tile, for bin size B.
size_t dsift_filter_lds_bytes(int B);
int dsift_filter_tile_cols(int B);
// Both kernels of the front end on `stream`: images [n_images][H][W] -> rows
// [n_images][ndesc][kDsiftDim]; fxy holds n_images * fxy_floats floats of scratch.
hipError_t launch_dsift(const DsiftPlan& p, const DsiftScale* dscales, const int* dlists,
                        const float* images, int n_images, float* fxy, float* rows,
                        hipStream_t stream);
// Host side (fv_dsift_host.cpp): the validated, cached plan of a geometry (FV_E_INVAL /
// FV_E_UNSUPPORTED for bad or oversized arguments); enqueueing on stream s of `device`
// (current) with images in device memory or, when images_dev is false, host memory copied
// into the stream's workspace; rows == nullptr puts the rows into the workspace and returns
// them in *rows_ws (valid until the next call on the stream).
int dsift_plan(int H, int W, int nsc, const double* scales, int B, int S, const DsiftPlan** out);
int dsift_enqueue(const DsiftPlan& p, int device, hipStream_t s, const float* images,
                  bool images_dev, int n_images, float* rows, float** rows_ws);
int dsift_release(int device, hipStream_t s);
bool dsift_in_use(int device, hipStream_t s);  // the pair holds a front-end workspace

}  // namespace fv

struct fv_pca {
  int Din = 0, D = 0, device = 0;
  uint64_t serial = 0;  // unique per load in the process (a freed handle's address can recur)
  fv::ProjConsts p{};
  void* dev_block = nullptr;
};

// The public handle (opaque in the C ABI).
struct fv_gmm {
  int K = 0, D = 0, device = 0;
  uint64_t serial = 0;  // unique per load in the process (a freed handle's address can recur)
  fv::Consts c{};
  void* dev_block = nullptr;  // one allocation holding every constant array
  bool f16_fits = true;       // every fp16 operand fragment is finite (else no fp16 form)
  // launch tuning (0 = automatic)
  int batch_chunk = 0;
  int batch_path = 0;
  int64_t single_split_below = 0;
  int batch_grid = 0;
  int fused16_variant = 0;
};

// Status of an arithmetic form for this model: FV_OK, FV_E_INVAL for an unknown form, or
// FV_E_UNSUPPORTED for the fp16 split when the model's operand entries overflow fp16.
inline int fv_form_status(const fv_gmm* g, int precision) {
  if (precision < FV_PREC_FP32 || precision > FV_PREC_BF16) return FV_E_INVAL;
  if (precision == FV_PREC_FP16_SPLIT && g != nullptr && !g->f16_fits) return FV_E_UNSUPPORTED;
  return FV_OK;
}
