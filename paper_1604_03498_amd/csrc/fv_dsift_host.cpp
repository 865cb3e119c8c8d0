// Host side of the dense-SIFT front end: the extraction plan of an image geometry (scaled
// sizes, descriptor grids, the rows and columns the filtered maps are needed at, the scale
// table), its device copy and scratch per (device, stream), and the C entry points
// fv_dsift_rows / fv_dsift.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <tuple>
#include <utility>
#include <vector>

#include "fv.h"
#include "fv_internal.h"

namespace fv {
namespace {

size_t al256(size_t n) { return (n + 255) & ~(size_t)255; }

// The n smallest of the nine scales 2, sqrt 2, 1, ..., 1/8 (Sec. 4: nine scales from 2 down to
// 1/8 by factors of sqrt 2; the 8-scale setting leaves out the largest).
void paper_scales(int n, std::vector<double>* out) {
  out->clear();
  for (int k = 9 - n; k < 9; ++k) out->push_back(std::pow(2.0, 1.0 - 0.5 * k));
}

// Scaled side: the side itself at factor 1, else s * side rounded to nearest, ties to even
// (the default rounding mode of nearbyint).
int64_t scaled_side(double s, int side) {
  if (s == 1.0) return side;
  return (int64_t)std::nearbyint(s * (double)side);
}

using PlanKey = std::tuple<int, int, int, int, std::vector<double>>;
std::mutex g_plan_mu;
std::map<PlanKey, std::unique_ptr<DsiftPlan>> g_plans;
constexpr size_t kMaxPlans = 256;

int build_plan(int H, int W, const std::vector<double>& f, int B, int S, DsiftPlan* p) {
  p->H = H;
  p->W = W;
  p->B = B;
  p->S = S;
  p->factors = f;
  p->scales.clear();
  p->lists.clear();
  const int TW = dsift_filter_tile_cols(B);
  int64_t desc = 0, fxy = 0, blk = 0;
  for (double s : f) {
    const int64_t Hs = scaled_side(s, H), Ws = scaled_side(s, W);
    if (Hs > kDsiftMaxScaled || Ws > kDsiftMaxScaled) return FV_E_UNSUPPORTED;
    // first-bin centres x0 = a S, a >= 0, with x0 + 3B <= Ws - 1 (every bin centre inside)
    const int64_t nx = Ws - 1 - 3 * B >= 0 ? (Ws - 1 - 3 * B) / S + 1 : 0;
    const int64_t ny = Hs - 1 - 3 * B >= 0 ? (Hs - 1 - 3 * B) / S + 1 : 0;
    if (nx == 0 || ny == 0) continue;
    DsiftScale d{};
    d.s = s;
    d.Hs = (int)Hs;
    d.Ws = (int)Ws;
    d.nx = (int)nx;
    d.ny = (int)ny;
    std::vector<int> R, C;
    for (int64_t b = 0; b < ny; ++b)
      for (int j = 0; j < 4; ++j) R.push_back((int)(b * S + j * B));
    for (int64_t a = 0; a < nx; ++a)
      for (int i = 0; i < 4; ++i) C.push_back((int)(a * S + i * B));
    std::sort(R.begin(), R.end());
    R.erase(std::unique(R.begin(), R.end()), R.end());
    std::sort(C.begin(), C.end());
    C.erase(std::unique(C.begin(), C.end()), C.end());
    d.nR = (int)R.size();
    d.nC = (int)C.size();
    d.ntx = C.back() / TW + 1;
    d.blk0 = (int)blk;
    d.desc0 = desc;
    d.fxy0 = fxy;
    d.row0 = (int)p->lists.size();
    p->lists.insert(p->lists.end(), R.begin(), R.end());
    d.col0 = (int)p->lists.size();
    p->lists.insert(p->lists.end(), C.begin(), C.end());
    d.ridx0 = (int)p->lists.size();
    for (int64_t b = 0; b < ny; ++b)
      for (int j = 0; j < 4; ++j)
        p->lists.push_back((int)(std::lower_bound(R.begin(), R.end(), (int)(b * S + j * B)) -
                                 R.begin()));
    d.cidx0 = (int)p->lists.size();
    for (int64_t a = 0; a < nx; ++a)
      for (int i = 0; i < 4; ++i)
        p->lists.push_back((int)(std::lower_bound(C.begin(), C.end(), (int)(a * S + i * B)) -
                                 C.begin()));
    desc += nx * ny;
    fxy += (int64_t)d.nR * d.nC * 8;
    blk += (int64_t)d.nR * d.ntx;
    if (blk > ((int64_t)1 << 30) || p->lists.size() > ((size_t)1 << 30)) return FV_E_UNSUPPORTED;
    p->scales.push_back(d);
  }
  p->nsc = (int)p->scales.size();
  p->ndesc = desc;
  p->fxy_floats = fxy;
  p->nblk = blk;
  return FV_OK;
}

// Per (device, stream): the device copy of the last plan's tables and the scratch of the
// filtered values, staged images and rows.  Work on one stream is ordered, so the buffers are
// reused between calls; they are replaced (and the tables rewritten) only after the stream
// has drained.
struct DsiftWs {
  std::mutex mu;
  char* dev = nullptr;
  size_t cap = 0;
  const DsiftPlan* tab = nullptr;  // plan whose tables are at the start of dev
  size_t tab_bytes = 0;
};

std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, std::unique_ptr<DsiftWs>> g_ws;

DsiftWs* ws_for(int device, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  auto& p = g_ws[{device, s}];
  if (!p) p.reset(new (std::nothrow) DsiftWs());
  return p.get();
}

}  // namespace

int dsift_plan(int H, int W, int nsc, const double* scales, int B, int S, const DsiftPlan** out) {
  if (!out) return FV_E_INVAL;
  *out = nullptr;
  if (H < 1 || W < 1 || B < 1 || S < 1) return FV_E_INVAL;
  if (H > kDsiftMaxSide || W > kDsiftMaxSide || B > kDsiftMaxBin || S > kDsiftMaxSide)
    return FV_E_UNSUPPORTED;
  std::vector<double> f;
  if (scales == nullptr) {
    if (nsc < 1 || nsc > 9) return FV_E_INVAL;
    paper_scales(nsc, &f);
  } else {
    if (nsc < 1) return FV_E_INVAL;
    if (nsc > kDsiftMaxScales) return FV_E_UNSUPPORTED;
    for (int i = 0; i < nsc; ++i) {
      if (!std::isfinite(scales[i]) || !(scales[i] > 0.0)) return FV_E_INVAL;
      f.push_back(scales[i]);
    }
  }
  PlanKey key{H, W, B, S, f};
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) {
    *out = it->second.get();
    return FV_OK;
  }
  std::unique_ptr<DsiftPlan> p(new (std::nothrow) DsiftPlan());
  if (!p) return FV_E_NOMEM;
  const int rc = build_plan(H, W, f, B, S, p.get());
  if (rc) return rc;
  // plans are never freed while the process runs (a workspace may point at one); beyond the
  // cap a new geometry is planned per call and kept in a side list
  if (g_plans.size() >= kMaxPlans) {
    static std::vector<std::unique_ptr<DsiftPlan>> extra;
    extra.push_back(std::move(p));
    *out = extra.back().get();
    return FV_OK;
  }
  *out = p.get();
  g_plans.emplace(std::move(key), std::move(p));
  return FV_OK;
}

int dsift_enqueue(const DsiftPlan& p, int device, hipStream_t s, const float* images,
                  bool images_dev, int n_images, float* rows, float** rows_ws) {
  if (n_images < 0 || (n_images > 0 && !images)) return FV_E_INVAL;
  if (n_images > 65535) return FV_E_UNSUPPORTED;
  if (rows_ws) *rows_ws = nullptr;
  DsiftWs* ws = ws_for(device, s);
  if (!ws) return FV_E_NOMEM;
  std::lock_guard<std::mutex> lk(ws->mu);
  const size_t b_tab = al256(p.scales.size() * sizeof(DsiftScale)) + al256(p.lists.size() * 4);
  const size_t b_fxy = al256((size_t)n_images * (size_t)p.fxy_floats * 4);
  const size_t b_img = images_dev ? 0 : al256((size_t)n_images * p.H * p.W * 4);
  const size_t b_rows = rows ? 0 : al256((size_t)n_images * (size_t)p.ndesc * kDsiftDim * 4);
  const size_t need = b_tab + b_fxy + b_img + b_rows;
  if (need > ws->cap) {
    if (ws->dev) {
      hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess) return device_error(e);
      e = hipFree(ws->dev);
      ws->dev = nullptr;
      ws->cap = 0;
      ws->tab = nullptr;
      if (e != hipSuccess) return device_error(e);
    }
    size_t cap = std::max(need, (size_t)(1u << 20));
    cap = al256(cap + cap / 4);
    hipError_t e = hipMalloc(&ws->dev, cap);
    if (e != hipSuccess) {
      ws->dev = nullptr;
      return device_error(e);
    }
    ws->cap = cap;
  }
  char* base = ws->dev;
  DsiftScale* dsc = reinterpret_cast<DsiftScale*>(base);
  int* dlists = reinterpret_cast<int*>(base + al256(p.scales.size() * sizeof(DsiftScale)));
  float* fxy = reinterpret_cast<float*>(base + b_tab);
  float* img_stage = reinterpret_cast<float*>(base + b_tab + b_fxy);
  float* rows_buf = reinterpret_cast<float*>(base + b_tab + b_fxy + b_img);
  if (ws->tab != &p) {
    // earlier launches on the stream may still read the old tables
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(e);
    if (!p.scales.empty()) {
      e = hipMemcpy(dsc, p.scales.data(), p.scales.size() * sizeof(DsiftScale),
                    hipMemcpyHostToDevice);
      if (e == hipSuccess)
        e = hipMemcpy(dlists, p.lists.data(), p.lists.size() * 4, hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        ws->tab = nullptr;
        return device_error(e);
      }
    }
    ws->tab = &p;
  }
  const float* img = images;
  if (!images_dev && n_images > 0) {
    hipError_t e = hipMemcpyAsync(img_stage, images, (size_t)n_images * p.H * p.W * 4,
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return device_error(e);
    img = img_stage;
  }
  float* dst = rows ? rows : rows_buf;
  if ((reinterpret_cast<uintptr_t>(dst) & 7) != 0) return FV_E_INVAL;
  hipError_t e = launch_dsift(p, dsc, dlists, img, n_images, fxy, dst, s);
  if (e != hipSuccess) return device_error(e);
  if (rows_ws) *rows_ws = rows_buf;
  return FV_OK;
}

bool dsift_in_use(int device, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  return g_ws.count({device, s}) != 0;
}

int dsift_release(int device, hipStream_t s) {
  std::unique_ptr<DsiftWs> ws;
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find({device, s});
    if (it == g_ws.end()) return FV_OK;
    ws = std::move(it->second);
    g_ws.erase(it);
  }
  if (!ws) return FV_OK;
  std::lock_guard<std::mutex> lk(ws->mu);
  int rc = FV_OK;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) rc = device_error(e);
  if (ws->dev && (e = hipFree(ws->dev)) != hipSuccess) rc = device_error(e);
  ws->dev = nullptr;
  return rc;
}

}  // namespace fv

extern "C" {

int fv_dsift_rows(int H, int W, int n_scales, const double* scales, int bin, int step,
                  int64_t* n_rows) {
  if (!n_rows) return FV_E_INVAL;
  *n_rows = 0;
  const fv::DsiftPlan* p = nullptr;
  const int rc = fv::dsift_plan(H, W, n_scales, scales, bin, step, &p);
  if (rc) return rc;
  *n_rows = p->ndesc;
  return FV_OK;
}

int fv_dsift(const float* images, int n_images, int H, int W, int n_scales,
             const double* scales, int bin, int step, float* rows, unsigned flags, int device,
             void* hip_stream) {
  if (flags & ~(unsigned)(FV_X_DEVICE | FV_OUT_DEVICE | FV_ASYNC)) return FV_E_INVAL;
  if (n_images < 0) return FV_E_INVAL;
  const fv::DsiftPlan* p = nullptr;
  int rc = fv::dsift_plan(H, W, n_scales, scales, bin, step, &p);
  if (rc) return rc;
  if (n_images == 0 || p->ndesc == 0) return FV_OK;
  if (!images || !rows) return FV_E_INVAL;
  const size_t out_bytes = (size_t)n_images * (size_t)p->ndesc * fv::kDsiftDim * 4;
  if (out_bytes > ((size_t)1 << 40)) return FV_E_UNSUPPORTED;
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  if (prev != device && (rc = fv::set_device(device)) != FV_OK) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  float* rows_ws = nullptr;
  const bool out_dev = (flags & FV_OUT_DEVICE) != 0;
  rc = fv::dsift_enqueue(*p, device, s, images, (flags & FV_X_DEVICE) != 0, n_images,
                         out_dev ? rows : nullptr, &rows_ws);
  if (rc == FV_OK && !out_dev) {
    hipError_t e = hipMemcpyAsync(rows, rows_ws, out_bytes, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) rc = fv::device_error(e);
  }
  if (rc == FV_OK && !(flags & FV_ASYNC)) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = fv::device_error(e);
  }
  if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
  return rc;
}

}  // extern "C"
