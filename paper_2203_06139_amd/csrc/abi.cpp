// abi.cpp -- the extern "C" boundary of libhistfit.so (declared in
// include/histfit.h): context and scratch ownership, host-side argument
// validation, launch-shape selection and kernel dispatch.  Every step of the
// computation runs in the HIP kernels; this file only checks and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <map>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>

#include "../../include/histfit.h"
#include "finish.hpp"
#include "fisher_kernels.hpp"
#include "fit_kernels.hpp"
#include "gradmap.hpp"
#include "unbinned.hpp"
#include "mlp.hpp"
#include "nll_avg.hpp"
#include "nll_kernels.hpp"

#define HF_EXPORT extern "C" __attribute__((visibility("default")))

static_assert(HF_NEYMAN == hf::OBJ_NEYMAN && HF_PEARSON == hf::OBJ_PEARSON &&
                  HF_POISSON == hf::OBJ_POISSON,
              "objective codes");
static_assert(HF_U32 == hf::DT_U32 && HF_F32 == hf::DT_F32 && HF_F64 == hf::DT_F64, "dtype codes");
static_assert(HF_ST_DOMAIN == hf::ST_DOMAIN && HF_ST_NONFINITE == hf::ST_NONFINITE, "status bits");
static_assert(HF_NORM_LISTING == hf::GRADMAP_NORM_LISTING && HF_NORM_PDF == hf::GRADMAP_NORM_PDF,
              "Gaussian normalisations");
static_assert(HF_MLP_IN == hf::kMlpIn && HF_MLP_HIDDEN == hf::kMlpHidden && HF_MLP_OUT == hf::kMlpOut &&
                  HF_MLP_OUT_PAD == hf::kMlpOutPad,
              "network shape");

namespace {

// Largest reduction width: P + 1 with P <= 16 for the objective, 64
// upper-triangle entries per pass for the Fisher matrix.
constexpr int kMaxNV = 64;
static_assert(hf::kFisherQ <= kMaxNV, "partials scratch");
// Upper bound on the objective kernels' grid; the partial-sum scratch is
// sized for it once, at context creation, so no call allocates afterwards.
constexpr int kMaxGrid = 8192;

}  // namespace

struct hf_ctx {
  int device = 0;
  int num_cu = 0;
  int max_grid = kMaxGrid;  // blocks whose partials the scratch holds
  int blocks_per_cu = 0;  // 0: as many as the kernel's occupancy allows
  std::map<hf::LaunchFn, std::pair<int, int>> occupancy;  // (blocks per CU, threads per block)
  std::map<hf::FisherFn, int> fisher_occupancy;
  std::string err;
  double* part = nullptr;
  int32_t* part_flags = nullptr;
  unsigned* ticket = nullptr;
  double2* log_lut = nullptr;
  hf::FitScratch fit;
};

namespace {

int fail(hf_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

int hip_fail(hf_ctx* c, hipError_t e, const char* what) {
  return fail(c, HF_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int use_device(hf_ctx* c) {
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(c, e, "hipGetDevice");
  if (cur != c->device) {
    e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  }
  return HF_OK;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// allow_avg: the caller evaluates bin-average models (nll_eval, nll_grad).
int check_model(hf_ctx* c, const hf_model* m, bool allow_avg = false) {
  if (!m) return fail(c, HF_EINVAL, "model is NULL");
  if (m->bin_average != 0 && m->bin_average != 1)
    return fail(c, HF_EINVAL, "model.bin_average must be 0 or 1");
  if (m->bin_average && m->kind == HF_GAUSS2D)
    return fail(c, HF_EUNSUPPORTED, "bin-average models are 1D only");
  if (m->bin_average && !allow_avg)
    return fail(c, HF_EUNSUPPORTED, "this call does not take bin-average models");
  switch (m->kind) {
    case HF_GAUSS_POLY:
      if (m->n_gauss < 0 || m->n_gauss > 4)
        return fail(c, HF_EUNSUPPORTED, "n_gauss %d outside 0..4", m->n_gauss);
      if (m->poly_degree < -1 || m->poly_degree > 3)
        return fail(c, HF_EUNSUPPORTED, "poly_degree %d outside -1..3", m->poly_degree);
      if (m->n_gauss == 0 && m->poly_degree < 0)
        return fail(c, HF_EINVAL, "model has no terms");
      break;
    case HF_GAUSS_EXP:
      if (m->n_gauss < 0 || m->n_gauss > 4)
        return fail(c, HF_EUNSUPPORTED, "n_gauss %d outside 0..4", m->n_gauss);
      break;
    case HF_GAUSS2D:
      return HF_OK;
    default:
      return fail(c, HF_EUNSUPPORTED, "unknown model kind %d", m->kind);
  }
  if (!std::isfinite(m->t_shift) || !std::isfinite(m->t_scale) || m->t_scale == 0.0)
    return fail(c, HF_EINVAL, "t_shift/t_scale must be finite and t_scale nonzero");
  return HF_OK;
}

int nparams(const hf_model* m) {
  switch (m->kind) {
    case HF_GAUSS_POLY:
      return 3 * m->n_gauss + m->poly_degree + 1;
    case HF_GAUSS_EXP:
      return 3 * m->n_gauss + 2;
    default:
      return 7;
  }
}

int bkg_code(const hf_model* m) {
  return m->kind == HF_GAUSS_EXP ? hf::BKG_EXP : m->poly_degree;
}

hf::LaunchFn pick_1d(int ng, int bkg, int obj, bool grad, bool f32) {
  switch (ng) {
    case 0:
      return hf::pick_1d_ng0(bkg, obj, grad, f32);
    case 1:
      return hf::pick_1d_ng1(bkg, obj, grad, f32);
    case 2:
      return hf::pick_1d_ng2(bkg, obj, grad, f32);
    case 3:
      return hf::pick_1d_ng3(bkg, obj, grad, f32);
    case 4:
      return hf::pick_1d_ng4(bkg, obj, grad, f32);
    default:
      return nullptr;
  }
}

// Grid for a grid-stride pass over nb bins in chunks of `chunk` bins with
// `block` threads per block: no more blocks than can be resident at once
// (occupancy per CU x CUs), so the grid runs in a single round, and the
// chunks split as evenly as that allows (every thread gets ceil or floor of
// the same count).
int objective_grid(const hf_ctx* c, int64_t nb, int chunk, int per_cu, int block = hf::kBlock) {
  const int64_t chunks = (nb + chunk - 1) / chunk;
  const int64_t per_block = block;
  int64_t gmax = static_cast<int64_t>(c->num_cu) * per_cu;
  if (gmax > c->max_grid) gmax = c->max_grid;
  if (gmax < 1) gmax = 1;
  int64_t need = (chunks + per_block - 1) / per_block;
  if (need <= gmax) return static_cast<int>(need < 1 ? 1 : need);
  const int64_t q = (chunks + gmax * per_block - 1) / (gmax * per_block);
  int64_t g = (chunks + per_block * q - 1) / (per_block * q);
  return static_cast<int>(g < 1 ? 1 : g);
}

int check_hist(hf_ctx* c, const hf_hist* h, bool two_d) {
  if (!h) return fail(c, HF_EINVAL, "hist is NULL");
  if (!h->counts) return fail(c, HF_EINVAL, "hist.counts is NULL");
  if (h->reserved != 0) return fail(c, HF_EINVAL, "hist.reserved must be 0");
  if (h->counts_dtype < HF_U32 || h->counts_dtype > HF_F64)
    return fail(c, HF_EINVAL, "counts_dtype %d unknown", h->counts_dtype);
  if (h->nx < 1 || h->ny < 1) return fail(c, HF_EINVAL, "nx, ny must be >= 1");
  if (!two_d && h->ny != 1) return fail(c, HF_EINVAL, "1D model needs ny == 1");
  if (h->nx > (int64_t(1) << 40) || h->ny > (int64_t(1) << 40) ||
      h->nx * h->ny > (int64_t(1) << 50))
    return fail(c, HF_EINVAL, "histogram too large");
  if (h->x_edges) {
    if (two_d) return fail(c, HF_EUNSUPPORTED, "x_edges is for 1D histograms");
    if ((reinterpret_cast<uintptr_t>(h->x_edges) & 7u) != 0)
      return fail(c, HF_EINVAL, "x_edges must be 8-byte aligned");
  } else if (!(std::isfinite(h->xlo) && std::isfinite(h->xhi) && h->xhi > h->xlo)) {
    return fail(c, HF_EINVAL, "x range must be finite with xhi > xlo");
  }
  if (two_d && !(std::isfinite(h->ylo) && std::isfinite(h->yhi) && h->yhi > h->ylo))
    return fail(c, HF_EINVAL, "y range must be finite with yhi > ylo");
  if (!aligned16(h->counts)) return fail(c, HF_EINVAL, "hist.counts must be 16-byte aligned");
  if (h->weights && !aligned16(h->weights))
    return fail(c, HF_EINVAL, "hist.weights must be 16-byte aligned");
  return HF_OK;
}

int run_objective(hf_ctx* c, const hf_hist* h, const hf_model* m, int32_t obj, int32_t prec,
                  const double* theta, const double* seed, double* nll_out, double* grad_out,
                  float* grad_w_out, uint32_t free_mask, int32_t* status_out, hipStream_t stream,
                  bool grad) {
  if (!c) return HF_EINVAL;
  int rc = check_model(c, m, true);
  if (rc) return rc;
  const bool two_d = m->kind == HF_GAUSS2D;
  rc = check_hist(c, h, two_d);
  if (rc) return rc;
  if (obj < HF_NEYMAN || obj > HF_POISSON) return fail(c, HF_EINVAL, "objective %d unknown", obj);
  if (prec != HF_FP64 && prec != HF_FP32_BIN)
    return fail(c, HF_EINVAL, "precision %d unknown", prec);
  const bool avg = m->bin_average != 0;
  const bool edges = h->x_edges != nullptr;
  if ((avg || edges) && prec != HF_FP64)
    return fail(c, HF_EUNSUPPORTED,
                "bin-average models and bins of any widths are evaluated in HF_FP64 only");
  if (!theta) return fail(c, HF_EINVAL, "theta is NULL");
  if (!nll_out) return fail(c, HF_EINVAL, "nll_out is NULL");
  if (grad && !grad_out) return fail(c, HF_EINVAL, "grad_out is NULL");
  if (grad_w_out && !aligned16(grad_w_out))
    return fail(c, HF_EINVAL, "grad_w_out must be 16-byte aligned");
  rc = use_device(c);
  if (rc) return rc;

  hf::LaunchFn fn = nullptr;
  if (two_d) {
    fn = hf::pick_2d(obj, grad, prec == HF_FP32_BIN);
  } else if (edges && !avg) {
    switch (m->n_gauss) {
      case 0: fn = hf::pick_edges_ng0(bkg_code(m), obj, grad); break;
      case 1: fn = hf::pick_edges_ng1(bkg_code(m), obj, grad); break;
      case 2: fn = hf::pick_edges_ng2(bkg_code(m), obj, grad); break;
      case 3: fn = hf::pick_edges_ng3(bkg_code(m), obj, grad); break;
      case 4: fn = hf::pick_edges_ng4(bkg_code(m), obj, grad); break;
      default: break;
    }
  } else if (avg) {
    switch (m->n_gauss) {
      case 0: fn = hf::pick_avg_ng0(bkg_code(m), obj, grad, edges); break;
      case 1: fn = hf::pick_avg_ng1(bkg_code(m), obj, grad, edges); break;
      case 2: fn = hf::pick_avg_ng2(bkg_code(m), obj, grad, edges); break;
      case 3: fn = hf::pick_avg_ng3(bkg_code(m), obj, grad, edges); break;
      case 4: fn = hf::pick_avg_ng4(bkg_code(m), obj, grad, edges); break;
      default: break;
    }
  } else {
    fn = pick_1d(m->n_gauss, bkg_code(m), obj, grad, prec == HF_FP32_BIN);
  }
  if (!fn) return fail(c, HF_EUNSUPPORTED, "no kernel for this model");

  hf::NllArgs a{};
  a.counts = h->counts;
  a.weights = h->weights;
  a.nx = h->nx;
  a.ny = two_d ? h->ny : 1;
  a.dtype = h->counts_dtype;
  a.obj = obj;
  a.hx = (h->xhi - h->xlo) / static_cast<double>(h->nx);
  // the bin-average kernels take the left edge of bin 0, the others its centre
  a.x0 = avg ? h->xlo : h->xlo + 0.5 * a.hx;
  if (two_d) {
    a.hy = (h->yhi - h->ylo) / static_cast<double>(h->ny);
    a.y0 = h->ylo + 0.5 * a.hy;
  }
  a.theta = theta;
  a.seed = seed;
  a.nll_out = nll_out;
  a.grad_out = grad_out;
  a.grad_w_out = grad_w_out;
  a.status_out = status_out;
  a.free_mask = free_mask;
  a.P = nparams(m);
  a.t_shift = m->t_shift;
  a.t_scale = m->t_scale;
  a.part = c->part;
  a.part_flags = c->part_flags;
  a.log_lut = c->log_lut;
  a.x_edges = h->x_edges;
  auto it = c->occupancy.find(fn);
  if (it == c->occupancy.end()) {
    int occ = 0, block = 0;
    hipError_t e = fn(a, 0, stream, &occ, &block);
    if (e != hipSuccess) return hip_fail(c, e, "occupancy query");
    it = c->occupancy.emplace(fn, std::make_pair(occ < 1 ? 1 : occ, block)).first;
  }
  // The 2D kernel runs at most two blocks per CU: measured on the 2048^2
  // workload with the two-kernel completion, 27.4 us at one block per CU,
  // 24.2 at two, 24.3 at three and 26.6 at four (with the one-kernel
  // completion one block had been faster, 41.0 against 52.0 us).
  const int occ = two_d ? std::min(2, it->second.first) : it->second.first;
  const int block = it->second.second;
  const int per_cu = c->blocks_per_cu > 0 ? c->blocks_per_cu : occ;
  // 2D work items are 16-bin pieces of one row (a row's tail is a short piece)
  const int64_t items_bins =
      two_d ? ((a.nx + hf::kChunk2D - 1) / hf::kChunk2D) * hf::kChunk2D * a.ny : a.nx;
  const int chunk = two_d ? hf::kChunk2D
                          : (avg ? hf::kAvgChunk : (edges ? 1 : hf::chunk_bins(m->n_gauss)));
  const int grid = objective_grid(c, items_bins, chunk, per_cu, block);
  hipError_t e = fn(a, grid, stream, nullptr, nullptr);
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  hf::FinishArgs f{};
  f.part = c->part;
  f.part_flags = c->part_flags;
  f.G = grid;
  f.NV = grad ? a.P + 1 : 1;
  f.seed = seed;
  f.nll_out = nll_out;
  f.grad_out = grad ? grad_out : nullptr;
  f.status_out = status_out;
  f.free_mask = free_mask;
  e = hf::launch_finish(f, stream);
  if (e != hipSuccess) return hip_fail(c, e, "finishing kernel launch");
  return HF_OK;
}

}  // namespace

HF_EXPORT int hf_ctx_create(hf_ctx** out, int device) {
  if (!out) return HF_EINVAL;
  *out = nullptr;
  hf_ctx* c = new hf_ctx();
  c->device = device;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) {
    delete c;
    return HF_EHIP;
  }
  e = hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess || c->num_cu < 1) {
    delete c;
    return HF_EHIP;
  }
  if (const char* s = std::getenv("HF_BLOCKS_PER_CU")) {
    const int v = std::atoi(s);
    if (v >= 1 && v <= 32) c->blocks_per_cu = v;
  }
  const size_t part_bytes = sizeof(double) * kMaxNV * kMaxGrid;
  double2 lut[hf::kLogLut];
  for (int j = 0; j < hf::kLogLut; ++j) hf::log_lut_entry(j, &lut[j].x, &lut[j].y);
  if (hipMalloc(&c->log_lut, sizeof lut) != hipSuccess ||
      hipMemcpy(c->log_lut, lut, sizeof lut, hipMemcpyHostToDevice) != hipSuccess ||
      hipMalloc(&c->part, part_bytes) != hipSuccess ||
      hipMalloc(&c->part_flags, sizeof(int32_t) * kMaxGrid) != hipSuccess ||
      hipMalloc(&c->ticket, 256) != hipSuccess || hipMemset(c->ticket, 0, 256) != hipSuccess ||
      hf::fit_scratch_init(&c->fit) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    hf_ctx_destroy(c);
    return HF_ENOMEM;
  }
  *out = c;
  return HF_OK;
}

HF_EXPORT void hf_ctx_destroy(hf_ctx* c) {
  if (!c) return;
  int cur = -1;
  if (hipGetDevice(&cur) == hipSuccess && cur != c->device) (void)hipSetDevice(c->device);
  if (c->part) (void)hipFree(c->part);
  if (c->part_flags) (void)hipFree(c->part_flags);
  if (c->ticket) (void)hipFree(c->ticket);
  if (c->log_lut) (void)hipFree(c->log_lut);
  hf::fit_scratch_free(&c->fit);
  if (cur >= 0 && cur != c->device) (void)hipSetDevice(cur);
  delete c;
}

namespace {
// Message of the last failing context-free call on this thread.
thread_local std::string g_noalloc_err;
}  // namespace

HF_EXPORT const char* hf_last_error(const hf_ctx* c) {
  return c ? c->err.c_str() : g_noalloc_err.c_str();
}

HF_EXPORT int hf_model_nparams(const hf_model* m) {
  const int rc = check_model(nullptr, m, true);
  if (rc) return rc;
  return nparams(m);
}

HF_EXPORT int nll_eval(hf_ctx* c, const hf_hist* h, const hf_model* m, int32_t obj, int32_t prec,
                       const double* theta, double* nll_out, int32_t* status_out,
                       hf_stream_t stream) {
  return run_objective(c, h, m, obj, prec, theta, nullptr, nll_out, nullptr, nullptr, 0u,
                       status_out, reinterpret_cast<hipStream_t>(stream), false);
}

HF_EXPORT int nll_grad(hf_ctx* c, const hf_hist* h, const hf_model* m, int32_t obj, int32_t prec,
                       const double* theta, const double* seed, double* nll_out, double* grad_out,
                       float* grad_w_out, uint32_t free_mask, int32_t* status_out,
                       hf_stream_t stream) {
  return run_objective(c, h, m, obj, prec, theta, seed, nll_out, grad_out, grad_w_out, free_mask,
                       status_out, reinterpret_cast<hipStream_t>(stream), true);
}

// ---------------------------------------------------------------------------
// nll_grad without a context: the scratch is a file-scope device array
// ---------------------------------------------------------------------------
namespace {

// Partials of up to kStaticMaxGrid blocks x kStaticNV values (P <= 16), the
// blocks' status flags and the log table, in one array per GPU:
//   [0, 2 kLogLut)                      log table (kLogLut double2)
//   [2 kLogLut, + kStaticNV kStaticMaxGrid)  block partials
//   [..., + kStaticMaxGrid / 2)         int32 flags, one per block
constexpr int kStaticMaxGrid = 2048;
constexpr int kStaticNV = 17;
constexpr size_t kScratchLut = 2 * static_cast<size_t>(hf::kLogLut);
constexpr size_t kScratchPart = static_cast<size_t>(kStaticNV) * kStaticMaxGrid;
constexpr size_t kScratchDoubles = kScratchLut + kScratchPart + kStaticMaxGrid / 2;
static_assert(kStaticMaxGrid % 2 == 0, "flags fill whole doubles");

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
hf_ctx* g_static_ctx[kMaxDevices] = {};

// The calling thread's current device's scratch, set up on first use: the
// array's device address (each GPU holds its own copy of `scratch`), the
// log table copied into it, the CU count.  Nothing is allocated on the
// device; the host-side record is created once per device and kept.
int static_context(hf_ctx** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    g_noalloc_err = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return HF_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    g_noalloc_err = "device index out of range";
    return HF_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ctx[dev]) {
    double* base = nullptr;
    e = hipGetSymbolAddress(reinterpret_cast<void**>(&base), HIP_SYMBOL(scratch));
    if (e != hipSuccess || !base) {
      g_noalloc_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return HF_EHIP;
    }
    int num_cu = 0;
    e = hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || num_cu < 1) {
      g_noalloc_err = "hipDeviceGetAttribute(multiprocessor count) failed";
      return HF_EHIP;
    }
    double2 lut[hf::kLogLut];
    for (int j = 0; j < hf::kLogLut; ++j) hf::log_lut_entry(j, &lut[j].x, &lut[j].y);
    e = hipMemcpy(base, lut, sizeof lut, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      g_noalloc_err = std::string("log table copy: ") + hipGetErrorString(e);
      return HF_EHIP;
    }
    hf_ctx* c = new hf_ctx();
    c->device = dev;
    c->num_cu = num_cu;
    c->max_grid = kStaticMaxGrid;
    c->log_lut = reinterpret_cast<double2*>(base);
    c->part = base + kScratchLut;
    c->part_flags = reinterpret_cast<int32_t*>(base + kScratchLut + kScratchPart);
    g_static_ctx[dev] = c;
  }
  *out = g_static_ctx[dev];
  return HF_OK;
}

}  // namespace

HF_EXPORT int nll_grad_noalloc(const hf_hist* h, const hf_model* m, int32_t obj, int32_t prec,
                               const double* theta, const double* seed, double* nll_out,
                               double* grad_out, float* grad_w_out, uint32_t free_mask,
                               int32_t* status_out, hf_stream_t stream) {
  g_noalloc_err.clear();
  if (!h || !m || !theta || !nll_out || !grad_out) {
    g_noalloc_err = "nll_grad_noalloc: hist, model, theta, nll_out and grad_out must not be NULL";
    return HF_EINVAL;
  }
  {
    const int P = hf_model_nparams(m);
    if (P > kStaticNV - 1) {
      g_noalloc_err = "nll_grad_noalloc: the static scratch holds partials of at most 16 "
                      "parameters";
      return HF_EINVAL;
    }
  }
  hf_ctx* c = nullptr;
  int rc = static_context(&c);
  if (rc) return rc;
  rc = run_objective(c, h, m, obj, prec, theta, seed, nll_out, grad_out, grad_w_out, free_mask,
                     status_out, reinterpret_cast<hipStream_t>(stream), true);
  if (rc) g_noalloc_err = c->err;
  return rc;
}

HF_EXPORT int nll_unbinned(hf_ctx* c, const double* events, const float* weights,
                           int64_t n_events, double lo, double hi, const hf_model* m,
                           const double* theta, double* nll_out, double* grad_out,
                           int32_t* status_out, hf_stream_t stream) {
  if (!c) return HF_EINVAL;
  int rc = check_model(c, m);
  if (rc) return rc;
  if (m->kind == HF_GAUSS2D)
    return fail(c, HF_EUNSUPPORTED, "the unbinned NLL takes 1D models");
  if (n_events < 0) return fail(c, HF_EINVAL, "n_events must be >= 0");
  if (n_events > 0 && !events) return fail(c, HF_EINVAL, "events is NULL");
  if (!(std::isfinite(lo) && std::isfinite(hi) && hi > lo))
    return fail(c, HF_EINVAL, "range must be finite with hi > lo");
  if (!theta) return fail(c, HF_EINVAL, "theta is NULL");
  if (!nll_out) return fail(c, HF_EINVAL, "nll_out is NULL");
  rc = use_device(c);
  if (rc) return rc;
  hf::UnbinnedFn fn = nullptr;
  switch (m->n_gauss) {
    case 0: fn = hf::pick_unbinned_ng0(bkg_code(m)); break;
    case 1: fn = hf::pick_unbinned_ng1(bkg_code(m)); break;
    case 2: fn = hf::pick_unbinned_ng2(bkg_code(m)); break;
    case 3: fn = hf::pick_unbinned_ng3(bkg_code(m)); break;
    case 4: fn = hf::pick_unbinned_ng4(bkg_code(m)); break;
    default: break;
  }
  if (!fn) return fail(c, HF_EUNSUPPORTED, "no unbinned kernel for this model");
  hf::UnbinnedArgs a{};
  a.x = events;
  a.w = weights;
  a.n = n_events;
  a.lo = lo;
  a.hi = hi;
  a.theta = theta;
  a.nll_out = nll_out;
  a.grad_out = grad_out;
  a.status_out = status_out;
  a.P = nparams(m);
  a.t_shift = m->t_shift;
  a.t_scale = m->t_scale;
  a.part = c->part;
  a.part_flags = c->part_flags;
  a.log_lut = c->log_lut;
  const bool vec = aligned16(events) && (reinterpret_cast<uintptr_t>(weights) & 7u) == 0;
  int grid = 0;
  // HF_BLOCKS_PER_CU caps the blocks per CU here as for the binned kernels
  const int cap = c->blocks_per_cu > 0 ? std::min(kMaxGrid, c->num_cu * c->blocks_per_cu) : kMaxGrid;
  hipError_t e = fn(a, vec, c->num_cu, cap, reinterpret_cast<hipStream_t>(stream), &grid);
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  hf::FinishArgs f{};
  f.part = c->part;
  f.part_flags = c->part_flags;
  f.G = grid;
  f.NV = grad_out ? a.P + 1 : 1;
  f.nll_out = nll_out;
  f.grad_out = grad_out;
  f.status_out = status_out;
  e = hf::launch_finish(f, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(c, e, "finishing kernel launch");
  return HF_OK;
}

HF_EXPORT int hf_nll_fisher(hf_ctx* c, const hf_hist* h, const hf_model* m, int32_t obj,
                            const double* theta, double* fisher_out, int32_t* status_out,
                            hf_stream_t stream_) {
  if (!c) return HF_EINVAL;
  int rc = check_model(c, m);
  if (rc) return rc;
  const bool two_d = m->kind == HF_GAUSS2D;
  rc = check_hist(c, h, two_d);
  if (rc) return rc;
  if (h->x_edges) return fail(c, HF_EUNSUPPORTED, "the Fisher matrix takes uniform bins only");
  if (obj < HF_NEYMAN || obj > HF_POISSON) return fail(c, HF_EINVAL, "objective %d unknown", obj);
  if (!theta) return fail(c, HF_EINVAL, "theta is NULL");
  if (!fisher_out) return fail(c, HF_EINVAL, "fisher_out is NULL");
  rc = use_device(c);
  if (rc) return rc;
  const bool ney = obj == HF_NEYMAN;
  hf::FisherFn fn = nullptr;
  if (two_d) {
    fn = hf::pick_fisher_2d(ney);
  } else {
    switch (m->n_gauss) {
      case 0: fn = hf::pick_fisher_ng0(bkg_code(m), ney); break;
      case 1: fn = hf::pick_fisher_ng1(bkg_code(m), ney); break;
      case 2: fn = hf::pick_fisher_ng2(bkg_code(m), ney); break;
      case 3: fn = hf::pick_fisher_ng3(bkg_code(m), ney); break;
      case 4: fn = hf::pick_fisher_ng4(bkg_code(m), ney); break;
      default: break;
    }
  }
  if (!fn) return fail(c, HF_EUNSUPPORTED, "no Fisher kernel for this model");
  const hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  hf::FisherArgs a{};
  a.counts = h->counts;
  a.weights = h->weights;
  a.nx = h->nx;
  a.ny = two_d ? h->ny : 1;
  a.dtype = h->counts_dtype;
  a.P = nparams(m);
  a.hx = (h->xhi - h->xlo) / static_cast<double>(h->nx);
  a.x0 = h->xlo + 0.5 * a.hx;
  if (two_d) {
    a.hy = (h->yhi - h->ylo) / static_cast<double>(h->ny);
    a.y0 = h->ylo + 0.5 * a.hy;
  }
  a.cfac = obj == HF_POISSON ? 1.0 : 2.0;
  a.theta = theta;
  a.fisher_out = fisher_out;
  a.status_out = status_out;
  a.t_shift = m->t_shift;
  a.t_scale = m->t_scale;
  a.part = c->part;
  a.part_flags = c->part_flags;
  auto it = c->fisher_occupancy.find(fn);
  if (it == c->fisher_occupancy.end()) {
    int occ = 0;
    hipError_t e = fn(a, 0, 0, stream, &occ);
    if (e != hipSuccess) return hip_fail(c, e, "occupancy query");
    it = c->fisher_occupancy.emplace(fn, occ < 1 ? 1 : occ).first;
  }
  // the 2D kernel runs one block per CU (measured on 2048^2: 27.1 us, 29.0 us
  // at the two its registers allow): each thread's share then amortises the
  // block's 28 wave reductions over twice the bins
  const int per_cu = c->blocks_per_cu > 0 ? c->blocks_per_cu : (two_d ? 1 : it->second);
  const int64_t items_bins =
      two_d ? ((a.nx + hf::kFisherChunk - 1) / hf::kFisherChunk) * hf::kFisherChunk * a.ny : a.nx;
  const int grid = objective_grid(c, items_bins, hf::kFisherChunk, per_cu);
  const int passes = hf::fisher_passes(a.P);
  const int entries = a.P * (a.P + 1) / 2;
  for (int p = 0; p < passes; ++p) {
    hipError_t e = fn(a, p, grid, stream, nullptr);
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
    hf::FinishSymArgs f{};
    f.part = c->part;
    f.part_flags = c->part_flags;
    f.G = grid;
    f.E0 = p * hf::kFisherQ;
    f.NQ = std::min(hf::kFisherQ, entries - f.E0);
    f.P = a.P;
    f.out = fisher_out;
    f.status_out = status_out;
    e = hf::launch_finish_sym(f, stream);
    if (e != hipSuccess) return hip_fail(c, e, "finishing kernel launch");
  }
  return HF_OK;
}

HF_EXPORT int hf_fisher_covariance(hf_ctx* c, int32_t B, int32_t P, int32_t obj,
                                   const double* fisher, uint32_t free_mask, double* cov_out,
                                   int32_t* status_out, hf_stream_t stream) {
  if (!c) return HF_EINVAL;
  if (B < 0) return fail(c, HF_EINVAL, "B must be >= 0");
  if (P < 1 || P > 16) return fail(c, HF_EINVAL, "P %d outside 1..16", P);
  if (obj < HF_NEYMAN || obj > HF_POISSON) return fail(c, HF_EINVAL, "objective %d unknown", obj);
  if (B > 0 && (!fisher || !cov_out)) return fail(c, HF_EINVAL, "fisher and cov_out must be non-NULL");
  if (P < 32 && (free_mask >> P) != 0u)
    return fail(c, HF_EINVAL, "free_mask has bits at or above P");
  int rc = use_device(c);
  if (rc) return rc;
  // F is the objective's expected curvature; one standard error is where the
  // objective rises by UP = 1/2 (Poisson NLL without the factor 2) or 1
  // (chi-square), so cov = 2 UP F^-1
  const double scale = obj == HF_POISSON ? 1.0 : 2.0;
  hipError_t e = hf::fisher_covariance(B, P, fisher, free_mask, scale, cov_out, status_out,
                                       reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  return HF_OK;
}

HF_EXPORT int hf_gauss_grad_map(hf_ctx* c, int64_t n, const double* x, const double* p,
                                int32_t p_shared, const double* sigma, int32_t sigma_shared,
                                int32_t norm, const double* seed, double* g_out, double* dx_out,
                                double* dp_out, double* dsigma_out, hf_stream_t stream) {
  if (!c) return HF_EINVAL;
  if (n < 0) return fail(c, HF_EINVAL, "n must be >= 0");
  if (norm != HF_NORM_LISTING && norm != HF_NORM_PDF)
    return fail(c, HF_EINVAL, "norm %d unknown", norm);
  if ((p_shared != 0 && p_shared != 1) || (sigma_shared != 0 && sigma_shared != 1))
    return fail(c, HF_EINVAL, "p_shared and sigma_shared must be 0 or 1");
  const bool shared = p_shared || sigma_shared;
  if (n == 0 && !shared) return HF_OK;
  if ((n > 0 && !x) || (n > 0 && !p_shared && !p) || (n > 0 && !sigma_shared && !sigma))
    return fail(c, HF_EINVAL, "x, p and sigma must be non-NULL");
  if ((p_shared && !p) || (sigma_shared && !sigma))
    return fail(c, HF_EINVAL, "a shared p or sigma must be non-NULL");
  int rc = use_device(c);
  if (rc) return rc;
  hf::GradMapArgs a{};
  a.n = n;
  a.x = x;
  a.p = p;
  a.sigma = sigma;
  a.seed = seed;
  a.p_shared = p_shared;
  a.sigma_shared = sigma_shared;
  a.norm = norm;
  a.g = g_out;
  a.dx = dx_out;
  a.dp = dp_out;
  a.ds = dsigma_out;
  a.part = c->part;
  a.part_flags = c->part_flags;
  a.ticket = c->ticket;
  // pairs of elements as 16-byte vectors when every per-element array allows
  bool vec = aligned16(x) && aligned16(seed) && aligned16(g_out) && aligned16(dx_out);
  if (!p_shared) vec = vec && aligned16(p) && aligned16(dp_out);
  if (!sigma_shared) vec = vec && aligned16(sigma) && aligned16(dsigma_out);
  hipError_t e = hf::gauss_grad_map(a, vec, c->num_cu, kMaxGrid,
                                    reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  return HF_OK;
}

HF_EXPORT int fit_batch(hf_ctx* c, int32_t B, const void* counts, int32_t dtype,
                        const int64_t* offsets, const double* ranges, const hf_model* m,
                        int32_t obj, int32_t prec, const double* theta0, const hf_fit_opts* o,
                        double* theta_out, double* nll_out, int32_t* status, int32_t* iters,
                        int32_t* nevals, hf_stream_t stream) {
  if (!c) return HF_EINVAL;
  int rc = check_model(c, m);
  if (rc) return rc;
  if (m->kind == HF_GAUSS2D) return fail(c, HF_EUNSUPPORTED, "fit_batch takes 1D models only");
  if (B < 0) return fail(c, HF_EINVAL, "B must be >= 0");
  if (B == 0) return HF_OK;
  if (!counts || !offsets || !ranges || !theta0 || !o || !theta_out || !nll_out || !status ||
      !iters || !nevals)
    return fail(c, HF_EINVAL, "a fit_batch pointer argument is NULL");
  if (dtype < HF_U32 || dtype > HF_F64) return fail(c, HF_EINVAL, "counts_dtype %d unknown", dtype);
  if (obj < HF_NEYMAN || obj > HF_POISSON) return fail(c, HF_EINVAL, "objective %d unknown", obj);
  if (prec != HF_FP64 && prec != HF_FP32_BIN)
    return fail(c, HF_EINVAL, "precision %d unknown", prec);
  if (o->max_iter < 1 || o->ls_max < 1 || o->ls_max > 60 || !(o->edm_tol >= 0.0))
    return fail(c, HF_EINVAL, "fit options out of range");
  if (o->hessian_init < 0 || o->hessian_init > 1)
    return fail(c, HF_EINVAL, "hessian_init must be 0 or 1");
  if (o->gradient < 0 || o->gradient > 1)
    return fail(c, HF_EINVAL, "gradient must be 0 (adjoint) or 1 (central differences)");
  if (o->gradient == 1 && prec != HF_FP64)
    return fail(c, HF_EINVAL, "central-difference gradients need FP64 bins");
  if (c->fit.cache_bins > 0) {
    const int cap = hf::fit_max_cache_bins(m->n_gauss, bkg_code(m), obj, c->fit.block);
    if (c->fit.cache_bins > cap)
      return fail(c, HF_EINVAL, "LDS cache of %d bins exceeds the %d this fit kernel can hold",
                  c->fit.cache_bins, cap);
  }
  if (c->fit.wave_bins > 0) {
    const int cap = hf::fit_max_wave_bins(m->n_gauss, bkg_code(m), obj, c->fit.block);
    if (c->fit.wave_bins > cap)
      return fail(c, HF_EINVAL, "wave_bins %d exceeds the %d this model's waves can hold in LDS",
                  c->fit.wave_bins, cap);
  }
  rc = use_device(c);
  if (rc) return rc;

  hf::FitArgs a{};
  a.B = B;
  a.counts = counts;
  a.dtype = dtype;
  a.offsets = offsets;
  a.ranges = ranges;
  a.obj = obj;
  a.f32 = prec == HF_FP32_BIN ? 1 : 0;
  a.theta0 = theta0;
  a.theta_out = theta_out;
  a.nll_out = nll_out;
  a.status = status;
  a.iters = iters;
  a.nevals = nevals;
  a.max_iter = o->max_iter;
  a.ls_max = o->ls_max;
  a.fixed_iters = o->fixed_iters;
  a.free_mask = o->free_mask;
  a.edm_tol = o->edm_tol;
  a.polish_edm = o->polish_edm;
  a.hessian_init = o->hessian_init;
  a.fd_grad = o->gradient;
  a.t_shift = m->t_shift;
  a.t_scale = m->t_scale;
  a.P = nparams(m);
  a.log_lut = c->log_lut;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hf::launch_fit(m->n_gauss, bkg_code(m), a, c->num_cu, &c->fit, s);
  if (e == hipErrorNotSupported) return fail(c, HF_EUNSUPPORTED, "no fit kernel for this model");
  if (e != hipSuccess) return hip_fail(c, e, "fit launch");
  return HF_OK;
}

// ---------------------------------------------------------------------------
// Learned initialiser
// ---------------------------------------------------------------------------
namespace {

int mlp_common(hf_ctx* c, int32_t B, const void* ws, int64_t ws_bytes) {
  if (!c) return HF_EINVAL;
  if (B < 64 || B % 64 != 0) return fail(c, HF_EINVAL, "batch must be a positive multiple of 64");
  if (!ws) return fail(c, HF_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(c, HF_EINVAL, "workspace must be 256-byte aligned");
  const int64_t need = hf::mlp_workspace_bytes(B);
  if (ws_bytes < need)
    return fail(c, HF_EINVAL, "workspace of %lld bytes, batch %d needs %lld",
                static_cast<long long>(ws_bytes), B, static_cast<long long>(need));
  return use_device(c);
}

int batch_common(hf_ctx* c, int32_t B, const void* counts, int32_t dtype, const int64_t* offsets) {
  if (!c) return HF_EINVAL;
  if (B < 1) return fail(c, HF_EINVAL, "B must be >= 1");
  if (!counts || !offsets) return fail(c, HF_EINVAL, "counts/offsets is NULL");
  if (dtype < HF_U32 || dtype > HF_F64) return fail(c, HF_EINVAL, "counts_dtype %d unknown", dtype);
  return use_device(c);
}

}  // namespace

HF_EXPORT int64_t hf_mlp_nparams(void) { return hf::MlpLayout::kTotal; }

HF_EXPORT int64_t hf_mlp_workspace_bytes(int32_t batch) {
  if (batch < 64 || batch % 64 != 0) return HF_EINVAL;
  return hf::mlp_workspace_bytes(batch);
}

HF_EXPORT int hf_mlp_workspace_layout(int32_t batch, int64_t* offsets) {
  if (batch < 64 || batch % 64 != 0 || !offsets) return HF_EINVAL;
  // carve from a fake base far from 0 so every view is a non-null offset
  char* base = reinterpret_cast<char*>(uintptr_t(1) << 40);
  const hf::MlpWorkspace w = hf::mlp_carve(base, batch);
  auto off = [base](const void* p) { return static_cast<int64_t>(static_cast<const char*>(p) - base); };
  for (int l = 0; l < 4; ++l) offsets[l] = off(w.a[l]);
  for (int l = 1; l <= 3; ++l) offsets[3 + l] = off(w.z[l]);
  offsets[7] = off(w.y);
  for (int l = 1; l <= 4; ++l) offsets[7 + l] = off(w.dz[l]);
  return HF_OK;
}

HF_EXPORT int hf_rebin_lognorm(hf_ctx* c, int32_t B, const void* counts, int32_t dtype,
                               const int64_t* offsets, float in_mean, float in_std, float* out,
                               hf_stream_t stream) {
  int rc = batch_common(c, B, counts, dtype, offsets);
  if (rc) return rc;
  if (!out) return fail(c, HF_EINVAL, "out is NULL");
  if (!(in_std > 0.0f) || !std::isfinite(in_mean)) return fail(c, HF_EINVAL, "bad in_mean/in_std");
  hipError_t e = hf::rebin_lognorm(B, counts, dtype, offsets, in_mean, in_std, out,
                                   reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? HF_OK : hip_fail(c, e, "rebin_lognorm");
}

HF_EXPORT int hf_default_starts(hf_ctx* c, int32_t B, const void* counts, int32_t dtype,
                                const int64_t* offsets, const double* ranges, const hf_model* m,
                                double* theta0, hf_stream_t stream) {
  int rc = batch_common(c, B, counts, dtype, offsets);
  if (rc) return rc;
  rc = check_model(c, m);
  if (rc) return rc;
  if (m->kind != HF_GAUSS_EXP || m->n_gauss != 1)
    return fail(c, HF_EUNSUPPORTED, "default starts exist for one Gaussian + exponential only");
  if (!ranges || !theta0) return fail(c, HF_EINVAL, "ranges/theta0 is NULL");
  hipError_t e = hf::default_starts(B, counts, dtype, offsets, ranges, m->t_shift, m->t_scale, theta0,
                                    reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? HF_OK : hip_fail(c, e, "default_starts");
}

HF_EXPORT int hf_column_stats(hf_ctx* c, int64_t n, int32_t cols, const float* x, float* mean,
                              float* std_out, hf_stream_t stream) {
  if (!c) return HF_EINVAL;
  if (n < 1 || cols < 1 || !x || !mean || !std_out) return fail(c, HF_EINVAL, "bad arguments");
  int rc = use_device(c);
  if (rc) return rc;
  hipError_t e = hf::column_stats(n, cols, x, mean, std_out, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? HF_OK : hip_fail(c, e, "column_stats");
}

HF_EXPORT int hf_theta_to_target(hf_ctx* c, int32_t B, const double* theta, const float* mean,
                                 const float* std_in, float* target, hf_stream_t stream) {
  if (!c) return HF_EINVAL;
  if (B < 1 || !theta || !mean || !std_in || !target) return fail(c, HF_EINVAL, "bad arguments");
  int rc = use_device(c);
  if (rc) return rc;
  hipError_t e = hf::theta_to_target(B, theta, mean, std_in, target,
                                     reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? HF_OK : hip_fail(c, e, "theta_to_target");
}

HF_EXPORT int hf_target_to_theta(hf_ctx* c, int32_t B, const float* y, const float* mean,
                                 const float* std_in, double* theta, hf_stream_t stream) {
  if (!c) return HF_EINVAL;
  if (B < 1 || !theta || !mean || !std_in || !y) return fail(c, HF_EINVAL, "bad arguments");
  int rc = use_device(c);
  if (rc) return rc;
  hipError_t e = hf::target_to_theta(B, y, mean, std_in, theta, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? HF_OK : hip_fail(c, e, "target_to_theta");
}

HF_EXPORT int hf_mlp_forward(hf_ctx* c, int32_t batch, const float* params, const float* x, float* y,
                             void* workspace, int64_t workspace_bytes, hf_stream_t stream) {
  int rc = mlp_common(c, batch, workspace, workspace_bytes);
  if (rc) return rc;
  if (!params || !x || !y) return fail(c, HF_EINVAL, "params/x/y is NULL");
  hipError_t e = hf::mlp_forward(batch, params, x, y, workspace, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? HF_OK : hip_fail(c, e, "mlp_forward");
}

HF_EXPORT int hf_mlp_train_step(hf_ctx* c, int32_t batch, float* params, float* adam_m, float* adam_v,
                                int32_t step, float lr, float wd, const float* x, const float* target,
                                float* grads, float* loss_out, void* workspace,
                                int64_t workspace_bytes, hf_stream_t stream) {
  int rc = mlp_common(c, batch, workspace, workspace_bytes);
  if (rc) return rc;
  if (!params || !adam_m || !adam_v || !x || !target || !grads || !loss_out)
    return fail(c, HF_EINVAL, "a pointer argument is NULL");
  if (step < 1 || !(lr > 0.0f) || !(wd >= 0.0f)) return fail(c, HF_EINVAL, "bad step/lr/wd");
  hipError_t e = hf::mlp_train_step(batch, params, adam_m, adam_v, step, lr, wd, x, target, grads,
                                    loss_out, workspace, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? HF_OK : hip_fail(c, e, "mlp_train_step");
}

HF_EXPORT int hf_fit_set_tuning(hf_ctx* c, int32_t wg_per_cu, int32_t cache_bins,
                                int32_t block_size) {
  if (!c) return HF_EINVAL;
  if (wg_per_cu < 1 || wg_per_cu > 16) return fail(c, HF_EINVAL, "wg_per_cu outside 1..16");
  if (cache_bins < 0) return fail(c, HF_EINVAL, "cache_bins must be >= 0");
  if (block_size != 256 && block_size != 512) return fail(c, HF_EINVAL, "block_size must be 256 or 512");
  c->fit.wg_per_cu = wg_per_cu;
  c->fit.cache_bins = cache_bins;
  c->fit.block = block_size;
  return HF_OK;
}

HF_EXPORT int hf_fit_set_wave_bins(hf_ctx* c, int32_t wave_bins) {
  if (!c) return HF_EINVAL;
  if (wave_bins < 0) return fail(c, HF_EINVAL, "wave_bins must be >= 0");
  c->fit.wave_bins = wave_bins;
  return HF_OK;
}

HF_EXPORT int hf_fit_get_wave_bins(const hf_ctx* c) {
  return c ? c->fit.wave_bins : HF_EINVAL;
}

HF_EXPORT int hf_fit_max_wave_bins(hf_ctx* c, const hf_model* m, int32_t objective,
                                   int32_t block_size) {
  if (!c) return HF_EINVAL;
  int rc = check_model(c, m);
  if (rc) return rc;
  if (m->kind == HF_GAUSS2D) return fail(c, HF_EUNSUPPORTED, "fit_batch takes 1D models only");
  if (objective < HF_NEYMAN || objective > HF_POISSON) return fail(c, HF_EINVAL, "objective unknown");
  rc = use_device(c);
  if (rc) return rc;
  if (block_size != 256 && block_size != 512) return fail(c, HF_EINVAL, "block_size must be 256 or 512");
  return hf::fit_max_wave_bins(m->n_gauss, bkg_code(m), objective, block_size);
}

HF_EXPORT int hf_fit_get_tuning(const hf_ctx* c, int32_t* wg_per_cu, int32_t* cache_bins,
                                int32_t* block_size) {
  if (!c || !wg_per_cu || !cache_bins || !block_size) return HF_EINVAL;
  *wg_per_cu = c->fit.wg_per_cu;
  *cache_bins = c->fit.cache_bins;
  *block_size = c->fit.block;
  return HF_OK;
}

HF_EXPORT int hf_fit_max_cache_bins(hf_ctx* c, const hf_model* m, int32_t objective,
                                    int32_t block_size) {
  if (!c) return HF_EINVAL;
  int rc = check_model(c, m);
  if (rc) return rc;
  if (m->kind == HF_GAUSS2D) return fail(c, HF_EUNSUPPORTED, "fit_batch takes 1D models only");
  if (objective < HF_NEYMAN || objective > HF_POISSON) return fail(c, HF_EINVAL, "objective unknown");
  rc = use_device(c);
  if (rc) return rc;
  if (block_size != 256 && block_size != 512) return fail(c, HF_EINVAL, "block_size must be 256 or 512");
  return hf::fit_max_cache_bins(m->n_gauss, bkg_code(m), objective, block_size);
}
