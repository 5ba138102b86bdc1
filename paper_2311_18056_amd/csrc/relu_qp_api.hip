// Host side of the C ABI declared in include/relu_qp.h: validation, device memory, the offline
// stage (Algorithm 1, "Offline") and the launch of the online stage.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "relu_qp.h"
#include "batch_kernel.h"
#include "layer_kernel.h"
#include "paper_layer.h"
#include "setup_kernels.h"
#include "small_kernel.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_OR_FAIL(expr)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(RQP_EHIP, "%s: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

// Entry points that touch the handle's device memory refuse an offloaded handle.
#define DEVICE_OR_FAIL(h)                                                                       \
  do {                                                                                         \
    if ((h)->offloaded) return fail(RQP_ESTATE, "the handle is offloaded (relu_qp_restore first)"); \
  } while (0)

// RAII device buffer used during setup
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 8); }
  double* d() const { return static_cast<double*>(p); }
};

}  // namespace

struct relu_qp_handle {
  int n = 0, m = 0, L = 0, batch = 1;
  int device = 0;  // the GPU the handle's memory lives on
  long ldw = 0;
  relu_qp_settings s{};
  size_t esize = 8;  // bytes per iterate element
  std::vector<double> grid, mid;
  std::vector<unsigned char> eq;
  int j0 = 0;
  int grid_wg = 0;     // workgroups of the persistent launch (closed loops, scaled problems)
  int grid_plain = 0;  // workgroups of the persistent launch of plain solves
  bool small = false;  // plain solves run on the single-workgroup kernel (n + m <= kSmallRows)
  rqp::LaunchPlan plan{};    // plain solves
  rqp::LaunchPlan plan_xt{}; // closed loops and Ruiz-scaled problems
  // device
  void* W = nullptr;
  long w_stride = 0;
  void* C = nullptr;
  void* q = nullptr;
  void* l = nullptr;
  void* u = nullptr;
  unsigned char* eq_d = nullptr;
  double* grid_d = nullptr;
  double* mid_d = nullptr;
  void* xs = nullptr;
  void* zs = nullptr;
  void* ys = nullptr;
  int* js = nullptr;
  uint64_t* xw = nullptr;
  uint64_t* xc = nullptr;
  uint64_t* xn = nullptr;
  uint64_t* xu = nullptr;  // closed loop: applied-control words, 2 parities x kMaxPlant x 2
  double* xpl = nullptr;   // closed loop: per-workgroup plant state, 2 x kMaxGrid x kMaxPlant
  double* axs = nullptr;   // A x of the last solve's x (m, FP64), for warm starts that continue it
  // Ruiz scaling (settings.scaling > 0): x = D xb, z = zb / E, y = E yb / c. Device copy scl:
  // c D (n), E (m), 1 / (c D) (n), 1 / E (m), D (n), E / c (m).
  std::vector<double> sD, sE;
  double sc = 1.0;
  double* scl = nullptr;
  // the paper's literal layer (built at first use): W (n+2m) x ldp and its exchange words
  void* Wp = nullptr;
  long ldp = 0;
  uint64_t* xwp = nullptr;
  size_t xw_words = 0, xn_words = 0;
  unsigned* err = nullptr;
  int* abort_h = nullptr;  // host-mapped
  int* abort_d = nullptr;
  uint32_t tag = 1;
  bool warm_mode = false, warm_pending = false, have_prev = false;
  // parametric data (Sec. IV): q = F x0, l = lo - E x0, u = hi - E x0
  int nx = 0;
  double* F_d = nullptr;
  double* E_d = nullptr;
  double* lo_d = nullptr;
  double* hi_d = nullptr;
  // batched engine
  bool batched = false;
  int bprec = 0;
  long ldk = 0, lpad = 0, cpad = 0, bpad = 0;
  void* bWa = nullptr;
  void* bWb = nullptr;
  double* bCd = nullptr;  // FP64 check matrix, K-blocked
  float* bX = nullptr;
  float* bZ = nullptr;
  float* bY = nullptr;
  void* bVa = nullptr;
  void* bVb = nullptr;
  double* bCVd = nullptr;  // FP64 check operands [x; 0] and [0; y], K-blocked
  double* bRpx = nullptr;  // check scratch: P x and A'y per list position (B x n each, FP64)
  double* bRaty = nullptr;
  int* bjb = nullptr;
  unsigned long long* bnorms = nullptr;
  int* blists = nullptr;
  int* bpos = nullptr;
  int* bmtiles = nullptr;
  unsigned* bbar = nullptr;
  int* bstatus = nullptr;   // slot states, persistent across launches
  int* biter = nullptr;     // iterations since admission
  float* bstage = nullptr;  // warm-start staging: n + m floats and one int
  rqp::BatchPlan bplan{};            // the tile shape in use
  rqp::BatchPlan bplans[rqp::kTileShapes]{};  // tile rows rqp::kTileRows (128, 64, 256)
  double tile_us[rqp::kTileShapes] = {};      // autotuner: microseconds per iteration of each shape
  bool tile_cached = false;          // the choice came from the autotuner's cache
  size_t dev_bytes = 0;              // requested bytes of the resident device allocations
  // every resident device allocation (the handle field that holds it, its size, and its pinned
  // host copy once the handle has been offloaded)
  struct DevAlloc {
    void** slot;
    size_t bytes;
    void* host;
  };
  std::vector<DevAlloc> allocs;
  bool offloaded = false;
};

namespace {

void free_handle(relu_qp_handle* h) {
  if (!h) return;
  void* ptrs[] = {h->W,    h->C,    h->q,    h->l,    h->u,     h->eq_d,   h->grid_d,  h->mid_d,
                  h->xs,   h->zs,   h->ys,   h->js,   h->xw,    h->xc,     h->xn,      h->err,  h->xu,  h->xpl, h->axs, h->scl, h->Wp, h->xwp,
                  h->F_d,  h->E_d,  h->lo_d, h->hi_d, h->bWa,   h->bWb,    h->bCd,
                  h->bX,   h->bZ,   h->bY,   h->bVa,  h->bVb,   h->bCVd,   h->bRpx, h->bRaty, h->bjb,
                  h->bnorms, h->blists, h->bmtiles, h->bbar, h->bstatus, h->biter, h->bstage, h->bpos};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (auto& e : h->allocs)
    if (e.host) (void)hipHostFree(e.host);
  if (h->abort_h) (void)hipHostFree(h->abort_h);
  delete h;
}

// Resident device allocation of a handle (counted in h->dev_bytes; freed by free_handle).
hipError_t dmalloc(relu_qp_handle* h, void** p, size_t bytes) {
  const size_t b = bytes ? bytes : 8;
  hipError_t e = hipMalloc(p, b);
  if (e == hipSuccess) {
    h->dev_bytes += b;
    h->allocs.push_back({p, b, nullptr});
  }
  return e;
}

// Frees one resident allocation (and its host copy) and forgets it.
void dfree(relu_qp_handle* h, void** p) {
  for (size_t i = 0; i < h->allocs.size(); ++i)
    if (h->allocs[i].slot == p) {
      if (*p) (void)hipFree(*p);
      if (h->allocs[i].host) (void)hipHostFree(h->allocs[i].host);
      h->dev_bytes -= h->allocs[i].bytes;
      h->allocs.erase(h->allocs.begin() + (long)i);
      break;
    }
  *p = nullptr;
}
template <typename T>
hipError_t dmalloc(relu_qp_handle* h, T** p, size_t bytes) {
  return dmalloc(h, reinterpret_cast<void**>(p), bytes);
}

// ---------------------------------------------------------------------------------------------
// Scratch of relu_qp_solve_x0_noalloc: the exchange words of one persistent launch (layer input,
// check vector, norm partials) and its error word, in a file-scope device array instead of the
// handle's allocations, so that the entry point allocates nothing. Every GPU the library runs on
// holds its own copy until the process ends. On the host, `scratch` names a host-side stand-in,
// not device memory: host code uses only the per-device address hipGetSymbolAddress returned
// (kept in g_scratch). Layout: error word at 0, norm partials (2 x kMaxGrid x 8 x 2 words) at
// 256, then the layer-input and check-vector words (2 x L x words each).
constexpr size_t kScratchBytes = (size_t)1 << 20;
constexpr size_t kScratchNormOff = 256;
constexpr size_t kScratchNormWords = (size_t)2 * rqp::kMaxGrid * 8 * 2;
constexpr size_t kScratchXwOff = kScratchNormOff + kScratchNormWords * 8;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
struct ScratchDev {
  void* ptr = nullptr;  // the device address of this GPU's scratch
  uint32_t tag = 1;     // next tag of the exchange words (monotone over every call on this GPU)
  bool clean = false;   // cleared since the process started
};
std::mutex g_scratch_mu;
ScratchDev g_scratch[kScratchDevices];

// Once per device, with that device current (called from relu_qp_setup).
int scratch_init(int dev) {
  if (dev < 0 || dev >= kScratchDevices) return fail(RQP_EINVAL, "device %d beyond %d", dev, kScratchDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev].ptr) return RQP_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return fail(RQP_EHIP, "scratch address on device %d: %s", dev, hipGetErrorString(e));
  g_scratch[dev].ptr = ptr;
  return RQP_OK;
}

// Zero fill by a kernel (no memset node, so a caller may capture the call in a graph).
__global__ void clear_words(uint64_t* p, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

int validate_settings(const relu_qp_settings* s) {
  if (!s) return fail(RQP_EINVAL, "settings is NULL");
  if (!(s->sigma > 0.0) || !std::isfinite(s->sigma)) return fail(RQP_EINVAL, "sigma must be finite and > 0");
  if (!(s->alpha > 0.0 && s->alpha < 2.0)) return fail(RQP_EINVAL, "alpha must be in (0, 2)");
  if (s->n_rho < 1 || s->n_rho > 64) return fail(RQP_EINVAL, "n_rho must be in [1, 64]");
  if (s->n_rho == 1 && !(s->rho0 > 0.0 && std::isfinite(s->rho0))) return fail(RQP_EINVAL, "rho0 must be > 0");
  if (s->n_rho > 1 && !(s->rho_min > 0.0 && s->rho_max > s->rho_min && std::isfinite(s->rho_max)))
    return fail(RQP_EINVAL, "need 0 < rho_min < rho_max");
  if (s->n_rho > 1 && !(s->rho0 > 0.0)) return fail(RQP_EINVAL, "rho0 must be > 0");
  if (!(s->rho_eq_scale > 0.0) || !std::isfinite(s->rho_eq_scale)) return fail(RQP_EINVAL, "rho_eq_scale must be > 0");
  if (!(s->eps_abs >= 0.0) || !(s->eps_rel >= 0.0)) return fail(RQP_EINVAL, "eps_abs and eps_rel must be >= 0");
  if (s->max_iter < 1 || s->max_iter > (1 << 28)) return fail(RQP_EINVAL, "max_iter must be in [1, 2^28]");
  if (s->check_interval < 1) return fail(RQP_EINVAL, "check_interval must be >= 1");
  if (s->precision != RQP_FP64 && s->precision != RQP_FP32 && s->precision != RQP_BF16X3)
    return fail(RQP_EINVAL, "unknown precision");
  if (s->batch < 1 || s->batch > (1 << 20)) return fail(RQP_EINVAL, "batch must be in [1, 2^20]");
  if (s->engine < RQP_ENGINE_AUTO || s->engine > RQP_ENGINE_BATCH) return fail(RQP_EINVAL, "unknown engine");
  if (s->scaling < 0 || s->scaling > 100) return fail(RQP_EINVAL, "scaling must be in [0, 100] passes");
  const bool batched = s->engine == RQP_ENGINE_BATCH ||
                       (s->engine == RQP_ENGINE_AUTO && (s->batch > 1 || s->precision == RQP_BF16X3));
  if (batched && s->precision == RQP_FP64) return fail(RQP_EINVAL, "the batched engine runs FP32 or BF16X3");
  if (!batched && s->precision == RQP_BF16X3) return fail(RQP_EINVAL, "BF16X3 needs the batched engine");
  if (!batched && s->batch != 1) return fail(RQP_EINVAL, "the single-instance engine needs batch == 1");
  return RQP_OK;
}

// Modified Ruiz equilibration (Algorithm 1 "scale problem"; Sec. III-D scales the KKT matrix
// and the cost as OSQP does), FP64 on the host at setup. Each pass: delta = 1 / sqrt of the
// inf-norm of every column of [[P, A'], [A, 0]] (1 for a zero column, clipped to
// [1e-4, 1e4]); P <- Dd P Dd, q <- Dd q, A <- De A Dd; then the cost scale
// gamma = 1 / max(mean column inf-norm of P, ||q||_inf) (clipped likewise), P, q <- gamma P, q.
// Returns the accumulated D (n), E (m) and c.
double clip_scale(double v) {
  const double d = v > 0.0 ? 1.0 / std::sqrt(v) : 1.0;
  return d < 1e-4 ? 1e-4 : (d > 1e4 ? 1e4 : d);
}

// q0 holds nq rows (the instances of a batch): the cost scale takes the largest |q| entry over
// all of them, so one scaling serves every instance (each pass scales q's entries by positive
// factors, so the entry-wise largest magnitudes over the rows are all that matters).
void ruiz(int n, int m, const double* P0, const double* q0, int nq, const double* A0, int passes,
          std::vector<double>& D, std::vector<double>& E, double& c) {
  std::vector<double> P(P0, P0 + (size_t)n * n), A(A0, A0 + (size_t)m * n), q(n, 0.0);
  for (int b = 0; b < nq; ++b)
    for (int i = 0; i < n; ++i) q[i] = std::max(q[i], std::fabs(q0[(size_t)b * n + i]));
  D.assign(n, 1.0);
  E.assign(m, 1.0);
  c = 1.0;
  std::vector<double> colx(n), colz(m), dd(n), de(m);
  for (int it = 0; it < passes; ++it) {
    std::fill(colx.begin(), colx.end(), 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) colx[j] = std::max(colx[j], std::fabs(P[(size_t)i * n + j]));
    for (int i = 0; i < m; ++i) {
      double r = 0.0;
      for (int j = 0; j < n; ++j) {
        const double v = std::fabs(A[(size_t)i * n + j]);
        colx[j] = std::max(colx[j], v);
        r = std::max(r, v);
      }
      colz[i] = r;
    }
    for (int j = 0; j < n; ++j) dd[j] = clip_scale(colx[j]);
    for (int i = 0; i < m; ++i) de[i] = clip_scale(colz[i]);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) P[(size_t)i * n + j] = dd[i] * P[(size_t)i * n + j] * dd[j];
    for (int i = 0; i < n; ++i) q[i] = dd[i] * q[i];
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = de[i] * A[(size_t)i * n + j] * dd[j];
    for (int j = 0; j < n; ++j) D[j] *= dd[j];
    for (int i = 0; i < m; ++i) E[i] *= de[i];
    // cost scaling
    std::fill(colx.begin(), colx.end(), 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) colx[j] = std::max(colx[j], std::fabs(P[(size_t)i * n + j]));
    double mean = 0.0, qn = 0.0;
    for (int j = 0; j < n; ++j) mean += colx[j];
    mean /= n;
    for (int i = 0; i < n; ++i) qn = std::max(qn, std::fabs(q[i]));
    const double sc = std::max(mean, qn);
    double g = 1.0;
    if (sc > 0.0) {
      g = 1.0 / sc;
      g = g < 1e-4 ? 1e-4 : (g > 1e4 ? 1e4 : g);
    }
    for (auto& v : P) v *= g;
    for (auto& v : q) v *= g;
    c *= g;
  }
}

// Penalty grid (Sec. III-C): {rho0}, or n_rho log-spaced values; start at the value nearest
// rho0 in log distance (ties to the smaller value); geometric midpoints for the rounding rule.
void make_grid(const relu_qp_settings& s, std::vector<double>& grid, std::vector<double>& mid, int& j0) {
  grid.clear();
  mid.clear();
  if (s.n_rho == 1) {
    grid.push_back(s.rho0);
    j0 = 0;
  } else {
    const double lo = std::log10(s.rho_min), hi = std::log10(s.rho_max);
    for (int i = 0; i < s.n_rho; ++i) grid.push_back(std::pow(10.0, lo + i * (hi - lo) / (s.n_rho - 1)));
    j0 = 0;
    double best = std::fabs(std::log(grid[0]) - std::log(s.rho0));
    for (int i = 1; i < s.n_rho; ++i) {
      const double d = std::fabs(std::log(grid[i]) - std::log(s.rho0));
      if (d < best) {
        best = d;
        j0 = i;
      }
    }
  }
  for (size_t i = 0; i + 1 < grid.size(); ++i) mid.push_back(std::sqrt(grid[i] * grid[i + 1]));
  if (mid.empty()) mid.push_back(0.0);
}

int validate_bounds(int m, const double* l, const double* u) {
  for (int i = 0; i < m; ++i) {
    if (std::isnan(l[i]) || std::isnan(u[i])) return fail(RQP_EINVAL, "l[%d] or u[%d] is NaN", i, i);
    if (l[i] > u[i]) return fail(RQP_EINVAL, "l[%d] > u[%d]", i, i);
    if (l[i] == INFINITY || u[i] == -INFINITY) return fail(RQP_EINVAL, "row %d has an empty box", i);
  }
  return RQP_OK;
}

template <typename T>
int upload_vec(void* dst, const double* src, size_t count) {
  std::vector<T> tmp(count);
  for (size_t i = 0; i < count; ++i) tmp[i] = (T)src[i];
  HIP_OR_FAIL(hipMemcpy(dst, tmp.data(), count * sizeof(T), hipMemcpyHostToDevice));
  return RQP_OK;
}

int upload(relu_qp_handle* h, void* dst, const double* src, size_t count) {
  return h->esize == 8 ? upload_vec<double>(dst, src, count) : upload_vec<float>(dst, src, count);
}

hipError_t cast_dev(relu_qp_handle* h, long count, const double* x, void* y, hipStream_t st,
                    const double* f = nullptr, long period = 1) {
  return h->esize == 8 ? rqp::cast_from_f64<double>(count, x, static_cast<double*>(y), st, f, period)
                       : rqp::cast_from_f64<float>(count, x, static_cast<float*>(y), st, f, period);
}

// Forms the compact layer matrices [D_j, D_j A'; A D_j, A D_j A'] for every grid value and the
// check matrix [P, A'; A, 0] (Algorithm 1, "compute KKT inverse, W and b for each rho").
template <typename T>
int build_weights(relu_qp_handle* h, const double* P, const double* A, hipStream_t st) {
  const int n = h->n, m = h->m;
  DevBuf P_d, A_d, Gw, K, DAt, ADAt, work, omega, info;
  const size_t nn = (size_t)n * n, mn = (size_t)m * n, mm = (size_t)m * m;
  if (P_d.alloc(nn * 8) || A_d.alloc(mn * 8) || Gw.alloc(nn * 8) || K.alloc(nn * 8) || DAt.alloc(mn * 8) ||
      ADAt.alloc(mm * 8) || work.alloc((2 * 32 * (size_t)n + 32 * 32) * 8) || omega.alloc((size_t)m * 8) ||
      info.alloc(sizeof(int)))
    return fail(RQP_ENOMEM, "setup workspace allocation failed (n=%d, m=%d)", n, m);
  HIP_OR_FAIL(hipMemcpyAsync(P_d.p, P, nn * 8, hipMemcpyHostToDevice, st));
  HIP_OR_FAIL(hipMemcpyAsync(A_d.p, A, mn * 8, hipMemcpyHostToDevice, st));
  std::vector<double> om(m);
  for (int i = 0; i < m; ++i) om[i] = h->eq[i] ? h->s.rho_eq_scale : 1.0;
  HIP_OR_FAIL(hipMemcpyAsync(omega.p, om.data(), (size_t)m * 8, hipMemcpyHostToDevice, st));
  HIP_OR_FAIL(hipMemsetAsync(info.p, 0, sizeof(int), st));
  // Gw = A' diag(omega) A
  HIP_OR_FAIL(rqp::gemm_f64(n, n, m, 1.0, A_d.d(), 1, n, omega.d(), A_d.d(), n, 1, 0.0, Gw.d(), n, st));
  T* W = static_cast<T*>(h->W);
  for (size_t j = 0; j < h->grid.size(); ++j) {
    HIP_OR_FAIL(rqp::kkt_form_f64(n, P_d.d(), Gw.d(), h->s.sigma, h->grid[j], K.d(), st));
    HIP_OR_FAIL(rqp::spd_inverse_f64(n, K.d(), work.d(), static_cast<int*>(info.p), st));
    // D A'  (n x m) and A D A' (m x m)
    HIP_OR_FAIL(rqp::gemm_f64(n, m, n, 1.0, K.d(), n, 1, nullptr, A_d.d(), 1, n, 0.0, DAt.d(), m, st));
    HIP_OR_FAIL(rqp::gemm_f64(m, m, n, 1.0, A_d.d(), n, 1, nullptr, DAt.d(), m, 1, 0.0, ADAt.d(), m, st));
    HIP_OR_FAIL(rqp::assemble_layer<T>(n, m, K.d(), DAt.d(), ADAt.d(), W + (long)j * h->w_stride, h->ldw, st));
  }
  HIP_OR_FAIL(rqp::assemble_check<T>(n, m, P_d.d(), A_d.d(), static_cast<T*>(h->C), h->ldw, st));
  int hinfo = 0;
  HIP_OR_FAIL(hipMemcpyAsync(&hinfo, info.p, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_OR_FAIL(hipStreamSynchronize(st));
  if (hinfo) return fail(RQP_ENOTPD, "P + sigma I + A' diag(rho) A is not positive definite");
  return RQP_OK;
}

rqp::LaunchPlan make_plan(const relu_qp_handle* h, int grid, bool xt) {
  return h->esize == 8 ? rqp::plan_layer<double>(h->L, grid, xt) : rqp::plan_layer<float>(h->L, grid, xt);
}

// Every workgroup's share of the check's x rows fits the kernel's buffers (kMaxCheckRows; true
// whenever a workgroup owns at most kMaxRows layer rows, checked once per grid).
bool check_split_fits(int n, int m, int grid) {
  int prev = rqp::check_split(0, grid, n, m, n + m);
  for (int g = 1; g <= grid; ++g) {
    const int next = rqp::check_split(g, grid, n, m, n + m);
    if (next < prev || next - prev > rqp::kMaxCheckRows) return false;
    prev = next;
  }
  return prev == n;
}

// An explicit launch shape for every persistent launch of the handle: at least one row and at
// most kMaxRows rows per workgroup, within the cooperative limit.
int set_grid(relu_qp_handle* h, int grid) {
  const int need = (h->L + rqp::kMaxRows - 1) / rqp::kMaxRows;
  const int top = h->L < 256 ? h->L : 256;  // the check gathers at most 8 * 256 norm partials
  if (grid < need || grid > top) return fail(RQP_EINVAL, "grid %d outside [%d, %d]", grid, need, top);
  if (!check_split_fits(h->n, h->m, grid)) return fail(RQP_EINVAL, "grid %d: check split does not fit", grid);
  rqp::LaunchPlan p = make_plan(h, grid, false), px = make_plan(h, grid, true);
  if (!p.fn || !px.fn) return fail(RQP_EHIP, "no kernel resources for n + m = %d", h->L);
  const int lim = p.max_grid < px.max_grid ? p.max_grid : px.max_grid;
  if (grid > lim) return fail(RQP_EINVAL, "grid %d exceeds the cooperative limit %d", grid, lim);
  h->plan = p;
  h->plan_xt = px;
  h->grid_wg = grid;
  h->grid_plain = grid;
  h->small = false;
  return RQP_OK;
}

// Rows per workgroup that plain solves aim at: few workgroups (exchange participants), but never
// more rows than a workgroup holds on chip (measured best at 2400 and 3200 rows in FP32).
constexpr double kPlainRowsPerGroup = 12.5;

int choose_grid(relu_qp_handle* h) {
  int cus = 0, dev = 0;
  HIP_OR_FAIL(hipGetDevice(&dev));
  HIP_OR_FAIL(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int need = (h->L + rqp::kMaxRows - 1) / rqp::kMaxRows;
  int g = cus < h->L ? cus : h->L;
  if (g > 256) g = 256;
  if (g < need) g = need;
  const int rc = set_grid(h, g);  // closed loops and scaled problems: one workgroup per CU
  if (rc != RQP_OK) return rc;
  // plain solves: about kPlainRowsPerGroup rows per workgroup, at most the rows the kernel keeps
  // on chip (registers + LDS), and at most the grid above
  const double on_chip = (double)(h->plan.reg_rows + h->plan.lds_rows);
  int gp = (int)std::ceil(h->L / std::min(kPlainRowsPerGroup, on_chip));
  if (gp > g) gp = g;
  if (gp < need) gp = need;
  if (gp != g) {
    const rqp::LaunchPlan p = make_plan(h, gp, false);
    if (p.fn && gp <= p.max_grid && check_split_fits(h->n, h->m, gp)) {
      h->plan = p;
      h->grid_plain = gp;
    }
  }
  if (h->L > rqp::kSmallRows) return RQP_OK;
  const hipError_t e = h->esize == 8 ? rqp::prepare_small<double>(h->L) : rqp::prepare_small<float>(h->L);
  if (e != hipSuccess) return fail(RQP_EHIP, "single-workgroup kernel: %s", hipGetErrorString(e));
  h->small = true;
  return RQP_OK;
}

int alloc_exchange(relu_qp_handle* h) {
  const size_t words = h->esize == 8 ? 2 : 1;
  h->xw_words = 2 * (size_t)h->L * words;
  h->xn_words = 2 * (size_t)h->L * 8 * 2;  // any grid has at most L workgroups
  HIP_OR_FAIL(dmalloc(h, &h->xw, h->xw_words * 8));
  HIP_OR_FAIL(dmalloc(h, &h->xc, h->xw_words * 8));
  HIP_OR_FAIL(dmalloc(h, &h->xn, h->xn_words * 8));
  HIP_OR_FAIL(dmalloc(h, &h->xu, (size_t)2 * rqp::kMaxPlant * 2 * 8));
  HIP_OR_FAIL(hipMemset(h->xu, 0, (size_t)2 * rqp::kMaxPlant * 2 * 8));
  HIP_OR_FAIL(dmalloc(h, &h->xpl, (size_t)2 * rqp::kMaxGrid * rqp::kMaxPlant * 8));
  HIP_OR_FAIL(dmalloc(h, &h->axs, (size_t)h->m * 8));
  HIP_OR_FAIL(hipMemset(h->axs, 0, (size_t)h->m * 8));
  HIP_OR_FAIL(hipMemset(h->xw, 0, h->xw_words * 8));
  HIP_OR_FAIL(hipMemset(h->xc, 0, h->xw_words * 8));
  HIP_OR_FAIL(hipMemset(h->xn, 0, h->xn_words * 8));
  h->tag = 1;
  return RQP_OK;
}


// Padded rows of the batched engine's FP64 check matrix: its constraint-row tiles (128 rows)
// start at row n, so rows up to L + 127 are read.
size_t check_rows(size_t L) { return (L + 127) / 128 * 128 + 128; }

bool is_batched(const relu_qp_settings& s) {
  return s.engine == RQP_ENGINE_BATCH || (s.engine == RQP_ENGINE_AUTO && (s.batch > 1 || s.precision == RQP_BF16X3));
}

int upload_f32(float* dst, const double* src, size_t count) { return upload_vec<float>(dst, src, count); }

// Layer matrices for the batched engine (FP32 or BF16 high/low, rows padded to ldk) from P and A,
// and the FP64 check matrix from P0 and A0 (the original problem when P and A are scaled).
int build_batch_weights(relu_qp_handle* h, const double* P, const double* A, const double* P0, const double* A0,
                        hipStream_t st) {
  const int n = h->n, m = h->m, L = h->L;
  DevBuf P_d, A_d, Gw, K, DAt, ADAt, work, omega, info, Wd;
  const size_t nn = (size_t)n * n, mn = (size_t)m * n, mm = (size_t)m * m, LL = (size_t)L * L;
  if (P_d.alloc(nn * 8) || A_d.alloc(mn * 8) || Gw.alloc(nn * 8) || K.alloc(nn * 8) || DAt.alloc(mn * 8) ||
      ADAt.alloc(mm * 8) || work.alloc((2 * 32 * (size_t)n + 32 * 32) * 8) || omega.alloc((size_t)m * 8) ||
      info.alloc(sizeof(int)) || Wd.alloc(LL * 8))
    return fail(RQP_ENOMEM, "setup workspace allocation failed (n=%d, m=%d)", n, m);
  HIP_OR_FAIL(hipMemcpyAsync(P_d.p, P, nn * 8, hipMemcpyHostToDevice, st));
  HIP_OR_FAIL(hipMemcpyAsync(A_d.p, A, mn * 8, hipMemcpyHostToDevice, st));
  std::vector<double> om(m);
  for (int i = 0; i < m; ++i) om[i] = h->eq[i] ? h->s.rho_eq_scale : 1.0;
  HIP_OR_FAIL(hipMemcpyAsync(omega.p, om.data(), (size_t)m * 8, hipMemcpyHostToDevice, st));
  HIP_OR_FAIL(hipMemsetAsync(info.p, 0, sizeof(int), st));
  HIP_OR_FAIL(rqp::gemm_f64(n, n, m, 1.0, A_d.d(), 1, n, omega.d(), A_d.d(), n, 1, 0.0, Gw.d(), n, st));
  const size_t es = h->bprec == rqp::kBatchBF16x3 ? 2 : 4;
  for (size_t j = 0; j < h->grid.size(); ++j) {
    HIP_OR_FAIL(rqp::kkt_form_f64(n, P_d.d(), Gw.d(), h->s.sigma, h->grid[j], K.d(), st));
    HIP_OR_FAIL(rqp::spd_inverse_f64(n, K.d(), work.d(), static_cast<int*>(info.p), st));
    HIP_OR_FAIL(rqp::gemm_f64(n, m, n, 1.0, K.d(), n, 1, nullptr, A_d.d(), 1, n, 0.0, DAt.d(), m, st));
    HIP_OR_FAIL(rqp::gemm_f64(m, m, n, 1.0, A_d.d(), n, 1, nullptr, DAt.d(), m, 1, 0.0, ADAt.d(), m, st));
    HIP_OR_FAIL(rqp::assemble_layer<double>(n, m, K.d(), DAt.d(), ADAt.d(), Wd.d(), L, st));
    const size_t off = j * (size_t)h->w_stride * es;
    if (h->bprec == rqp::kBatchBF16x3)
      HIP_OR_FAIL(rqp::split_bf16(L, L, Wd.d(), L, static_cast<char*>(h->bWa) + off, static_cast<char*>(h->bWb) + off,
                                  h->lpad, h->ldk, st));
    else
      HIP_OR_FAIL(rqp::pad_f32(L, L, Wd.d(), L, reinterpret_cast<float*>(static_cast<char*>(h->bWa) + off), h->lpad,
                               h->ldk, st));
  }
  // the check matrix stays FP64 (the residuals are FP64 evaluations of the iterates)
  if (P0 != P) HIP_OR_FAIL(hipMemcpyAsync(P_d.p, P0, nn * 8, hipMemcpyHostToDevice, st));
  if (A0 != A) HIP_OR_FAIL(hipMemcpyAsync(A_d.p, A0, mn * 8, hipMemcpyHostToDevice, st));
  HIP_OR_FAIL(rqp::assemble_check<double>(n, m, P_d.d(), A_d.d(), Wd.d(), L, st));
  HIP_OR_FAIL(rqp::pad_f64(L, L, Wd.d(), L, h->bCd, h->cpad, h->ldk, st));
  int hinfo = 0;
  HIP_OR_FAIL(hipMemcpyAsync(&hinfo, info.p, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_OR_FAIL(hipStreamSynchronize(st));
  if (hinfo) return fail(RQP_ENOTPD, "P + sigma I + A' diag(rho) A is not positive definite");
  return RQP_OK;
}

int autotune_tiles(relu_qp_handle* h, hipStream_t st);
int launch_batched(relu_qp_handle* h, int steps, hipStream_t st, relu_qp_result* out, bool copy_out,
                   bool fixed_iters = false);

int setup_batched(relu_qp_handle* h, const double* P, const double* q, const double* A, const double* l,
                  const double* u, const double* P0, const double* A0, hipStream_t st) {
  const int n = h->n, m = h->m, L = h->L, B = h->batch;
  h->batched = true;
  h->bprec = h->s.precision == RQP_BF16X3 ? rqp::kBatchBF16x3 : rqp::kBatchF32;
  // rows padded to a multiple of the K stage plus four stages (the GEMM may run up to three
  // stages past the end, into zeros)
  h->ldk = (L + rqp::kTileK - 1) / rqp::kTileK * rqp::kTileK + 4 * rqp::kTileK;
  h->lpad = (L + rqp::kTileN - 1) / rqp::kTileN * rqp::kTileN;
  h->cpad = check_rows(L);
  // list positions of a tile may run up to kTileM past the last running instance
  h->bpad = ((long)B + rqp::kTileM - 1) / rqp::kTileM * rqp::kTileM + rqp::kTileM;
  h->w_stride = h->lpad * h->ldk;
  // the kernel forms state and operand offsets in 32 bits
  if ((double)B * (n > m ? n : m) * 8 >= 4294967296.0 || (double)h->bpad * h->ldk * 8 >= 4294967296.0)
    return fail(RQP_EINVAL, "batch %d with n=%d, m=%d exceeds the batched engine's 4 GiB arrays", B, n, m);
  const size_t es = h->bprec == rqp::kBatchBF16x3 ? 2 : 4;
  const size_t nr = h->grid.size();
  const size_t wbytes = nr * (size_t)h->w_stride * es, cbytes = (size_t)h->cpad * h->ldk * 8;
  const size_t vbytes = (size_t)h->bpad * h->ldk * es, cvbytes = 2 * (size_t)h->bpad * h->ldk * 8;
  const size_t ntile_max = (size_t)B / rqp::kTileM + nr + 1;
  auto al = [h](void** p, size_t bytes) { return dmalloc(h, p, bytes) == hipSuccess; };
  const bool two = h->bprec == rqp::kBatchBF16x3;
  if (!al(&h->bWa, wbytes) || (two && !al(&h->bWb, wbytes)) || !al((void**)&h->bCd, cbytes) ||
      !al((void**)&h->bX, (size_t)B * n * 4) || !al((void**)&h->bZ, (size_t)B * m * 4) ||
      !al((void**)&h->bY, (size_t)B * m * 4) || !al(&h->bVa, 2 * vbytes) || (two && !al(&h->bVb, 2 * vbytes)) ||
      !al((void**)&h->bCVd, cvbytes) || !al((void**)&h->bRpx, (size_t)B * n * 8) ||
      !al((void**)&h->bRaty, (size_t)B * n * 8) || !al((void**)&h->bjb, (size_t)B * 4) ||
      !al((void**)&h->bnorms, (size_t)B * 8 * 8) || !al((void**)&h->blists, (size_t)B * 4) ||
      !al((void**)&h->bpos, (size_t)B * 4) ||
      !al((void**)&h->bmtiles, (1 + 3 * ntile_max) * 4) || !al((void**)&h->bbar, 1024 * 4) ||
      !al(&h->q, (size_t)B * n * 4) || !al(&h->l, (size_t)B * m * 4) || !al(&h->u, (size_t)B * m * 4) ||
      !al((void**)&h->bstatus, (size_t)B * 4) || !al((void**)&h->biter, (size_t)B * 4) ||
      !al((void**)&h->bstage, ((size_t)n + m + 1) * 4)) {
    (void)hipGetLastError();
    return fail(RQP_ENOMEM, "device allocation failed (batch %d, n=%d, m=%d)", B, n, m);
  }
  // operand padding columns must read as zero
  HIP_OR_FAIL(hipMemset(h->bVa, 0, 2 * vbytes));
  if (two) HIP_OR_FAIL(hipMemset(h->bVb, 0, 2 * vbytes));
  HIP_OR_FAIL(hipMemset(h->bCVd, 0, cvbytes));
  HIP_OR_FAIL(hipMemset(h->bnorms, 0, (size_t)B * 64));
  HIP_OR_FAIL(hipMemset(h->biter, 0, (size_t)B * 4));
  HIP_OR_FAIL(hipMemset(h->bX, 0, (size_t)B * n * 4));
  HIP_OR_FAIL(hipMemset(h->bZ, 0, (size_t)B * m * 4));
  HIP_OR_FAIL(hipMemset(h->bY, 0, (size_t)B * m * 4));
  HIP_OR_FAIL(rqp::fill_status(B, rqp::kSlotIdle, h->bstatus, st));
  std::vector<int> j0(B, h->j0);
  HIP_OR_FAIL(hipMemcpy(h->bjb, j0.data(), (size_t)B * 4, hipMemcpyHostToDevice));
  int rc;
  if ((rc = upload_f32(static_cast<float*>(h->q), q, (size_t)B * n)) ||
      (rc = upload_f32(static_cast<float*>(h->l), l, (size_t)B * m)) ||
      (rc = upload_f32(static_cast<float*>(h->u), u, (size_t)B * m)))
    return rc;
  if ((rc = build_batch_weights(h, P, A, P0, A0, st))) return rc;
  for (int v = 0; v < rqp::kTileShapes; ++v) {
    h->bplans[v] = rqp::plan_batch(h->bprec, rqp::kTileRows[v]);
    if (!h->bplans[v].fn) return fail(RQP_EHIP, "no resources for the batched kernel (%d-row tiles)", rqp::kTileRows[v]);
  }
  h->bplan = h->bplans[0];
  return autotune_tiles(h, st);
}

// One persistent launch of the batched kernel over every running or admitted slot, for at most
// `steps` iterations, then copies of the slot results into out. fixed_iters: no instance stops
// at a check (every one runs all `steps` iterations, as the timing of the autotuner needs).
int launch_batched(relu_qp_handle* h, int steps, hipStream_t st, relu_qp_result* out, bool copy_out,
                   bool fixed_iters) {
  const int B = h->batch;
  HIP_OR_FAIL(hipMemsetAsync(h->bbar, 0, 1024 * 4, st));
  __atomic_store_n(h->abort_h, 0, __ATOMIC_SEQ_CST);
  rqp::BatchArgs a{};
  a.n = h->n;
  a.m = h->m;
  a.L = h->L;
  a.B = B;
  a.ldk = h->ldk;
  a.lpad = h->lpad;
  a.cpad = h->cpad;
  a.bpad = h->bpad;
  a.prec = h->bprec;
  a.Wa = h->bWa;
  a.Wb = h->bWb;
  a.w_stride = h->w_stride;
  a.Cd = h->bCd;
  a.Q = static_cast<const float*>(h->q);
  a.Lo = static_cast<const float*>(h->l);
  a.Up = static_cast<const float*>(h->u);
  a.scl = h->scl;
  a.eq = h->eq_d;
  a.grid = h->grid_d;
  a.mid = h->mid_d;
  a.n_rho = (int)h->grid.size();
  a.sigma = h->s.sigma;
  a.alpha = h->s.alpha;
  a.eps_abs = h->s.eps_abs;
  a.eps_rel = h->s.eps_rel;
  a.rho_eq_scale = h->s.rho_eq_scale;
  // fixed_iters: no instance stops before the launch's last iteration (not even at max_iter)
  a.max_iter = fixed_iters && steps > h->s.max_iter ? steps : h->s.max_iter;
  a.check_interval = h->s.check_interval;
  a.terminate = !fixed_iters && !(h->s.eps_abs == 0.0 && h->s.eps_rel == 0.0);
  a.j0 = h->j0;
  a.steps = steps;
  a.X = h->bX;
  a.Z = h->bZ;
  a.Y = h->bY;
  a.Va = h->bVa;
  a.Vb = h->bVb;
  a.CVd = h->bCVd;
  a.Rpx = h->bRpx;
  a.Raty = h->bRaty;
  a.jb = h->bjb;
  a.status = h->bstatus;
  a.iterations = h->biter;
  a.rho_hist = out->rho_hist;
  a.prim_res = out->prim_res;
  a.dual_res = out->dual_res;
  a.max_checks = h->s.max_iter / h->s.check_interval + (h->s.max_iter % h->s.check_interval ? 1 : 0);
  a.norms = h->bnorms;
  a.lists = h->blists;
  a.pos_of = h->bpos;
  a.mtiles = h->bmtiles;
  a.bar = h->bbar;
  a.abort_flag = h->abort_d;
  hipError_t e = rqp::launch_batch(a, h->bplan, st);
  if (e != hipSuccess) return fail(RQP_EHIP, "batched launch failed: %s", hipGetErrorString(e));
  if (!copy_out) return RQP_OK;
  if (h->scl) {
    HIP_OR_FAIL(rqp::unscale_outputs(B, h->n, h->m, h->bX, h->bZ, h->bY, h->scl, static_cast<float*>(out->x),
                                     static_cast<float*>(out->z), static_cast<float*>(out->y), st));
  } else {
    HIP_OR_FAIL(hipMemcpyAsync(out->x, h->bX, (size_t)B * h->n * 4, hipMemcpyDeviceToDevice, st));
    HIP_OR_FAIL(hipMemcpyAsync(out->z, h->bZ, (size_t)B * h->m * 4, hipMemcpyDeviceToDevice, st));
    HIP_OR_FAIL(hipMemcpyAsync(out->y, h->bY, (size_t)B * h->m * 4, hipMemcpyDeviceToDevice, st));
  }
  HIP_OR_FAIL(hipMemcpyAsync(out->rho_index, h->bjb, (size_t)B * 4, hipMemcpyDeviceToDevice, st));
  HIP_OR_FAIL(hipMemcpyAsync(out->status, h->bstatus, (size_t)B * 4, hipMemcpyDeviceToDevice, st));
  HIP_OR_FAIL(hipMemcpyAsync(out->iterations, h->biter, (size_t)B * 4, hipMemcpyDeviceToDevice, st));
  return RQP_OK;
}

// Autotuner of the batched GEMM's tile shape (128 or 64 matrix rows per tile): each shape runs
// two check intervals of every slot from a cold start on the handle's own data, timed with HIP
// events; the faster one is kept. Slots, statuses and state are reset to idle afterwards. The
// shapes agree to rounding (every accumulator element sees the same products, in another
// interleaving on the matrix cores): few tiles (small batches) favour 64 rows, many 128.
// The choice is cached per process and device for the problem shape (n, m, batch, precision,
// penalties): a family loaded again (or another handle of the same shape) takes the cached
// choice and timings without timing again.
struct TileKey {
  int dev, n, m, B, prec, n_rho;
  bool operator<(const TileKey& o) const {
    return std::tie(dev, n, m, B, prec, n_rho) < std::tie(o.dev, o.n, o.m, o.B, o.prec, o.n_rho);
  }
};
struct TileChoice {
  int best;
  double us[rqp::kTileShapes];
};
std::mutex g_tile_mu;
std::map<TileKey, TileChoice> g_tile_cache;

// The shape with the fewest microseconds per iteration; a later candidate must be faster by more
// than 1 % (about the spread of repeated timings) to replace an earlier one, so near-ties go to
// the earlier shape in the candidate order (128, 64, 256 rows).
int best_tile(const relu_qp_handle* h) {
  int best = 0;
  for (int v = 1; v < rqp::kTileShapes; ++v)
    if (h->tile_us[v] < 0.99 * h->tile_us[best]) best = v;
  return best;
}

int autotune_tiles(relu_qp_handle* h, hipStream_t st) {
  const int B = h->batch, steps = 2 * h->s.check_interval;
  const TileKey key{h->device, h->n, h->m, B, h->bprec, (int)h->grid.size()};
  {
    std::lock_guard<std::mutex> lock(g_tile_mu);
    const auto it = g_tile_cache.find(key);
    if (it != g_tile_cache.end()) {
      for (int v = 0; v < rqp::kTileShapes; ++v) h->tile_us[v] = it->second.us[v];
      h->bplan = h->bplans[it->second.best];
      h->tile_cached = true;
      return RQP_OK;
    }
  }
  hipEvent_t e0, e1;
  HIP_OR_FAIL(hipEventCreate(&e0));
  HIP_OR_FAIL(hipEventCreate(&e1));
  relu_qp_result tmp{h->bX, h->bY, h->bZ, h->biter, h->bstatus, h->bjb, nullptr, nullptr, nullptr};
  int rc = RQP_OK;
  for (int v = 0; v < rqp::kTileShapes && rc == RQP_OK; ++v) {
    h->bplan = h->bplans[v];
    float best = 1e30f;
    for (int rep = 0; rep < 2 && rc == RQP_OK; ++rep) {  // the first run also warms caches
      if (hipSuccess != rqp::fill_status(B, rqp::kSlotAdmitCold, h->bstatus, st) ||
          hipSuccess != hipEventRecord(e0, st)) {
        rc = fail(RQP_EHIP, "autotuner launch failed");
        break;
      }
      rc = launch_batched(h, steps, st, &tmp, /*copy_out=*/false, /*fixed_iters=*/true);
      if (rc) break;
      float ms = 0.0f;
      if (hipSuccess != hipEventRecord(e1, st) || hipSuccess != hipEventSynchronize(e1) ||
          hipSuccess != hipEventElapsedTime(&ms, e0, e1)) {
        rc = fail(RQP_EHIP, "autotuner timing failed");
        break;
      }
      best = ms < best ? ms : best;
    }
    h->tile_us[v] = best * 1e3 / steps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  const int best = best_tile(h);
  h->bplan = h->bplans[best];
  {
    std::lock_guard<std::mutex> lock(g_tile_mu);
    TileChoice c{best, {}};
    for (int v = 0; v < rqp::kTileShapes; ++v) c.us[v] = h->tile_us[v];
    g_tile_cache[key] = c;
  }
  // back to idle slots with a zero state
  std::vector<int> j0(B, h->j0);
  HIP_OR_FAIL(rqp::fill_status(B, rqp::kSlotIdle, h->bstatus, st));
  HIP_OR_FAIL(hipMemsetAsync(h->biter, 0, (size_t)B * 4, st));
  HIP_OR_FAIL(hipMemsetAsync(h->bX, 0, (size_t)B * h->n * 4, st));
  HIP_OR_FAIL(hipMemsetAsync(h->bZ, 0, (size_t)B * h->m * 4, st));
  HIP_OR_FAIL(hipMemsetAsync(h->bY, 0, (size_t)B * h->m * 4, st));
  HIP_OR_FAIL(hipMemcpyAsync(h->bjb, j0.data(), (size_t)B * 4, hipMemcpyHostToDevice, st));
  HIP_OR_FAIL(hipStreamSynchronize(st));
  return RQP_OK;
}

int solve_batched(relu_qp_handle* h, hipStream_t st, relu_qp_result* out) {
  const bool warm = h->warm_pending || (h->warm_mode && h->have_prev);
  HIP_OR_FAIL(rqp::fill_status(h->batch, warm ? rqp::kSlotAdmitWarm : rqp::kSlotAdmitCold, h->bstatus, st));
  const int rc = launch_batched(h, h->s.max_iter, st, out, true);
  if (rc) return rc;
  h->warm_pending = false;
  h->have_prev = true;
  return RQP_OK;
}

// Host slot list -> chunks of at most kMaxSlotsPerCall passed by value.
template <typename F>
int for_slot_chunks(relu_qp_handle* h, const int* slots, int n_slots, F&& f) {
  if (!h->batched) return fail(RQP_ESTATE, "slots exist only with the batched engine");
  if (n_slots < 0 || (n_slots > 0 && !slots)) return fail(RQP_EINVAL, "bad slot list");
  std::vector<char> seen(h->batch, 0);
  for (int i = 0; i < n_slots; ++i) {
    if (slots[i] < 0 || slots[i] >= h->batch) return fail(RQP_EINVAL, "slot %d out of range [0, %d)", slots[i], h->batch);
    if (seen[slots[i]]++) return fail(RQP_EINVAL, "slot %d listed twice", slots[i]);
  }
  for (int i0 = 0; i0 < n_slots; i0 += rqp::kMaxSlotsPerCall) {
    rqp::SlotList sl{};
    sl.n = std::min(rqp::kMaxSlotsPerCall, n_slots - i0);
    for (int k = 0; k < sl.n; ++k) sl.s[k] = slots[i0 + k];
    const int rc = f(sl, i0);
    if (rc) return rc;
  }
  return RQP_OK;
}

}  // namespace

extern "C" {

void relu_qp_default_settings(relu_qp_settings* s) {
  if (!s) return;
  s->sigma = 1e-6;
  s->alpha = 1.6;
  s->rho0 = 0.1;
  s->n_rho = 1;
  s->rho_min = 1e-3;
  s->rho_max = 1e3;
  s->rho_eq_scale = 1e3;
  s->eps_abs = 1e-3;
  s->eps_rel = 1e-3;
  s->max_iter = 4000;
  s->check_interval = 25;
  s->precision = RQP_FP32;
  s->batch = 1;
  s->engine = RQP_ENGINE_AUTO;
  s->scaling = 0;
}

const char* relu_qp_last_error(void) { return g_last_error.c_str(); }

int relu_qp_setup(relu_qp_handle** hp, int n, int m, const double* P, const double* q, const double* A,
                  const double* l, const double* u, const relu_qp_settings* s, void* stream) {
  if (!hp) return fail(RQP_EINVAL, "handle pointer is NULL");
  *hp = nullptr;
  int rc = validate_settings(s);
  if (rc) return rc;
  if (n < 1 || m < 1) return fail(RQP_EINVAL, "need n >= 1 and m >= 1 (n=%d, m=%d)", n, m);
  if (!P || !q || !A || !l || !u) return fail(RQP_EINVAL, "NULL problem array");
  if ((long)n + m > 8L * rqp::kLayerBlock) return fail(RQP_EINVAL, "n + m = %ld exceeds %d", (long)n + m, 8 * rqp::kLayerBlock);
  double pmax = 0.0;
  for (long i = 0; i < (long)n * n; ++i) {
    if (!std::isfinite(P[i])) return fail(RQP_EINVAL, "P has a non-finite entry");
    pmax = std::fmax(pmax, std::fabs(P[i]));
  }
  for (int i = 0; i < n; ++i)
    for (int k = i + 1; k < n; ++k)
      if (std::fabs(P[(long)i * n + k] - P[(long)k * n + i]) > 1e-12 * (pmax > 0 ? pmax : 1.0))
        return fail(RQP_EINVAL, "P is not symmetric (%d, %d)", i, k);
  for (long i = 0; i < (long)m * n; ++i)
    if (!std::isfinite(A[i])) return fail(RQP_EINVAL, "A has a non-finite entry");
  const bool batched = is_batched(*s);
  const int B = s->batch;
  for (int b = 0; b < B; ++b) {
    rc = validate_bounds(m, l + (size_t)b * m, u + (size_t)b * m);
    if (rc) return rc;
    for (int i = 0; i < m; ++i)
      if ((l[(size_t)b * m + i] == u[(size_t)b * m + i]) != (l[i] == u[i]))
        return fail(RQP_EINVAL, "instance %d has another equality-row pattern (row %d)", b, i);
  }

  int dev = 0;
  HIP_OR_FAIL(hipGetDevice(&dev));
  rc = scratch_init(dev);
  if (rc) return rc;
  relu_qp_handle* h = new relu_qp_handle();
  h->device = dev;
  h->n = n;
  h->m = m;
  h->L = n + m;
  h->s = *s;
  h->batch = B;
  h->esize = s->precision == RQP_FP64 ? 8 : 4;
  h->ldw = (h->L + 3) / 4 * 4;  // 16-byte aligned rows
  h->w_stride = (long)h->L * h->ldw;
  make_grid(*s, h->grid, h->mid, h->j0);
  h->eq.resize(m);
  for (int i = 0; i < m; ++i) h->eq[i] = (l[i] == u[i]) ? 1 : 0;
  hipStream_t st = static_cast<hipStream_t>(stream);

  auto bail = [&](int code) {
    free_handle(h);
    return code;
  };
  const size_t nr = h->grid.size();
  if (dmalloc(h, &h->eq_d, (size_t)m) != hipSuccess || dmalloc(h, &h->grid_d, nr * 8) != hipSuccess ||
      dmalloc(h, &h->mid_d, h->mid.size() * 8) != hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(RQP_ENOMEM, "device allocation failed"));
  }
  if (hipHostMalloc(&h->abort_h, sizeof(int), hipHostMallocMapped) != hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(RQP_ENOMEM, "pinned allocation failed"));
  }
  *h->abort_h = 0;
  if (hipHostGetDevicePointer((void**)&h->abort_d, h->abort_h, 0) != hipSuccess)
    return bail(fail(RQP_EHIP, "hipHostGetDevicePointer failed"));
  if (hipMemcpy(h->eq_d, h->eq.data(), m, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->grid_d, h->grid.data(), nr * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->mid_d, h->mid.data(), h->mid.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(RQP_EHIP, "initial copies failed"));

  // Ruiz scaling: the device holds the scaled problem from here on (the batched engine's check
  // keeps the original P and A)
  const double *P0 = P, *A0 = A;
  std::vector<double> Ps, As, qs, ls, us;
  if (s->scaling > 0) {
    ruiz(n, m, P, q, B, A, s->scaling, h->sD, h->sE, h->sc);
    const std::vector<double>& D = h->sD;
    const std::vector<double>& E = h->sE;
    const double c = h->sc;
    Ps.resize((size_t)n * n);
    As.resize((size_t)m * n);
    qs.resize((size_t)B * n);
    ls.resize((size_t)B * m);
    us.resize((size_t)B * m);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) Ps[(size_t)i * n + j] = c * (D[i] * P[(size_t)i * n + j] * D[j]);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) As[(size_t)i * n + j] = E[i] * A[(size_t)i * n + j] * D[j];
    for (size_t b = 0; b < (size_t)B; ++b) {
      for (int i = 0; i < n; ++i) qs[b * n + i] = c * D[i] * q[b * n + i];
      for (int i = 0; i < m; ++i) {
        ls[b * m + i] = E[i] * l[b * m + i];
        us[b * m + i] = E[i] * u[b * m + i];
      }
    }
    P = Ps.data();
    A = As.data();
    q = qs.data();
    l = ls.data();
    u = us.data();
    std::vector<double> v(3 * ((size_t)n + m));
    for (int i = 0; i < n; ++i) {
      v[i] = c * D[i];
      v[(size_t)n + m + i] = 1.0 / (c * D[i]);
      v[2 * ((size_t)n + m) + i] = D[i];
    }
    for (int i = 0; i < m; ++i) {
      v[(size_t)n + i] = E[i];
      v[2 * (size_t)n + m + i] = 1.0 / E[i];
      v[3 * (size_t)n + 2 * m + i] = E[i] / c;
    }
    if (dmalloc(h, &h->scl, v.size() * 8) != hipSuccess ||
        hipMemcpy(h->scl, v.data(), v.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      return bail(fail(RQP_ENOMEM, "scaling vectors: device allocation failed"));
    }
  }
  if (batched) {
    if ((rc = setup_batched(h, P, q, A, l, u, P0, A0, st))) return bail(rc);
    *hp = h;
    return RQP_OK;
  }

  if (dmalloc(h, &h->W, nr * h->w_stride * h->esize) != hipSuccess ||
      dmalloc(h, &h->C, (size_t)h->w_stride * h->esize) != hipSuccess ||
      dmalloc(h, &h->q, (size_t)n * h->esize) != hipSuccess || dmalloc(h, &h->l, (size_t)m * h->esize) != hipSuccess ||
      dmalloc(h, &h->u, (size_t)m * h->esize) != hipSuccess || dmalloc(h, &h->xs, (size_t)n * h->esize) != hipSuccess ||
      dmalloc(h, &h->zs, (size_t)m * h->esize) != hipSuccess || dmalloc(h, &h->ys, (size_t)m * h->esize) != hipSuccess ||
      dmalloc(h, &h->js, sizeof(int)) != hipSuccess || dmalloc(h, &h->err, sizeof(unsigned)) != hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(RQP_ENOMEM, "device allocation failed (n=%d, m=%d, %zu penalties)", n, m, nr));
  }
  if ((rc = upload(h, h->q, q, n)) || (rc = upload(h, h->l, l, m)) || (rc = upload(h, h->u, u, m))) return bail(rc);
  if (hipMemset(h->xs, 0, (size_t)n * h->esize) != hipSuccess || hipMemset(h->zs, 0, (size_t)m * h->esize) != hipSuccess ||
      hipMemset(h->ys, 0, (size_t)m * h->esize) != hipSuccess || hipMemset(h->js, 0, sizeof(int)) != hipSuccess ||
      hipMemset(h->err, 0, sizeof(unsigned)) != hipSuccess)
    return bail(fail(RQP_EHIP, "initial copies failed"));

  rc = h->esize == 8 ? build_weights<double>(h, P, A, st) : build_weights<float>(h, P, A, st);
  if (rc) return bail(rc);
  if ((rc = choose_grid(h)) || (rc = alloc_exchange(h))) return bail(rc);
  *hp = h;
  return RQP_OK;
}

int relu_qp_update(relu_qp_handle* h, const double* q, const double* l, const double* u) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  DEVICE_OR_FAIL(h);
  if (h->batched) {
    const int B = h->batch, n = h->n, m = h->m;
    if ((l == nullptr) != (u == nullptr)) return fail(RQP_EINVAL, "the batched engine updates l and u together");
    if (l) {
      for (int b = 0; b < B; ++b) {
        int rc = validate_bounds(m, l + (size_t)b * m, u + (size_t)b * m);
        if (rc) return rc;
        for (int i = 0; i < m; ++i)
          if ((l[(size_t)b * m + i] == u[(size_t)b * m + i]) != (h->eq[i] != 0))
            return fail(RQP_EINVAL, "update changes the equality-row pattern (instance %d, row %d)", b, i);
      }
    }
    int rc;
    std::vector<double> qv, lv, uv;
    if (h->scl) {  // to scaled units: c D q, E l, E u
      if (q) {
        qv.resize((size_t)B * n);
        for (size_t b = 0; b < (size_t)B; ++b)
          for (int i = 0; i < n; ++i) qv[b * n + i] = h->sc * h->sD[i] * q[b * n + i];
        q = qv.data();
      }
      if (l) {
        lv.resize((size_t)B * m);
        uv.resize((size_t)B * m);
        for (size_t b = 0; b < (size_t)B; ++b)
          for (int i = 0; i < m; ++i) {
            lv[b * m + i] = h->sE[i] * l[b * m + i];
            uv[b * m + i] = h->sE[i] * u[b * m + i];
          }
        l = lv.data();
        u = uv.data();
      }
    }
    if (q && (rc = upload_f32(static_cast<float*>(h->q), q, (size_t)B * n))) return rc;
    if (l && ((rc = upload_f32(static_cast<float*>(h->l), l, (size_t)B * m)) ||
              (rc = upload_f32(static_cast<float*>(h->u), u, (size_t)B * m))))
      return rc;
    return RQP_OK;
  }
  std::vector<double> lv, uv;
  if (l || u) {
    lv.resize(h->m);
    uv.resize(h->m);
    std::vector<double> tmp(h->m);
    const size_t es = h->esize;
    // unchanged side comes from the device copy
    for (int side = 0; side < 2; ++side) {
      const double* src = side == 0 ? l : u;
      std::vector<double>& dst = side == 0 ? lv : uv;
      if (src) {
        std::memcpy(dst.data(), src, h->m * 8);
        if (h->scl)
          for (int i = 0; i < h->m; ++i) dst[i] *= h->sE[i];  // scaled rows (E > 0 keeps l <= u)
      } else {
        void* dev = side == 0 ? h->l : h->u;
        if (es == 8) {
          HIP_OR_FAIL(hipMemcpy(dst.data(), dev, h->m * 8, hipMemcpyDeviceToHost));
        } else {
          std::vector<float> f(h->m);
          HIP_OR_FAIL(hipMemcpy(f.data(), dev, h->m * 4, hipMemcpyDeviceToHost));
          for (int i = 0; i < h->m; ++i) dst[i] = f[i];
        }
      }
    }
    int rc = validate_bounds(h->m, lv.data(), uv.data());
    if (rc) return rc;
    for (int i = 0; i < h->m; ++i)
      if ((lv[i] == uv[i]) != (h->eq[i] != 0))
        return fail(RQP_EINVAL, "update changes the equality-row pattern at row %d", i);
  }
  int rc;
  // a non-finite q is accepted: the solve reports RQP_NONFINITE
  std::vector<double> qv;
  if (q && h->scl) {
    qv.resize(h->n);
    for (int i = 0; i < h->n; ++i) qv[i] = h->sc * h->sD[i] * q[i];
    q = qv.data();
  }
  if (q && (rc = upload(h, h->q, q, h->n))) return rc;
  if (l && (rc = upload(h, h->l, lv.data(), h->m))) return rc;
  if (u && (rc = upload(h, h->u, uv.data(), h->m))) return rc;
  return RQP_OK;
}

int relu_qp_update_device(relu_qp_handle* h, const double* q, const double* l, const double* u, void* stream) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  DEVICE_OR_FAIL(h);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long B = h->batch;
  // with Ruiz scaling: q <- c D q, l <- E l, u <- E u on the way
  const double* fq = h->scl;
  const double* fe = h->scl ? h->scl + h->n : nullptr;
  if (q) HIP_OR_FAIL(cast_dev(h, B * h->n, q, h->q, st, fq, h->n));
  if (l) HIP_OR_FAIL(cast_dev(h, B * h->m, l, h->l, st, fe, h->m));
  if (u) HIP_OR_FAIL(cast_dev(h, B * h->m, u, h->u, st, fe, h->m));
  return RQP_OK;
}

int relu_qp_set_parametric(relu_qp_handle* h, int nx, const double* F, const double* E, const double* lo,
                           const double* hi) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  DEVICE_OR_FAIL(h);
  if (nx < 1 || !F || !E || !lo || !hi) return fail(RQP_EINVAL, "bad parametric data");
  int rc = validate_bounds(h->m, lo, hi);
  if (rc) return rc;
  for (int i = 0; i < h->m; ++i)
    if ((lo[i] == hi[i]) != (h->eq[i] != 0)) return fail(RQP_EINVAL, "equality pattern of lo/hi differs at %d", i);
  for (void** p : {(void**)&h->F_d, (void**)&h->E_d, (void**)&h->lo_d, (void**)&h->hi_d})
    if (*p) dfree(h, p);
  h->nx = nx;
  HIP_OR_FAIL(dmalloc(h, &h->F_d, (size_t)h->n * nx * 8));
  HIP_OR_FAIL(dmalloc(h, &h->E_d, (size_t)h->m * nx * 8));
  HIP_OR_FAIL(dmalloc(h, &h->lo_d, (size_t)h->m * 8));
  HIP_OR_FAIL(dmalloc(h, &h->hi_d, (size_t)h->m * 8));
  std::vector<double> Fs, Es, los, his;
  if (h->scl) {  // scaled rows: q = (c D F) x0, l = E lo - (E E_x) x0, u likewise
    Fs.assign(F, F + (size_t)h->n * nx);
    Es.assign(E, E + (size_t)h->m * nx);
    los.assign(lo, lo + h->m);
    his.assign(hi, hi + h->m);
    for (int i = 0; i < h->n; ++i)
      for (int k = 0; k < nx; ++k) Fs[(size_t)i * nx + k] *= h->sc * h->sD[i];
    for (int i = 0; i < h->m; ++i) {
      for (int k = 0; k < nx; ++k) Es[(size_t)i * nx + k] *= h->sE[i];
      los[i] *= h->sE[i];
      his[i] *= h->sE[i];
    }
    F = Fs.data();
    E = Es.data();
    lo = los.data();
    hi = his.data();
  }
  HIP_OR_FAIL(hipMemcpy(h->F_d, F, (size_t)h->n * nx * 8, hipMemcpyHostToDevice));
  HIP_OR_FAIL(hipMemcpy(h->E_d, E, (size_t)h->m * nx * 8, hipMemcpyHostToDevice));
  HIP_OR_FAIL(hipMemcpy(h->lo_d, lo, (size_t)h->m * 8, hipMemcpyHostToDevice));
  HIP_OR_FAIL(hipMemcpy(h->hi_d, hi, (size_t)h->m * 8, hipMemcpyHostToDevice));
  return RQP_OK;
}

int relu_qp_update_x0_device(relu_qp_handle* h, const double* x0, void* stream) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  DEVICE_OR_FAIL(h);
  if (!h->F_d) return fail(RQP_ESTATE, "relu_qp_set_parametric has not been called");
  if (!x0) return fail(RQP_EINVAL, "x0 is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (h->batched)
    HIP_OR_FAIL(rqp::mpc_vectors_tiled<float>(h->batch, h->n, h->m, h->nx, h->F_d, h->E_d, h->lo_d, h->hi_d, x0,
                                              static_cast<float*>(h->q), static_cast<float*>(h->l),
                                              static_cast<float*>(h->u), st));
  else if (h->esize == 8)
    HIP_OR_FAIL(rqp::mpc_vectors<double>(h->batch, h->n, h->m, h->nx, h->F_d, h->E_d, h->lo_d, h->hi_d, x0,
                                         static_cast<double*>(h->q), static_cast<double*>(h->l),
                                         static_cast<double*>(h->u), st));
  else
    HIP_OR_FAIL(rqp::mpc_vectors<float>(h->batch, h->n, h->m, h->nx, h->F_d, h->E_d, h->lo_d, h->hi_d, x0,
                                        static_cast<float*>(h->q), static_cast<float*>(h->l),
                                        static_cast<float*>(h->u), st));
  return RQP_OK;
}

int relu_qp_warm_start(relu_qp_handle* h, const double* x, const double* y, int rho_index) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  DEVICE_OR_FAIL(h);
  if (!x || !y) return fail(RQP_EINVAL, "x or y is NULL");
  if (rho_index < 0 || rho_index >= (int)h->grid.size()) return fail(RQP_EINVAL, "rho_index out of range");
  int rc;
  if (h->batched) {
    const int B = h->batch, n = h->n, m = h->m;
    std::vector<double> xv, yv;
    if (h->scl) {  // to scaled units: xb = x / D, yb = c y / E
      xv.resize((size_t)B * n);
      yv.resize((size_t)B * m);
      for (size_t b = 0; b < (size_t)B; ++b) {
        for (int i = 0; i < n; ++i) xv[b * n + i] = x[b * n + i] / h->sD[i];
        for (int i = 0; i < m; ++i) yv[b * m + i] = h->sc * y[b * m + i] / h->sE[i];
      }
      x = xv.data();
      y = yv.data();
    }
    if ((rc = upload_f32(h->bX, x, (size_t)B * n)) || (rc = upload_f32(h->bY, y, (size_t)B * m))) return rc;
    std::vector<int> jv(B, rho_index);
    HIP_OR_FAIL(hipMemcpy(h->bjb, jv.data(), (size_t)B * 4, hipMemcpyHostToDevice));
    h->warm_pending = true;
    return RQP_OK;
  }
  std::vector<double> xv, yv;
  if (h->scl) {  // to scaled units: xb = x / D, yb = c y / E
    xv.resize(h->n);
    yv.resize(h->m);
    for (int i = 0; i < h->n; ++i) xv[i] = x[i] / h->sD[i];
    for (int i = 0; i < h->m; ++i) yv[i] = h->sc * y[i] / h->sE[i];
    x = xv.data();
    y = yv.data();
  }
  if ((rc = upload(h, h->xs, x, h->n)) || (rc = upload(h, h->ys, y, h->m))) return rc;
  HIP_OR_FAIL(hipMemcpy(h->js, &rho_index, sizeof(int), hipMemcpyHostToDevice));
  h->warm_pending = true;
  return RQP_OK;
}

int relu_qp_set_warm(relu_qp_handle* h, int enabled) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  h->warm_mode = enabled != 0;
  return RQP_OK;
}

}  // extern "C"

namespace {
// One persistent launch of `count` solves of the online loop; with x0 (count x nx), each solve
// first forms its q, l, u from its own initial state.
// A closed loop's plant and trajectory buffers (device, FP64).
struct ClosedLoop {
  const double* Ad;
  const double* Bd;
  int nu;
  double* traj_x;
  double* traj_u;
};

// Arguments of a single-instance launch from the handle (its exchange words and tag).
rqp::LayerArgs layer_args(relu_qp_handle* h, const double* x0, int count, relu_qp_result* out,
                          const ClosedLoop* cl) {
  rqp::LayerArgs a{};
  a.n = h->n;
  a.m = h->m;
  a.L = h->L;
  a.ldw = h->ldw;
  a.W = h->W;
  a.w_stride = h->w_stride;
  a.C = h->C;
  a.q = h->q;
  a.l = h->l;
  a.u = h->u;
  a.eq = h->eq_d;
  a.grid = h->grid_d;
  a.mid = h->mid_d;
  a.n_rho = (int)h->grid.size();
  a.sigma = h->s.sigma;
  a.alpha = h->s.alpha;
  a.eps_abs = h->s.eps_abs;
  a.eps_rel = h->s.eps_rel;
  a.rho_eq_scale = h->s.rho_eq_scale;
  a.max_iter = h->s.max_iter;
  a.check_interval = h->s.check_interval;
  a.terminate = !(h->s.eps_abs == 0.0 && h->s.eps_rel == 0.0);
  a.warm = (h->warm_pending || (h->warm_mode && h->have_prev)) ? 1 : 0;
  a.j0 = h->j0;
  a.xs = h->xs;
  a.zs = h->zs;
  a.ys = h->ys;
  a.js = h->js;
  a.axs = h->axs;
  a.warm_ax = (!h->warm_pending && h->warm_mode && h->have_prev) ? 1 : 0;
  a.xo = out->x;
  a.zo = out->z;
  a.yo = out->y;
  a.iterations = out->iterations;
  a.status = out->status;
  a.rho_index = out->rho_index;
  a.rho_hist = out->rho_hist;
  a.prim_res = out->prim_res;
  a.dual_res = out->dual_res;
  a.xw = h->xw;
  a.xc = h->xc;
  a.xn = h->xn;
  a.tag = h->tag;
  a.abort_flag = h->abort_d;
  a.err = h->err;
  a.count = count;
  a.chain = h->warm_mode ? 1 : 0;
  a.max_checks = h->s.max_iter / h->s.check_interval + (h->s.max_iter % h->s.check_interval ? 1 : 0);
  a.x0 = x0;
  a.F = h->F_d;
  a.E = h->E_d;
  a.plo = h->lo_d;
  a.phi = h->hi_d;
  a.nx = h->nx;
  a.final_check = 1;
  if (h->scl) {
    const size_t n = h->n, m = h->m;
    a.sc_dual = h->scl + n + m;
    a.sc_prim = h->scl + 2 * n + m;
    a.un_x = h->scl + 2 * (n + m);
    a.un_y = h->scl + 3 * n + 2 * m;
  }
  a.xu = h->xu;
  a.xpl = h->xpl;
  if (cl) {
    a.Ad = cl->Ad;
    a.Bd = cl->Bd;
    a.nu = cl->nu;
    a.traj_x = cl->traj_x;
    a.traj_u = cl->traj_u;
    a.chain = 1;
    a.final_check = 0;
  }
  return a;
}

// The launch itself: the single-workgroup kernel for small plain solves, else the persistent
// grid (the XT instantiation for closed loops and scaled problems). The handle's warm state
// advances with it.
int launch_single(relu_qp_handle* h, const rqp::LayerArgs& a, bool closed, hipStream_t st) {
  const bool xt = closed || h->scl;
  const rqp::LaunchPlan& plan = xt ? h->plan_xt : h->plan;
  const int grid = xt ? h->grid_wg : h->grid_plain;
  hipError_t e;
  if (h->small && !closed)
    e = h->esize == 8 ? rqp::launch_small<double>(a, st) : rqp::launch_small<float>(a, st);
  else
    e = h->esize == 8 ? rqp::launch_layer<double>(a, plan, grid, st) : rqp::launch_layer<float>(a, plan, grid, st);
  if (e != hipSuccess) return fail(RQP_EHIP, "persistent launch failed: %s", hipGetErrorString(e));
  h->warm_pending = false;
  h->have_prev = true;
  return RQP_OK;
}

int check_single_call(relu_qp_handle* h, const double* x0, int count, relu_qp_result* out) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  DEVICE_OR_FAIL(h);
  if (!out || !out->x || !out->y || !out->z || !out->iterations || !out->status || !out->rho_index)
    return fail(RQP_EINVAL, "result buffers x, y, z, iterations, status and rho_index are required");
  if (x0 && !h->F_d) return fail(RQP_ESTATE, "relu_qp_set_parametric has not been called");
  if (count < 1) return fail(RQP_EINVAL, "count must be >= 1");
  if (count > 1 && h->batched) return fail(RQP_EINVAL, "solve sequences run on the single-instance engine");
  const uint64_t span = (uint64_t)h->s.max_iter + 2u;
  if (span * (uint64_t)count >= 0x7fffffffull) return fail(RQP_EINVAL, "count * (max_iter + 2) must stay below 2^31");
  return RQP_OK;
}

int solve_impl(relu_qp_handle* h, const double* x0, int count, void* stream, relu_qp_result* out,
               const ClosedLoop* cl = nullptr) {
  int rc = check_single_call(h, x0, h && h->batched ? 1 : count, out);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (h->batched) {
    if (x0) HIP_OR_FAIL(rqp::mpc_vectors_tiled<float>(h->batch, h->n, h->m, h->nx, h->F_d, h->E_d, h->lo_d, h->hi_d, x0,
                                                static_cast<float*>(h->q), static_cast<float*>(h->l),
                                                static_cast<float*>(h->u), st));
    return solve_batched(h, st, out);
  }
  const uint32_t span = (uint32_t)h->s.max_iter + 2u;
  if ((uint64_t)h->tag + (uint64_t)span * count >= 0xffffffffull) {
    // restart the tag sequence: clear every exchange word so no stale tag can match
    HIP_OR_FAIL(hipMemsetAsync(h->xw, 0, h->xw_words * 8, st));
    HIP_OR_FAIL(hipMemsetAsync(h->xc, 0, h->xw_words * 8, st));
    HIP_OR_FAIL(hipMemsetAsync(h->xn, 0, h->xn_words * 8, st));
    HIP_OR_FAIL(hipMemsetAsync(h->xu, 0, (size_t)2 * rqp::kMaxPlant * 2 * 8, st));
    HIP_OR_FAIL(hipMemsetAsync(h->err, 0, sizeof(unsigned), st));
    h->tag = 1;
  }
  __atomic_store_n(h->abort_h, 0, __ATOMIC_SEQ_CST);
  const rqp::LayerArgs a = layer_args(h, x0, count, out, cl);
  rc = launch_single(h, a, cl != nullptr, st);
  if (rc) return rc;
  h->tag += span * (uint32_t)count;
  return RQP_OK;
}


}  // namespace

extern "C" {

int relu_qp_solve(relu_qp_handle* h, void* stream, relu_qp_result* out) {
  return solve_impl(h, nullptr, 1, stream, out);
}

int relu_qp_solve_x0(relu_qp_handle* h, const double* x0, void* stream, relu_qp_result* out) {
  if (!x0) return fail(RQP_EINVAL, "x0 is NULL");
  return solve_impl(h, x0, 1, stream, out);
}

int relu_qp_solve_sequence(relu_qp_handle* h, const double* x0s, int count, void* stream, relu_qp_result* out) {
  if (!x0s) return fail(RQP_EINVAL, "x0s is NULL");
  return solve_impl(h, x0s, count, stream, out);
}

int relu_qp_solve_x0_noalloc(relu_qp_handle* h, const double* x0, void* stream, relu_qp_result* out) {
  if (!x0) return fail(RQP_EINVAL, "x0 is NULL");
  int rc = check_single_call(h, x0, 1, out);
  if (rc) return rc;
  if (h->batched) return fail(RQP_ESTATE, "relu_qp_solve_x0_noalloc runs on the single-instance engine");
  const size_t words = h->esize == 8 ? 2 : 1;
  const size_t need = kScratchXwOff + (size_t)2 * 2 * h->L * words * 8;
  if (need > kScratchBytes)
    return fail(RQP_EINVAL, "n + m = %d needs %zu bytes of scratch; the library holds %zu", h->L, need, kScratchBytes);
  int cur = -1;
  HIP_OR_FAIL(hipGetDevice(&cur));
  if (cur != h->device) return fail(RQP_ESTATE, "the current device %d is not the handle's device %d", cur, h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  rqp::LayerArgs a = layer_args(h, x0, 1, out, nullptr);
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ScratchDev& sd = g_scratch[h->device];
    if (!sd.ptr) return fail(RQP_ESTATE, "no scratch on device %d", h->device);
    const uint32_t span = (uint32_t)h->s.max_iter + 2u;
    unsigned char* base = static_cast<unsigned char*>(sd.ptr);
    if (!sd.clean || (uint64_t)sd.tag + span >= 0xffffffffull) {
      // first use on this GPU, or the tag sequence restarts: no stale tag may match
      hipLaunchKernelGGL(clear_words, dim3(256), dim3(256), 0, st, reinterpret_cast<uint64_t*>(base),
                         kScratchBytes / 8);
      HIP_OR_FAIL(hipGetLastError());
      sd.tag = 1;
      sd.clean = true;
    }
    a.err = reinterpret_cast<unsigned*>(base);
    a.xn = reinterpret_cast<uint64_t*>(base + kScratchNormOff);
    a.xw = reinterpret_cast<uint64_t*>(base + kScratchXwOff);
    a.xc = a.xw + (size_t)2 * h->L * words;
    a.tag = sd.tag;
    sd.tag += span;
  }
  __atomic_store_n(h->abort_h, 0, __ATOMIC_SEQ_CST);
  return launch_single(h, a, false, st);
}

int relu_qp_solve_paper_form(relu_qp_handle* h, int iters, void* stream, relu_qp_result* out) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  DEVICE_OR_FAIL(h);
  if (h->batched) return fail(RQP_ESTATE, "the paper's layer form runs on the single-instance engine");
  if (h->grid.size() != 1 || h->s.alpha != 1.0)
    return fail(RQP_EINVAL, "the paper's layer form needs alpha = 1 and a fixed penalty (n_rho = 1)");
  if (h->scl) return fail(RQP_EINVAL, "the paper's layer form runs without Ruiz scaling");
  if (iters < 1 || iters > (1 << 24)) return fail(RQP_EINVAL, "iters must be in [1, 2^24]");
  if (!out || !out->x || !out->y || !out->z || !out->iterations || !out->status)
    return fail(RQP_EINVAL, "result buffers x, y, z, iterations and status are required");
  const int n = h->n, m = h->m;
  const long Lp = (long)n + 2L * m;
  if (Lp > rqp::kPaperMaxL) return fail(RQP_EINVAL, "n + 2m = %ld above %d", Lp, rqp::kPaperMaxL);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t words = h->esize == 8 ? 2 : 1;
  if (!h->Wp) {
    const long ldp = (Lp + 3) / 4 * 4;
    if (dmalloc(h, &h->Wp, (size_t)Lp * ldp * h->esize) != hipSuccess ||
        dmalloc(h, &h->xwp, 2 * (size_t)Lp * words * 8) != hipSuccess) {
      (void)hipGetLastError();
      return fail(RQP_ENOMEM, "paper-form weights: device allocation failed");
    }
    HIP_OR_FAIL(hipMemset(h->xwp, 0, 2 * (size_t)Lp * words * 8));
    std::vector<double> rv(m);
    for (int i = 0; i < m; ++i) rv[i] = h->grid[0] * (h->eq[i] ? h->s.rho_eq_scale : 1.0);
    DevBuf rho;
    if (rho.alloc((size_t)m * 8)) return fail(RQP_ENOMEM, "paper-form setup: device allocation failed");
    HIP_OR_FAIL(hipMemcpy(rho.p, rv.data(), (size_t)m * 8, hipMemcpyHostToDevice));
    hipError_t e = h->esize == 8
                       ? rqp::assemble_paper_w<double>(n, m, static_cast<const double*>(h->W), h->ldw,
                                                       static_cast<const double*>(h->C), rho.d(), h->s.sigma,
                                                       static_cast<double*>(h->Wp), ldp, st)
                       : rqp::assemble_paper_w<float>(n, m, static_cast<const float*>(h->W), h->ldw,
                                                      static_cast<const float*>(h->C), rho.d(), h->s.sigma,
                                                      static_cast<float*>(h->Wp), ldp, st);
    if (e != hipSuccess) return fail(RQP_EHIP, "paper-form setup failed: %s", hipGetErrorString(e));
    h->ldp = ldp;
  }
  const uint32_t span = (uint32_t)iters + 2u;
  if ((uint64_t)h->tag + span >= 0xffffffffull) {
    // restart the tag sequence: clear every exchange word so no stale tag can match
    HIP_OR_FAIL(hipMemsetAsync(h->xw, 0, h->xw_words * 8, st));
    HIP_OR_FAIL(hipMemsetAsync(h->xc, 0, h->xw_words * 8, st));
    HIP_OR_FAIL(hipMemsetAsync(h->xn, 0, h->xn_words * 8, st));
    HIP_OR_FAIL(hipMemsetAsync(h->xu, 0, (size_t)2 * rqp::kMaxPlant * 2 * 8, st));
    HIP_OR_FAIL(hipMemsetAsync(h->xwp, 0, 2 * (size_t)Lp * words * 8, st));
    HIP_OR_FAIL(hipMemsetAsync(h->err, 0, sizeof(unsigned), st));
    h->tag = 1;
  }
  int cus = 0, dev = 0;
  HIP_OR_FAIL(hipGetDevice(&dev));
  HIP_OR_FAIL(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  int grid = cus < 256 ? cus : 256;
  if (grid > Lp) grid = (int)Lp;
  if ((Lp + grid - 1) / grid > rqp::kPaperMaxRows) return fail(RQP_EINVAL, "too many rows per workgroup");
  rqp::PaperArgs a{};
  a.n = n;
  a.m = m;
  a.Lp = (int)Lp;
  a.ldp = h->ldp;
  a.W = h->Wp;
  a.Wc = h->W;
  a.ldw = h->ldw;
  a.q = h->q;
  a.l = h->l;
  a.u = h->u;
  a.iters = iters;
  a.xw = h->xwp;
  a.tag = h->tag;
  a.err = h->err;
  a.xo = out->x;
  a.zo = out->z;
  a.yo = out->y;
  a.iterations = out->iterations;
  a.status = out->status;
  hipError_t e = h->esize == 8 ? rqp::launch_paper_layer<double>(a, grid, st) : rqp::launch_paper_layer<float>(a, grid, st);
  if (e != hipSuccess) return fail(RQP_EHIP, "paper-form launch failed: %s", hipGetErrorString(e));
  h->tag += span;
  return RQP_OK;
}

int relu_qp_closed_loop(relu_qp_handle* h, const double* x0, int steps, const double* Ad, const double* Bd, int nu,
                        double* traj_x, double* traj_u, void* stream, relu_qp_result* out) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  if (h->batched) return fail(RQP_ESTATE, "closed loops run on the single-instance engine");
  if (!h->F_d) return fail(RQP_ESTATE, "relu_qp_set_parametric has not been called");
  if (!x0 || !Ad || !Bd || !traj_x || !traj_u) return fail(RQP_EINVAL, "x0, Ad, Bd, traj_x and traj_u are required");
  if (nu < 1 || nu > h->m || nu > rqp::kMaxPlant)
    return fail(RQP_EINVAL, "nu = %d outside [1, min(m, %d)]", nu, rqp::kMaxPlant);
  if (h->nx > rqp::kMaxPlant) return fail(RQP_EINVAL, "nx = %d above %d", h->nx, rqp::kMaxPlant);
  if (h->scl) return fail(RQP_EINVAL, "closed loops run without Ruiz scaling");
  const ClosedLoop cl{Ad, Bd, nu, traj_x, traj_u};
  return solve_impl(h, x0, steps, stream, out, &cl);
}

int relu_qp_load_slots(relu_qp_handle* h, const int* slots, int n_slots, const double* q, const double* l,
                       const double* u, void* stream) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  DEVICE_OR_FAIL(h);
  hipStream_t st = static_cast<hipStream_t>(stream);
  return for_slot_chunks(h, slots, n_slots, [&](const rqp::SlotList& sl, int i0) -> int {
    const size_t n = h->n, m = h->m;
    HIP_OR_FAIL(rqp::load_slots(sl, h->n, h->m, q ? q + i0 * n : nullptr, l ? l + i0 * m : nullptr,
                                u ? u + i0 * m : nullptr, static_cast<float*>(h->q), static_cast<float*>(h->l),
                                static_cast<float*>(h->u), h->scl, st));
    return RQP_OK;
  });
}

int relu_qp_load_slots_x0(relu_qp_handle* h, const int* slots, int n_slots, const double* x0, void* stream) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  DEVICE_OR_FAIL(h);
  if (!h->F_d) return fail(RQP_ESTATE, "relu_qp_set_parametric has not been called");
  if (!x0 && n_slots > 0) return fail(RQP_EINVAL, "x0 is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  return for_slot_chunks(h, slots, n_slots, [&](const rqp::SlotList& sl, int i0) -> int {
    HIP_OR_FAIL(rqp::load_x0_slots(sl, h->n, h->m, h->nx, h->F_d, h->E_d, h->lo_d, h->hi_d,
                                   x0 + (size_t)i0 * h->nx, static_cast<float*>(h->q), static_cast<float*>(h->l),
                                   static_cast<float*>(h->u), st));
    return RQP_OK;
  });
}

int relu_qp_admit(relu_qp_handle* h, const int* slots, int n_slots, int src_slot, int shift_x, int shift_y,
                  void* stream) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  DEVICE_OR_FAIL(h);
  if (h->batched && (src_slot < -1 || src_slot >= h->batch))
    return fail(RQP_EINVAL, "src_slot %d out of range [-1, %d)", src_slot, h->batch);
  if (shift_x < 0 || shift_x > h->n || shift_y < 0 || shift_y > h->m) return fail(RQP_EINVAL, "bad shift");
  hipStream_t st = static_cast<hipStream_t>(stream);
  bool first = true;
  return for_slot_chunks(h, slots, n_slots, [&](const rqp::SlotList& sl, int) -> int {
    // the source state is staged once, before any listed slot (which may include it) is written
    if (src_slot >= 0 && !first) {
      HIP_OR_FAIL(rqp::admit_slots(sl, -2, shift_x, shift_y, h->n, h->m, h->bX, h->bY, h->bjb, h->bstatus,
                                   h->bstage, h->scl, st));
    } else {
      HIP_OR_FAIL(rqp::admit_slots(sl, src_slot, shift_x, shift_y, h->n, h->m, h->bX, h->bY, h->bjb, h->bstatus,
                                   h->bstage, h->scl, st));
    }
    first = false;
    return RQP_OK;
  });
}

int relu_qp_step(relu_qp_handle* h, int n_checks, void* stream, relu_qp_result* out) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  DEVICE_OR_FAIL(h);
  if (!h->batched) return fail(RQP_ESTATE, "relu_qp_step needs the batched engine");
  if (!out || !out->x || !out->y || !out->z || !out->iterations || !out->status || !out->rho_index)
    return fail(RQP_EINVAL, "result buffers x, y, z, iterations, status and rho_index are required");
  if (h->s.max_iter % h->s.check_interval != 0)
    return fail(RQP_EINVAL, "serving needs max_iter to be a multiple of check_interval");
  if (n_checks < 1 || n_checks > h->s.max_iter / h->s.check_interval)
    return fail(RQP_EINVAL, "n_checks must be in [1, max_iter / check_interval]");
  return launch_batched(h, n_checks * h->s.check_interval, static_cast<hipStream_t>(stream), out, true);
}

int relu_qp_get_tile(const relu_qp_handle* h, int* tile_rows, double* us_per_iter) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  if (!h->batched) return fail(RQP_ESTATE, "tile shapes exist only with the batched engine");
  if (tile_rows) *tile_rows = h->bplan.tn;
  if (us_per_iter)
    for (int v = 0; v < rqp::kTileShapes; ++v) us_per_iter[v] = h->tile_us[v];
  return RQP_OK;
}

int relu_qp_set_tile(relu_qp_handle* h, int tile_rows) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  if (!h->batched) return fail(RQP_ESTATE, "tile shapes exist only with the batched engine");
  int v = -1;
  for (int c = 0; c < rqp::kTileShapes; ++c)
    if (tile_rows == rqp::kTileRows[c]) v = c;
  if (tile_rows == 0) v = best_tile(h);
  if (v < 0) return fail(RQP_EINVAL, "tile_rows must be 128, 64, 256 or 0 (the autotuner's choice)");
  h->bplan = h->bplans[v];
  return RQP_OK;
}

int relu_qp_abort(relu_qp_handle* h) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  __atomic_store_n(h->abort_h, 1, __ATOMIC_SEQ_CST);
  return RQP_OK;
}

int relu_qp_max_checks(const relu_qp_handle* h) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  return h->s.max_iter / h->s.check_interval + (h->s.max_iter % h->s.check_interval ? 1 : 0);
}

int relu_qp_get_rho_grid(const relu_qp_handle* h, double* grid, int* n_rho) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  if (n_rho) *n_rho = (int)h->grid.size();
  if (grid) std::memcpy(grid, h->grid.data(), h->grid.size() * 8);
  return RQP_OK;
}

int relu_qp_offload(relu_qp_handle* h) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  if (h->offloaded) return RQP_OK;
  HIP_OR_FAIL(hipDeviceSynchronize());  // no launch may still use the buffers
  // host copies first (kept for later offloads), so that a failure leaves the device intact
  for (auto& e : h->allocs)
    if (!e.host && hipHostMalloc(&e.host, e.bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      e.host = nullptr;
      return fail(RQP_ENOMEM, "pinned host memory for the offload failed (%zu bytes)", e.bytes);
    }
  for (auto& e : h->allocs) HIP_OR_FAIL(hipMemcpy(e.host, *e.slot, e.bytes, hipMemcpyDeviceToHost));
  for (auto& e : h->allocs) {
    (void)hipFree(*e.slot);
    *e.slot = nullptr;
  }
  h->offloaded = true;
  h->dev_bytes = 0;
  return RQP_OK;
}

int relu_qp_restore(relu_qp_handle* h) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  if (!h->offloaded) return RQP_OK;
  size_t total = 0;
  for (size_t i = 0; i < h->allocs.size(); ++i) {
    auto& e = h->allocs[i];
    if (hipMalloc(e.slot, e.bytes) != hipSuccess) {
      (void)hipGetLastError();
      for (size_t k = 0; k < i; ++k) {
        (void)hipFree(*h->allocs[k].slot);
        *h->allocs[k].slot = nullptr;
      }
      *e.slot = nullptr;
      return fail(RQP_ENOMEM, "device memory for the restore failed (%zu bytes)", e.bytes);
    }
    total += e.bytes;
  }
  for (auto& e : h->allocs) HIP_OR_FAIL(hipMemcpy(*e.slot, e.host, e.bytes, hipMemcpyHostToDevice));
  h->offloaded = false;
  h->dev_bytes = total;
  return RQP_OK;
}

int relu_qp_set_launch(relu_qp_handle* h, int grid) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  if (h->batched) return grid == 0 ? RQP_OK : fail(RQP_EINVAL, "the batched engine uses one workgroup per CU");
  return grid == 0 ? choose_grid(h) : set_grid(h, grid);
}

int relu_qp_get_launch(const relu_qp_handle* h, int* grid, int* block) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  if (grid) *grid = h->batched ? h->bplan.grid : (h->small ? 1 : h->grid_plain);
  if (block) *block = h->batched ? rqp::kBatchBlock : rqp::kLayerBlock;
  return RQP_OK;
}

int relu_qp_device_bytes(const relu_qp_handle* h, size_t* bytes) {
  if (!h) return fail(RQP_ESTATE, "NULL handle");
  if (!bytes) return fail(RQP_EINVAL, "bytes is NULL");
  *bytes = h->dev_bytes;
  return RQP_OK;
}

// The resident allocations of relu_qp_setup (and relu_qp_set_parametric), size by size, with
// the same expressions the allocating code uses, and the FP64 workspace setup holds on top of
// them while it factors; no device call.
int relu_qp_footprint(int n, int m, const relu_qp_settings* s, int nx, size_t* bytes, size_t* setup_extra) {
  if (!bytes) return fail(RQP_EINVAL, "bytes is NULL");
  if (n < 1 || m < 1 || nx < 0) return fail(RQP_EINVAL, "need n >= 1, m >= 1, nx >= 0");
  int rc = validate_settings(s);
  if (rc) return rc;
  std::vector<double> grid, mid;
  int j0 = 0;
  make_grid(*s, grid, mid, j0);
  const size_t nr = grid.size(), L = (size_t)n + m;
  auto a8 = [](size_t b) { return b ? b : (size_t)8; };
  size_t t = a8(m) + a8(nr * 8) + a8(mid.size() * 8);
  if (is_batched(*s)) {
    const size_t B = s->batch;
    const bool two = s->precision == RQP_BF16X3;
    const size_t es = two ? 2 : 4;
    const size_t ldk = (L + rqp::kTileK - 1) / rqp::kTileK * rqp::kTileK + 4 * rqp::kTileK;
    const size_t lpad = (L + rqp::kTileN - 1) / rqp::kTileN * rqp::kTileN;
    const size_t bpad = (B + rqp::kTileM - 1) / rqp::kTileM * rqp::kTileM + rqp::kTileM;
    const size_t w_stride = lpad * ldk, vbytes = bpad * ldk * es;
    const size_t ntile_max = B / rqp::kTileM + nr + 1;
    const size_t nw = two ? 2 : 1;
    t += nw * (nr * w_stride * es + 2 * vbytes);                   // layer weights, V (two parities)
    t += check_rows(L) * ldk * 8 + 2 * bpad * ldk * 8;             // FP64 check matrix and operands
    t += 2 * B * n * 8;                                            // check scratch (P x, A'y)
    t += B * n * 4 + 2 * B * m * 4;                                // x, z, y
    t += B * 4 + B * 64 + B * 4 + B * 4;                           // penalty index, norms, lists, positions
    t += (1 + 3 * ntile_max) * 4 + 1024 * 4;                       // tile lists, barrier words
    t += B * n * 4 + 2 * B * m * 4;                                // q, l, u
    t += 2 * B * 4 + (L + 1) * 4;                                  // status, iterations, staging
    if (s->scaling > 0) t += 3 * L * 8;                            // Ruiz scaling vectors
  } else {
    const size_t es = s->precision == RQP_FP64 ? 8 : 4;
    const size_t ldw = (L + 3) / 4 * 4, w_stride = L * ldw;
    t += nr * w_stride * es + w_stride * es;  // layer and check matrices
    t += 2 * ((size_t)n + 2 * m) * es;        // q, l, u and x, z, y
    t += 4 + 4 + (size_t)m * 8;               // penalty index, error word, carried A x
    const size_t words = es == 8 ? 2 : 1;
    t += 2 * (2 * L * words * 8) + 2 * L * 8 * 2 * 8;  // exchange buffers
    t += (size_t)2 * rqp::kMaxPlant * 2 * 8;           // closed-loop control words
    t += (size_t)2 * rqp::kMaxGrid * rqp::kMaxPlant * 8;  // closed-loop plant states
    if (s->scaling > 0) t += 3 * L * 8;                    // Ruiz scaling vectors
  }
  if (nx > 0) t += ((size_t)n + m) * nx * 8 + 2 * (size_t)m * 8;
  *bytes = t;
  if (setup_extra) {
    const size_t nn = (size_t)n * n, mn = (size_t)m * n, mm = (size_t)m * m;
    size_t w = (3 * nn + 2 * mn + mm + 2 * 32 * (size_t)n + 32 * 32 + m) * 8 + sizeof(int);
    if (is_batched(*s)) w += L * L * 8;
    *setup_extra = w;
  }
  return RQP_OK;
}

int relu_qp_cleanup(relu_qp_handle* h) {
  if (!h) return RQP_OK;
  (void)hipDeviceSynchronize();
  free_handle(h);
  return RQP_OK;
}

}  // extern "C"
