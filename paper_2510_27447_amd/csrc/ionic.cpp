// Host side of the C ABI declared in include/ionic_sdc.h: argument checking,
// parameter derivation, Gauss-Lobatto nodes and quadrature, launch
// assembly and the handle's bookkeeping.  All numerical work of the
// reaction + SDC stage runs in the kernels of sdc_kernel.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "grid_ops.h"
#include "implicit_ops.h"
#include "ionic_sdc.h"
#include "kernel_ops.h"

using ionic::AdaptCtl;
using ionic::DevStats;
using ionic::ErrSlot;
using ionic::kSlots;
using ionic::kBlock;
using ionic::kMaxBatch;
using ionic::kMaxNodes;
using ionic::LaunchCommon;
using ionic::ModelOps;
using ionic::SimDesc;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(IONIC_EHIP, std::string(what) + ": " + hipGetErrorName(e) + " (" +
                              hipGetErrorString(e) + ")");
}

#define IONIC_HIP(call)                                   \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return hip_fail(e_, #call);     \
  } while (0)

const ModelOps* ops_for(int model) {
  switch (model) {
    case IONIC_LR91: return &ionic::kOpsLR91;
    case IONIC_TT06_EPI: return &ionic::kOpsTT06;
    case IONIC_TEST_LINEAR: return &ionic::kOpsTestLinear;
    case IONIC_TEST_LOGISTIC: return &ionic::kOpsTestLogistic;
    default: return nullptr;
  }
}

bool valid_precision(int p) { return p == IONIC_FP64 || p == IONIC_MIXED; }

int64_t stride_of(int64_t n) { return (n + 63) / 64 * 64; }

size_t bytes_of(const ModelOps* o, int precision, int64_t n) {
  const size_t s = size_t(stride_of(n));
  if (precision == IONIC_FP64) return size_t(o->n_states) * s * 8;
  return size_t(o->n_fp64) * s * 8 + size_t(o->n_states - o->n_fp64) * s * 4;
}

// Gauss-Lobatto nodes on [0, 1]: endpoints plus the roots of P'_{M-1}
// mapped from [-1, 1] (closed forms for M <= 5).
void lobatto_nodes(int M, double* c) {
  c[0] = 0.0;
  c[M - 1] = 1.0;
  if (M == 3) c[1] = 0.5;
  if (M == 4) {
    const double s5 = std::sqrt(5.0);
    c[1] = (5.0 - s5) / 10.0;
    c[2] = (5.0 + s5) / 10.0;
  }
  if (M == 5) {
    const double s21 = std::sqrt(21.0);
    c[1] = (7.0 - s21) / 14.0;
    c[2] = 0.5;
    c[3] = (7.0 + s21) / 14.0;
  }
}

// S[m][j] = integral_{c_m}^{c_{m+1}} l_j(s) ds by 5-point Gauss-Legendre
// quadrature, exact for the degree <= 4 Lagrange polynomials.
void lobatto_matrix(int M, const double* c, double* S /* (M-1) x M */) {
  const double a = std::sqrt(5.0 - 2.0 * std::sqrt(10.0 / 7.0)) / 3.0;
  const double b = std::sqrt(5.0 + 2.0 * std::sqrt(10.0 / 7.0)) / 3.0;
  const double wa = (322.0 + 13.0 * std::sqrt(70.0)) / 900.0;
  const double wb = (322.0 - 13.0 * std::sqrt(70.0)) / 900.0;
  const double gx[5] = {-b, -a, 0.0, a, b};
  const double gw[5] = {wb, wa, 128.0 / 225.0, wa, wb};
  for (int m = 0; m < M - 1; ++m) {
    const double lo = c[m], hi = c[m + 1], half = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
    for (int j = 0; j < M; ++j) {
      double acc = 0.0;
      for (int q = 0; q < 5; ++q) {
        const double s = mid + half * gx[q];
        double l = 1.0;
        for (int k = 0; k < M; ++k)
          if (k != j) l *= (s - c[k]) / (c[j] - c[k]);
        acc += gw[q] * l;
      }
      S[m * M + j] = half * acc;
    }
  }
}

// library-owned device memory of one handle
struct DevBlock {
  DevStats stats[kSlots];
  ErrSlot err[kSlots];
  AdaptCtl ctl;
  double rest[32];  // resting state computed by ionic_init when x0 is NULL
};

// Blocks of destroyed handles are kept per device and handed to the next
// ionic_init on that device, so that neither creating nor destroying a handle
// frees device memory (hipFree waits for the whole device).
constexpr int kMaxDevices = 64;
std::mutex g_pool_mu;
std::vector<DevBlock*> g_pool[kMaxDevices];

// Staging of state_readback_noalloc: one file-scope device array per GPU,
// held until the process ends.  On the host its name is only a stand-in: the
// array's address on a device comes from hipGetSymbolAddress, taken once per
// device with that device current (scratch_on_current_device).
constexpr size_t kScratchBytes = size_t(8) << 20;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

// Device address of `scratch` on the current device (0 = OK).
int scratch_on_current_device(int device, double** out) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(IONIC_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[device] = p;
  }
  *out = static_cast<double*>(g_scratch_ptr[device]);
  return IONIC_OK;
}

}  // namespace

struct ionic_sim {
  const ModelOps* ops = nullptr;
  int model = 0;
  int precision = 0;
  int64_t n = 0;
  int64_t stride = 0;
  void* state = nullptr;
  std::vector<double> raw;
  alignas(16) unsigned char p64[1024];
  alignas(16) unsigned char p32[1024];
  double tol = 0.0;
  int maxit = 0;
  int predictor = IONIC_PRED_NEWTON;
  DevBlock* dev = nullptr;  // statistics slots and the adaptive control block
  DevStats* stats = nullptr;
  int device = 0;           // the HIP device of the state buffer
  // streams this handle has enqueued work on (ionic_destroy and the stats
  // calls wait for these only); more than kMaxStreams distinct streams
  // falls back to waiting for the device
  static constexpr int kMaxStreams = 8;
  hipStream_t streams[kMaxStreams] = {};
  int n_streams = 0;
  bool many_streams = false;
  // inputs for the batched entry
  bool inputs_set = false;
  double t0 = 0.0, dt = 0.0, t_on = 0.0, t_off = 0.0;
  int M = 0, K = 0;
  const double* i_stim = nullptr;
  const double* i_diff = nullptr;
  long long step_offset = 0;
  const int32_t* order = nullptr;  // vertex processing order (device, caller-owned) or null
  // multigrid tables of the last bidomain grid (the coarsest inverse costs
  // O(n^3) on the host, so it is formed once per grid and conductivities)
  long long mg_dims[3] = {0, 0, 0};
  double mg_sie[3] = {0.0, 0.0, 0.0};
  std::vector<double> mg_tables;

  const void* params() const { return precision == IONIC_FP64 ? (const void*)p64 : (const void*)p32; }
};

namespace {

// Record that work of handle s is enqueued on stream st.
void touch(ionic_sim* s, hipStream_t st) {
  for (int i = 0; i < s->n_streams; ++i)
    if (s->streams[i] == st) return;
  if (s->n_streams < ionic_sim::kMaxStreams)
    s->streams[s->n_streams++] = st;
  else
    s->many_streams = true;
}

// Wait until every piece of work the handle has enqueued has completed.
hipError_t wait_handle(const ionic_sim* s) {
  if (s->many_streams) return hipDeviceSynchronize();
  for (int i = 0; i < s->n_streams; ++i) {
    hipError_t e = hipStreamSynchronize(s->streams[i]);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void fill_quadrature(int M, LaunchCommon& c) {
  std::memset(&c, 0, sizeof(c));
  double nodes[kMaxNodes], S[(kMaxNodes - 1) * kMaxNodes];
  lobatto_nodes(M, nodes);
  lobatto_matrix(M, nodes, S);
  for (int m = 0; m < M - 1; ++m) {
    c.dc[m] = nodes[m + 1] - nodes[m];
    for (int j = 0; j < M; ++j) c.S[m][j] = S[m * M + j];
  }
}

SimDesc desc_of(const ionic_sim* s, double t0, double dt, const double* stim, double t_on,
                double t_off, const double* diff, long long offset, int n_steps, int K,
                int first_block) {
  SimDesc d;
  std::memset(&d, 0, sizeof(d));
  d.state = s->state;
  d.n = s->n;
  d.stride = s->stride;
  d.i_stim = stim;
  d.i_diff = diff;
  d.t0 = t0;
  d.dt = dt;
  d.t_on = t_on;
  d.t_off = t_off;
  d.step_offset = offset;
  d.n_steps = n_steps;
  d.n_sweeps = K;
  d.stats = s->stats;
  d.order = s->order;
  d.first_block = first_block;
  return d;
}

int check_step_args(double t0, double dt, int n_steps, int n_nodes, int n_sweeps, double t_on,
                    double t_off) {
  if (n_steps < 0) return fail(IONIC_EINVAL, "n_steps must be >= 0");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(IONIC_EINVAL, "dt must be positive and finite");
  if (!std::isfinite(t0)) return fail(IONIC_EINVAL, "t0 must be finite");
  if (n_nodes < 2 || n_nodes > IONIC_MAX_NODES)
    return fail(IONIC_EUNSUPPORTED, "n_nodes must be in [2, " + std::to_string(IONIC_MAX_NODES) + "]");
  if (n_sweeps < 0 || n_sweeps > IONIC_MAX_SWEEPS)
    return fail(IONIC_EINVAL, "n_sweeps must be in [0, " + std::to_string(IONIC_MAX_SWEEPS) + "]");
  if (std::isnan(t_on) || std::isnan(t_off)) return fail(IONIC_EINVAL, "stimulus window is NaN");
  return IONIC_OK;
}

}  // namespace

extern "C" {

const char* ionic_last_error(void) { return g_err.c_str(); }

int ionic_n_states(int model) {
  const ModelOps* o = ops_for(model);
  return o ? o->n_states : fail(IONIC_EUNSUPPORTED, "unknown model");
}

int ionic_n_fp64_states(int model) {
  const ModelOps* o = ops_for(model);
  return o ? o->n_fp64 : fail(IONIC_EUNSUPPORTED, "unknown model");
}

const char* ionic_state_name(int model, int idx) {
  const ModelOps* o = ops_for(model);
  if (!o || idx < 0 || idx >= o->n_states) return nullptr;
  return o->state_names[idx];
}

int ionic_n_params(int model) {
  const ModelOps* o = ops_for(model);
  return o ? o->n_params : fail(IONIC_EUNSUPPORTED, "unknown model");
}

const char* ionic_param_name(int model, int idx) {
  const ModelOps* o = ops_for(model);
  if (!o || idx < 0 || idx >= o->n_params) return nullptr;
  return o->param_names[idx];
}

int64_t ionic_plane_stride(int64_t n) { return n < 1 ? 0 : stride_of(n); }

size_t ionic_state_bytes(int model, int precision, int64_t n) {
  const ModelOps* o = ops_for(model);
  if (!o || !valid_precision(precision) || n < 1) return 0;
  return bytes_of(o, precision, n);
}

int ionic_lobatto(int M, double* c, double* S) {
  if (M < 2 || M > IONIC_MAX_NODES) return fail(IONIC_EUNSUPPORTED, "n_nodes must be in [2, 5]");
  double nodes[kMaxNodes];
  lobatto_nodes(M, nodes);
  if (c) std::memcpy(c, nodes, sizeof(double) * M);
  if (S) lobatto_matrix(M, nodes, S);
  return IONIC_OK;
}

int ionic_init(ionic_sim** out, const ionic_config* cfg, void* state_dev, size_t state_bytes,
               const double* x0, int x0_on_device, void* hip_stream) {
  if (!out) return fail(IONIC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(IONIC_EINVAL, "cfg is NULL");
  const ModelOps* o = ops_for(cfg->model);
  if (!o) return fail(IONIC_EUNSUPPORTED, "unknown model " + std::to_string(cfg->model));
  if (!valid_precision(cfg->precision)) return fail(IONIC_EUNSUPPORTED, "unknown precision");
  if (cfg->n_vertices < 1) return fail(IONIC_EINVAL, "n_vertices must be >= 1");
  if (cfg->n_vertices > (int64_t(1) << 36)) return fail(IONIC_EINVAL, "n_vertices too large");
  if (!(cfg->newton_tol >= 0.0) || !std::isfinite(cfg->newton_tol))
    return fail(IONIC_EINVAL, "newton_tol must be finite and >= 0");
  if (cfg->newton_maxit < 1 || cfg->newton_maxit > 64)
    return fail(IONIC_EINVAL, "newton_maxit must be in [1, 64]");
  if (cfg->n_params < 0 || cfg->n_params > o->n_params)
    return fail(IONIC_EINVAL, "n_params out of range (max " + std::to_string(o->n_params) + ")");
  if (cfg->n_params > 0 && !cfg->params) return fail(IONIC_EINVAL, "params is NULL");
  if (!state_dev) return fail(IONIC_EINVAL, "state_dev is NULL");
  const size_t need = bytes_of(o, cfg->precision, cfg->n_vertices);
  if (state_bytes < need)
    return fail(IONIC_EINVAL, "state buffer too small: need " + std::to_string(need) + " bytes");
  if (o->params_bytes[0] > 1024 || o->params_bytes[1] > 1024)
    return fail(IONIC_EUNSUPPORTED, "parameter block too large");

  ionic_sim* s = new ionic_sim();
  s->ops = o;
  s->model = cfg->model;
  s->precision = cfg->precision;
  s->n = cfg->n_vertices;
  s->stride = stride_of(s->n);
  s->state = state_dev;
  s->raw.assign(o->param_defaults, o->param_defaults + o->n_raw);
  for (int i = 0; i < cfg->n_params; ++i) s->raw[i] = cfg->params[i];
  o->derive(s->raw.data(), s->p64, s->p32);
  s->tol = cfg->precision == IONIC_MIXED ? std::max(cfg->newton_tol, 1e-6) : cfg->newton_tol;
  s->maxit = cfg->newton_maxit;

  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "hipGetDevice");
  }
  if (s->device < 0 || s->device >= kMaxDevices) {
    delete s;
    return fail(IONIC_EUNSUPPORTED, "device index beyond " + std::to_string(kMaxDevices - 1));
  }
  {  // a pooled block of this device, else a new one
    std::lock_guard<std::mutex> g(g_pool_mu);
    std::vector<DevBlock*>& pool = g_pool[s->device];
    if (!pool.empty()) {
      s->dev = pool.back();
      pool.pop_back();
    }
  }
  if (!s->dev) {
    e = hipMalloc(&s->dev, sizeof(DevBlock));
    if (e != hipSuccess) {
      s->dev = nullptr;
      delete s;
      return hip_fail(e, "hipMalloc(stats)");
    }
  }
  auto cleanup = [&](int rc) {
    (void)hipStreamSynchronize(st);
    std::lock_guard<std::mutex> g(g_pool_mu);
    g_pool[s->device].push_back(s->dev);
    delete s;
    return rc;
  };
  s->stats = s->dev->stats;
  touch(s, st);
  e = hipMemsetAsync(s->dev, 0, sizeof(DevBlock), st);
  if (e != hipSuccess) return cleanup(hip_fail(e, "hipMemsetAsync(stats)"));

  if (!x0) {
    e = o->rest(s->precision, s->p64, s->dev->rest, s->state, s->stride, s->n, st);
    if (e != hipSuccess) return cleanup(hip_fail(e, "resting state"));
    *out = s;
    return IONIC_OK;
  }
  const double* src = x0;
  double* staging = nullptr;
  const size_t x0_bytes = size_t(o->n_states) * size_t(s->n) * sizeof(double);
  if (!x0_on_device && s->precision == IONIC_FP64) {
    // the double layout is the SoA rows of x0 with a padded row stride: copy
    // them straight into the state buffer
    e = hipMemcpy2DAsync(s->state, size_t(s->stride) * sizeof(double), x0,
                         size_t(s->n) * sizeof(double), size_t(s->n) * sizeof(double),
                         size_t(o->n_states), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return cleanup(hip_fail(e, "copy initial state"));
    *out = s;
    return IONIC_OK;
  }
  if (!x0_on_device) {
    e = hipMalloc(&staging, x0_bytes);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipMalloc(x0 staging)"));
    e = hipMemcpyAsync(staging, x0, x0_bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(st);
      (void)hipFree(staging);
      return cleanup(hip_fail(e, "hipMemcpyAsync(x0)"));
    }
    src = staging;
  }
  e = o->pack(s->precision, src, s->n, s->state, s->stride, 0, s->n, st);
  if (staging) {  // the staging buffer is released only after the pack has read it
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(staging);
  }
  if (e != hipSuccess) return cleanup(hip_fail(e, "pack initial state"));
  *out = s;
  return IONIC_OK;
}

void ionic_destroy(ionic_sim* s) {
  if (!s) return;
  // the block goes back to the pool once no work of this handle can still
  // write it
  (void)wait_handle(s);
  if (s->dev) {
    std::lock_guard<std::mutex> g(g_pool_mu);
    g_pool[s->device].push_back(s->dev);
  }
  delete s;
}

int reaction_sdc_step(ionic_sim* s, double t0, double dt, int n_steps, int n_nodes, int n_sweeps,
                      const double* i_stim_dev, double stim_t_on, double stim_t_off,
                      const double* i_diff_dev, void* hip_stream) {
  if (!s) return fail(IONIC_EINVAL, "sim is NULL");
  int rc = check_step_args(t0, dt, n_steps, n_nodes, n_sweeps, stim_t_on, stim_t_off);
  if (rc != IONIC_OK) return rc;
  if (n_steps == 0) return IONIC_OK;
  LaunchCommon c;
  fill_quadrature(n_nodes, c);
  c.tol = s->tol;
  c.maxit = s->maxit;
  c.n_sims = 1;
  c.sims[0] = desc_of(s, t0, dt, i_stim_dev, stim_t_on, stim_t_off, i_diff_dev, 0, n_steps,
                      n_sweeps, 0);
  const int blocks = int((s->n + kBlock - 1) / kBlock);
  touch(s, static_cast<hipStream_t>(hip_stream));
  hipError_t e = s->ops->sdc[s->precision][s->predictor](n_nodes, s->params(), c, blocks,
                                                         static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "launch sdc_kernel");
  return IONIC_OK;
}

static int check_grid(const ionic_sim* s, const ionic_grid* g) {
  if (!g) return fail(IONIC_EINVAL, "grid is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(IONIC_EINVAL, "grid extents must be >= 1");
  if ((__int128)g->nx * g->ny * g->nz != (__int128)s->n)
    return fail(IONIC_EINVAL, "grid nx*ny*nz must equal the vertex count");
  if (s->n >= (int64_t(1) << 31)) return fail(IONIC_EINVAL, "grid must have fewer than 2^31 nodes");
  if (!(g->h > 0.0) || !std::isfinite(g->h)) return fail(IONIC_EINVAL, "grid h must be positive");
  if (!(g->sigma >= 0.0) || !std::isfinite(g->sigma))
    return fail(IONIC_EINVAL, "grid sigma must be finite and >= 0");
  return IONIC_OK;
}

int ionic_diffusion_current(ionic_sim* s, const ionic_grid* g, double* i_diff_dev,
                            void* hip_stream) {
  if (!s) return fail(IONIC_EINVAL, "sim is NULL");
  int rc = check_grid(s, g);
  if (rc != IONIC_OK) return rc;
  if (!i_diff_dev) return fail(IONIC_EINVAL, "i_diff_dev is NULL");
  touch(s, static_cast<hipStream_t>(hip_stream));
  IONIC_HIP(ionic::diffusion_launch(static_cast<const double*>(s->state), g->nx, g->ny, g->nz,
                                    g->h, g->sigma, i_diff_dev,
                                    static_cast<hipStream_t>(hip_stream)));
  return IONIC_OK;
}

int reaction_diffusion_step(ionic_sim* s, const ionic_grid* g, double t0, double dt, int n_steps,
                            int n_nodes, int n_sweeps, const double* i_stim_dev, double stim_t_on,
                            double stim_t_off, double* i_diff_work_dev, void* hip_stream) {
  if (!s) return fail(IONIC_EINVAL, "sim is NULL");
  int rc = check_grid(s, g);
  if (rc != IONIC_OK) return rc;
  rc = check_step_args(t0, dt, n_steps, n_nodes, n_sweeps, stim_t_on, stim_t_off);
  if (rc != IONIC_OK) return rc;
  if (!i_diff_work_dev) return fail(IONIC_EINVAL, "i_diff_work_dev is NULL");
  if (dt * g->sigma * 4.0 / (g->h * g->h) > 2.0)
    return fail(IONIC_EINVAL, "explicit diffusion unstable: dt must be <= h^2 / (2 sigma) = " +
                                  std::to_string(g->h * g->h / (2.0 * g->sigma)));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  touch(s, st);
  LaunchCommon c;
  fill_quadrature(n_nodes, c);
  c.tol = s->tol;
  c.maxit = s->maxit;
  c.n_sims = 1;
  const int blocks = int((s->n + kBlock - 1) / kBlock);
  const ionic::SdcLaunch launch = s->ops->sdc[s->precision][s->predictor];
  for (int k = 0; k < n_steps; ++k) {
    IONIC_HIP(ionic::diffusion_launch(static_cast<const double*>(s->state), g->nx, g->ny, g->nz,
                                      g->h, g->sigma, i_diff_work_dev, st));
    c.sims[0] = desc_of(s, t0, dt, i_stim_dev, stim_t_on, stim_t_off, i_diff_work_dev, k, 1,
                        n_sweeps, 0);
    hipError_t e = launch(n_nodes, s->params(), c, blocks, st);
    if (e != hipSuccess) return hip_fail(e, "launch sdc_kernel (reaction-diffusion)");
  }
  return IONIC_OK;
}

// Work of a solve: the CG vectors and scalars, then (when the grid has a
// multigrid hierarchy) the level tables and vectors.
static size_t elliptic_bytes(long long nx, long long ny, long long nz, int max_iter) {
  const long long n = nx * ny * nz;
  return ionic::CgWork::bytes(n, ionic::cg_params(nx, ny, nz).nb, max_iter) +
         sizeof(double) * ionic::mg_doubles(ionic::mg_plan(nx, ny, nz));
}

int ionic_multigrid_levels(int64_t nx, int64_t ny, int64_t nz) {
  if (nx < 1 || ny < 1 || nz < 1) return fail(IONIC_EINVAL, "grid extents must be >= 1");
  if ((__int128)nx * ny * nz >= ((__int128)1 << 31))
    return fail(IONIC_EINVAL, "grid must have fewer than 2^31 nodes");
  const ionic::MgPlan plan = ionic::mg_plan(nx, ny, nz);
  return plan.usable ? plan.levels : 0;
}

size_t ionic_elliptic_work_bytes(int64_t nx, int64_t ny, int64_t nz, int max_iter) {
  if (nx < 1 || ny < 1 || nz < 1 || max_iter < 0 || max_iter > (1 << 24)) return 0;
  if ((__int128)nx * ny * nz >= ((__int128)1 << 31)) return 0;
  return elliptic_bytes(nx, ny, nz, max_iter);
}

static int check_bidomain_grid(const ionic_sim* s, const ionic_bidomain_grid* g) {
  if (!g) return fail(IONIC_EINVAL, "grid is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(IONIC_EINVAL, "grid extents must be >= 1");
  if ((__int128)g->nx * g->ny * g->nz != (__int128)s->n)
    return fail(IONIC_EINVAL, "grid nx*ny*nz must equal the vertex count");
  if (s->n >= (int64_t(1) << 31)) return fail(IONIC_EINVAL, "grid must have fewer than 2^31 nodes");
  if (!(g->h > 0.0) || !std::isfinite(g->h)) return fail(IONIC_EINVAL, "grid h must be positive");
  for (int a = 0; a < 3; ++a) {
    if (!(g->sigma_i[a] >= 0.0) || !(g->sigma_e[a] >= 0.0) || !std::isfinite(g->sigma_i[a]) ||
        !std::isfinite(g->sigma_e[a]))
      return fail(IONIC_EINVAL, "conductivities must be finite and >= 0");
    const int64_t ext = a == 0 ? g->nx : (a == 1 ? g->ny : g->nz);
    if (ext > 1 && !(g->sigma_i[a] + g->sigma_e[a] > 0.0))
      return fail(IONIC_EINVAL, "sigma_i + sigma_e must be > 0 along every grid direction");
  }
  return IONIC_OK;
}

// CG parameters of a bidomain grid.
static ionic::CgParams cg_params_of(const ionic_bidomain_grid* g, double rtol) {
  ionic::CgParams c = ionic::cg_params(g->nx, g->ny, g->nz);
  for (int a = 0; a < 3; ++a) {
    c.si[a] = g->sigma_i[a];
    c.sie[a] = g->sigma_i[a] + g->sigma_e[a];
  }
  c.rtol = rtol;
  return c;
}

// The vectors and scalars of a solve in the caller's work buffer.
static ionic::CgWork carve_cg_work(void* work, long long n, long long nb) {
  double* base = static_cast<double*>(work);
  ionic::CgWork w;
  w.r = base;
  w.z = w.r + n;
  w.p[0] = w.z + n;
  w.p[1] = w.p[0] + n;
  w.q = w.p[1] + n;
  w.u_prev = w.q + n;
  w.u_prev2 = w.u_prev + n;
  w.part_a = w.u_prev2 + n;
  w.part_b = w.part_a + nb;
  w.part_c = w.part_b + nb;
  w.sc = w.part_c + nb;
  return w;
}

// The preconditioner of the solves of one call: multigrid when the grid has
// a hierarchy (its tables uploaded and its inverse diagonals formed once per
// call; the host tables are kept in the handle), else Jacobi.
struct Preconditioner {
  bool mg = false;
  ionic::MgLevels levels{};
};

static int prepare_preconditioner(ionic_sim* s, const ionic::CgParams& c, void* work,
                                  int max_iter, Preconditioner& pc, hipStream_t st) {
  const ionic::MgPlan plan = ionic::mg_plan(c.nx, c.ny, c.nz);
  pc.mg = plan.usable;
  if (!pc.mg) return IONIC_OK;
  const bool same = s->mg_dims[0] == c.nx && s->mg_dims[1] == c.ny && s->mg_dims[2] == c.nz &&
                    s->mg_sie[0] == c.sie[0] && s->mg_sie[1] == c.sie[1] &&
                    s->mg_sie[2] == c.sie[2] && s->mg_tables.size() == plan.table_doubles;
  if (!same) {
    s->mg_tables = ionic::mg_tables(plan);
    ionic::mg_coarse_inverse(plan, c.sie, s->mg_tables);
    s->mg_dims[0] = c.nx;
    s->mg_dims[1] = c.ny;
    s->mg_dims[2] = c.nz;
    for (int a = 0; a < 3; ++a) s->mg_sie[a] = c.sie[a];
  }
  double* region = static_cast<double*>(work) + ionic::CgWork::bytes(c.n, c.nb, max_iter) / sizeof(double);
  IONIC_HIP(hipMemcpyAsync(region, s->mg_tables.data(), s->mg_tables.size() * sizeof(double),
                           hipMemcpyHostToDevice, st));
  pc.levels = ionic::mg_bind(plan, c.sie, region);
  IONIC_HIP(ionic::mg_setup(pc.levels, st));
  return IONIC_OK;
}

// One elliptic solve on stream st; info accumulates.  The device decides
// convergence after every iteration (iterations after it are launched but do
// nothing); the host reads that decision between batches of iterations (see
// below).  work_bytes has been checked by the caller; the mean removal at the
// end is only enqueued.
static int elliptic_solve_impl(ionic_sim* s, const ionic::CgParams& c, double* u, void* work,
                               double rtol, int max_iter, const Preconditioner& pc,
                               ionic_elliptic_info* info, hipStream_t st, long long expect = 0,
                               const double* V = nullptr) {
  const long long n = s->n;
  ionic::CgWork w = carve_cg_work(work, n, c.nb);
  if (!V) V = static_cast<const double*>(s->state);
  const bool jacobi = !pc.mg;
  // z = M^-1 r and its r.z parts when multigrid preconditions; with iter >= 0
  // the cycle first tests ||r_iter|| (xtmp and ytmp are dead vectors of the CG
  // at that point)
  auto cycle = [&](double* ytmp, long long iter) {
    return ionic::mg_apply(pc.levels, w.r, w.z, w.q, ytmp, w.ctl(), w.part_b, w.part_c, c.nb,
                           w.bb(), rtol, iter >= 0 ? w.rr(iter) : nullptr, iter, st);
  };
  IONIC_HIP(ionic::cg_start(c, V, u, w, jacobi, st));
  if (!jacobi) IONIC_HIP(cycle(w.p_k(0), -1));
  IONIC_HIP(ionic::cg_start_sums(c, w, st));
  // Iterations in batches.  After each batch one synchronisation reads the
  // stop flag, b.b and the r.r of the batch's iterations.  The first batch is
  // the expected count (the previous solve of a time loop; with Jacobi, four
  // fewer), so a time loop usually synchronises once per solve; launches after
  // the stop return at once.
  constexpr int kBatch = 8, kBatchMg = 2;
  long long batch = jacobi ? std::max<long long>(kBatch, expect - 4)
                           : std::max<long long>(kBatchMg, expect);
  int k = 0;
  double head[8];                 // the scalars before the per-iteration triples
  std::vector<double> triples;    // (r.z, p.q, r.r) of iterations k0 .. k
  int k0 = 0;
  for (;;) {
    k0 = k;
    const int until = int(std::min<long long>(max_iter, k + batch));
    batch = jacobi ? kBatch : kBatchMg;
    for (; k < until; ++k) {
      IONIC_HIP(ionic::cg_iteration(c, k, u, w, jacobi, st));
      if (!jacobi) IONIC_HIP(cycle(w.p_k(k + 1), k + 1));
    }
    if (k == max_iter) IONIC_HIP(ionic::cg_end(c, k, w, st));
    triples.resize(size_t(3 * (k - k0 + 1)));
    IONIC_HIP(hipMemcpyAsync(head, w.sc, sizeof(head), hipMemcpyDeviceToHost, st));
    IONIC_HIP(hipMemcpyAsync(triples.data(), w.rz(k0), triples.size() * sizeof(double),
                             hipMemcpyDeviceToHost, st));
    IONIC_HIP(hipStreamSynchronize(st));
    ionic::CgCtl ctl;
    std::memcpy(&ctl, &head[3], sizeof(ctl));
    if (ctl.done || k >= max_iter) {
      // a stop in an earlier batch would have ended the loop there, so the
      // stopping iteration lies in this batch (or is 0, the first batch's k0)
      const long long iters = ctl.done ? ctl.iters : k;
      const double bb = head[0], rr = triples[size_t(3 * (iters - k0) + 2)];
      const double rel = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
      if (info) {
        info->cg_iterations += iters;
        info->relative_residual = rel;
        info->converged = info->converged && rel <= rtol ? 1 : 0;
      }
      break;
    }
  }
  // enqueued only: the caller synchronises before u is read
  IONIC_HIP(ionic::cg_remove_mean(c, u, w, st));
  return IONIC_OK;
}

static int check_elliptic_work(const ionic::CgParams& c, size_t work_bytes, int max_iter) {
  const size_t need = elliptic_bytes(c.nx, c.ny, c.nz, max_iter);
  if (work_bytes < need)
    return fail(IONIC_EINVAL, "elliptic work buffer too small: need " + std::to_string(need) +
                                  " bytes");
  return IONIC_OK;
}

int ionic_elliptic_solve(ionic_sim* s, const ionic_bidomain_grid* g, double* u_dev,
                         void* work_dev, size_t work_bytes, double rtol, int max_iter,
                         ionic_elliptic_info* info, void* hip_stream) {
  if (!s) return fail(IONIC_EINVAL, "sim is NULL");
  int rc = check_bidomain_grid(s, g);
  if (rc != IONIC_OK) return rc;
  if (!u_dev || !work_dev) return fail(IONIC_EINVAL, "u_dev or work_dev is NULL");
  if (!(rtol >= 0.0) || !std::isfinite(rtol)) return fail(IONIC_EINVAL, "rtol must be >= 0");
  if (max_iter < 0 || max_iter > (1 << 24)) return fail(IONIC_EINVAL, "max_iter out of range");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const ionic::CgParams c = cg_params_of(g, rtol);
  rc = check_elliptic_work(c, work_bytes, max_iter);
  if (rc != IONIC_OK) return rc;
  touch(s, st);
  Preconditioner pc;
  rc = prepare_preconditioner(s, c, work_dev, max_iter, pc, st);
  if (rc != IONIC_OK) return rc;
  ionic_elliptic_info local{0, 0.0, 1, 0};
  rc = elliptic_solve_impl(s, c, u_dev, work_dev, rtol, max_iter, pc, &local, st);
  if (rc != IONIC_OK) return rc;
  IONIC_HIP(hipStreamSynchronize(st));
  if (info) *info = local;
  return IONIC_OK;
}

int reaction_bidomain_step(ionic_sim* s, const ionic_bidomain_grid* g, double t0, double dt,
                           int n_steps, int n_nodes, int n_sweeps, const double* i_stim_dev,
                           double stim_t_on, double stim_t_off, double* u_dev, void* work_dev,
                           size_t work_bytes, double rtol, int max_iter, double* i_diff_work_dev,
                           ionic_elliptic_info* info, void* hip_stream) {
  if (!s) return fail(IONIC_EINVAL, "sim is NULL");
  int rc = check_bidomain_grid(s, g);
  if (rc != IONIC_OK) return rc;
  rc = check_step_args(t0, dt, n_steps, n_nodes, n_sweeps, stim_t_on, stim_t_off);
  if (rc != IONIC_OK) return rc;
  if (!u_dev || !work_dev || !i_diff_work_dev)
    return fail(IONIC_EINVAL, "u_dev, work_dev or i_diff_work_dev is NULL");
  if (!(rtol >= 0.0) || !std::isfinite(rtol)) return fail(IONIC_EINVAL, "rtol must be >= 0");
  if (max_iter < 0 || max_iter > (1 << 24)) return fail(IONIC_EINVAL, "max_iter out of range");
  double smax = 0.0;
  for (int a = 0; a < 3; ++a) {
    const int64_t ext = a == 0 ? g->nx : (a == 1 ? g->ny : g->nz);
    if (ext > 1) smax = std::max(smax, g->sigma_i[a]);
  }
  if (dt * smax * 4.0 / (g->h * g->h) > 2.0)
    return fail(IONIC_EINVAL, "explicit parabolic term unstable: dt must be <= h^2 / (2 max sigma_i) = " +
                                  std::to_string(g->h * g->h / (2.0 * smax)));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const ionic::CgParams c = cg_params_of(g, rtol);
  LaunchCommon lc;
  fill_quadrature(n_nodes, lc);
  lc.tol = s->tol;
  lc.maxit = s->maxit;
  lc.n_sims = 1;
  const int blocks = int((s->n + kBlock - 1) / kBlock);
  const ionic::SdcLaunch launch = s->ops->sdc[s->precision][s->predictor];
  rc = check_elliptic_work(c, work_bytes, max_iter);
  if (rc != IONIC_OK) return rc;
  touch(s, st);
  Preconditioner pc;
  rc = prepare_preconditioner(s, c, work_dev, max_iter, pc, st);
  if (rc != IONIC_OK) return rc;
  ionic_elliptic_info acc{0, 0.0, 1, 0};
  long long expect = 0;
  ionic::CgWork w = carve_cg_work(work_dev, s->n, c.nb);
  for (int k = 0; k < n_steps; ++k) {
    // the guess: the caller's u, then the last solution, then the linear
    // extrapolation from the last two, then the quadratic one from the last three
    if (k >= 1) IONIC_HIP(ionic::cg_extrapolate(c, u_dev, w, k < 3 ? k - 1 : 2, st));
    const long long before = acc.cg_iterations;
    rc = elliptic_solve_impl(s, c, u_dev, work_dev, rtol, max_iter, pc, &acc, st, expect);
    if (rc != IONIC_OK) return rc;
    expect = acc.cg_iterations - before;
    IONIC_HIP(ionic::bidomain_current(c, static_cast<const double*>(s->state), u_dev, g->h,
                                      i_diff_work_dev, st));
    lc.sims[0] = desc_of(s, t0, dt, i_stim_dev, stim_t_on, stim_t_off, i_diff_work_dev, k, 1,
                         n_sweeps, 0);
    hipError_t e = launch(n_nodes, s->params(), lc, blocks, st);
    if (e != hipSuccess) return hip_fail(e, "launch sdc_kernel (bidomain)");
  }
  IONIC_HIP(hipStreamSynchronize(st));
  if (info) *info = acc;
  return IONIC_OK;
}

// ---- partitioned stepping with the parabolic term implicit ------------------------------

namespace {

// Layout of the work buffer of reaction_bidomain_implicit_step: the elliptic
// solve's work, six state-sized vectors (n_states planes of stride doubles),
// five fields of stride doubles, the BiCGSTAB work, the solutions of the three
// systems of a pass (each the guess of the same system in the next pass) and
// one change slot.
struct ImpWork {
  void* elliptic;
  double *XK, *K1, *K2, *XT, *FN, *B;  // state-sized
  double* XN;  // state-sized: X^n in double planes (handles in the mixed layout)
  double *idiff, *idiff2, *S, *r, *uK;  // fields
  ionic::BiCgWork bw;
  double* xs[3];  // xs[0] is the BiCGSTAB work's own x
  unsigned long long* change;
};

size_t imp_bytes(int n_states, long long nx, long long ny, long long nz, int max_iter) {
  const long long n = nx * ny * nz, stride = stride_of(n);
  const ionic::CgParams c = ionic::cg_params(nx, ny, nz);
  const size_t ell = (elliptic_bytes(nx, ny, nz, max_iter) + 255) / 256 * 256;
  return ell + sizeof(double) * size_t(7 * n_states * stride + 5 * stride + 2 * n) +
         ionic::BiCgWork::bytes(n, c.nb, max_iter) + 256;
}

ImpWork carve_imp(void* work, int n_states, long long nx, long long ny, long long nz,
                  int max_iter) {
  const long long n = nx * ny * nz, stride = stride_of(n);
  const ionic::CgParams c = ionic::cg_params(nx, ny, nz);
  ImpWork w;
  w.elliptic = work;
  const size_t ell = (elliptic_bytes(nx, ny, nz, max_iter) + 255) / 256 * 256;
  double* q = reinterpret_cast<double*>(static_cast<char*>(work) + ell);
  double** state_vecs[7] = {&w.XK, &w.K1, &w.K2, &w.XT, &w.FN, &w.B, &w.XN};
  for (double** v : state_vecs) {
    *v = q;
    q += size_t(n_states) * size_t(stride);
  }
  double** fields[5] = {&w.idiff, &w.idiff2, &w.S, &w.r, &w.uK};
  for (double** v : fields) {
    *v = q;
    q += stride;
  }
  double** bv[10] = {&w.bw.x, &w.bw.r, &w.bw.rh, &w.bw.p, &w.bw.ph,
                     &w.bw.v, &w.bw.s, &w.bw.sh, &w.bw.t, &w.bw.dinv};
  for (double** v : bv) {
    *v = q;
    q += n;
  }
  w.xs[0] = w.bw.x;
  for (int a = 1; a < 3; ++a) {
    w.xs[a] = q;
    q += n;
  }
  for (int a = 0; a < 5; ++a) {
    w.bw.part[a] = q;
    q += c.nb;
  }
  w.bw.sc = q;
  q += 8 + 4 * (max_iter + 2);
  w.change = reinterpret_cast<unsigned long long*>(q);
  return w;
}

// One BiCGSTAB solve of (S + cst M_L^{-1} A_i) x = r into w.xs[sys], from the
// value xs[sys] holds when warm (the same system's solution in the previous
// pass or step), else from zero.  Iterations go in batches with one
// synchronisation each, the first sized from `expect` (the previous solve's
// count); launches queued after convergence return at once.  Adds to the
// counters of info and returns the iteration count in *iters_out.
int bicg_solve(const ionic::CgParams& c, double h, double cst, ImpWork& w, int sys, int warm,
               long long expect, int max_iter, ionic_implicit_info* acc, long long* iters_out,
               hipStream_t st) {
  w.bw.x = w.xs[sys];
  IONIC_HIP(ionic::bicg_start(c, h, cst, w.S, w.r, w.bw, warm, st));
  constexpr int kBatch = 4;
  int k = 0;
  ionic::BiCgCtl ctl{0, 0, 0};
  // iteration k's first launch tests ||r_k||: a solve of m iterations ends in launch m
  int batch = int(std::min<long long>(std::max<long long>(kBatch, expect + 1), max_iter + 1));
  for (;;) {
    const int until = std::min(max_iter + 1, k + batch);
    batch = kBatch;
    for (; k < until; ++k) IONIC_HIP(ionic::bicg_iteration(c, h, cst, w.S, k, w.bw, st));
    IONIC_HIP(hipMemcpyAsync(&ctl, w.bw.sc + 4, sizeof(ctl), hipMemcpyDeviceToHost, st));
    IONIC_HIP(hipStreamSynchronize(st));
    if (ctl.done || k > max_iter) break;
  }
  const long long iters = ctl.done ? ctl.iters : max_iter;
  *iters_out = iters;
  acc->krylov_iterations += iters;
  acc->krylov_max = std::max<int32_t>(acc->krylov_max, int32_t(iters));
  if (!ctl.done) acc->krylov_converged = 0;
  return IONIC_OK;
}

}  // namespace

size_t ionic_implicit_work_bytes(int model, int64_t nx, int64_t ny, int64_t nz, int max_iter) {
  const ModelOps* o = ops_for(model);
  if (!o || nx < 1 || ny < 1 || nz < 1 || max_iter < 1 || max_iter > (1 << 20)) return 0;
  if ((__int128)nx * ny * nz >= ((__int128)1 << 31)) return 0;
  return imp_bytes(o->n_states, nx, ny, nz, max_iter);
}

int reaction_bidomain_implicit_step(ionic_sim* s, const ionic_bidomain_grid* g, double t0,
                                    double dt, int n_steps, const double* i_stim_dev,
                                    double stim_t_on, double stim_t_off, double* u_dev,
                                    void* work_dev, size_t work_bytes, double elliptic_rtol,
                                    double krylov_rtol, double inner_tol, int max_inner,
                                    int max_iter, ionic_implicit_info* info, void* hip_stream) {
  if (!s) return fail(IONIC_EINVAL, "sim is NULL");
  int rc = check_bidomain_grid(s, g);
  if (rc != IONIC_OK) return rc;
  rc = check_step_args(t0, dt, n_steps, 2, 1, stim_t_on, stim_t_off);
  if (rc != IONIC_OK) return rc;
  if (!u_dev || !work_dev) return fail(IONIC_EINVAL, "u_dev or work_dev is NULL");
  if (!(elliptic_rtol >= 0.0) || !std::isfinite(elliptic_rtol) || !(krylov_rtol >= 0.0) ||
      !std::isfinite(krylov_rtol) || !(inner_tol >= 0.0) || !std::isfinite(inner_tol))
    return fail(IONIC_EINVAL, "tolerances must be finite and >= 0");
  if (max_inner < 1 || max_inner > 1000) return fail(IONIC_EINVAL, "max_inner must be in [1, 1000]");
  if (max_iter < 1 || max_iter > (1 << 20)) return fail(IONIC_EINVAL, "max_iter out of range");
  const int ns = s->ops->n_states;
  const size_t need = imp_bytes(ns, g->nx, g->ny, g->nz, max_iter);
  if (work_bytes < need)
    return fail(IONIC_EINVAL, "implicit work buffer too small: need " + std::to_string(need) +
                                  " bytes");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  touch(s, st);
  ionic::CgParams ce = cg_params_of(g, elliptic_rtol);
  ionic::CgParams ck = cg_params_of(g, krylov_rtol);
  ImpWork w = carve_imp(work_dev, ns, g->nx, g->ny, g->nz, max_iter);
  Preconditioner pc;
  rc = prepare_preconditioner(s, ce, w.elliptic, max_iter, pc, st);
  if (rc != IONIC_OK) return rc;

  const long long n = s->n, stride = s->stride;
  const long long elems = (long long)ns * stride;
  const size_t state_bytes = sizeof(double) * size_t(elems);
  // the mixed layout: the step runs on a double copy of the state (planes of
  // stride doubles) with F, J and the eliminations in float, and stores the
  // result back in the handle's layout at the end
  const bool mixed = s->precision == IONIC_MIXED;
  double* Xn = mixed ? w.XN : static_cast<double*>(s->state);
  if (mixed) IONIC_HIP(s->ops->unpack(IONIC_MIXED, s->state, stride, 0, n, Xn, stride, st));
  const int model = s->model;
  const int ef = mixed ? 1 : 0;
  const void* pp = s->params();
  constexpr double kG = ionic::kRosGamma;
  ionic_implicit_info acc{};
  acc.converged = 1;
  acc.krylov_converged = 1;
  ionic_elliptic_info ell{0, 0.0, 1, 0};
  long long cg_last = 0;

  // one stage or correction system (sys 0, 1, 2): reduce at X, BiCGSTAB, expand
  // into out.  Each system's solve starts from its own solution in the last pass
  // (of this step or the previous one), from zero in the first pass of the call.
  long long krylov_last[3] = {0, 0, 0};
  int have_guess[3] = {0, 0, 0};
  auto stage = [&](int sys, const double* X, double c, double cf, const double* base,
                   const double* idiff, int stim_on, double* out) -> int {
    ionic::ImpBlock b{};
    b.X = X;
    b.n = n;
    b.stride = stride;
    b.stim = i_stim_dev;
    b.stim_on = stim_on;
    b.idiff = idiff;
    b.c = c;
    b.cf = cf;
    b.base = base;
    b.expand = 0;
    b.S = w.S;
    b.r = w.r;
    IONIC_HIP(ionic::imp_block(model, ef, pp, b, st));
    int rc2 = bicg_solve(ck, g->h, c, w, sys, have_guess[sys], krylov_last[sys], max_iter, &acc,
                         &krylov_last[sys], st);
    if (rc2 != IONIC_OK) return rc2;
    have_guess[sys] = 1;
    b.expand = 1;
    b.dv = w.xs[sys];
    b.out = out;
    IONIC_HIP(ionic::imp_block(model, ef, pp, b, st));
    return IONIC_OK;
  };

  for (int step = 0; step < n_steps; ++step) {
    const double t_mid = t0 + (double(step) + 0.5) * dt;
    const int on = (stim_t_on <= t_mid && t_mid < stim_t_off) ? 1 : 0;
    // G(X^n; u^n) for the correction
    IONIC_HIP(ionic::bidomain_current(ce, Xn, u_dev, g->h, w.idiff, st));
    IONIC_HIP(ionic::imp_rhs(model, ef, pp, Xn, n, stride, i_stim_dev, on, w.idiff, 1.0, 0.0, nullptr,
                             w.FN, st));
    IONIC_HIP(hipMemcpyAsync(w.XK, Xn, state_bytes, hipMemcpyDeviceToDevice, st));
    IONIC_HIP(hipMemcpyAsync(w.uK, u_dev, sizeof(double) * size_t(n), hipMemcpyDeviceToDevice, st));
    int passes = 0;
    double change = 0.0;
    for (int k = 0; k < max_inner; ++k) {
      ++passes;
      // 1. u^{k+1} from v^k
      const long long cg_before = ell.cg_iterations;
      rc = elliptic_solve_impl(s, ce, w.uK, w.elliptic, elliptic_rtol, max_iter, pc, &ell, st,
                               cg_last, w.XK);
      if (rc != IONIC_OK) return rc;
      cg_last = ell.cg_iterations - cg_before;
      // 2. ROS2 from X^n with u^{k+1}, both stages on I - gamma tau J(X^n)
      IONIC_HIP(ionic::bidomain_current(ce, Xn, w.uK, g->h, w.idiff, st));
      rc = stage(0, Xn, kG * dt, kG * dt, nullptr, w.idiff, on, w.K1);
      if (rc != IONIC_OK) return rc;
      IONIC_HIP(ionic::soa_lincomb(w.XT, Xn, ionic::kRosA21, w.K1, 0.0, nullptr, elems, st));
      IONIC_HIP(ionic::bidomain_current(ce, w.XT, w.uK, g->h, w.idiff2, st));
      IONIC_HIP(ionic::imp_rhs(model, ef, pp, w.XT, n, stride, i_stim_dev, on, w.idiff2, kG * dt,
                               -2.0, w.K1, w.B, st));
      rc = stage(1, Xn, kG * dt, 0.0, w.B, w.idiff, on, w.K2);
      if (rc != IONIC_OK) return rc;
      IONIC_HIP(ionic::soa_lincomb(w.XT, Xn, ionic::kRosM1, w.K1, ionic::kRosM2, w.K2, elems, st));
      // 3. the correction at X~ = XT: b = (X^n - X~ + tau/2 G(X^n; u^n)) + tau/2 G(X~; u^{k+1})
      IONIC_HIP(ionic::bidomain_current(ce, w.XT, w.uK, g->h, w.idiff2, st));
      IONIC_HIP(ionic::soa_lincomb(w.B, Xn, -1.0, w.XT, 0.5 * dt, w.FN, elems, st));
      rc = stage(2, w.XT, dt, 0.5 * dt, w.B, w.idiff2, on, w.K1);
      if (rc != IONIC_OK) return rc;
      // 4. X^{k+1} = X~ + eps and its scaled change from X^k
      IONIC_HIP(hipMemsetAsync(w.change, 0, sizeof(unsigned long long), st));
      IONIC_HIP(ionic::imp_finish(w.XT, w.K1, w.XK, n, stride, ns, s->ops->scale, w.change, st));
      unsigned long long bits = 0;
      IONIC_HIP(hipMemcpyAsync(&bits, w.change, sizeof(bits), hipMemcpyDeviceToHost, st));
      IONIC_HIP(hipStreamSynchronize(st));
      std::memcpy(&change, &bits, sizeof(change));
      if (change <= inner_tol) break;
    }
    if (!(change <= inner_tol)) acc.converged = 0;
    acc.steps += 1;
    acc.inner_passes += passes;
    acc.inner_max = std::max<int32_t>(acc.inner_max, passes);
    acc.last_change = change;
    IONIC_HIP(hipMemcpyAsync(Xn, w.XK, state_bytes, hipMemcpyDeviceToDevice, st));
    IONIC_HIP(hipMemcpyAsync(u_dev, w.uK, sizeof(double) * size_t(n), hipMemcpyDeviceToDevice, st));
  }
  if (mixed) IONIC_HIP(s->ops->pack(IONIC_MIXED, Xn, stride, s->state, stride, 0, n, st));
  IONIC_HIP(hipStreamSynchronize(st));
  acc.cg_iterations = ell.cg_iterations;
  if (info) *info = acc;
  return IONIC_OK;
}

int ionic_set_vertex_order(ionic_sim* s, const int32_t* order_dev, int64_t n) {
  if (!s) return fail(IONIC_EINVAL, "sim is NULL");
  if (!order_dev) {
    s->order = nullptr;
    return IONIC_OK;
  }
  if (n != s->n) return fail(IONIC_EINVAL, "order must hold one entry per vertex");
  // a non-permutation would make lanes share or leave vertices, an index out of
  // range would read outside the state: check the caller's array once, here
  std::vector<int32_t> h(static_cast<size_t>(n));
  IONIC_HIP(hipMemcpy(h.data(), order_dev, sizeof(int32_t) * size_t(n), hipMemcpyDeviceToHost));
  std::vector<unsigned char> seen(static_cast<size_t>(n), 0);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t v = h[size_t(i)];
    if (v < 0 || int64_t(v) >= n || seen[size_t(v)])
      return fail(IONIC_EINVAL, "order is not a permutation of the vertices (entry " +
                                    std::to_string(i) + ")");
    seen[size_t(v)] = 1;
  }
  s->order = order_dev;
  return IONIC_OK;
}

int ionic_set_predictor(ionic_sim* s, int predictor) {
  if (!s) return fail(IONIC_EINVAL, "sim is NULL");
  if (predictor != IONIC_PRED_NEWTON && predictor != IONIC_PRED_ROS2 &&
      predictor != IONIC_PRED_RUSH_LARSEN)
    return fail(IONIC_EUNSUPPORTED, "unknown predictor " + std::to_string(predictor));
  s->predictor = predictor;
  return IONIC_OK;
}

int reaction_sdc_adaptive(ionic_sim* s, double t0, double t_end, double dt_init, double dt_max,
                          double err_tol, int n_nodes, int n_sweeps, const double* i_stim_dev,
                          double stim_t_on, double stim_t_off, const double* i_diff_dev,
                          void* work_dev, size_t work_bytes, int64_t max_attempts,
                          double* history_dev, ionic_adapt_result* out, void* hip_stream) {
  if (!s) return fail(IONIC_EINVAL, "sim is NULL");
  if (!out) return fail(IONIC_EINVAL, "out is NULL");
  int rc = check_step_args(t0, 1.0, 0, n_nodes, n_sweeps, stim_t_on, stim_t_off);
  if (rc != IONIC_OK) return rc;
  if (!std::isfinite(t_end) || !(t_end > t0)) return fail(IONIC_EINVAL, "t_end must be finite and > t0");
  if (!(dt_init > 0.0) || !std::isfinite(dt_init)) return fail(IONIC_EINVAL, "dt_init must be positive and finite");
  if (!(dt_max > 0.0) || !std::isfinite(dt_max)) return fail(IONIC_EINVAL, "dt_max must be positive and finite");
  if (!(err_tol > 0.0) || !std::isfinite(err_tol)) return fail(IONIC_EINVAL, "err_tol must be positive and finite");
  if (max_attempts < 1) return fail(IONIC_EINVAL, "max_attempts must be >= 1");
  if (!work_dev) return fail(IONIC_EINVAL, "work_dev is NULL");
  const size_t need = bytes_of(s->ops, s->precision, s->n);
  if (work_bytes < need)
    return fail(IONIC_EINVAL, "work buffer too small: need " + std::to_string(need) + " bytes");
  if (work_dev == s->state) return fail(IONIC_EINVAL, "work_dev must differ from the state buffer");

  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  touch(s, st);
  constexpr double kDtMin = 1e-12;
  AdaptCtl* ctl = &s->dev->ctl;
  ErrSlot* err = s->dev->err;
  IONIC_HIP(ionic::adapt_init(ctl, err, t0, t_end, dt_init, dt_max, err_tol, kDtMin, stim_t_on,
                              stim_t_off, (long long)max_attempts, st));
  LaunchCommon c;
  fill_quadrature(n_nodes, c);
  c.tol = s->tol;
  c.maxit = s->maxit;
  c.n_sims = 1;
  c.ctl = ctl;
  c.err = err;
  c.state_alt = work_dev;
  // one step per attempt; t0, dt and the buffers come from the control block
  c.sims[0] = desc_of(s, t0, 1.0, i_stim_dev, stim_t_on, stim_t_off, i_diff_dev, 0, 1, n_sweeps, 0);
  const int blocks = int((s->n + kBlock - 1) / kBlock);
  const ionic::SdcLaunch launch = s->ops->sdc[s->precision][IONIC_PRED_ROS2];

  AdaptCtl h;
  std::memset(&h, 0, sizeof(h));
  h.t = t0;
  h.dt_try = std::min(dt_init, dt_max);
  int64_t enqueued = 0;
  for (;;) {
    // enough attempts to reach t_end at the current step, plus room for rejections
    const double est = std::ceil((t_end - h.t) / std::max(h.dt_try, kDtMin));
    int64_t chunk = int64_t(std::min(est, 4096.0)) + 8;
    chunk = std::min<int64_t>(chunk, max_attempts - enqueued);
    for (int64_t a = 0; a < chunk; ++a) {
      hipError_t e = launch(n_nodes, s->params(), c, blocks, st);
      if (e != hipSuccess) return hip_fail(e, "launch sdc_kernel (adaptive)");
      IONIC_HIP(ionic::adapt_control(ctl, err, history_dev, (long long)max_attempts, st));
    }
    enqueued += chunk;
    IONIC_HIP(hipMemcpyAsync(&h, ctl, sizeof(h), hipMemcpyDeviceToHost, st));
    IONIC_HIP(hipStreamSynchronize(st));
    if (h.done || enqueued >= max_attempts) break;
  }
  if (h.cur == 1)  // the last accepted state sits in the work buffer
    IONIC_HIP(hipMemcpyAsync(s->state, work_dev, need, hipMemcpyDeviceToDevice, st));
  IONIC_HIP(hipStreamSynchronize(st));
  out->t = h.t;
  out->dt_next = h.dt_try;
  out->err_last = h.err_last;
  out->accepted = h.accepted;
  out->rejected = h.rejected;
  out->reached = h.t >= t_end ? 1 : 0;
  out->failed = h.failed || !(h.t >= t_end) ? 1 : 0;
  return IONIC_OK;
}

int ionic_set_inputs(ionic_sim* s, double t0, double dt, int n_nodes, int n_sweeps,
                     const double* i_stim_dev, double stim_t_on, double stim_t_off,
                     const double* i_diff_dev) {
  if (!s) return fail(IONIC_EINVAL, "sim is NULL");
  int rc = check_step_args(t0, dt, 0, n_nodes, n_sweeps, stim_t_on, stim_t_off);
  if (rc != IONIC_OK) return rc;
  s->inputs_set = true;
  s->t0 = t0;
  s->dt = dt;
  s->M = n_nodes;
  s->K = n_sweeps;
  s->i_stim = i_stim_dev;
  s->t_on = stim_t_on;
  s->t_off = stim_t_off;
  s->i_diff = i_diff_dev;
  s->step_offset = 0;
  return IONIC_OK;
}

int reaction_sdc_step_batch(ionic_sim* const* sims, const int* n_steps, int n_sims,
                            void* hip_stream) {
  if (n_sims < 0) return fail(IONIC_EINVAL, "n_sims must be >= 0");
  if (n_sims == 0) return IONIC_OK;
  if (!sims || !n_steps) return fail(IONIC_EINVAL, "sims or n_steps is NULL");
  const ionic_sim* s0 = sims[0];
  if (!s0) return fail(IONIC_EINVAL, "sims[0] is NULL");
  for (int i = 0; i < n_sims; ++i) {
    const ionic_sim* s = sims[i];
    if (!s) return fail(IONIC_EINVAL, "sims[" + std::to_string(i) + "] is NULL");
    if (n_steps[i] < 0) return fail(IONIC_EINVAL, "n_steps[" + std::to_string(i) + "] < 0");
    if (!s->inputs_set)
      return fail(IONIC_ESTATE, "sims[" + std::to_string(i) + "]: ionic_set_inputs not called");
    if (s->model != s0->model || s->precision != s0->precision || s->M != s0->M ||
        s->predictor != s0->predictor || s->tol != s0->tol || s->maxit != s0->maxit ||
        s->raw != s0->raw)
      return fail(IONIC_ESTATE, "batched handles must share model, precision, predictor, "
                                "n_nodes, parameters and Newton settings");
    for (int k = 0; k < i; ++k)
      if (sims[k] == s) return fail(IONIC_EINVAL, "a handle appears twice in the batch");
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  LaunchCommon c;
  fill_quadrature(s0->M, c);
  c.tol = s0->tol;
  c.maxit = s0->maxit;
  int i = 0;
  while (i < n_sims) {
    int cnt = 0, blocks = 0;
    for (; i < n_sims && cnt < kMaxBatch; ++i) {
      ionic_sim* s = sims[i];
      if (n_steps[i] == 0) continue;
      c.sims[cnt] = desc_of(s, s->t0, s->dt, s->i_stim, s->t_on, s->t_off, s->i_diff,
                            s->step_offset, n_steps[i], s->K, blocks);
      blocks += int((s->n + kBlock - 1) / kBlock);
      ++cnt;
    }
    if (cnt == 0) continue;
    c.n_sims = cnt;
    hipError_t e = s0->ops->sdc[s0->precision][s0->predictor](s0->M, s0->params(), c, blocks, st);
    if (e != hipSuccess) return hip_fail(e, "launch sdc_kernel (batch)");
  }
  for (int k = 0; k < n_sims; ++k) {
    sims[k]->step_offset += n_steps[k];
    touch(sims[k], st);
  }
  return IONIC_OK;
}

int state_readback(ionic_sim* s, double* out, int64_t first, int64_t count, int out_on_device,
                   void* hip_stream) {
  if (!s) return fail(IONIC_EINVAL, "sim is NULL");
  if (!out) return fail(IONIC_EINVAL, "out is NULL");
  if (first < 0 || count < 0 || first + count > s->n)
    return fail(IONIC_EINVAL, "vertex range out of bounds");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (count == 0) return IONIC_OK;
  touch(s, st);
  const size_t bytes = size_t(s->ops->n_states) * size_t(count) * sizeof(double);
  if (out_on_device) {
    IONIC_HIP(s->ops->unpack(s->precision, s->state, s->stride, first, count, out, count, st));
    IONIC_HIP(hipStreamSynchronize(st));
    return IONIC_OK;
  }
  double* tmp = nullptr;
  IONIC_HIP(hipMalloc(&tmp, bytes));
  hipError_t e = s->ops->unpack(s->precision, s->state, s->stride, first, count, tmp, count, st);
  if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, bytes, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(tmp);
  if (e != hipSuccess) return hip_fail(e, "state_readback");
  return IONIC_OK;
}

int state_readback_noalloc(ionic_sim* s, double* out, int64_t first, int64_t count,
                           void* hip_stream) {
  if (!s) return fail(IONIC_EINVAL, "sim is NULL");
  if (!out) return fail(IONIC_EINVAL, "out is NULL");
  if (first < 0 || count < 0 || first + count > s->n)
    return fail(IONIC_EINVAL, "vertex range out of bounds");
  if (count == 0) return IONIC_OK;
  const size_t bytes = size_t(s->ops->n_states) * size_t(count) * sizeof(double);
  if (bytes > kScratchBytes)
    return fail(IONIC_EINVAL, "readback of " + std::to_string(bytes) + " bytes exceeds the " +
                                  std::to_string(kScratchBytes) + "-byte static staging buffer (" +
                                  std::to_string(kScratchBytes / (size_t(s->ops->n_states) * 8)) +
                                  " vertices of this model)");
  int dev = -1;
  IONIC_HIP(hipGetDevice(&dev));
  if (dev != s->device)
    return fail(IONIC_EINVAL, "the current device is not the handle's device");
  double* stage = nullptr;
  int rc = scratch_on_current_device(dev, &stage);
  if (rc != IONIC_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  touch(s, st);
  IONIC_HIP(s->ops->unpack(s->precision, s->state, s->stride, first, count, stage, count, st));
  IONIC_HIP(hipMemcpyAsync(out, stage, bytes, hipMemcpyDeviceToHost, st));
  IONIC_HIP(hipStreamSynchronize(st));
  return IONIC_OK;
}

int ionic_gates_to_steady_state(ionic_sim* s, void* hip_stream) {
  if (!s) return fail(IONIC_EINVAL, "sim is NULL");
  touch(s, static_cast<hipStream_t>(hip_stream));
  IONIC_HIP(s->ops->steady(s->precision, s->params(), s->state, s->stride, s->n,
                           static_cast<hipStream_t>(hip_stream)));
  return IONIC_OK;
}

int ionic_get_stats(ionic_sim* s, ionic_stats* out) {
  if (!s) return fail(IONIC_EINVAL, "sim is NULL");
  if (!out) return fail(IONIC_EINVAL, "out is NULL");
  std::vector<DevStats> d(kSlots);
  IONIC_HIP(wait_handle(s));
  const hipStream_t cs = s->n_streams ? s->streams[0] : nullptr;
  IONIC_HIP(hipMemcpyAsync(d.data(), s->stats, sizeof(DevStats) * kSlots, hipMemcpyDeviceToHost,
                           cs));
  IONIC_HIP(hipStreamSynchronize(cs));
  std::memset(out, 0, sizeof(*out));
  for (const DevStats& x : d) {  // fold the slots
    out->vertex_steps += int64_t(x.vertex_steps);
    out->newton_iters += int64_t(x.newton_iters);
    out->newton_solves += int64_t(x.newton_solves);
    out->n_nonconverged += int64_t(x.nonconverged);
    out->n_nonfinite += int64_t(x.nonfinite);
    out->newton_it_max = std::max(out->newton_it_max, int32_t(x.it_max));
  }
  return IONIC_OK;
}

int ionic_reset_stats(ionic_sim* s) {
  if (!s) return fail(IONIC_EINVAL, "sim is NULL");
  IONIC_HIP(wait_handle(s));
  const hipStream_t cs = s->n_streams ? s->streams[0] : nullptr;
  IONIC_HIP(hipMemsetAsync(s->stats, 0, sizeof(DevStats) * kSlots, cs));
  IONIC_HIP(hipStreamSynchronize(cs));
  return IONIC_OK;
}

int ionic_debug_jacobian(ionic_sim* s, int64_t vertex, double i_stim, double i_diff,
                         double* F_out, double* J_out, void* hip_stream) {
  if (!s) return fail(IONIC_EINVAL, "sim is NULL");
  if (vertex < 0 || vertex >= s->n) return fail(IONIC_EINVAL, "vertex out of range");
  if (!F_out || !J_out) return fail(IONIC_EINVAL, "F_out or J_out is NULL");
  const int n = s->ops->n_states;
  const size_t bytes = size_t(n + n * n) * sizeof(double);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  touch(s, st);
  double* tmp = nullptr;
  IONIC_HIP(hipMalloc(&tmp, bytes));
  std::vector<double> host(size_t(n + n * n));
  hipError_t e = s->ops->debug_jac(s->precision, s->params(), s->state, s->stride, vertex, i_stim,
                                   i_diff, tmp, st);
  if (e == hipSuccess) e = hipMemcpyAsync(host.data(), tmp, bytes, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(tmp);
  if (e != hipSuccess) return hip_fail(e, "ionic_debug_jacobian");
  std::memcpy(F_out, host.data(), sizeof(double) * n);
  std::memcpy(J_out, host.data() + n, sizeof(double) * n * n);
  return IONIC_OK;
}

}  // extern "C"
