// C ABI of the ADER-DG library: context, argument checks, allocation and
// the launch sequence of one step.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ader.h"
#include "kernel_set.hpp"

using namespace ader;

namespace {

constexpr size_t kLdsBytes = 160 * 1024;  // LDS per workgroup on gfx950
constexpr size_t kSmallSpill = 16;        // scratch bytes per lane a candidate may use in the first passes
constexpr int kTotBlocks = 512;           // blocks of the conservation-sum reduction

struct ProbState {
  ader_problem desc{};
  int D = 0, N = 0, n = 0, m = 0, nd = 0, nst = 0, nf = 0;
  int64_t E = 0;
  Geom g{};
  double h[3] = {1, 1, 1};
  Ops ops{};
  double coef = 0.0;  // cfl * alpha_N
  int sweeps = 0;
  int64_t u_off = 0, u_cnt = 0, q_off = 0, q_cnt = 0;
  KernelSet ks{};
  int cls = 0;                      // kernel class (batched launches)
  PredVariant pv{};                 // chosen predictor variant (the class's)
  bool tuned = false;               // chosen by timing (else default or forced)
  double tune_ms = 0.0;             // measured time of the chosen variant on the sample
  std::vector<PredVariant> cand;    // predictor variants that fit this problem
  size_t trace_elt = 8;             // bytes per trace value
  OpsSweep sw{};            // sweep operators (host copy)
  OpsSweep *sw_dev = nullptr;  // device copy read by the predictor
  Ops *ops_dev = nullptr;   // device copy of the tables (outputs, faces, update read them by pointer)
  double *mat = nullptr, *ustar = nullptr, *acc = nullptr;
  double *summ = nullptr;           // detection: [E][m][2] extremes of the state before a step
  void *hist = nullptr;             // guess 3: [E][m][N][nd] Taylor coefficients of the last predictor
  int64_t e_off = 0;                // offset of the problem's elements in the flag array
  void *trace[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
  void *GL[3] = {nullptr, nullptr, nullptr}, *GR[3] = {nullptr, nullptr, nullptr};  // trace type
};

// Problems that share every kernel (dimension, degree, PDE, precision) run
// as one batched launch per stage: per-problem argument records and tile
// prefixes live in device memory, and persistent workgroups stride over the
// tiles of all problems of the class.
struct KClass {
  std::vector<int> probs;
  PredVariant pv{};
  bool tuned = false;
  double tune_ms = 0.0;
  int D = 0;
  const void *face[3] = {nullptr, nullptr, nullptr};
  const void *update = nullptr, *cfl = nullptr, *detect = nullptr;
  bool face_avg = false;                   // face integrals from time-averaged traces
  PredArgs *pargs = nullptr;               // device [np]
  DetArgs *dargs = nullptr;                // device [np], once detection is enabled
  FaceArgs *fargs[3] = {nullptr, nullptr, nullptr};
  UpdArgs *uargs = nullptr;
  CflArgs *cargs = nullptr;
  int64_t *pstart = nullptr, *cstart = nullptr;  // device [np+1]
  RowTile *ftiles = nullptr, *utiles = nullptr;   // device [ftot], [utot]
  int64_t ptot = 0, ftot = 0, utot = 0, ctot = 0;  // tiles
  int pgrid = 0, fgrid[3] = {0, 0, 0}, ugrid = 0, cgrid = 0;  // persistent grid sizes
};

}  // namespace

struct ader_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  hipStream_t cur = nullptr;   // stream the launches go to (the capture stream while capturing)
  hipStream_t gstream = nullptr;  // graph replays (created on first use)
  hipGraphExec_t gexec = nullptr;
  double *g_u = nullptr;
  int g_steps = 0;
  hipEvent_t g_in = nullptr, g_out = nullptr;
  std::vector<ProbState> P;
  std::vector<KClass> K;
  double *dt = nullptr, *t = nullptr, *tnext = nullptr;  // device [nprob]
  double *coef = nullptr, *tend = nullptr;               // device [nprob]
  bool detect = false;                                   // a posteriori detection after each step
  int *flags = nullptr;                                  // device [total elements]
  int64_t total_e = 0;
  std::vector<double> tend_host;                         // values held by tend
  unsigned long long *smax = nullptr;    // device [nprob][kSmaxPerProblem] slots, time-step kernel maxima
  unsigned long long *smax_f = nullptr;  // device, the same slots: maxima taken by the update
  const double *fused_u = nullptr;  // state buffer whose maxima smax_f holds (written by the last step)
  int *hist_ok = nullptr;           // device [1]: the guess-3 history belongs to the state in hist_u
  double *dtprev = nullptr;         // device [nprob]: step of the last completed step
  const double *hist_u = nullptr;   // state buffer of the last completed ader_step / ader_run
  int *err = nullptr;                                      // device [1]
  double *partial = nullptr, *sums = nullptr;              // totals scratch
  int64_t total_u = 0, total_q = 0, total_m = 0;
  std::string msg;
  std::vector<void *> allocs;
  bool profile = false;
  std::vector<hipEvent_t> ev_pool, ev_used;  // 5 boundaries per profiled step
};

namespace {

thread_local std::string g_create_msg = "";  // message of the last failed ader_create

ader_status fail(ader_ctx *c, ader_status s, const std::string &m) {
  if (c) c->msg = m;
  return s;
}

#define HIP_OR_FAIL(ctx, call)                                                          \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(ctx, ADER_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

ader_status dalloc(ader_ctx *c, void **p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(c, ADER_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  c->allocs.push_back(*p);
  return ADER_OK;
}

KernelSet kernels_for(const ader_problem &d) {
  if (d.pde == ADER_EULER) return d.dim == 2 ? kernels_euler2(d.degree) : kernels_euler3(d.degree);
  return kernels_elastic3(d.degree);
}

ader_status validate(ader_ctx *c, const ader_problem &d, int i) {
  const std::string w = "problem " + std::to_string(i) + ": ";
  if (d.dim != 2 && d.dim != 3) return fail(c, ADER_ERR_INVALID, w + "dim must be 2 or 3");
  if (d.degree < 0) return fail(c, ADER_ERR_INVALID, w + "degree must be >= 0");
  if (d.degree > 7) return fail(c, ADER_ERR_UNSUPPORTED, w + "degree > 7 is not built");
  for (int a = 0; a < d.dim; a++) {
    if (d.nelem[a] < 1) return fail(c, ADER_ERR_INVALID, w + "nelem must be >= 1");
    if (d.nelem[a] > 65535) return fail(c, ADER_ERR_UNSUPPORTED, w + "nelem must be <= 65535");
    if (!(d.hi[a] > d.lo[a]) || !isfinite(d.hi[a] - d.lo[a]))
      return fail(c, ADER_ERR_INVALID, w + "hi must exceed lo");
  }
  if (d.pde != ADER_EULER && d.pde != ADER_ELASTIC) return fail(c, ADER_ERR_INVALID, w + "unknown pde");
  if (d.pde == ADER_EULER && !(d.gamma > 1.0)) return fail(c, ADER_ERR_INVALID, w + "gamma must exceed 1");
  if (d.pde == ADER_ELASTIC) {
    if (d.dim != 3) return fail(c, ADER_ERR_UNSUPPORTED, w + "elasticity is 3-D only");
    if (!d.material) return fail(c, ADER_ERR_INVALID, w + "elasticity needs a material array");
    const int64_t E = (int64_t)d.nelem[0] * d.nelem[1] * d.nelem[2];
    for (int64_t e = 0; e < E; e++) {
      const double *mt = d.material + 3 * e;
      if (!(mt[0] > 0.0) || !(mt[2] >= 0.0) || !(mt[1] + 2.0 * mt[2] > 0.0) || !isfinite(mt[0]) ||
          !isfinite(mt[1]) || !isfinite(mt[2]))
        return fail(c, ADER_ERR_INVALID, w + "invalid material at element " + std::to_string(e));
    }
  }
  if (d.prec != ADER_FP64 && d.prec != ADER_FP32 && d.prec != ADER_BF16)
    return fail(c, ADER_ERR_INVALID, w + "unknown precision");
  if (d.picard_iters < 0) return fail(c, ADER_ERR_INVALID, w + "picard_iters must be >= 0");
  if (d.guess < 0 || d.guess > 3) return fail(c, ADER_ERR_INVALID, w + "guess must be 0, 1, 2 or 3");
  if (d.face_avg != 0 && d.face_avg != 1) return fail(c, ADER_ERR_INVALID, w + "face_avg must be 0 or 1");
  if (!(d.cfl > 0.0) || d.cfl > 1.0) return fail(c, ADER_ERR_INVALID, w + "cfl must be in (0, 1]");
  return ADER_OK;
}

// dt of every problem from its mesh maximum S: dt = coef / S, clipped so
// that the last step lands on t_end (when clip is set); resets the maximum.
// One workgroup: it first decides whether any S is not a positive finite
// number, then writes every dt.  While the error flag is raised (by the
// time-step kernel, by an earlier step, or here) every problem takes dt = 0,
// independently of thread timing.
constexpr int kFinBlock = 256;
// Maximum over the slots of problem i (bit patterns of positive doubles).
__device__ __forceinline__ double slots_max(unsigned long long *smax, int i) {
  unsigned long long m = 0ull;
  for (int k = 0; k < kSmaxSlots; k++) m = max(m, *smax_slot(smax, i, k));
  return __longlong_as_double((long long)m);
}
// smax is the buffer of maxima this step uses; both it and smax_f (the
// update's buffer, filled again by this step's update) are cleared.
__global__ void __launch_bounds__(kFinBlock) k_finalize(unsigned long long *smax, unsigned long long *smax_f,
                                                        int *err, const double *coef, const double *tend, int clip,
                                                        const double *t, double *dt, double *tnext, int np) {
  const int prior = *err;  // written before this kernel (it writes err only after the barrier)
  int bad = 0;
  for (int i = threadIdx.x; i < np; i += kFinBlock) {
    const double S = slots_max(smax, i);
    if (!(S > 0.0) || isinf(S)) bad = 1;
  }
  const bool stop = __syncthreads_or(bad) || prior;
  for (int i = threadIdx.x; i < np; i += kFinBlock) {
    const double S = slots_max(smax, i);
    for (int k = 0; k < kSmaxSlots; k++) {
      *smax_slot(smax, i, k) = 0ull;
      *smax_slot(smax_f, i, k) = 0ull;
    }
    double d = stop ? 0.0 : coef[i] / S;
    double tn = t[i] + d;
    if (clip) {
      const double rem = tend[i] - t[i];
      if (rem <= d) {  // the last step lands exactly on t_end
        d = rem > 0.0 ? rem : 0.0;
        tn = rem > 0.0 ? tend[i] : t[i];
      }
    }
    dt[i] = d;
    tnext[i] = tn;
  }
  if (bad) atomicOr(err, 1);
}

__global__ void k_zero_u64(unsigned long long *p, int n) {
  const int i = threadIdx.x + blockIdx.x * blockDim.x;
  if (i < n) p[i] = 0ull;
}

// End of a step: the new time, the step just taken (the previous interval
// of the next step's guess 3) and the mark that the history is current.
__global__ void k_commit(double *t, const double *tnext, const double *dt, double *dtprev, int *hist_ok, int np) {
  const int i = threadIdx.x + blockIdx.x * blockDim.x;
  if (i < np) {
    t[i] = tnext[i];
    dtprev[i] = dt[i];
  }
  if (i == 0) *hist_ok = 1;
}

__global__ void k_set_int(int *p, int v) { *p = v; }

// Conservation sums: per-block partial sums in a fixed order, then a
// sequential pass over the blocks; deterministic for a given grid.
__global__ void __launch_bounds__(kBlock) k_totals_partial(const double *u, int64_t E, int m, int nd,
                                                          int n, int D, Ops ops, double vol,
                                                          double *partial) {
  __shared__ double red[kBlock];
  for (int v = 0; v < m; v++) {
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < E * nd;
         i += (int64_t)gridDim.x * kBlock) {
      const int64_t e = i / nd;
      const int k = (int)(i - e * nd);
      double wk = vol;
      int kk = k;
      for (int a = 0; a < D; a++) {
        wk *= ops.w[kk % n];
        kk /= n;
      }
      s += wk * u[(e * m + v) * nd + k];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * m + v] = red[0];
    __syncthreads();
  }
}

__global__ void k_totals_final(const double *partial, int nblk, int m, double *out) {
  const int v = threadIdx.x;
  if (v >= m) return;
  double s = 0.0;
  for (int b = 0; b < nblk; b++) s += partial[(int64_t)b * m + v];
  out[v] = s;
}

// Scratch of ader_totals_noalloc: the per-block partial sums of
// k_totals_partial, kTotBlocks x (at most 9 variables) doubles (36 KB).  Each
// device holds its own copy until the process ends.  In host code the name
// only stands for the array; kernels get its device address, taken once per
// device with hipGetSymbolAddress.
constexpr int kScratchVars = 9;
__device__ __align__(256) double scratch[kTotBlocks * kScratchVars];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

// The device address of `scratch` on the current device (looked up on the
// first call per device).
hipError_t scratch_address(double **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double *)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// One batched launch: `grid` persistent workgroups over `tiles` tiles.
ader_status launch(ader_ctx *c, const void *fn, int64_t tiles, int grid, int threads, size_t shmem,
                   void **args) {
  if (tiles <= 0) return ADER_OK;
  if (grid < 1) return fail(c, ADER_ERR_UNSUPPORTED, "grid too large");
  HIP_OR_FAIL(c, hipLaunchKernel(fn, dim3((unsigned)grid), dim3(threads), args, shmem, c->cur));
  return ADER_OK;
}

// Uniform state u[e][v][k] = val[v] (used to time predictor variants).
__global__ void k_fill_state(double *u, int64_t count, int m, int nd, double v0, double v1, double v2,
                             double v3, double v4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int v = (int)((i / nd) % m);
  const double vals[5] = {v0, v1, v2, v3, v4};
  u[i] = v < 5 ? vals[v] : 0.0;
}

std::mutex g_tune_mu;
std::map<std::string, std::string> g_tune_cache;  // configuration -> variant name

PredArgs pred_args(const ader_ctx *c, const ProbState &s, int p) {
  PredArgs a{};
  a.hist = s.hist;
  a.dtprev = c->dtprev;
  a.hist_ok = c->hist_ok;
  a.sw = s.sw_dev;
  a.ops = s.ops_dev;
  a.g = s.g;
  a.u_off = s.u_off;
  a.q_off = s.q_off;
  a.pidx = p;
  a.mat = s.mat;
  a.ustar = s.ustar;
  for (int ax = 0; ax < 3; ax++)
    for (int sd = 0; sd < 2; sd++) a.trace[ax][sd] = s.trace[ax][sd];
  a.acc_glob = s.acc;
  a.sweeps = s.sweeps;
  a.guess = s.desc.guess;
  a.face_avg = s.desc.face_avg != 0;
  return a;
}

ader_status upload(ader_ctx *c, void **dst, const void *src, size_t bytes) {
  ader_status st = dalloc(c, dst, bytes);
  if (st) return st;
  HIP_OR_FAIL(c, hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
  return ADER_OK;
}

// Time every candidate predictor variant of a class on a uniform state of
// up to 32768 elements of its largest problem (the kernels have no
// data-dependent branches) and keep the fastest.  Results are cached per
// configuration for the process.
ader_status tune_class(ader_ctx *c, KClass &k, const std::vector<PredVariant> &cand) {
  int pl = k.probs[0];
  for (int p : k.probs)
    if (c->P[p].E > c->P[pl].E) pl = p;
  ProbState &s = c->P[pl];
  const int64_t Et = s.E < 32768 ? s.E : 32768;
  const std::string key = std::to_string(s.D) + "/" + std::to_string(s.N) + "/" +
                          std::to_string(s.desc.pde) + "/" + std::to_string(s.desc.prec) + "/" +
                          std::to_string(Et) + "/" + std::to_string(s.sweeps) + "/" + std::to_string(s.desc.guess);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end())
      for (const PredVariant &v : cand)
        if (it->second == v.name) {
          k.pv = v;
          k.tuned = true;
          return ADER_OK;
        }
  }
  // the timing state, released on every return (hipFree waits for the launches)
  struct Scratch {
    double *ut = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Scratch() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      if (ut) (void)hipFree(ut);
    }
  } sc;
  const int64_t cnt = Et * s.m * s.nd;
  if (hipMalloc(&sc.ut, cnt * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    sc.ut = nullptr;
    return ADER_OK;  // no room to tune: keep the default
  }
  double *ut = sc.ut;
  PredArgs a = pred_args(c, s, pl);
  a.u_off = 0;
  const int64_t start[2] = {0, Et};
  PredArgs *a_dev = nullptr;
  int64_t *st_dev = nullptr;
  ader_status st;
  if ((st = upload(c, (void **)&a_dev, &a, sizeof(a))) || (st = upload(c, (void **)&st_dev, start, sizeof(start))))
    return st;
  const double ie = 1.0 / (s.desc.gamma - 1.0);  // Euler: rho = 1, v = 0, p = 1
  const unsigned nb = (unsigned)((cnt + 255) / 256);
  if (s.desc.pde == ADER_EULER)
    hipLaunchKernelGGL(k_fill_state, dim3(nb), dim3(256), 0, c->cur, ut, cnt, s.m, s.nd, 1.0, 0.0, 0.0,
                       s.D == 2 ? ie : 0.0, s.D == 3 ? ie : 0.0);
  else
    hipLaunchKernelGGL(k_fill_state, dim3(nb), dim3(256), 0, c->cur, ut, cnt, s.m, s.nd, 0.0, 0.0, 0.0,
                       1.0, 1.0);
  const double dt_tune = 1e-6;
  HIP_OR_FAIL(c, hipMemcpyAsync(c->dt + pl, &dt_tune, sizeof(double), hipMemcpyHostToDevice, c->cur));
  if (s.desc.guess == 3) {  // time the steady state: a previous interval (zero history) of the same step
    const int one = 1;
    HIP_OR_FAIL(c, hipMemcpyAsync(c->dtprev + pl, &dt_tune, sizeof(double), hipMemcpyHostToDevice, c->cur));
    HIP_OR_FAIL(c, hipMemcpyAsync(c->hist_ok, &one, sizeof(int), hipMemcpyHostToDevice, c->cur));
  }
  HIP_OR_FAIL(c, hipEventCreate(&sc.e0));
  HIP_OR_FAIL(c, hipEventCreate(&sc.e1));
  hipEvent_t e0 = sc.e0, e1 = sc.e1;
  Batch b{st_dev, 1};
  const double *dtp = c->dt;
  double *qn = nullptr;
  void *args[] = {&a_dev, &b, &ut, &dtp, &qn};
  double best = 1e30;
  PredVariant bestv = k.pv;
  const char *tl = getenv("ADER_TUNE_LOG");  // print every candidate's time
  const bool tune_log = tl && *tl && strcmp(tl, "0") != 0;
  st = ADER_OK;
  for (const PredVariant &v : cand) {
    const int grid = (int)Et;  // one element per workgroup
    if ((st = launch(c, v.fn, Et, grid, v.threads, v.lds, args))) break;  // warm-up
    HIP_OR_FAIL(c, hipEventRecord(e0, c->cur));
    for (int r = 0; r < 3 && !st; r++) st = launch(c, v.fn, Et, grid, v.threads, v.lds, args);
    HIP_OR_FAIL(c, hipEventRecord(e1, c->cur));
    HIP_OR_FAIL(c, hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_OR_FAIL(c, hipEventElapsedTime(&ms, e0, e1));
    if (st) break;
    if (tune_log) fprintf(stderr, "[ader tune] %s %s %.4f ms\n", key.c_str(), v.name, ms / 3.0);
    if (ms / 3.0 < best) {
      best = ms / 3.0;
      bestv = v;
    }
  }
  HIP_OR_FAIL(c, hipStreamSynchronize(c->cur));
  if (st) return st;
  const double zero = 0.0;
  const int izero = 0;
  HIP_OR_FAIL(c, hipMemcpy(c->dt + pl, &zero, sizeof(double), hipMemcpyHostToDevice));
  HIP_OR_FAIL(c, hipMemcpy(c->dtprev + pl, &zero, sizeof(double), hipMemcpyHostToDevice));
  HIP_OR_FAIL(c, hipMemcpy(c->hist_ok, &izero, sizeof(int), hipMemcpyHostToDevice));
  k.pv = bestv;
  k.tuned = true;
  k.tune_ms = best;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = bestv.name;
  return ADER_OK;
}

// Argument records, tile prefixes and persistent grids of a class.
ader_status build_class(ader_ctx *c, KClass &k) {
  const int np = (int)k.probs.size();
  std::vector<PredArgs> pa(np);
  std::vector<FaceArgs> fa[3];
  std::vector<UpdArgs> ua(np);
  std::vector<CflArgs> ca(np);
  std::vector<int64_t> ps(np + 1, 0), cs(np + 1, 0);
  std::vector<RowTile> ft, ut;
  const int fpb = k.face_avg ? face_avg_per_block(k.D, c->P[k.probs[0]].N) : face_per_block(k.D, c->P[k.probs[0]].N);
  for (int a = 0; a < 3; a++) fa[a].resize(np);
  for (int i = 0; i < np; i++) {
    const int p = k.probs[i];
    ProbState &s = c->P[p];
    s.pv = k.pv;
    s.tuned = k.tuned;
    s.tune_ms = k.tune_ms;
    pa[i] = pred_args(c, s, p);
    const int nx = s.g.nel[0], rows = s.g.nel[1] * s.g.nel[2];
    for (int ax = 0; ax < s.D; ax++) {
      FaceArgs &f = fa[ax][i];
      f.ops = s.ops_dev;
      f.g = s.g;
      f.trace0 = s.trace[ax][0];
      f.trace1 = s.trace[ax][1];
      f.mat = s.mat;
      f.GL = s.GL[ax];
      f.GR = s.GR[ax];
      f.cx = (nx + fpb - 1) / fpb;
    }
    UpdArgs &u = ua[i];
    u.ops = s.ops_dev;
    u.g = s.g;
    u.ustar = s.ustar;
    for (int ax = 0; ax < 3; ax++) {
      u.GL[ax] = s.GL[ax];
      u.GR[ax] = s.GR[ax];
    }
    u.u_off = s.u_off;
    u.pidx = p;
    const int ept = upd_elems(s.D, s.N, s.m);
    u.cx = (nx + ept - 1) / ept;
    for (int ax = 0; ax < 3; ax++) u.h[ax] = s.h[ax];
    u.mat = s.mat;
    CflArgs &cf = ca[i];
    cf.g = s.g;
    for (int ax = 0; ax < 3; ax++) cf.h[ax] = s.h[ax];
    cf.u_off = s.u_off;
    cf.mat = s.mat;
    cf.pidx = p;
    cf.summ = c->detect ? s.summ : nullptr;
    ps[i + 1] = ps[i] + s.E;
    cs[i + 1] = cs[i] + rows;
    for (int r = 0; r < rows; r++) {
      const int iy = r % s.g.nel[1], iz = r / s.g.nel[1];
      for (int bx = 0; bx < fa[0][i].cx; bx++) ft.push_back(RowTile{i, p, bx, (uint32_t)iy | (uint32_t)iz << 16});
      for (int bx = 0; bx < u.cx; bx++) ut.push_back(RowTile{i, p, bx, (uint32_t)iy | (uint32_t)iz << 16});
    }
  }
  ader_status st;
  const size_t b64 = (np + 1) * sizeof(int64_t);
  if ((st = upload(c, (void **)&k.pargs, pa.data(), np * sizeof(PredArgs))) ||
      (st = upload(c, (void **)&k.uargs, ua.data(), np * sizeof(UpdArgs))) ||
      (st = upload(c, (void **)&k.cargs, ca.data(), np * sizeof(CflArgs))) ||
      (st = upload(c, (void **)&k.pstart, ps.data(), b64)) || (st = upload(c, (void **)&k.cstart, cs.data(), b64)) ||
      (st = upload(c, (void **)&k.ftiles, ft.data(), ft.size() * sizeof(RowTile))) ||
      (st = upload(c, (void **)&k.utiles, ut.data(), ut.size() * sizeof(RowTile))))
    return st;
  for (int ax = 0; ax < k.D; ax++)
    if ((st = upload(c, (void **)&k.fargs[ax], fa[ax].data(), np * sizeof(FaceArgs)))) return st;
  k.ptot = ps[np];
  k.ftot = (int64_t)ft.size();
  k.utot = (int64_t)ut.size();
  k.ctot = cs[np];
  if (k.ptot > 0x7fffffff) return fail(c, ADER_ERR_UNSUPPORTED, "more than 2^31-1 elements in one kernel class");
  k.pgrid = (int)k.ptot;  // the predictor takes one element per workgroup
  // face, update and time-step kernels: one tile per workgroup as well (the
  // grid-stride loops then run once); these stages are bound by HBM and
  // gain from every workgroup the device can hold
  if (k.ftot > 0x7fffffff || k.utot > 0x7fffffff) return fail(c, ADER_ERR_UNSUPPORTED, "grid too large");
  for (int ax = 0; ax < k.D; ax++) k.fgrid[ax] = (int)k.ftot;
  k.ugrid = (int)k.utot;
  k.cgrid = (int)k.ctot;
  return ADER_OK;
}

// Per-problem maxima of the wave speed of u into `out` (the time-step kernel).
ader_status run_maxima(ader_ctx *c, const double *u, unsigned long long *out) {
  for (KClass &k : c->K) {
    Batch b{k.cstart, (int)k.probs.size()};
    void *args[] = {&k.cargs, &b, &u, &out, &c->err};
    ader_status st = launch(c, k.cfl, k.ctot, k.cgrid, kBlock, 0, args);
    if (st) return st;
  }
  return ADER_OK;
}

// Every problem's dt (clipped to the t_end values held by c->tend when
// clip is set) from the maxima of u: taken here by the time-step kernel,
// or (fused) those the previous step's update took of the state it wrote.
ader_status run_cfl(ader_ctx *c, const double *u, int clip, bool fused = false) {
  ader_status st;
  if (!fused && (st = run_maxima(c, u, c->smax))) return st;
  const int np = (int)c->P.size();
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinBlock), 0, c->cur, fused ? c->smax_f : c->smax, c->smax_f,
                     c->err, c->coef, c->tend, clip, c->t, c->dt, c->tnext, np);
  HIP_OR_FAIL(c, hipGetLastError());
  return ADER_OK;
}

ader_status run_predictor(ader_ctx *c, const double *u, const double *dt_dev, double *qhat) {
  const double *dt = dt_dev ? dt_dev : c->dt;
  for (KClass &k : c->K) {
    Batch b{k.pstart, (int)k.probs.size()};
    void *args[] = {&k.pargs, &b, &u, &dt, &qhat};
    ader_status st = launch(c, k.pv.fn, k.ptot, k.pgrid, k.pv.threads, k.pv.lds, args);
    if (st) return st;
  }
  return ADER_OK;
}

ader_status run_faces(ader_ctx *c) {
  for (KClass &k : c->K) {
    for (int ax = 0; ax < k.D; ax++) {
      void *args[] = {&k.fargs[ax], &k.ftiles, &k.ftot};
      ader_status st = launch(c, k.face[ax], k.ftot, k.fgrid[ax], kBlock, 0, args);
      if (st) return st;
    }
  }
  return ADER_OK;
}

// The update; with `maxima` it also takes the wave-speed maxima of the new
// state into smax_f (the next step's time step then needs no pass over u).
ader_status run_update(ader_ctx *c, double *u, const double *dt_dev, bool maxima = false) {
  const double *dt = dt_dev ? dt_dev : c->dt;
  unsigned long long *sm = maxima ? c->smax_f : nullptr;
  for (KClass &k : c->K) {
    void *args[] = {&k.uargs, &k.utiles, &k.utot, &u, &dt, &sm, &c->err};
    ader_status st = launch(c, k.update, k.utot, k.ugrid, kBlock, 0, args);
    if (st) return st;
  }
  return ADER_OK;
}

ader_status run_corrector(ader_ctx *c, double *u, const double *dt_dev) {
  ader_status st = run_faces(c);
  return st ? st : run_update(c, u, dt_dev);
}

ader_status mark(ader_ctx *c) {
  if (!c->profile) return ADER_OK;
  hipEvent_t ev;
  if (!c->ev_pool.empty()) {
    ev = c->ev_pool.back();
    c->ev_pool.pop_back();
  } else {
    HIP_OR_FAIL(c, hipEventCreate(&ev));
  }
  c->ev_used.push_back(ev);
  HIP_OR_FAIL(c, hipEventRecord(ev, c->cur));
  return ADER_OK;
}

ader_status check_flag(ader_ctx *c) {
  int flag = 0;
  HIP_OR_FAIL(c, hipMemcpyAsync(&flag, c->err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  if (flag) {
    int zero = 0;
    HIP_OR_FAIL(c, hipMemcpyAsync(c->err, &zero, sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return fail(c, ADER_ERR_NONFINITE, "non-finite or non-physical state (NaN/Inf, rho <= 0 or p <= 0)");
  }
  return ADER_OK;
}

// Detection records of a class, and the time-step records with or without
// the per-element extremes (re-uploaded when detection is switched).
ader_status refresh_detection(ader_ctx *c, KClass &k) {
  const int np = (int)k.probs.size();
  std::vector<CflArgs> ca(np);
  HIP_OR_FAIL(c, hipMemcpy(ca.data(), k.cargs, np * sizeof(CflArgs), hipMemcpyDeviceToHost));
  for (int i = 0; i < np; i++) ca[i].summ = c->detect ? c->P[k.probs[i]].summ : nullptr;
  HIP_OR_FAIL(c, hipMemcpy(k.cargs, ca.data(), np * sizeof(CflArgs), hipMemcpyHostToDevice));
  if (c->detect && !k.dargs) {
    std::vector<DetArgs> da(np);
    for (int i = 0; i < np; i++) {
      const ProbState &s = c->P[k.probs[i]];
      da[i].g = s.g;
      da[i].u_off = s.u_off;
      da[i].summ = s.summ;
      da[i].flags = c->flags + s.e_off;
    }
    ader_status st = upload(c, (void **)&k.dargs, da.data(), np * sizeof(DetArgs));
    if (st) return st;
  }
  return ADER_OK;
}

ader_status run_detect(ader_ctx *c, const double *u) {
  for (KClass &k : c->K) {
    Batch b{k.cstart, (int)k.probs.size()};
    void *args[] = {&k.dargs, &b, &u};
    ader_status st = launch(c, k.detect, k.ctot, k.cgrid, kBlock, 0, args);
    if (st) return st;
  }
  return ADER_OK;
}

// Make the device t_end values equal to t_end_host (a synchronous copy,
// only when they change).
ader_status set_tend(ader_ctx *c, const double *t_end_host) {
  const size_t np = c->P.size();
  bool same = true;
  for (size_t i = 0; i < np && same; i++) same = c->tend_host[i] == t_end_host[i];
  if (same) return ADER_OK;
  if (c->gexec) {  // a captured replay may still read the old values
    HIP_OR_FAIL(c, hipStreamSynchronize(c->gstream));
  }
  c->tend_host.assign(t_end_host, t_end_host + np);
  HIP_OR_FAIL(c, hipMemcpyAsync(c->tend, c->tend_host.data(), np * sizeof(double), hipMemcpyHostToDevice,
                                c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return ADER_OK;
}

// The guess-3 history (the previous interval's predictor) is current only
// for the state the last step of this context wrote: before a step on any
// other buffer, mark it stale (that step is then the plain scheme).
ader_status history_for(ader_ctx *c, const double *u) {
  if (c->hist_u == u) return ADER_OK;
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, c->stream, c->hist_ok, 0);
  HIP_OR_FAIL(c, hipGetLastError());
  c->hist_u = nullptr;
  return ADER_OK;
}

// The launches of one step on c->cur: dt, predictor, faces, update, commit
// of the new time.  Profiling events are recorded only outside captures.
// With `fused` the step's dt comes from the maxima the previous step's
// update took (smax_f holds them for this u); else the time-step kernel
// reads u.  The update takes the maxima of the new state unless detection is
// on (the time-step kernel then also records the per-element extremes the
// detection needs).
ader_status step_launches(ader_ctx *c, double *u, bool marks, bool fused) {
  ader_status st;
  const bool m = marks && c->profile;
  if ((m && (st = mark(c))) || (st = run_cfl(c, u, 1, fused))) return st;
  if ((m && (st = mark(c))) || (st = run_predictor(c, u, nullptr, nullptr))) return st;
  if ((m && (st = mark(c))) || (st = run_faces(c))) return st;
  if ((m && (st = mark(c))) || (st = run_update(c, u, nullptr, !c->detect))) return st;
  if (c->detect && (st = run_detect(c, u))) return st;  // timed with the update stage
  if (m && (st = mark(c))) return st;
  const int np = (int)c->P.size();
  hipLaunchKernelGGL(k_commit, dim3((np + 255) / 256), dim3(256), 0, c->cur, c->t, c->tnext, c->dt, c->dtprev,
                     c->hist_ok, np);
  HIP_OR_FAIL(c, hipGetLastError());
  return ADER_OK;
}

}  // namespace

extern "C" {

const char *ader_version(void) { return "ader-mi355x 0.1 (gfx950)"; }

ader_status ader_stability_alpha(int32_t degree, double *alpha) {
  if (!alpha || degree < 0) return ADER_ERR_INVALID;
  if (degree > 7) return ADER_ERR_UNSUPPORTED;
  *alpha = stability_alpha(degree);
  return ADER_OK;
}

ader_status ader_basis(int32_t degree, double *xi, double *w, double *dhat, double *tmat) {
  if (degree < 0) return ADER_ERR_INVALID;
  if (degree > 7) return ADER_ERR_UNSUPPORTED;
  Ops o;
  if (build_ops(degree, &o)) return ADER_ERR_INVALID;
  const int n = degree + 1;
  for (int i = 0; i < n; i++) {
    if (xi) xi[i] = o.xi[i];
    if (w) w[i] = o.w[i];
    for (int j = 0; j < n; j++) {
      if (dhat) dhat[i * n + j] = o.D[i * kMaxN + j];
      if (tmat) tmat[i * n + j] = o.T[i * kMaxN + j];
    }
  }
  return ADER_OK;
}

ader_status ader_create(const ader_problem *probs, int32_t nprob, void *hip_stream, ader_ctx **out) {
  if (!out) return ADER_ERR_INVALID;
  *out = nullptr;
  if (!probs || nprob < 1) {
    g_create_msg = "probs is NULL or nprob < 1";
    return ADER_ERR_INVALID;
  }
  ader_ctx *c = new ader_ctx();
  c->stream = (hipStream_t)hip_stream;
  c->cur = c->stream;
  ader_status st = ADER_OK;
  auto bail = [&](ader_status s) {
    g_create_msg = c->msg;  // readable through ader_last_error(NULL)
    ader_destroy(c);
    return s;
  };
  for (int i = 0; i < nprob; i++)  // argument checks first: they need no device
    if ((st = validate(c, probs[i], i))) return bail(st);
  if (hipGetDevice(&c->device) != hipSuccess) {
    (void)hipGetLastError();
    c->msg = "no HIP device";
    return bail(ADER_ERR_DEVICE);
  }
  c->P.resize(nprob);
  int64_t uoff = 0, qoff = 0, moff = 0;
  for (int i = 0; i < nprob; i++) {
    const ader_problem &d = probs[i];
    ProbState &s = c->P[i];
    s.desc = d;
    s.D = d.dim;
    s.N = d.degree;
    s.ks = kernels_for(d);
    if (!s.ks.cfl) {
      c->msg = "no kernels for this configuration";
      return bail(ADER_ERR_UNSUPPORTED);
    }
    s.n = s.ks.n;
    s.m = s.ks.M;
    s.nd = s.ks.ND;
    s.nst = s.ks.NST;
    s.nf = s.ks.NF;
    s.E = 1;
    for (int a = 0; a < 3; a++) {
      s.g.nel[a] = a < s.D ? d.nelem[a] : 1;
      s.h[a] = a < s.D ? (d.hi[a] - d.lo[a]) / d.nelem[a] : 1.0;
      s.g.inv_h[a] = 1.0 / s.h[a];
      s.E *= s.g.nel[a];
    }
    s.g.E = s.E;
    s.g.gamma = d.gamma;
    if (build_ops(s.N, &s.ops)) {
      c->msg = "basis construction failed";
      return bail(ADER_ERR_INVALID);
    }
    s.coef = d.cfl * stability_alpha(s.N);
    s.sweeps = d.picard_iters > 0 ? d.picard_iters
               : d.guess == 3      ? 1
                                   : (s.N + 1 - d.guess > 1 ? s.N + 1 - d.guess : 1);
    s.u_off = uoff;
    s.u_cnt = s.E * s.m * s.nd;
    s.q_off = qoff;
    s.q_cnt = s.E * s.m * s.nst;
    s.e_off = c->total_e;
    c->total_e += s.E;
    uoff += s.u_cnt;
    qoff += s.q_cnt;
    moff += s.m;
    for (int k = 0; k < kMaxN * kMaxN; k++) {
      for (int a = 0; a < 3; a++) {
        s.sw.DA[a][k] = -s.g.inv_h[a] * s.ops.D[k];
        s.sw.DAf[a][k] = (float)s.sw.DA[a][k];
      }
      s.sw.T[k] = s.ops.T[k];
      s.sw.Tf[k] = (float)s.ops.T[k];
      s.sw.Dhf[k] = (float)s.ops.D[k];
      for (int a = 0; a < 3; a++) s.sw.VA[a][k] = s.g.inv_h[a] * s.ops.V[k];
    }
    for (int a = 0; a < 3; a++) line_slots(s.D, s.N, a < s.D ? a : 0, s.sw.ls[a]);
    for (int k = 0; k < kMaxN; k++) {
      s.sw.Trow[k] = s.ops.Trow[k];
      s.sw.Trowf[k] = (float)s.ops.Trow[k];
      s.sw.xi[k] = s.ops.xi[k];
      s.sw.xif[k] = (float)s.ops.xi[k];
    }
    const size_t acc_bytes = (size_t)s.m * s.ks.ACC * sizeof(double);
    s.trace_elt = d.prec == ADER_FP64 ? sizeof(double) : sizeof(float);
    // candidate predictor variants: this precision, within the LDS budget;
    // for FP64 the HBM-accumulator variant only when no LDS variant fits
    std::vector<PredVariant> cand;
    const int want = d.prec == ADER_FP64 ? kFP64 : (d.prec == ADER_FP32 ? kFP32 : kBF16);
    // preference: accumulator in LDS over HBM, then no scratch spills over spills
    for (int pass = 0; pass < 4 && cand.empty(); pass++)
      for (int v = 0; v < s.ks.npred; v++) {
        const PredVariant &pv = s.ks.pred[v];
        if (pv.prec != want || pv.lds > kLdsBytes || pv.acc_lds != (pass < 2)) continue;
        hipFuncAttributes fa;
        if (hipFuncGetAttributes(&fa, pv.fn) != hipSuccess) {
          (void)hipGetLastError();
          continue;
        }
        // "no spills" admits a few bytes of scratch (the timing decides)
        if ((fa.localSizeBytes > kSmallSpill) != (pass % 2 == 1)) continue;
        if (hipFuncSetAttribute(pv.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pv.lds) !=
            hipSuccess) {
          (void)hipGetLastError();
          continue;
        }
        cand.push_back(pv);
      }
    if (cand.empty()) {
      c->msg = "problem " + std::to_string(i) + ": space-time DOFs of one element exceed LDS";
      return bail(ADER_ERR_UNSUPPORTED);
    }
    s.pv = cand[0];
    s.cand = cand;
    // device buffers
    if ((st = dalloc(c, (void **)&s.ops_dev, sizeof(Ops)))) return bail(st);
    if ((st = dalloc(c, (void **)&s.sw_dev, sizeof(OpsSweep)))) return bail(st);
    if (hipMemcpy(s.ops_dev, &s.ops, sizeof(Ops), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s.sw_dev, &s.sw, sizeof(OpsSweep), hipMemcpyHostToDevice) != hipSuccess) {
      c->msg = "operator table upload failed";
      return bail(ADER_ERR_DEVICE);
    }
    const size_t ub = (size_t)s.u_cnt * sizeof(double);
    const size_t gb = (size_t)s.E * s.m * s.nf * s.trace_elt;  // face integrals share the trace type
    if ((st = dalloc(c, (void **)&s.ustar, ub))) return bail(st);
    // traces per element and side: every time node, or the time averages
    const int ncomp = d.pde == ADER_ELASTIC ? s.m : 2 * s.m;
    const size_t tb = d.face_avg ? (size_t)s.E * ncomp * s.nf * s.trace_elt : (size_t)s.u_cnt * s.trace_elt;
    for (int a = 0; a < s.D; a++) {
      for (int sd = 0; sd < 2; sd++)
        if ((st = dalloc(c, (void **)&s.trace[a][sd], tb))) return bail(st);
      if ((st = dalloc(c, (void **)&s.GL[a], gb))) return bail(st);
      if (d.pde == ADER_ELASTIC && (st = dalloc(c, (void **)&s.GR[a], gb))) return bail(st);
    }
    if (d.guess == 3 && s.N > 0) {  // previous interval: N Taylor coefficients per node and variable
      const size_t hb = (size_t)s.E * s.m * s.N * s.nd * s.trace_elt;
      if ((st = dalloc(c, &s.hist, hb))) return bail(st);
      if (hipMemset(s.hist, 0, hb) != hipSuccess) {
        c->msg = "history initialisation failed";
        return bail(ADER_ERR_DEVICE);
      }
    }
    // every candidate shares acc_lds (the first pass that finds any fixes it)
    if (!s.pv.acc_lds && (st = dalloc(c, (void **)&s.acc, (size_t)s.E * acc_bytes))) return bail(st);
    if (d.pde == ADER_ELASTIC) {
      if ((st = dalloc(c, (void **)&s.mat, (size_t)s.E * 3 * sizeof(double)))) return bail(st);
      if (hipMemcpy(s.mat, d.material, (size_t)s.E * 3 * sizeof(double), hipMemcpyHostToDevice) !=
          hipSuccess) {
        c->msg = "material upload failed";
        return bail(ADER_ERR_DEVICE);
      }
    }
  }
  c->total_u = uoff;
  c->total_q = qoff;
  c->total_m = moff;
  if ((st = dalloc(c, (void **)&c->dt, nprob * sizeof(double)))) return bail(st);
  if ((st = dalloc(c, (void **)&c->t, nprob * sizeof(double)))) return bail(st);
  if ((st = dalloc(c, (void **)&c->tnext, nprob * sizeof(double)))) return bail(st);
  const size_t smax_bytes = (size_t)nprob * kSmaxPerProblem * sizeof(unsigned long long);
  if ((st = dalloc(c, (void **)&c->smax, smax_bytes))) return bail(st);
  if ((st = dalloc(c, (void **)&c->smax_f, smax_bytes))) return bail(st);
  if ((st = dalloc(c, (void **)&c->dtprev, nprob * sizeof(double)))) return bail(st);
  if ((st = dalloc(c, (void **)&c->hist_ok, sizeof(int)))) return bail(st);
  {
    std::vector<double> coef(nprob);
    for (int i = 0; i < nprob; i++) coef[i] = c->P[i].coef;
    c->tend_host.assign(nprob, INFINITY);
    if ((st = upload(c, (void **)&c->coef, coef.data(), nprob * sizeof(double))) ||
        (st = upload(c, (void **)&c->tend, c->tend_host.data(), nprob * sizeof(double))))
      return bail(st);
  }
  if ((st = dalloc(c, (void **)&c->err, sizeof(int)))) return bail(st);
  if ((st = dalloc(c, (void **)&c->partial, (size_t)kTotBlocks * 9 * sizeof(double)))) return bail(st);
  if ((st = dalloc(c, (void **)&c->sums, (size_t)c->total_m * sizeof(double)))) return bail(st);
  if (hipMemset(c->dt, 0, nprob * sizeof(double)) != hipSuccess ||
      hipMemset(c->t, 0, nprob * sizeof(double)) != hipSuccess ||
      hipMemset(c->tnext, 0, nprob * sizeof(double)) != hipSuccess ||
      hipMemset(c->smax, 0, smax_bytes) != hipSuccess || hipMemset(c->smax_f, 0, smax_bytes) != hipSuccess ||
      hipMemset(c->dtprev, 0, nprob * sizeof(double)) != hipSuccess ||
      hipMemset(c->hist_ok, 0, sizeof(int)) != hipSuccess ||
      hipMemset(c->err, 0, sizeof(int)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    c->msg = "initialisation failed";
    return bail(ADER_ERR_DEVICE);
  }
  // kernel classes: problems with the same kernels share every launch
  const char *force = getenv("ADER_VARIANT");
  const char *tune_env = getenv("ADER_AUTOTUNE");
  for (int i = 0; i < nprob; i++) {
    ProbState &s = c->P[i];
    int k = 0;
    for (; k < (int)c->K.size(); k++) {
      const ProbState &r = c->P[c->K[k].probs[0]];
      if (r.D == s.D && r.N == s.N && r.desc.pde == s.desc.pde && r.desc.prec == s.desc.prec &&
          (r.desc.face_avg != 0) == (s.desc.face_avg != 0))
        break;
    }
    if (k == (int)c->K.size()) {
      KClass kc;
      kc.D = s.D;
      kc.pv = s.cand[0];
      const bool f64 = s.desc.prec == ADER_FP64;
      kc.face_avg = s.desc.face_avg != 0;
      for (int ax = 0; ax < 3; ax++)
        kc.face[ax] = kc.face_avg ? (f64 ? s.ks.faceavg64[ax] : s.ks.faceavg32[ax])
                                  : (f64 ? s.ks.face64[ax] : s.ks.face32[ax]);
      kc.update = f64 ? s.ks.update64 : s.ks.update32;
      kc.cfl = s.ks.cfl;
      kc.detect = s.ks.detect;
      c->K.push_back(kc);
    }
    s.cls = k;
    c->K[k].probs.push_back(i);
  }
  for (KClass &k : c->K) {
    const std::vector<PredVariant> &cand = c->P[k.probs[0]].cand;
    bool forced = false;
    if (force && *force)
      for (const PredVariant &pv : cand)
        if (strcmp(pv.name, force) == 0) {
          k.pv = pv;
          forced = true;
        }
    const bool tune = !forced && cand.size() > 1 && !(tune_env && strcmp(tune_env, "0") == 0);
    if (tune && (st = tune_class(c, k, cand))) return bail(st);
    if ((st = build_class(c, k))) return bail(st);
  }
  *out = c;
  return ADER_OK;
}

ader_status ader_profile(ader_ctx *c, int32_t enable) {
  if (!c) return ADER_ERR_INVALID;
  c->profile = enable != 0;
  return ADER_OK;
}

ader_status ader_stage_times(ader_ctx *c, double *ms_host, int64_t *launches_host) {
  if (!c || !ms_host) return ADER_ERR_INVALID;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < 4; i++) {
    ms_host[i] = 0.0;
    if (launches_host) launches_host[i] = 0;
  }
  for (size_t b = 0; b + 5 <= c->ev_used.size(); b += 5)
    for (int i = 0; i < 4; i++) {
      float ms = 0.0f;
      HIP_OR_FAIL(c, hipEventElapsedTime(&ms, c->ev_used[b + i], c->ev_used[b + i + 1]));
      ms_host[i] += ms;
      if (launches_host) launches_host[i] += 1;
    }
  for (hipEvent_t e : c->ev_used) c->ev_pool.push_back(e);
  c->ev_used.clear();
  return ADER_OK;
}

ader_status ader_destroy(ader_ctx *c) {
  if (!c) return ADER_OK;
  if (!c->allocs.empty() || !c->ev_used.empty() || !c->ev_pool.empty() || c->gstream)
    (void)hipDeviceSynchronize();
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->g_in) (void)hipEventDestroy(c->g_in);
  if (c->g_out) (void)hipEventDestroy(c->g_out);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  for (hipEvent_t e : c->ev_used) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  for (void *p : c->allocs) (void)hipFree(p);
  delete c;
  return ADER_OK;
}

ader_status ader_layout(const ader_ctx *c, int32_t prob, int64_t *offset, int64_t *count) {
  if (!c || prob < 0 || prob >= (int32_t)c->P.size()) return ADER_ERR_INVALID;
  if (offset) *offset = c->P[prob].u_off;
  if (count) *count = c->P[prob].u_cnt;
  return ADER_OK;
}

ader_status ader_qhat_layout(const ader_ctx *c, int32_t prob, int64_t *offset, int64_t *count) {
  if (!c || prob < 0 || prob >= (int32_t)c->P.size()) return ADER_ERR_INVALID;
  if (offset) *offset = c->P[prob].q_off;
  if (count) *count = c->P[prob].q_cnt;
  return ADER_OK;
}

ader_status ader_state_size(const ader_ctx *c, int64_t *count) {
  if (!c || !count) return ADER_ERR_INVALID;
  *count = c->total_u;
  return ADER_OK;
}

ader_status ader_cfl_dt(ader_ctx *c, const double *u, double *dt_host) {
  if (!c) return ADER_ERR_INVALID;
  if (!u) return fail(c, ADER_ERR_INVALID, "u is NULL");
  c->fused_u = nullptr;  // the finalisation clears the update's maxima
  ader_status st = run_cfl(c, u, 0);
  if (st || !dt_host) return st;
  HIP_OR_FAIL(c, hipMemcpyAsync(dt_host, c->dt, c->P.size() * sizeof(double), hipMemcpyDeviceToHost,
                                c->stream));
  return check_flag(c);
}

ader_status ader_predictor(ader_ctx *c, const double *u, const double *dt_dev, double *qhat_out) {
  if (!c) return ADER_ERR_INVALID;
  if (!u) return fail(c, ADER_ERR_INVALID, "u is NULL");
  c->fused_u = nullptr;
  c->hist_u = nullptr;
  return run_predictor(c, u, dt_dev, qhat_out);
}

ader_status ader_corrector(ader_ctx *c, double *u, const double *dt_dev) {
  if (!c) return ADER_ERR_INVALID;
  if (!u) return fail(c, ADER_ERR_INVALID, "u is NULL");
  c->fused_u = nullptr;
  c->hist_u = nullptr;
  return run_corrector(c, u, dt_dev);
}

ader_status ader_step(ader_ctx *c, double *u, const double *t_end_host) {
  if (!c) return ADER_ERR_INVALID;
  if (!u || !t_end_host) return fail(c, ADER_ERR_INVALID, "u and t_end must not be NULL");
  ader_status st = set_tend(c, t_end_host);
  if (st) return st;
  const bool fused = !c->detect && c->fused_u == u;
  c->fused_u = nullptr;
  if ((st = history_for(c, u))) return st;
  if ((st = step_launches(c, u, true, fused))) return st;
  c->fused_u = c->detect ? nullptr : u;
  c->hist_u = u;
  return ADER_OK;
}

ader_status ader_run(ader_ctx *c, double *u, const double *t_end_host, int32_t nsteps) {
  if (!c) return ADER_ERR_INVALID;
  if (!u || !t_end_host) return fail(c, ADER_ERR_INVALID, "u and t_end must not be NULL");
  if (nsteps < 1) return fail(c, ADER_ERR_INVALID, "nsteps must be >= 1");
  ader_status st = set_tend(c, t_end_host);
  if (st) return st;
  if (!c->gstream) {
    HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
    HIP_OR_FAIL(c, hipEventCreateWithFlags(&c->g_in, hipEventDisableTiming));
    HIP_OR_FAIL(c, hipEventCreateWithFlags(&c->g_out, hipEventDisableTiming));
  }
  if (!c->gexec || c->g_u != u || c->g_steps != nsteps) {
    if (c->gexec) {
      HIP_OR_FAIL(c, hipStreamSynchronize(c->gstream));
      (void)hipGraphExecDestroy(c->gexec);
      c->gexec = nullptr;
    }
    HIP_OR_FAIL(c, hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
    c->cur = c->gstream;
    // every captured step takes its dt from the maxima the update before it
    // took (the first one from those of the previous replay, or of the pass
    // below); with detection on, every step runs the time-step kernel
    for (int i = 0; i < nsteps && !st; i++) st = step_launches(c, u, false, !c->detect);
    c->cur = c->stream;
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->gstream, &g);
    if (st) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (ec != hipSuccess) return fail(c, ADER_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      c->gexec = nullptr;
      return fail(c, ADER_ERR_DEVICE, std::string("graph instantiation: ") + hipGetErrorString(ei));
    }
    c->g_u = u;
    c->g_steps = nsteps;
  }
  if (!c->detect && c->fused_u != u) {
    // the replay's first step needs the maxima of u in smax_f
    c->fused_u = nullptr;
    const int np = (int)c->P.size();
    hipLaunchKernelGGL(k_zero_u64, dim3((np * kSmaxPerProblem + 255) / 256), dim3(256), 0, c->stream, c->smax_f,
                       np * kSmaxPerProblem);
    HIP_OR_FAIL(c, hipGetLastError());
    if ((st = run_maxima(c, u, c->smax_f))) return st;
  }
  if ((st = history_for(c, u))) return st;
  // order the replay after earlier work on the context stream, and later work after it
  HIP_OR_FAIL(c, hipEventRecord(c->g_in, c->stream));
  HIP_OR_FAIL(c, hipStreamWaitEvent(c->gstream, c->g_in, 0));
  HIP_OR_FAIL(c, hipGraphLaunch(c->gexec, c->gstream));
  HIP_OR_FAIL(c, hipEventRecord(c->g_out, c->gstream));
  HIP_OR_FAIL(c, hipStreamWaitEvent(c->stream, c->g_out, 0));
  c->fused_u = c->detect ? nullptr : u;
  c->hist_u = u;
  return ADER_OK;
}

ader_status ader_set_detection(ader_ctx *c, int32_t enable) {
  if (!c) return ADER_ERR_INVALID;
  const bool on = enable != 0;
  if (on == c->detect) return ADER_OK;
  ader_status st;
  if (on) {  // buffers kept from an earlier call (also one that failed part-way) are reused
    if (!c->flags) {
      if ((st = dalloc(c, (void **)&c->flags, (size_t)c->total_e * sizeof(int)))) return st;
      HIP_OR_FAIL(c, hipMemset(c->flags, 0, (size_t)c->total_e * sizeof(int)));
    }
    for (ProbState &s : c->P)
      if (!s.summ && (st = dalloc(c, (void **)&s.summ, (size_t)s.E * s.m * 2 * sizeof(double)))) return st;
  }
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  if (c->gexec) {  // the captured steps no longer match
    HIP_OR_FAIL(c, hipStreamSynchronize(c->gstream));
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  c->detect = on;
  c->fused_u = nullptr;
  for (KClass &k : c->K)
    if ((st = refresh_detection(c, k))) {
      // incomplete records: leave detection off (steps then launch no detection kernel)
      c->detect = false;
      for (KClass &r : c->K) (void)refresh_detection(c, r);
      return st;
    }
  return ADER_OK;
}

ader_status ader_detect_flags(ader_ctx *c, int32_t *flags_host) {
  if (!c || !flags_host) return ADER_ERR_INVALID;
  if (!c->flags) return fail(c, ADER_ERR_INVALID, "detection was never enabled (ader_set_detection)");
  HIP_OR_FAIL(c, hipMemcpyAsync(flags_host, c->flags, (size_t)c->total_e * sizeof(int), hipMemcpyDeviceToHost,
                                c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return ADER_OK;
}

ader_status ader_time(ader_ctx *c, double *t_host) {
  if (!c || !t_host) return ADER_ERR_INVALID;
  HIP_OR_FAIL(c, hipMemcpyAsync(t_host, c->t, c->P.size() * sizeof(double), hipMemcpyDeviceToHost,
                                c->stream));
  return check_flag(c);
}

ader_status ader_last_dt(ader_ctx *c, double *dt_host) {
  if (!c || !dt_host) return ADER_ERR_INVALID;
  HIP_OR_FAIL(c, hipMemcpyAsync(dt_host, c->dt, c->P.size() * sizeof(double), hipMemcpyDeviceToHost,
                                c->stream));
  return check_flag(c);
}

ader_status ader_set_time(ader_ctx *c, const double *t_host) {
  if (!c || !t_host) return ADER_ERR_INVALID;
  HIP_OR_FAIL(c, hipMemcpyAsync(c->t, t_host, c->P.size() * sizeof(double), hipMemcpyHostToDevice,
                                c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return ADER_OK;
}

ader_status ader_totals(ader_ctx *c, const double *u, double *sums_host) {
  if (!c || !sums_host) return ADER_ERR_INVALID;
  if (!u) return fail(c, ADER_ERR_INVALID, "u is NULL");
  int64_t moff = 0;
  for (size_t p = 0; p < c->P.size(); p++) {
    ProbState &s = c->P[p];
    double vol = 1.0;
    for (int a = 0; a < s.D; a++) vol *= s.h[a];
    hipLaunchKernelGGL(k_totals_partial, dim3(kTotBlocks), dim3(kBlock), 0, c->stream, u + s.u_off,
                       s.E, s.m, s.nd, s.n, s.D, s.ops, vol, c->partial);
    hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(64), 0, c->stream, c->partial, kTotBlocks, s.m,
                       c->sums + moff);
    HIP_OR_FAIL(c, hipGetLastError());
    moff += s.m;
  }
  HIP_OR_FAIL(c, hipMemcpyAsync(sums_host, c->sums, (size_t)c->total_m * sizeof(double),
                                hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return ADER_OK;
}

ader_status ader_totals_noalloc(const ader_problem *prob, const double *u, double *sums_dev, void *hip_stream) {
  if (!prob || !u || !sums_dev) {
    g_create_msg = "prob, u and sums_dev must not be NULL";
    return ADER_ERR_INVALID;
  }
  ader_ctx tmp;  // only carries the message of validate()
  ader_status st = validate(&tmp, *prob, 0);
  if (st) {
    g_create_msg = tmp.msg;
    return st;
  }
  const int D = prob->dim, N = prob->degree, n = N + 1;
  const int m = prob->pde == ADER_EULER ? D + 2 : 9;
  if (m > kScratchVars) {  // the scratch holds kTotBlocks partial sums of at most kScratchVars variables
    g_create_msg = "more variables than the static scratch holds";
    return ADER_ERR_UNSUPPORTED;
  }
  int nd = 1;
  int64_t E = 1;
  double vol = 1.0;
  for (int a = 0; a < D; a++) {
    nd *= n;
    E *= prob->nelem[a];
    vol *= (prob->hi[a] - prob->lo[a]) / prob->nelem[a];
  }
  Ops ops;
  if (build_ops(N, &ops)) {
    g_create_msg = "basis construction failed";
    return ADER_ERR_INVALID;
  }
  double *part = nullptr;
  hipError_t e = scratch_address(&part);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    g_create_msg = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return ADER_ERR_DEVICE;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  // the same kernels and grid as ader_totals: the same sums bit for bit
  hipLaunchKernelGGL(k_totals_partial, dim3(kTotBlocks), dim3(kBlock), 0, s, u, E, m, nd, n, D, ops, vol, part);
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(64), 0, s, part, kTotBlocks, m, sums_dev);
  e = hipGetLastError();
  if (e != hipSuccess) {
    g_create_msg = std::string("totals launch: ") + hipGetErrorString(e);
    return ADER_ERR_DEVICE;
  }
  return ADER_OK;
}

ader_status ader_describe(const ader_ctx *c, int32_t prob, char *buf, int32_t len) {
  if (!c || !buf || len <= 0 || prob < 0 || prob >= (int32_t)c->P.size()) return ADER_ERR_INVALID;
  const ProbState &s = c->P[prob];
  snprintf(buf, (size_t)len,
           "predictor=%s threads=%d lds_bytes=%zu sweeps=%d selection=%s tuned_ms=%.4f trace_bytes=%zu",
           s.pv.name, s.pv.threads, s.pv.lds, s.sweeps, s.tuned ? "autotuned" : "default", s.tune_ms,
           s.trace_elt);
  return ADER_OK;
}

const char *ader_last_error(const ader_ctx *c) {
  if (!c) return g_create_msg.c_str();
  return c->msg.c_str();
}

}  // extern "C"
