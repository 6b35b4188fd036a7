// cmflb_capi.hip -- implementation of the C ABI declared in include/cmflb.h:
// lattice objects, the FP64 per-mode constants, launch geometry, captured
// step graphs and the statistics ring.
//
// Method: De Rosis & Zhou, "A fluctuating lattice Boltzmann formulation based
// on orthogonal central moments" (arXiv 2602.16486).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hipfft/hipfft.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cmflb.h"
#include "cmflb_device.h"
#include "cmflb_internal.h"

using namespace cmf;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_TRY(call)                                                      \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess)                                                  \
      return fail(CMF_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

constexpr double kCs2 = 1.0 / 3.0;
constexpr int kGraphSteps = 32;
// most steps whose statistics one forked reduction handles (lattices): the
// partial sums go to a ring of 2 K slots, K = kStatBatch, or fewer steps
// (down to 1) when the ring would exceed kStatRingBytes
constexpr int kStatBatch = 8;
constexpr size_t kStatRingBytes = (size_t)256 << 20;
static_assert(kGraphSteps % kStatBatch == 0, "a captured run is whole batches");
// noise counters are distinct for steps below 2^56 (see site_normals)
constexpr int64_t kMaxStep = (int64_t)1 << 56;

// one-axis weights of the rest state: w(0) = 2/3, w(+-1) = 1/6; the D2Q9 and
// D3Q27 weights of Sec. 2.2 / 2.3 are their products (4/9, 1/9, 1/36 and
// 8/27, 2/27, 1/54, 1/216).
double axis_weight(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
// one-axis norms sum_c w(c) P_p(c)^2 of P_0 = 1, P_1 = c, P_2 = c^2 - c_s^2
const double kAxisNorm[3] = {1.0, 1.0 / 3.0, 2.0 / 9.0};

template <class L>
void lattice_weights(double *w) {
  for (int i = 0; i < L::Q; ++i)
    w[i] = axis_weight(L::cx[i]) * axis_weight(L::cy[i]) *
           (L::D == 3 ? axis_weight(L::cz[i]) : 1.0);
}

// D3Q19 weights (Sec. 2.4): 1/3 at rest, 1/18 on the axes, 1/36 on the
// face diagonals
void d3q19_weights(double *w) {
  for (int i = 0; i < 19; ++i) w[i] = i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// the D3Q19 basis polynomials of Sec. 2.4 at c
void d3q19_basis(double x, double y, double z, double *P) {
  const double c2 = x * x + y * y + z * z;
  const double row[19] = {1.0, x, y, z, c2 - 1.0, 3.0 * x * x - c2, y * y - z * z, x * y, y * z,
                          x * z, x * (3.0 * c2 - 5.0), y * (3.0 * c2 - 5.0), z * (3.0 * c2 - 5.0),
                          x * (y * y - z * z), y * (z * z - x * x), z * (x * x - y * y),
                          3.0 * c2 * c2 - 6.0 * c2 + 1.0, (2.0 * c2 - 3.0) * (3.0 * x * x - c2),
                          (2.0 * c2 - 3.0) * (y * y - z * z)};
  for (int v = 0; v < 19; ++v) P[v] = row[v];
}

// b_v of the paper's orthogonal bases (Sec. 2.2 and 2.3): products of the
// one-axis norms; D2Q9 rows 3 and 4 are sums/differences of two orthogonal
// products and have norm 2/9 + 2/9.  D3Q19 (Sec. 2.4): sum_i w_i P_v(c_i)^2.
void mode_norms(int q, double *b) {
  if (q == 19) {
    double w[19];
    d3q19_weights(w);
    for (int v = 0; v < 19; ++v) b[v] = 0.0;
    for (int i = 0; i < 19; ++i) {
      double P[19];
      d3q19_basis(D3Q19::cx[i], D3Q19::cy[i], D3Q19::cz[i], P);
      for (int v = 0; v < 19; ++v) b[v] += w[i] * P[v] * P[v];
    }
  } else if (q == 27) {
    for (int v = 0; v < 27; ++v) {
      const int pos = D3Q27::mode_pos[v];
      b[v] = kAxisNorm[pos % 3] * kAxisNorm[(pos / 3) % 3] * kAxisNorm[pos / 9];
    }
  } else {
    const int px[9] = {0, 1, 0, -1, -1, 1, 2, 1, 2};
    const int py[9] = {0, 0, 1, -1, -1, 1, 1, 2, 2};
    for (int v = 0; v < 9; ++v)
      b[v] = px[v] < 0 ? 2.0 * kAxisNorm[2] * kAxisNorm[0]
                       : kAxisNorm[px[v]] * kAxisNorm[py[v]];
  }
}

// the compile-time sqrt(b_v) of the kernels against the norms computed here
bool sqrt_norms_consistent(int q) {
  double b[27];
  mode_norms(q, b);
  for (int v = 0; v < q; ++v) {
    const double s = q == 9 ? sqrt_norm<D2Q9>(v) : (q == 19 ? sqrt_norm<D3Q19>(v) : sqrt_norm<D3Q27>(v));
    if (fabs(s * s - b[v]) > 1e-14 * b[v]) return false;
  }
  return true;
}

bool is_omega_mode(int q, int v) {
  return q == 9 ? (v == 4 || v == 5) : (v >= 7 && v <= 9);
}

int first_noisy(int q) { return q == 9 ? 3 : 4; }

size_t storage_bytes(int storage) {
  switch (storage) {
    case kF64: return 8;
    case kF32: return 4;
    case kF16:
    case kBF16: return 2;
  }
  return 0;
}

int env_int(const char *name, int dflt) {
  const char *s = getenv(name);
  if (!s || !*s) return dflt;
  return atoi(s);
}

// env_int clamped to [lo, hi]
int env_int(const char *name, int dflt, int lo, int hi) {
  const int v = env_int(name, dflt);
  return v < lo ? lo : (v > hi ? hi : v);
}

}  // namespace

namespace {

// FP64 per-mode constants of one descriptor: rates, weights, mode noise
// factors amp_v = I~_v sqrt(Lambda_v (2 - Lambda_v) b_v) (eq. phi_general
// is phi_v = sqrt(rho kT / c_s^2) amp_v), storage scales.
struct ModeConstants {
  double lambda[27], w[27], amp[27];
  float scale[27];
  bool general;
};

void mode_constants(const cmf_desc *desc, ModeConstants &mc) {
  const int q = desc->q;
  const double omega = 1.0 / desc->tau;
  for (int v = 0; v < q; ++v)
    mc.lambda[v] = desc->lambda ? desc->lambda[v] : (is_omega_mode(q, v) ? omega : 1.0);
  mc.general = false;
  for (int v = first_noisy(q); v < q; ++v)
    if (!is_omega_mode(q, v) && mc.lambda[v] != 1.0) mc.general = true;
  double b[27];
  if (q == 9)
    lattice_weights<D2Q9>(mc.w);
  else if (q == 19)
    d3q19_weights(mc.w);
  else
    lattice_weights<D3Q27>(mc.w);
  mode_norms(q, b);
  for (int v = 0; v < q; ++v) {
    const double lv = mc.lambda[v];
    mc.amp[v] = v >= first_noisy(q) ? sqrt(lv * (2.0 - lv) * b[v]) : 0.0;
  }
  for (int i = 0; i < q; ++i) {
    if (desc->storage == kF16 || desc->storage == kBF16) {
      const double sigma = desc->kT > 0.0 ? sqrt(desc->rho0 * desc->kT * mc.w[i] / kCs2)
                                          : 1e-2 * mc.w[i];
      mc.scale[i] = (float)ldexp(1.0, (int)ceil(log2(sigma)));
    } else {
      mc.scale[i] = 1.0f;
    }
  }
}

// Captured runs of kGraphSteps steps: step j passes step offset j and runs
// on the caller's stream; the steps go in batches of K consecutive steps
// (K = the lattice's stat_batch, at most kStatBatch; 1 for an ensemble),
// step j writing its partial sums to slot j mod 2K; once a batch is done,
// one statistics reduction for all its steps runs on a second stream
// (default priority), overlapping the next batch; the first step of batch
// b + 2 waits for it (it reuses the slots); the step counter advances once,
// after the last reduction.  One fork per batch instead of one per step:
// the event records and waits between the streams cost microseconds each.
struct ForkedRun {
  hipStream_t aux = nullptr;
  hipEvent_t ev_step[kGraphSteps] = {};
  hipEvent_t ev_fin[kGraphSteps] = {};
  bool ready = false;
};

void forked_release(ForkedRun &F) {
  for (int j = 0; j < kGraphSteps; ++j) {
    if (F.ev_step[j]) (void)hipEventDestroy(F.ev_step[j]);
    if (F.ev_fin[j]) (void)hipEventDestroy(F.ev_fin[j]);
    F.ev_step[j] = F.ev_fin[j] = nullptr;
  }
  if (F.aux) (void)hipStreamDestroy(F.aux);
  F.aux = nullptr;
  F.ready = false;
}

int forked_init(ForkedRun &F) {
  if (F.ready) return CMF_OK;
  hipError_t e = hipStreamCreate(&F.aux);
  for (int j = 0; j < kGraphSteps && e == hipSuccess; ++j) {
    e = hipEventCreateWithFlags(&F.ev_step[j], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&F.ev_fin[j], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    forked_release(F);
    return fail(CMF_EHIP, "stream/event creation failed: %s", hipGetErrorString(e));
  }
  F.ready = true;
  return CMF_OK;
}

// Enqueue a run of n <= kGraphSteps steps in the forked form on stream s,
// in batches of K steps: step(j, stream) enqueues step j (step offset j,
// partial-sum slot j mod 2K); fin(j0, count, stream) the statistics
// reduction of steps j0 .. j0 + count - 1 (only when `stats`), on the second
// stream; the step counter advances by n at the end.  Used inside a graph
// capture (runs of kGraphSteps) and directly (the remainder of a cmf_step
// call), so the statistics of direct steps overlap the next steps as well.
template <class StepFn, class FinFn>
hipError_t enqueue_forked(hipStream_t s, ForkedRun &F, bool stats, int K, int64_t *step_dev,
                          StepFn step, FinFn fin, int n) {
  hipError_t e = hipSuccess;
  const int nbatch = (n + K - 1) / K;
  for (int b = 0; b < nbatch && e == hipSuccess; ++b) {
    const int j0 = b * K, j1 = j0 + K < n ? j0 + K : n;
    if (stats && b >= 2) e = hipStreamWaitEvent(s, F.ev_fin[b - 2], 0);
    for (int j = j0; j < j1 && e == hipSuccess; ++j) e = step(j, s);
    if (stats) {
      if (e == hipSuccess) e = hipEventRecord(F.ev_step[b], s);
      if (e == hipSuccess) e = hipStreamWaitEvent(F.aux, F.ev_step[b], 0);
      if (e == hipSuccess) e = fin(j0, j1 - j0, F.aux);
      if (e == hipSuccess) e = hipEventRecord(F.ev_fin[b], F.aux);
    }
  }
  if (stats && e == hipSuccess) e = hipStreamWaitEvent(s, F.ev_fin[nbatch - 1], 0);
  if (e == hipSuccess) e = launch_bump_step(step_dev, n, s);
  return e;
}

template <class StepFn, class FinFn>
int run_forked(hipStream_t s, ForkedRun &F, bool stats, int K, int64_t *step_dev, StepFn step,
               FinFn fin, int n) {
  if (n < 1 || n > kGraphSteps) return fail(CMF_EINVAL, "internal: forked run of %d steps", n);
  if (stats) {
    int rc = forked_init(F);
    if (rc != CMF_OK) return rc;
  }
  const hipError_t e = enqueue_forked(s, F, stats, K, step_dev, step, fin, n);
  if (e != hipSuccess) return fail(CMF_EHIP, "step launch failed: %s", hipGetErrorString(e));
  return CMF_OK;
}

template <class StepFn, class FinFn>
int capture_forked(hipStream_t s, ForkedRun &F, bool stats, int K, int64_t *step_dev,
                   StepFn step, FinFn fin, hipGraphExec_t *out) {
  if (stats) {
    int rc = forked_init(F);
    if (rc != CMF_OK) return rc;
  }
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  hipError_t e = enqueue_forked(s, F, stats, K, step_dev, step, fin, kGraphSteps);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(s, &g);
  if (e == hipSuccess) e = ec;
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(CMF_EHIP, "graph capture failed: %s", hipGetErrorString(e));
  return CMF_OK;
}

}  // namespace

struct cmf_lattice {
  cmf_desc desc;
  int q = 0;
  int storage = 0;
  bool general = false;
  bool nt_stores = true;  // population rows are whole cache lines
  bool in_place = false;  // AA streaming on one buffer (buf[1] == buf[0])
  bool own_stream = false;
  bool own_bufs = true;  // false: the population buffers belong to the caller
  hipStream_t stream = nullptr;
  int device = 0;
  int64_t N = 0;
  void *buf[2] = {nullptr, nullptr};
  int parity = 0;  // buf[parity] holds the state of the current step
  double *partials = nullptr;
  double *level2 = nullptr;
  int nparts = 0;
  int partials_cap = 0;    // partial rows per slot
  int partials_slots = 0;  // slots allocated (2 stat_batch needed)
  int stat_batch = 1;      // steps per forked statistics reduction
  int cus = 256;
  double *series = nullptr;
  int cap = 0;
  int64_t *step_dev = nullptr;
  int64_t read_step = 0;   // first step whose statistics were not returned
  int block = 256;
  int grid = 1;
  double lambda[27];
  double w[27];
  double amp[27];
  float scale[27];
  double mass0 = 0.0;
  StepParams<float> pf;
  StepParams<double> pd;
  ConvParams cp;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  ForkedRun forked;
  // structure factor
  int sk_nbins = 0;
  int64_t sk_M = 0, sk_samples = 0;
  float *sk_fields = nullptr;
  void *sk_F = nullptr;
  double *sk_acc = nullptr, *sk_out = nullptr;
  int32_t *sk_perm = nullptr;
  int64_t *sk_off = nullptr;
  hipfftHandle sk_plan = 0;
  bool sk_has_plan = false;
};

namespace {

// weight class |c_i|^2 of population i of a q-velocity lattice
int weight_class_of(int q, int i) {
  if (q == 9) return weight_class<D2Q9>(i);
  if (q == 19) return weight_class<D3Q19>(i);
  return weight_class<D3Q27>(i);
}

// per-class storage scales (and reciprocals) from the per-population ones.
// With 16-bit storage the tensor-product lattices (D2Q9, D3Q27) hand the
// stores 2^|c_i|^2 d*_i (their inverse one-axis maps skip the halvings), so
// the store scale of class k carries 2^-k: the stored values are the same.
void class_scales(int q, int storage, const float *scale, float *cs, float *ics) {
  const bool doubled = (storage == kF16 || storage == kBF16) && q != 19;
  for (int k = 0; k < 4; ++k) {
    cs[k] = 1.0f;
    ics[k] = doubled ? ldexpf(1.0f, -k) : 1.0f;
  }
  for (int i = 0; i < q; ++i) {
    const int k = weight_class_of(q, i);
    cs[k] = scale[i];
    ics[k] = doubled ? ldexpf(1.0f / scale[i], -k) : 1.0f / scale[i];
  }
}

// Step-kernel parameters of a lattice description with workgroups of
// `block` threads.
template <typename R>
void fill_params(const cmf_desc &d, const double *lambda, const double *amp, const float *scale,
                 int block, StepParams<R> &p) {
  memset(&p, 0, sizeof p);
  p.nx = d.nx;
  p.ny = d.ny;
  p.nz = d.nz;
  p.nxb = (d.nx + block - 1) / block;
  p.ntiles = p.nxb * p.ny * p.nz;
  p.noise = d.kT > 0.0 ? 1 : 0;
  p.rho0 = (R)d.rho0;
  for (int v = 0; v < d.q; ++v) {
    p.amp[v] = (R)amp[v];
    p.oml[v] = (R)(1.0 - lambda[v]);
    p.lam[v] = (R)lambda[v];
  }
  p.amp1 = (R)sqrt(d.kT / kCs2);
  class_scales(d.q, d.storage, scale, p.scale, p.iscale);
  p.key0 = (uint32_t)d.seed;
  p.key1 = (uint32_t)(d.seed >> 32);
  p.replica = d.replica;
}

template <typename R>
void fill_step_params(const cmf_lattice *L, const double *amp,
                      const float *scale, StepParams<R> &p) {
  fill_params(L->desc, L->lambda, amp, scale, L->block, p);
}

// tuned launch shapes of this process, keyed by device/lattice/storage/box
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tuned;
bool g_tune_file_loaded = false;

std::string tune_key(const cmf_lattice *L) {
  char b[160];
  snprintf(b, sizeof b, "dev%d:q%d:s%d:g%d:%dx%dx%d%s", L->device, L->q, L->storage,
           L->general ? 1 : 0, L->desc.nx, L->desc.ny, L->desc.nz, L->in_place ? ":aa" : "");
  return b;
}

// launch shapes the step kernels support: block threads per workgroup a
// multiple of 64 up to 256 (the statistics reduction assumes it), grid >= 1
bool valid_launch(int block, int grid) {
  return (block == 64 || block == 128 || block == 192 || block == 256) && grid >= 1;
}

void load_tune_file_locked() {
  if (g_tune_file_loaded) return;
  g_tune_file_loaded = true;
  const char *path = getenv("CMFLB_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  char key[160];
  int block, grid;
  double ms;
  // only shapes that cmf_set_launch would accept; other lines are skipped
  while (fscanf(f, "%159s %d %d %lf", key, &block, &grid, &ms) == 4)
    if (valid_launch(block, grid)) g_tuned[key] = {block, grid};
  fclose(f);
}

void remember_tuned(const cmf_lattice *L, int block, int grid, double ms) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_tune_file_locked();
  const std::string key = tune_key(L);
  g_tuned[key] = {block, grid};
  const char *path = getenv("CMFLB_TUNE_CACHE");
  if (path && *path) {
    FILE *f = fopen(path, "a");
    if (f) {
      fprintf(f, "%s %d %d %.6f\n", key.c_str(), block, grid, ms);
      fclose(f);
    }
  }
}

bool lookup_tuned(const cmf_lattice *L, int *block, int *grid) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_tune_file_locked();
  auto it = g_tuned.find(tune_key(L));
  if (it == g_tuned.end()) return false;
  *block = it->second.first;
  *grid = it->second.second;
  return true;
}

int default_block(int nx) { return nx >= 192 ? 256 : ((nx + 63) / 64) * 64; }

int ntiles_for(const cmf_lattice *L, int block) {
  return ((L->desc.nx + block - 1) / block) * L->desc.ny * L->desc.nz;
}

void drop_graphs(cmf_lattice *L) {
  for (int k = 0; k < 2; ++k)
    if (L->graph[k]) {
      (void)hipGraphExecDestroy(L->graph[k]);
      L->graph[k] = nullptr;
    }
}

// Apply a launch shape: step parameters, partials capacity, graphs.
int apply_launch(cmf_lattice *L, int block, int grid, const double *amp,
                 const float *scale) {
  // new parameters and buffers first: on failure the current shape stays
  const int block0 = L->block;
  L->block = block;
  StepParams<double> pd;
  StepParams<float> pf;
  fill_step_params(L, amp, scale, pd);
  fill_step_params(L, amp, scale, pf);
  L->block = block0;
  const int nt = pf.ntiles;
  const int g = grid < nt ? grid : nt;
  const size_t slot_bytes = sizeof(double) * kPartStride * (size_t)g;
  int K = kStatBatch;
  while (K > 1 && 2 * (size_t)K * slot_bytes > kStatRingBytes) K /= 2;
  if (g > L->partials_cap || 2 * K > L->partials_slots) {
    double *parts = nullptr;
    if (hipMalloc((void **)&parts, 2 * (size_t)K * slot_bytes) != hipSuccess)
      return fail(CMF_ENOMEM, "hipMalloc of the statistics partials failed");
    if (L->partials) (void)hipFree(L->partials);
    L->partials = parts;
    L->partials_cap = g;
    L->partials_slots = 2 * K;
  }
  L->stat_batch = K;
  L->block = block;
  L->pd = pd;
  L->pf = pf;
  L->grid = g;
  L->nparts = g;
  drop_graphs(L);
  return CMF_OK;
}

const void *step_params(const cmf_lattice *L) {
  return L->storage == kF64 ? (const void *)&L->pd : (const void *)&L->pf;
}

// partial-sum slot b (0 .. 2 stat_batch - 1) of the lattice
double *partials_buf(const cmf_lattice *L, int b) {
  return L->partials + (size_t)b * kPartStride * L->partials_cap;
}

// Streaming form of a step that starts from state parity b: the pull from
// buffer b into buffer 1 - b, or in place the even half of an AA pair from
// parity 0 (populations at their own sites) and the odd half from parity 1.
int stream_mode(const cmf_lattice *L, int b) {
  return !L->in_place ? kStreamPull : b == 0 ? kStreamAAEven : kStreamAAOdd;
}

// conversion parameters for the current state parity
ConvParams conv(const cmf_lattice *L) {
  ConvParams cp = L->cp;
  cp.layout = !L->in_place ? kLayoutPull : L->parity == 0 ? kLayoutNatural : kLayoutSwapped;
  return cp;
}

// the fused step from state parity b, step index *step_dev + off
hipError_t launch_lattice_step(const cmf_lattice *L, int b, int off, double *partials,
                               hipStream_t s) {
  return launch_step(L->q, L->storage, L->general, L->nt_stores, stream_mode(L, b), step_params(L),
                     L->buf[b], L->buf[b ^ 1], L->step_dev, off, partials, L->grid, L->block, s);
}

// One direct step: the fused kernel, then its statistics and the step
// counter on the same stream.
int enqueue_one_step(cmf_lattice *L) {
  HIP_TRY(launch_lattice_step(L, L->parity, 0, partials_buf(L, 0), L->stream));
  HIP_TRY(launch_finalize(partials_buf(L, 0), L->nparts, L->level2, L->series, L->cap,
                          L->step_dev, 0, 1, L->mass0,
                          !(L->desc.flags & CMF_FLAG_NO_STATS), L->stream));
  L->parity ^= 1;
  return CMF_OK;
}

// Time n full steps (fused step + statistics finalize) as direct launches.
int time_full_steps(cmf_lattice *L, int n, double *ms_out) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, L->stream);
  int rc = CMF_OK;
  for (int s = 0; s < n && e == hipSuccess && rc == CMF_OK; ++s) rc = enqueue_one_step(L);
  if (e == hipSuccess) e = hipEventRecord(e1, L->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc != CMF_OK) return rc;
  if (e != hipSuccess) return fail(CMF_EHIP, "timing failed: %s", hipGetErrorString(e));
  *ms_out = ms;
  return CMF_OK;
}

// Steps of a forked run starting from buffer `parity` (step j reads
// buf[parity ^ (j & 1)]) and the statistics reductions of their batches.
struct LatticeRun {
  cmf_lattice *L;
  int parity;
  hipError_t operator()(int j, hipStream_t s) const {
    return launch_lattice_step(L, parity ^ (j & 1), j, partials_buf(L, j % (2 * L->stat_batch)), s);
  }
};
struct LatticeFin {
  cmf_lattice *L;
  hipError_t operator()(int j0, int count, hipStream_t s) const {
    // j0 is a multiple of stat_batch: the batch's slots are consecutive
    return launch_finalize_batch(partials_buf(L, j0 % (2 * L->stat_batch)),
                                 (int64_t)kPartStride * L->partials_cap, count, L->nparts,
                                 L->level2, L->series, L->cap, L->step_dev, j0, 0, L->mass0, true,
                                 s);
  }
};

int capture_graph(cmf_lattice *L, int parity) {
  const bool stats = !(L->desc.flags & CMF_FLAG_NO_STATS);
  return capture_forked(L->stream, L->forked, stats, L->stat_batch, L->step_dev,
                        LatticeRun{L, parity}, LatticeFin{L}, &L->graph[parity]);
}

// n <= kGraphSteps direct steps in the forked form
int run_direct(cmf_lattice *L, int n) {
  const bool stats = !(L->desc.flags & CMF_FLAG_NO_STATS);
  int rc = run_forked(L->stream, L->forked, stats, L->stat_batch, L->step_dev,
                      LatticeRun{L, L->parity}, LatticeFin{L}, n);
  if (rc == CMF_OK) L->parity ^= (n & 1);
  return rc;
}

void release(cmf_lattice *L) {
  if (!L) return;
  if (L->stream) (void)hipStreamSynchronize(L->stream);
  for (int k = 0; k < 2; ++k) {
    if (L->graph[k]) (void)hipGraphExecDestroy(L->graph[k]);
    if (L->buf[k] && L->own_bufs && !(k == 1 && L->buf[1] == L->buf[0])) (void)hipFree(L->buf[k]);
  }
  if (L->partials) (void)hipFree(L->partials);
  if (L->level2) (void)hipFree(L->level2);
  if (L->series) (void)hipFree(L->series);
  if (L->step_dev) (void)hipFree(L->step_dev);
  if (L->sk_has_plan) (void)hipfftDestroy(L->sk_plan);
  for (void *p : {(void *)L->sk_fields, L->sk_F, (void *)L->sk_acc, (void *)L->sk_out,
                  (void *)L->sk_perm, (void *)L->sk_off})
    if (p) (void)hipFree(p);
  forked_release(L->forked);
  if (L->own_stream && L->stream) (void)hipStreamDestroy(L->stream);
  delete L;
}

int validate(const cmf_desc *d) {
  if (!d) return fail(CMF_EINVAL, "desc is NULL");
  if (d->q != 9 && d->q != 19 && d->q != 27)
    return fail(CMF_EINVAL, "q must be 9, 19 or 27, got %d", d->q);
  if (d->nx < 1 || d->ny < 1 || d->nz < 1)
    return fail(CMF_EINVAL, "box edges must be >= 1 (%d, %d, %d)", d->nx, d->ny, d->nz);
  if (d->q == 9 && d->nz != 1) return fail(CMF_EINVAL, "D2Q9 needs nz = 1, got %d", d->nz);
  if (!sqrt_norms_consistent(d->q))
    return fail(CMF_EINVAL, "internal: the kernels' sqrt(b_v) table does not match the basis");
  const int64_t N = (int64_t)d->nx * d->ny * d->nz;
  if (N >= (int64_t)1 << 31) return fail(CMF_EINVAL, "N = %lld sites exceeds 2^31 - 1", (long long)N);
  if (d->nx >= (1 << 28)) return fail(CMF_EINVAL, "nx = %d is not below 2^28", d->nx);
  if (d->storage < kF64 || d->storage > kBF16) return fail(CMF_EINVAL, "unknown storage %d", d->storage);
  if (!(d->rho0 > 0.0) || !isfinite(d->rho0)) return fail(CMF_EINVAL, "rho0 must be > 0");
  if (!(d->tau >= 0.5) || !isfinite(d->tau)) return fail(CMF_EINVAL, "tau must be >= 0.5");
  if (!(d->kT >= 0.0) || !isfinite(d->kT)) return fail(CMF_EINVAL, "kT must be >= 0");
  if (d->lambda)
    for (int v = 0; v < d->q; ++v)
      if (!(d->lambda[v] >= 0.0 && d->lambda[v] <= 2.0))
        return fail(CMF_EINVAL, "lambda[%d] = %g outside [0, 2]", v, d->lambda[v]);
  if (d->series_capacity < 0) return fail(CMF_EINVAL, "series_capacity < 0");
  return CMF_OK;
}

}  // namespace

extern "C" {

const char *cmf_version(void) { return "cmflb 0.1 (gfx950)"; }

const char *cmf_last_error(void) { return g_last_error.c_str(); }

int cmf_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return 0;
  return n;
}

namespace {

// host checks of the fields of an equilibrium initialisation: positive
// finite densities, finite velocities
int check_init_fields(int64_t N, const double *rho, const double *u) {
  if (rho)
    for (int64_t s = 0; s < N; ++s)
      if (!(rho[s] > 0.0) || !isfinite(rho[s]))
        return fail(CMF_EINVAL, "rho[%lld] = %g is not a positive density", (long long)s, rho[s]);
  if (u)
    for (int64_t s = 0; s < 3 * N; ++s)
      if (!isfinite(u[s]))
        return fail(CMF_EINVAL, "u[%lld] = %g is not finite", (long long)s, u[s]);
  return CMF_OK;
}

// device copies of the optional rho (N) and u (3 N) fields; on failure
// nothing stays allocated
hipError_t upload_init_fields(int64_t N, const double *rho, const double *u, double **drho,
                              double **du) {
  *drho = *du = nullptr;
  hipError_t e = hipSuccess;
  if (rho) {
    e = hipMalloc((void **)drho, sizeof(double) * N);
    if (e == hipSuccess) e = hipMemcpy(*drho, rho, sizeof(double) * N, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && u) {
    e = hipMalloc((void **)du, sizeof(double) * 3 * N);
    if (e == hipSuccess) e = hipMemcpy(*du, u, sizeof(double) * 3 * N, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    if (*drho) (void)hipFree(*drho);
    if (*du) (void)hipFree(*du);
    *drho = *du = nullptr;
  }
  return e;
}

// timing events, all or none
int create_events(std::vector<hipEvent_t> &ev) {
  for (auto &x : ev) {
    const hipError_t e = hipEventCreate(&x);
    if (e != hipSuccess) {
      for (auto &y : ev)
        if (y) (void)hipEventDestroy(y);
      return fail(CMF_EHIP, "hipEventCreate failed: %s", hipGetErrorString(e));
    }
  }
  return CMF_OK;
}

// bytes of one population buffer (q x N elements, rounded up to 256)
size_t buffer_bytes(const cmf_desc *d) {
  return ((size_t)d->q * d->nx * d->ny * d->nz * storage_bytes(d->storage) + 255) / 256 * 256;
}

// `p` must point into a device allocation of the current device with at
// least `bytes` bytes from p to the allocation's end (host-side queries
// only: a wrong pointer or a short buffer becomes CMF_EINVAL instead of a
// kernel access out of bounds).
int check_device_span(const void *p, size_t bytes, const char *what) {
  hipPointerAttribute_t attr;
  int dev = 0;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess || attr.type != hipMemoryTypeDevice ||
      hipGetDevice(&dev) != hipSuccess || attr.device != dev) {
    (void)hipGetLastError();
    return fail(CMF_EINVAL, "%s is not device memory of the current device", what);
  }
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void *>(p)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(CMF_EINVAL, "%s: the allocation holding it is not known to HIP", what);
  }
  const uintptr_t b = reinterpret_cast<uintptr_t>(base), a = reinterpret_cast<uintptr_t>(p);
  if (a < b || a - b > size || size - (a - b) < bytes)
    return fail(CMF_EINVAL, "%s: %zu bytes from it to the end of its allocation, %zu needed",
                what, a < b || a - b > size ? (size_t)0 : size - (a - b), bytes);
  return CMF_OK;
}

// population buffers of a lattice: one with in-place streaming, else two
int buffer_count(const cmf_desc *d) { return (d->flags & CMF_FLAG_IN_PLACE) ? 1 : 2; }

// in-place streaming addresses each z plane (ny q nx values) with 32-bit
// byte offsets
int check_in_place(const cmf_desc *d) {
  if (!(d->flags & CMF_FLAG_IN_PLACE)) return CMF_OK;
  const int64_t plane = (int64_t)d->ny * d->q * d->nx * storage_bytes(d->storage);
  if (plane >= ((int64_t)1 << 32))
    return fail(CMF_EUNSUPPORTED, "in-place streaming needs each z plane below 4 GiB (%lld bytes)",
                (long long)plane);
  return CMF_OK;
}

int create_lattice(const cmf_desc *desc, void *hip_stream, void *ext, size_t ext_bytes,
                   cmf_lattice **out) {
  if (!out) return fail(CMF_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(desc);
  if (rc != CMF_OK) return rc;
  rc = check_in_place(desc);
  if (rc != CMF_OK) return rc;
  if (ext) {
    const size_t need = buffer_count(desc) * buffer_bytes(desc);
    if (reinterpret_cast<uintptr_t>(ext) % 256 != 0)
      return fail(CMF_EINVAL, "external buffer is not 256-byte aligned");
    if (ext_bytes < need)
      return fail(CMF_EINVAL, "external buffer holds %zu bytes, the lattice needs %zu", ext_bytes, need);
    rc = check_device_span(ext, need, "external buffer");
    if (rc != CMF_OK) return rc;
  }
  cmf_lattice *L = new cmf_lattice();
  L->desc = *desc;
  L->desc.lambda = nullptr;
  L->q = desc->q;
  L->storage = desc->storage;
  L->N = (int64_t)desc->nx * desc->ny * desc->nz;
  L->cap = desc->series_capacity > 0 ? desc->series_capacity : 4096;
  const int q = L->q;

  // rates (the paper's pattern unless given) and the FP64 per-mode
  // constants
  ModeConstants mc;
  mode_constants(desc, mc);
  L->general = mc.general;
  L->nt_stores = ((int64_t)desc->nx * storage_bytes(desc->storage)) % kLineBytes == 0;
  L->in_place = (desc->flags & CMF_FLAG_IN_PLACE) != 0;
  double amp[27];
  float scale[27];
  for (int v = 0; v < q; ++v) {
    L->lambda[v] = mc.lambda[v];
    L->w[v] = mc.w[v];
    amp[v] = mc.amp[v];
    scale[v] = mc.scale[v];
  }
  L->mass0 = (double)L->N * desc->rho0;
  for (int v = 0; v < q; ++v) {
    L->amp[v] = amp[v];
    L->scale[v] = scale[v];
  }

  L->cp.nx = desc->nx;
  L->cp.ny = desc->ny;
  L->cp.nz = desc->nz;
  L->cp.pitch = 0;
  L->cp.layout = kLayoutPull;
  L->cp.rho0 = desc->rho0;
  for (int i = 0; i < q; ++i) {
    L->cp.w[i] = L->w[i];
    L->cp.scale[i] = scale[i];
    L->cp.iscale[i] = 1.0f / scale[i];
  }

  hipError_t e = hipGetDevice(&L->device);
  if (e != hipSuccess) {
    release(L);
    return fail(CMF_EHIP, "hipGetDevice failed: %s", hipGetErrorString(e));
  }
  if (hip_stream) {
    L->stream = (hipStream_t)hip_stream;
  } else {
    e = hipStreamCreate(&L->stream);
    if (e != hipSuccess) {
      release(L);
      return fail(CMF_EHIP, "hipStreamCreate failed: %s", hipGetErrorString(e));
    }
    L->own_stream = true;
  }
  const size_t bytes = buffer_bytes(desc);
  if (ext) {
    L->own_bufs = false;
    L->buf[0] = ext;
    L->buf[1] = L->in_place ? ext : static_cast<char *>(ext) + bytes;
  } else {
    for (int k = 0; k < buffer_count(desc); ++k) {
      if (hipMalloc(&L->buf[k], bytes) != hipSuccess) {
        release(L);
        return fail(CMF_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
      }
    }
    if (L->in_place) L->buf[1] = L->buf[0];
  }
  if (hipMalloc((void **)&L->series, sizeof(double) * kSeriesStride * L->cap) != hipSuccess ||
      hipMalloc((void **)&L->level2, sizeof(double) * kPartStride * kMaxLevel2 * kStatBatch) !=
          hipSuccess ||
      hipMalloc((void **)&L->step_dev, sizeof(int64_t)) != hipSuccess) {
    release(L);
    return fail(CMF_ENOMEM, "hipMalloc of statistics buffers failed");
  }
  // launch shape: a tuned one for this key if known, else the defaults
  // (persistent grid of 2 x CUs for 4- and 8-byte storage, 16 x CUs for
  // 16-bit storage, which is issue-bound and wants more waves)
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, L->device) == hipSuccess && prop.multiProcessorCount > 0)
      L->cus = prop.multiProcessorCount;
    int block = default_block(desc->nx);
    int grid = (storage_bytes(L->storage) >= 4 ? 2 : 16) * L->cus;
    lookup_tuned(L, &block, &grid);
    const int be = env_int("CMF_BLOCK", 0), ge = env_int("CMF_GRID", 0);
    if (be == 64 || be == 128 || be == 192 || be == 256) block = be;
    if (ge > 0) grid = ge;
    rc = apply_launch(L, block, grid, L->amp, L->scale);
    if (rc != CMF_OK) {
      release(L);
      return rc;
    }
  }
  *out = L;
  rc = cmf_init_equilibrium(L, nullptr, nullptr);
  if (rc != CMF_OK) {
    release(L);
    *out = nullptr;
    return rc;
  }
  return CMF_OK;
}

}  // namespace

int cmf_create(const cmf_desc *desc, void *hip_stream, cmf_lattice **out) {
  return create_lattice(desc, hip_stream, nullptr, 0, out);
}

int cmf_create_external(const cmf_desc *desc, void *dev_ptr, size_t bytes, void *hip_stream,
                        cmf_lattice **out) {
  if (!dev_ptr) return fail(CMF_EINVAL, "dev_ptr is NULL");
  return create_lattice(desc, hip_stream, dev_ptr, bytes, out);
}

size_t cmf_external_bytes(const cmf_desc *desc) {
  if (validate(desc) != CMF_OK || check_in_place(desc) != CMF_OK) return 0;
  return buffer_count(desc) * buffer_bytes(desc);
}

int cmf_destroy(cmf_lattice *L) {
  if (!L) return fail(CMF_EINVAL, "lattice is NULL");
  release(L);
  return CMF_OK;
}

int cmf_init_equilibrium(cmf_lattice *L, const double *rho, const double *u) {
  if (!L) return fail(CMF_EINVAL, "lattice is NULL");
  int rc = check_init_fields(L->N, rho, u);
  if (rc != CMF_OK) return rc;
  HIP_TRY(hipStreamSynchronize(L->stream));
  double *drho = nullptr, *du = nullptr;
  hipError_t e = upload_init_fields(L->N, rho, u, &drho, &du);
  if (e == hipSuccess) {
    L->parity = 0;
    e = launch_init_eq(L->q, L->storage, conv(L), drho, du, L->buf[0], L->stream);
  }
  if (e == hipSuccess) e = launch_zero_i64(L->step_dev, 1, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (drho) (void)hipFree(drho);
  if (du) (void)hipFree(du);
  if (e != hipSuccess) return fail(CMF_EHIP, "equilibrium initialisation failed: %s", hipGetErrorString(e));
  L->read_step = 0;
  return CMF_OK;
}

int cmf_set_populations(cmf_lattice *L, const double *f) {
  if (!L || !f) return fail(CMF_EINVAL, "NULL argument");
  HIP_TRY(hipStreamSynchronize(L->stream));
  double *df = nullptr;
  const size_t bytes = sizeof(double) * L->q * L->N;
  if (hipMalloc((void **)&df, bytes) != hipSuccess)
    return fail(CMF_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
  hipError_t e = hipMemcpy(df, f, bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_set_state(L->q, L->storage, conv(L), df, L->buf[L->parity], L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  (void)hipFree(df);
  if (e != hipSuccess) return fail(CMF_EHIP, "set_populations failed: %s", hipGetErrorString(e));
  return CMF_OK;
}

int cmf_get_populations(cmf_lattice *L, double *f) {
  if (!L || !f) return fail(CMF_EINVAL, "NULL argument");
  HIP_TRY(hipStreamSynchronize(L->stream));
  double *df = nullptr;
  const size_t bytes = sizeof(double) * L->q * L->N;
  if (hipMalloc((void **)&df, bytes) != hipSuccess)
    return fail(CMF_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
  hipError_t e = launch_get_state(L->q, L->storage, conv(L), L->buf[L->parity], df, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e == hipSuccess) e = hipMemcpy(f, df, bytes, hipMemcpyDeviceToHost);
  (void)hipFree(df);
  if (e != hipSuccess) return fail(CMF_EHIP, "get_populations failed: %s", hipGetErrorString(e));
  return CMF_OK;
}

int cmf_gather_sites(cmf_lattice *L, const int64_t *sites, int64_t n, double *out) {
  if (!L || (n > 0 && (!sites || !out))) return fail(CMF_EINVAL, "NULL argument");
  if (n < 0) return fail(CMF_EINVAL, "n < 0");
  if (n == 0) return CMF_OK;
  for (int64_t k = 0; k < n; ++k)
    if (sites[k] < 0 || sites[k] >= L->N)
      return fail(CMF_EINVAL, "site %lld outside [0, %lld)", (long long)sites[k], (long long)L->N);
  HIP_TRY(hipStreamSynchronize(L->stream));
  int64_t *ds = nullptr;
  double *dout = nullptr;
  if (hipMalloc((void **)&ds, sizeof(int64_t) * n) != hipSuccess ||
      hipMalloc((void **)&dout, sizeof(double) * L->q * n) != hipSuccess) {
    if (ds) (void)hipFree(ds);
    return fail(CMF_ENOMEM, "hipMalloc failed");
  }
  hipError_t e = hipMemcpy(ds, sites, sizeof(int64_t) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_gather(L->q, L->storage, conv(L), L->buf[L->parity], ds, n, dout, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e == hipSuccess) e = hipMemcpy(out, dout, sizeof(double) * L->q * n, hipMemcpyDeviceToHost);
  (void)hipFree(ds);
  (void)hipFree(dout);
  if (e != hipSuccess) return fail(CMF_EHIP, "gather_sites failed: %s", hipGetErrorString(e));
  return CMF_OK;
}

int cmf_step(cmf_lattice *L, int64_t nsteps) {
  if (!L) return fail(CMF_EINVAL, "lattice is NULL");
  if (nsteps < 0) return fail(CMF_EINVAL, "nsteps < 0");
  const bool graphs = !(L->desc.flags & CMF_FLAG_NO_GRAPH);
  int64_t left = nsteps;
  while (graphs && left >= kGraphSteps) {
    if (!L->graph[L->parity]) {
      int rc = capture_graph(L, L->parity);
      if (rc != CMF_OK) return rc;
    }
    HIP_TRY(hipGraphLaunch(L->graph[L->parity], L->stream));
    left -= kGraphSteps;  // an even number of steps: parity unchanged
  }
  while (left > 0) {
    const int n = left < kGraphSteps ? (int)left : kGraphSteps;
    int rc = run_direct(L, n);
    if (rc != CMF_OK) return rc;
    left -= n;
  }
  return CMF_OK;
}

int cmf_profile_steps(cmf_lattice *L, int64_t nsteps, double *kernel_ms) {
  if (!L || !kernel_ms) return fail(CMF_EINVAL, "NULL argument");
  if (nsteps < 0) return fail(CMF_EINVAL, "nsteps < 0");
  *kernel_ms = 0.0;
  if (nsteps == 0) return CMF_OK;
  std::vector<hipEvent_t> ev(2 * nsteps, nullptr);
  int rc = create_events(ev);
  if (rc != CMF_OK) return rc;
  // batches of stat_batch steps, each kernel between its own event pair and
  // the batch's statistics reduction after the batch, so that only event
  // markers separate consecutive step kernels
  const int K = L->stat_batch;
  const bool stats = !(L->desc.flags & CMF_FLAG_NO_STATS);
  for (int64_t s0 = 0; s0 < nsteps && rc == CMF_OK; s0 += K) {
    const int cnt = nsteps - s0 < K ? (int)(nsteps - s0) : K;
    hipError_t e = hipSuccess;
    for (int j = 0; j < cnt && e == hipSuccess; ++j) {
      e = hipEventRecord(ev[2 * (s0 + j)], L->stream);
      if (e == hipSuccess) e = launch_lattice_step(L, L->parity, j, partials_buf(L, j), L->stream);
      if (e == hipSuccess) e = hipEventRecord(ev[2 * (s0 + j) + 1], L->stream);
      if (e == hipSuccess) L->parity ^= 1;
    }
    if (e == hipSuccess && stats)
      e = launch_finalize_batch(partials_buf(L, 0), (int64_t)kPartStride * L->partials_cap, cnt,
                                L->nparts, L->level2, L->series, L->cap, L->step_dev, 0, 0,
                                L->mass0, true, L->stream);
    if (e == hipSuccess) e = launch_bump_step(L->step_dev, cnt, L->stream);
    if (e != hipSuccess) rc = fail(CMF_EHIP, "profiled step failed: %s", hipGetErrorString(e));
  }
  hipError_t e = hipStreamSynchronize(L->stream);
  if (rc == CMF_OK && e != hipSuccess) rc = fail(CMF_EHIP, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
  double total = 0.0;
  for (int64_t s = 0; s < nsteps && rc == CMF_OK; ++s) {
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, ev[2 * s], ev[2 * s + 1]);
    if (e != hipSuccess) rc = fail(CMF_EHIP, "hipEventElapsedTime failed: %s", hipGetErrorString(e));
    total += ms;
  }
  for (auto &x : ev) (void)hipEventDestroy(x);
  *kernel_ms = total;
  return rc;
}

int cmf_sk_reset(cmf_lattice *L, int32_t nbins) {
  if (!L) return fail(CMF_EINVAL, "lattice is NULL");
  if (nbins < 1 || nbins > 1024) return fail(CMF_EINVAL, "nbins must be in [1, 1024], got %d", nbins);
  HIP_TRY(hipStreamSynchronize(L->stream));
  const int nx = L->desc.nx, ny = L->desc.ny, nz = L->desc.nz;
  const int64_t M = (int64_t)(nx / 2 + 1) * ny * nz;
  if (!L->sk_has_plan) {
    // all buffers and the plan, or none of them
    auto drop = [&]() {
      for (void **p : {(void **)&L->sk_fields, &L->sk_F, (void **)&L->sk_acc, (void **)&L->sk_perm}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
      }
    };
    drop();
    if (hipMalloc((void **)&L->sk_fields, sizeof(float) * 4 * L->N) != hipSuccess ||
        hipMalloc(&L->sk_F, sizeof(float) * 2 * 4 * M) != hipSuccess ||
        hipMalloc((void **)&L->sk_acc, sizeof(double) * 4 * M) != hipSuccess ||
        hipMalloc((void **)&L->sk_perm, sizeof(int32_t) * M) != hipSuccess) {
      drop();
      return fail(CMF_ENOMEM, "structure-factor allocation failed");
    }
    hipfftResult fr = nz > 1 ? hipfftPlan3d(&L->sk_plan, nz, ny, nx, HIPFFT_R2C)
                             : hipfftPlan2d(&L->sk_plan, ny, nx, HIPFFT_R2C);
    if (fr != HIPFFT_SUCCESS) {
      drop();
      return fail(CMF_EHIP, "hipfft plan failed (%d)", (int)fr);
    }
    if (hipfftSetStream(L->sk_plan, L->stream) != HIPFFT_SUCCESS) {
      (void)hipfftDestroy(L->sk_plan);
      drop();
      return fail(CMF_EHIP, "hipfftSetStream failed");
    }
    L->sk_has_plan = true;
    L->sk_M = M;
  }
  if (L->sk_nbins != nbins) {
    L->sk_nbins = 0;  // no shells until the new ones are in place
    // shell of every mode on the device, counting sort by shell on the host
    std::vector<int32_t> bin(M), perm(M);
    std::vector<int64_t> off(nbins + 1, 0);
    HIP_TRY(launch_sk_shell_index(nx, ny, nz, nbins, M, L->sk_perm, L->stream));
    HIP_TRY(hipStreamSynchronize(L->stream));
    HIP_TRY(hipMemcpy(bin.data(), L->sk_perm, sizeof(int32_t) * M, hipMemcpyDeviceToHost));
    for (int64_t m = 0; m < M; ++m)
      if (bin[m] >= 0) ++off[bin[m] + 1];
    for (int b = 0; b < nbins; ++b) off[b + 1] += off[b];
    std::vector<int64_t> pos(off.begin(), off.end() - 1);
    for (int64_t m = 0; m < M; ++m)
      if (bin[m] >= 0) perm[pos[bin[m]]++] = (int32_t)m;
    if (L->sk_off) (void)hipFree(L->sk_off);
    if (L->sk_out) (void)hipFree(L->sk_out);
    L->sk_off = nullptr;
    L->sk_out = nullptr;
    if (hipMalloc((void **)&L->sk_off, sizeof(int64_t) * (nbins + 1)) != hipSuccess ||
        hipMalloc((void **)&L->sk_out, sizeof(double) * 6 * nbins) != hipSuccess)
      return fail(CMF_ENOMEM, "structure-factor allocation failed");
    HIP_TRY(hipMemcpy(L->sk_perm, perm.data(), sizeof(int32_t) * off[nbins], hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(L->sk_off, off.data(), sizeof(int64_t) * (nbins + 1), hipMemcpyHostToDevice));
    L->sk_nbins = nbins;
  }
  HIP_TRY(hipMemsetAsync(L->sk_acc, 0, sizeof(double) * 4 * M, L->stream));
  HIP_TRY(hipStreamSynchronize(L->stream));
  L->sk_samples = 0;
  return CMF_OK;
}

int cmf_sk_accumulate(cmf_lattice *L) {
  if (!L) return fail(CMF_EINVAL, "lattice is NULL");
  if (!L->sk_nbins) return fail(CMF_EINVAL, "call cmf_sk_reset first");
  HIP_TRY(launch_macro_dev(L->q, L->storage, conv(L), L->buf[L->parity], L->sk_fields, L->stream));
  for (int f = 0; f < 4; ++f) {
    hipfftResult fr = hipfftExecR2C(L->sk_plan, (hipfftReal *)(L->sk_fields + f * L->N),
                                    (hipfftComplex *)L->sk_F + f * L->sk_M);
    if (fr != HIPFFT_SUCCESS) return fail(CMF_EHIP, "hipfftExecR2C failed (%d)", (int)fr);
  }
  HIP_TRY(launch_sk_accumulate(L->sk_F, L->sk_M, 1.0 / (double)L->N, L->sk_acc, L->stream));
  ++L->sk_samples;
  return CMF_OK;
}

int cmf_sk_shells(cmf_lattice *L, double *out, int64_t *nsamples) {
  if (!L || !out) return fail(CMF_EINVAL, "NULL argument");
  if (!L->sk_nbins) return fail(CMF_EINVAL, "call cmf_sk_reset first");
  const int nb = L->sk_nbins;
  HIP_TRY(launch_sk_segments(L->sk_acc, L->sk_M, L->desc.nx, L->desc.ny, L->desc.nz, nb,
                             L->sk_perm, L->sk_off, L->sk_out, L->stream));
  HIP_TRY(hipStreamSynchronize(L->stream));
  std::vector<double> raw(6 * nb);
  HIP_TRY(hipMemcpy(raw.data(), L->sk_out, sizeof(double) * 6 * nb, hipMemcpyDeviceToHost));
  const double ns = L->sk_samples > 0 ? (double)L->sk_samples : 1.0;
  for (int b = 0; b < nb; ++b) {
    const double w = raw[6 * b + 1];
    out[6 * b + 0] = w > 0 ? raw[6 * b] / w : 0.0;
    out[6 * b + 1] = w;
    for (int c = 2; c < 6; ++c) out[6 * b + c] = w > 0 ? raw[6 * b + c] / w / ns : 0.0;
  }
  if (nsamples) *nsamples = L->sk_samples;
  return CMF_OK;
}

int cmf_get_launch(cmf_lattice *L, cmf_launch *out) {
  if (!L || !out) return fail(CMF_EINVAL, "NULL argument");
  out->block = L->block;
  out->grid = L->grid;
  out->ms_per_step = 0.0;
  return CMF_OK;
}

int cmf_set_launch(cmf_lattice *L, int32_t block, int32_t grid) {
  if (!L) return fail(CMF_EINVAL, "lattice is NULL");
  if (!(block == 64 || block == 128 || block == 192 || block == 256))
    return fail(CMF_EINVAL, "block must be 64, 128, 192 or 256, got %d", block);
  if (grid < 1) return fail(CMF_EINVAL, "grid must be >= 1, got %d", grid);
  HIP_TRY(hipStreamSynchronize(L->stream));
  return apply_launch(L, block, grid, L->amp, L->scale);
}

int cmf_autotune(cmf_lattice *L, int32_t steps_per_trial, cmf_launch *trials, int32_t cap,
                 int32_t *n_out) {
  if (!L) return fail(CMF_EINVAL, "lattice is NULL");
  if (steps_per_trial < 1) return fail(CMF_EINVAL, "steps_per_trial must be >= 1");
  if (n_out) *n_out = 0;
  HIP_TRY(hipStreamSynchronize(L->stream));
  // snapshot: current population buffer, step counter, series ring
  const size_t bytes = ((size_t)L->q * L->N * storage_bytes(L->storage) + 255) / 256 * 256;
  void *saved = nullptr;
  double *saved_series = nullptr;
  if (hipMalloc(&saved, bytes) != hipSuccess) return fail(CMF_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
  if (hipMalloc((void **)&saved_series, sizeof(double) * kSeriesStride * L->cap) != hipSuccess) {
    (void)hipFree(saved);
    return fail(CMF_ENOMEM, "hipMalloc of the statistics snapshot failed");
  }
  int64_t step0 = 0;
  const int parity0 = L->parity;
  const int block0 = L->block, grid0 = L->grid;
  hipError_t e = hipMemcpyAsync(saved, L->buf[parity0], bytes, hipMemcpyDeviceToDevice, L->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(saved_series, L->series, sizeof(double) * kSeriesStride * L->cap,
                       hipMemcpyDeviceToDevice, L->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&step0, L->step_dev, sizeof(int64_t), hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) {
    (void)hipFree(saved);
    (void)hipFree(saved_series);
    return fail(CMF_EHIP, "autotune snapshot failed: %s", hipGetErrorString(e));
  }
  std::vector<int> blocks;
  for (int b = 64; b <= 256; b += 64)
    if (b == 64 || b - 64 < L->desc.nx) blocks.push_back(b);
  std::vector<cmf_launch> done;
  int rc = CMF_OK;
  for (int b : blocks) {
    std::vector<int> grids;
    for (int m : {1, 2, 4, 8, 16, 32}) grids.push_back(m * L->cus);
    grids.push_back(ntiles_for(L, b));
    int last = -1;
    for (int g : grids) {
      const int gg = g < ntiles_for(L, b) ? g : ntiles_for(L, b);
      if (gg == last) continue;
      last = gg;
      rc = apply_launch(L, b, gg, L->amp, L->scale);
      if (rc != CMF_OK) break;
      double warm = 0.0, ms = 0.0;
      rc = time_full_steps(L, 1, &warm);
      if (rc == CMF_OK) rc = time_full_steps(L, steps_per_trial, &ms);
      if (rc != CMF_OK) break;
      done.push_back(cmf_launch{b, gg, ms / steps_per_trial});
    }
    if (rc != CMF_OK) break;
  }
  // restore the state exactly
  L->parity = parity0;
  e = hipMemcpyAsync(L->buf[parity0], saved, bytes, hipMemcpyDeviceToDevice, L->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(L->series, saved_series, sizeof(double) * kSeriesStride * L->cap,
                       hipMemcpyDeviceToDevice, L->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(L->step_dev, &step0, sizeof(int64_t), hipMemcpyHostToDevice, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  (void)hipFree(saved);
  (void)hipFree(saved_series);
  if (rc == CMF_OK && e != hipSuccess) rc = fail(CMF_EHIP, "autotune restore failed: %s", hipGetErrorString(e));
  if (rc != CMF_OK) {
    (void)apply_launch(L, block0, grid0, L->amp, L->scale);
    return rc;
  }
  size_t best = 0;
  for (size_t k = 1; k < done.size(); ++k)
    if (done[k].ms_per_step < done[best].ms_per_step) best = k;
  rc = apply_launch(L, done[best].block, done[best].grid, L->amp, L->scale);
  if (rc != CMF_OK) return rc;
  remember_tuned(L, done[best].block, done[best].grid, done[best].ms_per_step);
  if (trials)
    for (size_t k = 0; k < done.size() && (int32_t)k < cap; ++k) trials[k] = done[k];
  if (n_out) *n_out = (int32_t)done.size();
  return CMF_OK;
}

int cmf_synchronize(cmf_lattice *L) {
  if (!L) return fail(CMF_EINVAL, "lattice is NULL");
  HIP_TRY(hipStreamSynchronize(L->stream));
  return CMF_OK;
}

int cmf_get_step(cmf_lattice *L, int64_t *step) {
  if (!L || !step) return fail(CMF_EINVAL, "NULL argument");
  HIP_TRY(hipStreamSynchronize(L->stream));
  HIP_TRY(hipMemcpy(step, L->step_dev, sizeof(int64_t), hipMemcpyDeviceToHost));
  return CMF_OK;
}

int cmf_set_step(cmf_lattice *L, int64_t step) {
  if (!L) return fail(CMF_EINVAL, "lattice is NULL");
  if (step < 0 || step >= kMaxStep)
    return fail(CMF_EINVAL, "step %lld outside [0, 2^56)", (long long)step);
  HIP_TRY(hipStreamSynchronize(L->stream));
  HIP_TRY(hipMemcpy(L->step_dev, &step, sizeof(int64_t), hipMemcpyHostToDevice));
  L->read_step = step;
  return CMF_OK;
}

int cmf_stats(cmf_lattice *L, cmf_moments *out, int64_t cap, int64_t *n_out) {
  if (!L || !n_out || (cap > 0 && !out)) return fail(CMF_EINVAL, "NULL argument");
  if (cap < 0) return fail(CMF_EINVAL, "cap < 0");
  *n_out = 0;
  int64_t step = 0;
  int rc = cmf_get_step(L, &step);
  if (rc != CMF_OK) return rc;
  if (L->desc.flags & CMF_FLAG_NO_STATS) {
    L->read_step = step;
    return CMF_OK;
  }
  int64_t first = L->read_step;
  if (step - first > L->cap) first = step - L->cap;
  if (step - first > cap) first = step - cap;
  std::vector<double> ring((size_t)L->cap * kSeriesStride);
  if (step > first)
    HIP_TRY(hipMemcpy(ring.data(), L->series, sizeof(double) * ring.size(),
                      hipMemcpyDeviceToHost));
  std::vector<double> rows((size_t)(step - first) * kSeriesStride);
  for (int64_t s = first; s < step; ++s)
    memcpy(rows.data() + (s - first) * kSeriesStride,
           ring.data() + (s % L->cap) * kSeriesStride, sizeof(double) * kSeriesStride);
  bool bad = false;
  for (int64_t s = first; s < step; ++s) {
    const double *r = rows.data() + (s - first) * kSeriesStride;
    cmf_moments &m = out[s - first];
    m.step = r[0];
    m.sum_rho = r[1];
    for (int a = 0; a < 3; ++a) {
      m.sum_j[a] = r[2 + a];
      m.sum_u[a] = r[5 + a];
      m.sum_u2[a] = r[8 + a];
    }
    m.nonfinite = r[11];
    if (m.nonfinite != 0.0) bad = true;
  }
  *n_out = step - first;
  L->read_step = step;
  if (bad) return fail(CMF_ENONFINITE, "non-finite density or velocity in a recorded step");
  return CMF_OK;
}

int cmf_sample_macro(cmf_lattice *L, void *rho_dev, void *u_dev) {
  if (!L) return fail(CMF_EINVAL, "lattice is NULL");
  int rc = rho_dev ? check_device_span(rho_dev, sizeof(float) * L->N, "rho_dev") : CMF_OK;
  if (rc == CMF_OK && u_dev) rc = check_device_span(u_dev, sizeof(float) * 3 * L->N, "u_dev");
  if (rc != CMF_OK) return rc;
  HIP_TRY(launch_macro(L->q, L->storage, conv(L), L->buf[L->parity], (float *)rho_dev,
                       (float *)u_dev, L->stream));
  return CMF_OK;
}

int cmf_get_macro(cmf_lattice *L, double *rho, double *u) {
  if (!L) return fail(CMF_EINVAL, "lattice is NULL");
  if (!rho && !u) return CMF_OK;
  HIP_TRY(hipStreamSynchronize(L->stream));
  double *d = nullptr;
  const size_t bytes = sizeof(double) * 4 * L->N;
  if (hipMalloc((void **)&d, bytes) != hipSuccess)
    return fail(CMF_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
  hipError_t e = launch_macro(L->q, L->storage, conv(L), L->buf[L->parity], d, d + L->N, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e == hipSuccess && rho) e = hipMemcpy(rho, d, sizeof(double) * L->N, hipMemcpyDeviceToHost);
  if (e == hipSuccess && u) e = hipMemcpy(u, d + L->N, sizeof(double) * 3 * L->N, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(CMF_EHIP, "get_macro failed: %s", hipGetErrorString(e));
  return CMF_OK;
}

int cmf_velocity_pdf(cmf_lattice *L, int32_t nbins, double xmax, double *moments,
                     int64_t *counts) {
  if (!L) return fail(CMF_EINVAL, "lattice is NULL");
  if (counts && (nbins < 1 || nbins > kVelMaxBins))
    return fail(CMF_EINVAL, "nbins = %d outside [1, %d]", nbins, kVelMaxBins);
  if (counts && !(xmax > 0.0 && isfinite(xmax))) return fail(CMF_EINVAL, "xmax must be > 0");
  if (!moments && !counts) return CMF_OK;
  HIP_TRY(hipStreamSynchronize(L->stream));
  const int grid = (int)std::min<int64_t>((L->N + 255) / 256, 1024);
  const int nb2 = nbins + 2;
  double *partials = nullptr, *sums = nullptr;
  unsigned long long *dcounts = nullptr;
  if (hipMalloc((void **)&partials, sizeof(double) * kVelCols * grid) != hipSuccess ||
      hipMalloc((void **)&sums, sizeof(double) * kVelCols) != hipSuccess ||
      (counts && hipMalloc((void **)&dcounts, sizeof(unsigned long long) * 3 * nb2) != hipSuccess)) {
    if (partials) (void)hipFree(partials);
    if (sums) (void)hipFree(sums);
    return fail(CMF_ENOMEM, "hipMalloc failed");
  }
  const double n = (double)L->N;
  double h[kVelCols];
  // pass 1: the means; pass 2: central moments about them; pass 3: histogram
  VelNorm c = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  double mean[3], var[3], m3[3], m4[3];
  hipError_t e = launch_vel_moments(L->q, L->storage, conv(L), L->buf[L->parity], c, grid,
                                    partials, sums, L->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h, sums, sizeof h, hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e == hipSuccess) {
    for (int a = 0; a < 3; ++a) c.centre[a] = mean[a] = h[4 * a] / n;
    e = launch_vel_moments(L->q, L->storage, conv(L), L->buf[L->parity], c, grid, partials, sums,
                           L->stream);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h, sums, sizeof h, hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e == hipSuccess) {
    for (int a = 0; a < 3; ++a) {
      // central moments about the FP64 mean; the residual first moment
      // d = sum (u - mean) / N corrects them to the exact mean
      const double d = h[4 * a] / n, s2 = h[4 * a + 1] / n, s3 = h[4 * a + 2] / n,
                   s4 = h[4 * a + 3] / n;
      var[a] = s2 - d * d;
      m3[a] = s3 - 3.0 * d * s2 + 2.0 * d * d * d;
      m4[a] = s4 - 4.0 * d * s3 + 6.0 * d * d * s2 - 3.0 * d * d * d * d;
      mean[a] += d;
      c.centre[a] = mean[a];
      c.inv_sigma[a] = var[a] > 0.0 ? 1.0 / sqrt(var[a]) : 0.0;
    }
    if (moments)
      for (int a = 0; a < 3; ++a) {
        moments[4 * a] = mean[a];
        moments[4 * a + 1] = var[a];
        moments[4 * a + 2] = var[a] > 0.0 ? m3[a] / (var[a] * sqrt(var[a])) : 0.0;
        moments[4 * a + 3] = var[a] > 0.0 ? m4[a] / (var[a] * var[a]) : 0.0;
      }
  }
  if (e == hipSuccess && counts) {
    e = launch_zero_i64(reinterpret_cast<int64_t *>(dcounts), 3 * nb2, L->stream);
    if (e == hipSuccess)
      e = launch_vel_hist(L->q, L->storage, conv(L), L->buf[L->parity], c, grid, nbins, xmax,
                          dcounts, L->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(counts, dcounts, sizeof(unsigned long long) * 3 * nb2,
                         hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  }
  (void)hipFree(partials);
  (void)hipFree(sums);
  if (dcounts) (void)hipFree(dcounts);
  if (e != hipSuccess) return fail(CMF_EHIP, "velocity_pdf failed: %s", hipGetErrorString(e));
  return CMF_OK;
}

int cmf_noise_sample(int32_t q, uint64_t seed, uint32_t replica, int64_t step, int64_t site0,
                     int64_t n, int32_t fp64, double *out) {
  if (q != 9 && q != 19 && q != 27) return fail(CMF_EINVAL, "q must be 9, 19 or 27");
  if (step < 0 || step >= kMaxStep) return fail(CMF_EINVAL, "step outside [0, 2^56)");
  if (n < 0 || site0 < 0 || site0 + n > ((int64_t)1 << 32)) return fail(CMF_EINVAL, "bad site range");
  if (n == 0) return CMF_OK;
  if (!out) return fail(CMF_EINVAL, "out is NULL");
  double *d = nullptr;
  if (hipMalloc((void **)&d, sizeof(double) * q * n) != hipSuccess) return fail(CMF_ENOMEM, "hipMalloc failed");
  hipError_t e = launch_noise(q, fp64, (uint32_t)seed, (uint32_t)(seed >> 32), replica, (uint64_t)step,
                              site0, n, d,
                              nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(out, d, sizeof(double) * q * n, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(CMF_EHIP, "noise_sample failed: %s", hipGetErrorString(e));
  return CMF_OK;
}

int cmf_philox_words(const uint32_t *ctr, int64_t n, uint32_t key0, uint32_t key1, uint32_t *out) {
  if (n < 0) return fail(CMF_EINVAL, "n < 0");
  if (n == 0) return CMF_OK;
  if (!ctr || !out) return fail(CMF_EINVAL, "NULL argument");
  uint32_t *dc = nullptr, *dout = nullptr;
  if (hipMalloc((void **)&dc, 16 * n) != hipSuccess || hipMalloc((void **)&dout, 16 * n) != hipSuccess) {
    if (dc) (void)hipFree(dc);
    return fail(CMF_ENOMEM, "hipMalloc failed");
  }
  hipError_t e = hipMemcpy(dc, ctr, 16 * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_philox(dc, n, key0, key1, dout, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(out, dout, 16 * n, hipMemcpyDeviceToHost);
  (void)hipFree(dc);
  (void)hipFree(dout);
  if (e != hipSuccess) return fail(CMF_EHIP, "philox_words failed: %s", hipGetErrorString(e));
  return CMF_OK;
}

int cmf_stream_copy(size_t bytes, int32_t reps, double *best_ms) {
  if (!best_ms || reps < 1 || bytes == 0) return fail(CMF_EINVAL, "bad arguments");
  const size_t n16 = (bytes + 15) / 16;
  void *a = nullptr, *b = nullptr;
  if (hipMalloc(&a, n16 * 16) != hipSuccess || hipMalloc(&b, n16 * 16) != hipSuccess) {
    if (a) (void)hipFree(a);
    return fail(CMF_ENOMEM, "hipMalloc of %zu bytes failed", n16 * 16);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMemset(a, 0, n16 * 16);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = launch_stream_copy(a, b, n16, nullptr);  // warm-up
  double best = 1e30;
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, nullptr);
    if (e == hipSuccess) e = launch_stream_copy(a, b, n16, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && ms < best) best = ms;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(a);
  (void)hipFree(b);
  if (e != hipSuccess) return fail(CMF_EHIP, "stream copy failed: %s", hipGetErrorString(e));
  *best_ms = best;
  return CMF_OK;
}

}  // extern "C"

// ---- one step without allocation ------------------------------------------
// Device scratch of cmf_step_noalloc, one copy per GPU the library runs on
// (held until the process ends): the per-workgroup partial sums of the
// statistics (kNoAllocMaxGrid rows), the second-level rows of their
// reduction (kMaxLevel2 rows) and the step counter the kernels read.  In
// host code `scratch` only names the symbol; its device address comes from
// hipGetSymbolAddress, once per device (scratch_address).
namespace {
constexpr int kNoAllocMaxGrid = 65536;
constexpr size_t kScratchPartials = (size_t)kNoAllocMaxGrid * kPartStride;
constexpr size_t kScratchLevel2 = (size_t)kMaxLevel2 * kPartStride;
constexpr size_t kScratchDoubles = kScratchPartials + kScratchLevel2 + 1;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with that device current).
int scratch_address(double **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(CMF_EHIP, "hipGetDevice failed: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(CMF_EUNSUPPORTED, "device %d: at most %d devices are supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(CMF_EHIP, "hipGetSymbolAddress of the scratch array failed: %s",
                  hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<double *>(ptr);
  }
  *out = g_scratch_dev[dev];
  return CMF_OK;
}
}  // namespace

extern "C" int cmf_step_noalloc(const cmf_desc *desc, const void *src, void *dst, int64_t step,
                                int32_t block, int32_t grid, double *stats_dev,
                                void *hip_stream) {
  int rc = validate(desc);
  if (rc != CMF_OK) return rc;
  if (desc->flags & CMF_FLAG_IN_PLACE)
    return fail(CMF_EUNSUPPORTED, "cmf_step_noalloc is a two-buffer pull step (no CMF_FLAG_IN_PLACE)");
  if (!src || !dst || src == dst) return fail(CMF_EINVAL, "src and dst must be two different buffers");
  if (reinterpret_cast<uintptr_t>(src) % 256 != 0 || reinterpret_cast<uintptr_t>(dst) % 256 != 0)
    return fail(CMF_EINVAL, "src and dst must be 256-byte aligned");
  if (step < 0 || step >= kMaxStep)
    return fail(CMF_EINVAL, "step %lld outside [0, 2^56)", (long long)step);
  if (!valid_launch(block, grid))
    return fail(CMF_EINVAL, "block must be 64, 128, 192 or 256 and grid >= 1, got (%d, %d)", block,
                grid);
  if (grid > kNoAllocMaxGrid)
    return fail(CMF_EINVAL,
                "grid %d exceeds %d: the scratch holds the partial sums of at most %d workgroups",
                grid, kNoAllocMaxGrid, kNoAllocMaxGrid);
  const size_t state_bytes =
      (size_t)desc->q * desc->nx * desc->ny * desc->nz * storage_bytes(desc->storage);
  rc = check_device_span(src, state_bytes, "src");
  if (rc == CMF_OK) rc = check_device_span(dst, state_bytes, "dst");
  if (rc == CMF_OK && stats_dev)
    rc = check_device_span(stats_dev, kSeriesStride * sizeof(double), "stats_dev");
  if (rc != CMF_OK) return rc;
  double *scr = nullptr;
  rc = scratch_address(&scr);
  if (rc != CMF_OK) return rc;
  ModeConstants mc;
  mode_constants(desc, mc);
  StepParams<double> pd;
  StepParams<float> pf;
  const bool f64 = desc->storage == kF64;
  if (f64)
    fill_params(*desc, mc.lambda, mc.amp, mc.scale, block, pd);
  else
    fill_params(*desc, mc.lambda, mc.amp, mc.scale, block, pf);
  const int ntiles = f64 ? pd.ntiles : pf.ntiles;
  const int g = grid < ntiles ? grid : ntiles;
  const bool nt = ((int64_t)desc->nx * storage_bytes(desc->storage)) % kLineBytes == 0;
  const double mass0 = (double)desc->nx * desc->ny * desc->nz * desc->rho0;
  int64_t *step_dev = reinterpret_cast<int64_t *>(scr + kScratchPartials + kScratchLevel2);
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = launch_set_i64(step_dev, step, s);
  if (e == hipSuccess)
    e = launch_step(desc->q, desc->storage, mc.general, nt, kStreamPull,
                    f64 ? (const void *)&pd : (const void *)&pf,
                    src, dst, step_dev, 0, scr, g, block, s);
  if (e == hipSuccess && stats_dev)
    e = launch_finalize(scr, g, scr + kScratchPartials, stats_dev, 1, step_dev, 0, 0, mass0, true, s);
  if (e != hipSuccess) return fail(CMF_EHIP, "step launch failed: %s", hipGetErrorString(e));
  return CMF_OK;
}

// ===========================================================================
// batched ensembles
// ===========================================================================
struct cmf_ensemble {
  struct Rep {
    cmf_desc desc;
    int64_t N = 0;
    int64_t offset = 0;  // elements
    int64_t pitch = 0;   // elements per population array: N rounded up to 64
    int tile0 = 0, ntiles = 0, spt = 1, tsites = 0;
    ConvParams cp;
  };
  int n = 0;
  int storage = 1;
  uint32_t flags = 0;
  bool general = false;
  bool own_stream = false;
  hipStream_t stream = nullptr;
  std::vector<Rep> reps;
  std::vector<ModeConstants> mcs;
  int spt9 = kEnsembleSpt9, spt3d = kEnsembleSpt27;  // sites per thread of a tile
  int tiles_cap = 0;  // tiles the tile map and the partials are allocated for
  void *arena[2] = {nullptr, nullptr};
  size_t arena_bytes = 0;
  int parity = 0;
  void *d_reps = nullptr;
  int32_t *d_tile_rep = nullptr;
  int ntiles = 0;
  int64_t total_sites = 0;
  double *partials = nullptr;
  double *series = nullptr;
  double *d_mass0 = nullptr;
  int cap = 4096;
  int64_t *step_dev = nullptr;
  std::vector<int64_t> read_step;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  ForkedRun forked;
};

namespace {

// multiplier and shifts of the exact division by d >= 1 that
// udiv_invariant applies (Granlund and Montgomery, PLDI 1994, Fig. 4.1):
// l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1, s1 = min(l, 1),
// s2 = max(l - 1, 0)
void invariant_divisor(uint32_t d, uint32_t *m, uint32_t *sh) {
  int l = 0;
  while ((1ull << l) < d) ++l;
  *m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
  *sh = (uint32_t)(l < 1 ? l : 1) | ((uint32_t)(l > 1 ? l - 1 : 0) << 8);
}

template <typename R>
void fill_replica(const cmf_desc &d, const ModeConstants &mc, const cmf_ensemble::Rep &rp,
                  ReplicaParams<R> &p) {
  memset(&p, 0, sizeof p);
  p.q = d.q;
  p.nx = d.nx;
  p.ny = d.ny;
  p.nz = d.nz;
  p.nsites = (int32_t)rp.N;
  p.tile0 = rp.tile0;
  p.ntiles = rp.ntiles;
  p.spt = rp.spt;
  p.tsites = rp.tsites;
  p.pitch = (int32_t)rp.pitch;
  invariant_divisor((uint32_t)d.nx, &p.div_nx, &p.sh_nx);
  invariant_divisor((uint32_t)d.ny, &p.div_ny, &p.sh_ny);
  p.noise = d.kT > 0.0 ? 1 : 0;
  p.offset = rp.offset;
  p.key0 = (uint32_t)d.seed;
  p.key1 = (uint32_t)(d.seed >> 32);
  p.replica = d.replica;
  p.rho0 = (R)d.rho0;
  for (int v = 0; v < d.q; ++v) {
    p.amp[v] = (R)mc.amp[v];
    p.oml[v] = (R)(1.0 - mc.lambda[v]);
    p.lam[v] = (R)mc.lambda[v];
  }
  p.amp1 = (R)sqrt(d.kT / kCs2);
  class_scales(d.q, d.storage, mc.scale, p.scale, p.iscale);
}

void ens_release(cmf_ensemble *E) {
  if (!E) return;
  if (E->stream) (void)hipStreamSynchronize(E->stream);
  for (int k = 0; k < 2; ++k) {
    if (E->graph[k]) (void)hipGraphExecDestroy(E->graph[k]);
    if (E->arena[k]) (void)hipFree(E->arena[k]);
  }
  if (E->d_reps) (void)hipFree(E->d_reps);
  if (E->d_tile_rep) (void)hipFree(E->d_tile_rep);
  if (E->partials) (void)hipFree(E->partials);
  if (E->series) (void)hipFree(E->series);
  if (E->d_mass0) (void)hipFree(E->d_mass0);
  if (E->step_dev) (void)hipFree(E->step_dev);
  forked_release(E->forked);
  if (E->own_stream && E->stream) (void)hipStreamDestroy(E->stream);
  delete E;
}

double *ens_partials_buf(const cmf_ensemble *E, int b) {
  return E->partials + (size_t)b * kPartStride * E->ntiles;
}

// One direct step (as enqueue_one_step of a lattice).
int ens_enqueue_step(cmf_ensemble *E) {
  HIP_TRY(launch_ensemble_step(E->storage, E->general, E->d_reps, E->d_tile_rep, E->ntiles,
                               E->arena[E->parity], E->arena[1 - E->parity], E->step_dev, 0,
                               ens_partials_buf(E, 0), E->stream));
  HIP_TRY(launch_ensemble_finalize(E->storage, E->d_reps, E->n, ens_partials_buf(E, 0), E->series,
                                   E->cap, E->step_dev, 0, 1, E->d_mass0,
                                   !(E->flags & CMF_FLAG_NO_STATS), E->stream));
  E->parity ^= 1;
  return CMF_OK;
}

struct EnsembleRun {
  cmf_ensemble *E;
  int parity;
  hipError_t operator()(int j, hipStream_t s) const {
    const int b = parity ^ (j & 1);
    return launch_ensemble_step(E->storage, E->general, E->d_reps, E->d_tile_rep,
                                E->ntiles, E->arena[b], E->arena[b ^ 1], E->step_dev, j,
                                ens_partials_buf(E, j & 1), s);
  }
};
struct EnsembleFin {
  cmf_ensemble *E;
  hipError_t operator()(int j, int count, hipStream_t s) const {
    if (count != 1) return hipErrorInvalidValue;  // ensembles reduce step by step
    return launch_ensemble_finalize(E->storage, E->d_reps, E->n, ens_partials_buf(E, j & 1),
                                    E->series, E->cap, E->step_dev, j, 0, E->d_mass0, true, s);
  }
};

int ens_capture(cmf_ensemble *E, int parity) {
  const bool stats = !(E->flags & CMF_FLAG_NO_STATS);
  return capture_forked(E->stream, E->forked, stats, 1, E->step_dev, EnsembleRun{E, parity},
                        EnsembleFin{E}, &E->graph[parity]);
}

int ens_run_direct(cmf_ensemble *E, int n) {
  const bool stats = !(E->flags & CMF_FLAG_NO_STATS);
  int rc = run_forked(E->stream, E->forked, stats, 1, E->step_dev, EnsembleRun{E, E->parity},
                      EnsembleFin{E}, n);
  if (rc == CMF_OK) E->parity ^= (n & 1);
  return rc;
}

int ens_check_index(cmf_ensemble *E, int32_t index) {
  if (!E) return fail(CMF_EINVAL, "ensemble is NULL");
  if (index < 0 || index >= E->n) return fail(CMF_EINVAL, "replica index %d outside [0, %d)", index, E->n);
  return CMF_OK;
}

void *ens_replica_buffer(cmf_ensemble *E, int index) {
  return (char *)E->arena[E->parity] + E->reps[index].offset * storage_bytes(E->storage);
}

// Tile the replicas, 3-D replicas first, then D2Q9, each in creation order:
// a tile of a replica is spt x kEnsembleBlock consecutive sites, spt = spt9
// (D2Q9) or spt3d (D3Q19, D3Q27), the last tile of a replica ragged.  Uploads the tile map and the replica
// records, grows the tile map and the partial-sum buffers when needed and
// drops captured graphs.  The stream must be idle.
int ens_build_tiles(cmf_ensemble *E, int spt9, int spt3d) {
  std::vector<int32_t> tile_rep;
  std::vector<int> tile0(E->n), ntl(E->n), spt(E->n), tsites(E->n);
  for (int pass = 0; pass < 2; ++pass)
    for (int r = 0; r < E->n; ++r) {
      const int q = E->reps[r].desc.q;
      if ((pass == 0) != (q != 9)) continue;
      tile0[r] = (int)tile_rep.size();
      spt[r] = q == 9 ? spt9 : spt3d;
      tsites[r] = spt[r] * kEnsembleBlock;
      const int64_t n = (E->reps[r].N + tsites[r] - 1) / tsites[r];
      if ((int64_t)tile_rep.size() + n >= ((int64_t)1 << 31))
        return fail(CMF_EINVAL, "ensemble has too many tiles");
      ntl[r] = (int)n;
      tile_rep.insert(tile_rep.end(), ntl[r], r);
    }
  const int nt = (int)tile_rep.size();
  if (nt > E->tiles_cap) {
    // allocate first, so that a failure leaves the current tiling usable
    int32_t *map = nullptr;
    double *parts = nullptr;
    if (hipMalloc((void **)&map, sizeof(int32_t) * nt) != hipSuccess ||
        hipMalloc((void **)&parts, 2 * sizeof(double) * kPartStride * nt) != hipSuccess) {
      if (map) (void)hipFree(map);
      return fail(CMF_ENOMEM, "allocation of the tile map (%d tiles) failed", nt);
    }
    if (E->d_tile_rep) (void)hipFree(E->d_tile_rep);
    if (E->partials) (void)hipFree(E->partials);
    E->d_tile_rep = map;
    E->partials = parts;
    E->tiles_cap = nt;
  }
  for (int r = 0; r < E->n; ++r) {
    E->reps[r].tile0 = tile0[r];
    E->reps[r].ntiles = ntl[r];
    E->reps[r].spt = spt[r];
    E->reps[r].tsites = tsites[r];
  }
  E->ntiles = nt;
  E->spt9 = spt9;
  E->spt3d = spt3d;
  hipError_t e = hipMemcpy(E->d_tile_rep, tile_rep.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    if (E->storage == kF64) {
      std::vector<ReplicaParams<double>> h(E->n);
      for (int r = 0; r < E->n; ++r) fill_replica(E->reps[r].desc, E->mcs[r], E->reps[r], h[r]);
      e = hipMemcpy(E->d_reps, h.data(), sizeof(ReplicaParams<double>) * E->n, hipMemcpyHostToDevice);
    } else {
      std::vector<ReplicaParams<float>> h(E->n);
      for (int r = 0; r < E->n; ++r) fill_replica(E->reps[r].desc, E->mcs[r], E->reps[r], h[r]);
      e = hipMemcpy(E->d_reps, h.data(), sizeof(ReplicaParams<float>) * E->n, hipMemcpyHostToDevice);
    }
  }
  for (int k = 0; k < 2; ++k)
    if (E->graph[k]) {
      (void)hipGraphExecDestroy(E->graph[k]);
      E->graph[k] = nullptr;
    }
  if (e != hipSuccess) return fail(CMF_EHIP, "tile map upload failed: %s", hipGetErrorString(e));
  return CMF_OK;
}

}  // namespace

extern "C" {

int cmf_ensemble_create(const cmf_desc *descs, int32_t n, void *hip_stream, cmf_ensemble **out) {
  if (!out) return fail(CMF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!descs || n < 1) return fail(CMF_EINVAL, "need at least one descriptor");
  for (int r = 0; r < n; ++r) {
    int rc = validate(&descs[r]);
    if (rc != CMF_OK) return fail(rc, "replica %d: %s", r, g_last_error.c_str());
    if (descs[r].storage != descs[0].storage) return fail(CMF_EINVAL, "replica %d: storage differs from replica 0", r);
    if (descs[r].flags != descs[0].flags) return fail(CMF_EINVAL, "replica %d: flags differ from replica 0", r);
    if (descs[r].flags & CMF_FLAG_IN_PLACE)
      return fail(CMF_EUNSUPPORTED, "replica %d: in-place streaming is for single lattices", r);
    // ensemble tiles address a replica's buffer (q arrays of N rounded up
    // to 64) with 32-bit byte offsets
    const int64_t n_pad = ((int64_t)descs[r].nx * descs[r].ny * descs[r].nz + 63) / 64 * 64;
    const int64_t bytes = (int64_t)descs[r].q * n_pad * storage_bytes(descs[r].storage);
    if (bytes >= ((int64_t)1 << 32))
      return fail(CMF_EINVAL, "replica %d: %lld population bytes; an ensemble member holds below 4 GiB",
                  r, (long long)bytes);
  }
  cmf_ensemble *E = new cmf_ensemble();
  E->n = n;
  E->storage = descs[0].storage;
  E->flags = descs[0].flags;
  E->cap = descs[0].series_capacity > 0 ? descs[0].series_capacity : 4096;
  E->reps.resize(n);
  E->read_step.assign(n, 0);
  E->mcs.resize(n);
  std::vector<ModeConstants> &mcs = E->mcs;
  int64_t offset = 0;
  for (int r = 0; r < n; ++r) {
    cmf_ensemble::Rep &rp = E->reps[r];
    rp.desc = descs[r];
    rp.desc.lambda = nullptr;
    rp.N = (int64_t)descs[r].nx * descs[r].ny * descs[r].nz;
    rp.offset = offset;
    rp.pitch = (rp.N + 63) / 64 * 64;
    offset += (int64_t)descs[r].q * rp.pitch;
    mode_constants(&descs[r], mcs[r]);
    if (mcs[r].general) E->general = true;
    rp.cp.nx = descs[r].nx;
    rp.cp.ny = descs[r].ny;
    rp.cp.nz = descs[r].nz;
    rp.cp.pitch = rp.pitch;
    rp.cp.layout = kLayoutPull;
    rp.cp.rho0 = descs[r].rho0;
    for (int i = 0; i < descs[r].q; ++i) {
      rp.cp.w[i] = mcs[r].w[i];
      rp.cp.scale[i] = mcs[r].scale[i];
      rp.cp.iscale[i] = 1.0f / mcs[r].scale[i];
    }
    E->total_sites += rp.N;
  }
  // sites per thread of the tiles (cmf_ensemble_set_tiles / _autotune;
  // CMF_ENSEMBLE_SPT9 / CMF_ENSEMBLE_SPT27, the latter for both 3-D
  // lattices, override the defaults, 1..16)
  const int spt9 = env_int("CMF_ENSEMBLE_SPT9", kEnsembleSpt9, 1, 16);
  const int spt27 = env_int("CMF_ENSEMBLE_SPT27", kEnsembleSpt27, 1, 16);
  E->arena_bytes = ((size_t)offset * storage_bytes(E->storage) + 255) / 256 * 256;
  hipError_t e = hip_stream ? hipSuccess : hipStreamCreate(&E->stream);
  if (hip_stream) E->stream = (hipStream_t)hip_stream; else E->own_stream = true;
  if (e != hipSuccess) {
    ens_release(E);
    return fail(CMF_EHIP, "hipStreamCreate failed: %s", hipGetErrorString(e));
  }
  const size_t rec = E->storage == kF64 ? sizeof(ReplicaParams<double>) : sizeof(ReplicaParams<float>);
  bool ok = hipMalloc(&E->arena[0], E->arena_bytes) == hipSuccess &&
            hipMalloc(&E->arena[1], E->arena_bytes) == hipSuccess &&
            hipMalloc(&E->d_reps, rec * n) == hipSuccess &&
            hipMalloc((void **)&E->series, sizeof(double) * kSeriesStride * E->cap * n) == hipSuccess &&
            hipMalloc((void **)&E->d_mass0, sizeof(double) * n) == hipSuccess &&
            hipMalloc((void **)&E->step_dev, sizeof(int64_t)) == hipSuccess;
  if (!ok) {
    ens_release(E);
    return fail(CMF_ENOMEM, "ensemble allocation (%zu bytes per arena) failed", E->arena_bytes);
  }
  {
    const int rc = ens_build_tiles(E, spt9, spt27);
    if (rc != CMF_OK) {
      const std::string msg = g_last_error;
      ens_release(E);
      return fail(rc, "%s", msg.c_str());
    }
  }
  std::vector<double> mass0(n);
  for (int r = 0; r < n; ++r) mass0[r] = (double)E->reps[r].N * descs[r].rho0;
  e = hipMemcpy(E->d_mass0, mass0.data(), sizeof(double) * n, hipMemcpyHostToDevice);
  // at rest every deviation is exactly zero
  if (e == hipSuccess) e = hipMemsetAsync(E->arena[0], 0, E->arena_bytes, E->stream);
  if (e == hipSuccess) e = launch_zero_i64(E->step_dev, 1, E->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(E->stream);
  if (e != hipSuccess) {
    ens_release(E);
    return fail(CMF_EHIP, "ensemble initialisation failed: %s", hipGetErrorString(e));
  }
  *out = E;
  return CMF_OK;
}

int cmf_ensemble_destroy(cmf_ensemble *E) {
  if (!E) return fail(CMF_EINVAL, "ensemble is NULL");
  ens_release(E);
  return CMF_OK;
}

int cmf_ensemble_info(cmf_ensemble *E, int32_t *n_replicas, int64_t *total_sites, int64_t *n_tiles) {
  if (!E) return fail(CMF_EINVAL, "ensemble is NULL");
  if (n_replicas) *n_replicas = E->n;
  if (total_sites) *total_sites = E->total_sites;
  if (n_tiles) *n_tiles = E->ntiles;
  return CMF_OK;
}

int cmf_ensemble_get_tiles(cmf_ensemble *E, cmf_ensemble_tiles *out) {
  if (!E || !out) return fail(CMF_EINVAL, "NULL argument");
  out->spt9 = E->spt9;
  out->spt3d = E->spt3d;
  out->ms_per_step = 0.0;
  return CMF_OK;
}

int cmf_ensemble_set_tiles(cmf_ensemble *E, int32_t spt9, int32_t spt3d) {
  if (!E) return fail(CMF_EINVAL, "ensemble is NULL");
  if (spt9 < 1 || spt9 > 16 || spt3d < 1 || spt3d > 16)
    return fail(CMF_EINVAL, "sites per thread must be in [1, 16], got %d and %d", spt9, spt3d);
  HIP_TRY(hipStreamSynchronize(E->stream));
  return ens_build_tiles(E, spt9, spt3d);
}

int cmf_ensemble_autotune(cmf_ensemble *E, int32_t steps_per_trial, cmf_ensemble_tiles *trials,
                          int32_t cap, int32_t *n_out) {
  if (!E) return fail(CMF_EINVAL, "ensemble is NULL");
  if (steps_per_trial < 1) return fail(CMF_EINVAL, "steps_per_trial must be >= 1");
  if (n_out) *n_out = 0;
  HIP_TRY(hipStreamSynchronize(E->stream));
  bool has2d = false, has3d = false;
  for (const auto &rp : E->reps) (rp.desc.q == 9 ? has2d : has3d) = true;
  std::vector<int> c9 = has2d ? std::vector<int>{1, 2, 3, 4, 6, 8} : std::vector<int>{E->spt9};
  std::vector<int> c3 = has3d ? std::vector<int>{1, 2, 3, 4, 6, 8} : std::vector<int>{E->spt3d};
  // snapshot: current arena, step counter, statistics rings
  const size_t series_bytes = sizeof(double) * kSeriesStride * E->cap * E->n;
  void *saved = nullptr, *saved_series = nullptr;
  if (hipMalloc(&saved, E->arena_bytes) != hipSuccess) return fail(CMF_ENOMEM, "hipMalloc of %zu bytes failed", E->arena_bytes);
  if (hipMalloc(&saved_series, series_bytes) != hipSuccess) {
    (void)hipFree(saved);
    return fail(CMF_ENOMEM, "hipMalloc of the statistics snapshot failed");
  }
  const int parity0 = E->parity, spt9_0 = E->spt9, spt3d_0 = E->spt3d;
  int64_t step0 = 0;
  hipError_t e = hipMemcpyAsync(saved, E->arena[parity0], E->arena_bytes, hipMemcpyDeviceToDevice, E->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(saved_series, E->series, series_bytes, hipMemcpyDeviceToDevice, E->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&step0, E->step_dev, sizeof(int64_t), hipMemcpyDeviceToHost, E->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(E->stream);
  if (e != hipSuccess) {
    (void)hipFree(saved);
    (void)hipFree(saved_series);
    return fail(CMF_EHIP, "ensemble autotune snapshot failed: %s", hipGetErrorString(e));
  }
  std::vector<cmf_ensemble_tiles> done;
  int rc = CMF_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(CMF_EHIP, "hipEventCreate failed");
  for (int a : c9) {
    for (int b : c3) {
      if (rc != CMF_OK) break;
      rc = ens_build_tiles(E, a, b);
      if (rc != CMF_OK) break;
      rc = ens_enqueue_step(E);  // untimed
      hipError_t x = hipSuccess;
      if (rc == CMF_OK) x = hipEventRecord(e0, E->stream);
      for (int k = 0; k < steps_per_trial && rc == CMF_OK && x == hipSuccess; ++k) rc = ens_enqueue_step(E);
      if (rc == CMF_OK && x == hipSuccess) x = hipEventRecord(e1, E->stream);
      if (rc == CMF_OK && x == hipSuccess) x = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (rc == CMF_OK && x == hipSuccess) x = hipEventElapsedTime(&ms, e0, e1);
      if (rc == CMF_OK && x != hipSuccess) rc = fail(CMF_EHIP, "ensemble autotune timing failed: %s", hipGetErrorString(x));
      if (rc == CMF_OK) done.push_back(cmf_ensemble_tiles{a, b, (double)ms / steps_per_trial});
    }
    if (rc != CMF_OK) break;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  // restore the state exactly
  (void)hipStreamSynchronize(E->stream);
  E->parity = parity0;
  e = hipMemcpyAsync(E->arena[parity0], saved, E->arena_bytes, hipMemcpyDeviceToDevice, E->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(E->series, saved_series, series_bytes, hipMemcpyDeviceToDevice, E->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(E->step_dev, &step0, sizeof(int64_t), hipMemcpyHostToDevice, E->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(E->stream);
  (void)hipFree(saved);
  (void)hipFree(saved_series);
  if (rc == CMF_OK && e != hipSuccess) rc = fail(CMF_EHIP, "ensemble autotune restore failed: %s", hipGetErrorString(e));
  if (rc != CMF_OK || done.empty()) {
    const std::string msg = rc != CMF_OK ? g_last_error : std::string("no trial ran");
    (void)ens_build_tiles(E, spt9_0, spt3d_0);
    return fail(rc != CMF_OK ? rc : CMF_EHIP, "%s", msg.c_str());
  }
  size_t best = 0;
  for (size_t k = 1; k < done.size(); ++k)
    if (done[k].ms_per_step < done[best].ms_per_step) best = k;
  rc = ens_build_tiles(E, done[best].spt9, done[best].spt3d);
  if (rc != CMF_OK) return rc;
  if (trials)
    for (size_t k = 0; k < done.size() && (int32_t)k < cap; ++k) trials[k] = done[k];
  if (n_out) *n_out = (int32_t)done.size();
  return CMF_OK;
}

int cmf_ensemble_init_equilibrium(cmf_ensemble *E, int32_t index, const double *rho, const double *u) {
  int rc = ens_check_index(E, index);
  if (rc != CMF_OK) return rc;
  cmf_ensemble::Rep &rp = E->reps[index];
  rc = check_init_fields(rp.N, rho, u);
  if (rc != CMF_OK) return rc;
  HIP_TRY(hipStreamSynchronize(E->stream));
  double *drho = nullptr, *du = nullptr;
  hipError_t e = upload_init_fields(rp.N, rho, u, &drho, &du);
  if (e == hipSuccess)
    e = launch_init_eq(rp.desc.q, E->storage, rp.cp, drho, du, ens_replica_buffer(E, index), E->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(E->stream);
  if (drho) (void)hipFree(drho);
  if (du) (void)hipFree(du);
  if (e != hipSuccess) return fail(CMF_EHIP, "ensemble init failed: %s", hipGetErrorString(e));
  return CMF_OK;
}

int cmf_ensemble_set_populations(cmf_ensemble *E, int32_t index, const double *f) {
  int rc = ens_check_index(E, index);
  if (rc != CMF_OK) return rc;
  if (!f) return fail(CMF_EINVAL, "f is NULL");
  cmf_ensemble::Rep &rp = E->reps[index];
  HIP_TRY(hipStreamSynchronize(E->stream));
  const size_t bytes = sizeof(double) * rp.desc.q * rp.N;
  double *df = nullptr;
  if (hipMalloc((void **)&df, bytes) != hipSuccess) return fail(CMF_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
  hipError_t e = hipMemcpy(df, f, bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_set_state(rp.desc.q, E->storage, rp.cp, df, ens_replica_buffer(E, index), E->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(E->stream);
  (void)hipFree(df);
  if (e != hipSuccess) return fail(CMF_EHIP, "ensemble set_populations failed: %s", hipGetErrorString(e));
  return CMF_OK;
}

int cmf_ensemble_get_populations(cmf_ensemble *E, int32_t index, double *f) {
  int rc = ens_check_index(E, index);
  if (rc != CMF_OK) return rc;
  if (!f) return fail(CMF_EINVAL, "f is NULL");
  cmf_ensemble::Rep &rp = E->reps[index];
  HIP_TRY(hipStreamSynchronize(E->stream));
  const size_t bytes = sizeof(double) * rp.desc.q * rp.N;
  double *df = nullptr;
  if (hipMalloc((void **)&df, bytes) != hipSuccess) return fail(CMF_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
  hipError_t e = launch_get_state(rp.desc.q, E->storage, rp.cp, ens_replica_buffer(E, index), df, E->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(E->stream);
  if (e == hipSuccess) e = hipMemcpy(f, df, bytes, hipMemcpyDeviceToHost);
  (void)hipFree(df);
  if (e != hipSuccess) return fail(CMF_EHIP, "ensemble get_populations failed: %s", hipGetErrorString(e));
  return CMF_OK;
}

int cmf_ensemble_step(cmf_ensemble *E, int64_t nsteps) {
  if (!E) return fail(CMF_EINVAL, "ensemble is NULL");
  if (nsteps < 0) return fail(CMF_EINVAL, "nsteps < 0");
  const bool graphs = !(E->flags & CMF_FLAG_NO_GRAPH);
  int64_t left = nsteps;
  while (graphs && left >= kGraphSteps) {
    if (!E->graph[E->parity]) {
      int rc = ens_capture(E, E->parity);
      if (rc != CMF_OK) return rc;
    }
    HIP_TRY(hipGraphLaunch(E->graph[E->parity], E->stream));
    left -= kGraphSteps;
  }
  while (left > 0) {
    const int n = left < kGraphSteps ? (int)left : kGraphSteps;
    int rc = ens_run_direct(E, n);
    if (rc != CMF_OK) return rc;
    left -= n;
  }
  return CMF_OK;
}

int cmf_ensemble_profile_steps(cmf_ensemble *E, int64_t nsteps, double *kernel_ms) {
  if (!E || !kernel_ms) return fail(CMF_EINVAL, "NULL argument");
  if (nsteps < 0) return fail(CMF_EINVAL, "nsteps < 0");
  *kernel_ms = 0.0;
  std::vector<hipEvent_t> ev(2 * nsteps, nullptr);
  const int rc = create_events(ev);
  if (rc != CMF_OK) return rc;
  hipError_t e = hipSuccess;
  for (int64_t s = 0; s < nsteps && e == hipSuccess; ++s) {
    e = hipEventRecord(ev[2 * s], E->stream);
    if (e == hipSuccess)
      e = launch_ensemble_step(E->storage, E->general, E->d_reps, E->d_tile_rep, E->ntiles,
                               E->arena[E->parity], E->arena[1 - E->parity], E->step_dev, 0,
                               ens_partials_buf(E, 0), E->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[2 * s + 1], E->stream);
    if (e == hipSuccess)
      e = launch_ensemble_finalize(E->storage, E->d_reps, E->n, ens_partials_buf(E, 0), E->series,
                                   E->cap, E->step_dev, 0, 1, E->d_mass0,
                                   !(E->flags & CMF_FLAG_NO_STATS), E->stream);
    E->parity ^= 1;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(E->stream);
  double total = 0.0;
  for (int64_t s = 0; s < nsteps && e == hipSuccess; ++s) {
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, ev[2 * s], ev[2 * s + 1]);
    total += ms;
  }
  for (auto &x : ev) (void)hipEventDestroy(x);
  if (e != hipSuccess) return fail(CMF_EHIP, "ensemble profiling failed: %s", hipGetErrorString(e));
  *kernel_ms = total;
  return CMF_OK;
}

int cmf_ensemble_synchronize(cmf_ensemble *E) {
  if (!E) return fail(CMF_EINVAL, "ensemble is NULL");
  HIP_TRY(hipStreamSynchronize(E->stream));
  return CMF_OK;
}

int cmf_ensemble_get_step(cmf_ensemble *E, int64_t *step) {
  if (!E || !step) return fail(CMF_EINVAL, "NULL argument");
  HIP_TRY(hipStreamSynchronize(E->stream));
  HIP_TRY(hipMemcpy(step, E->step_dev, sizeof(int64_t), hipMemcpyDeviceToHost));
  return CMF_OK;
}

int cmf_ensemble_set_step(cmf_ensemble *E, int64_t step) {
  if (!E) return fail(CMF_EINVAL, "ensemble is NULL");
  if (step < 0 || step >= kMaxStep)
    return fail(CMF_EINVAL, "step %lld outside [0, 2^56)", (long long)step);
  HIP_TRY(hipStreamSynchronize(E->stream));
  HIP_TRY(hipMemcpy(E->step_dev, &step, sizeof(int64_t), hipMemcpyHostToDevice));
  for (auto &r : E->read_step) r = step;
  return CMF_OK;
}

int cmf_ensemble_stats(cmf_ensemble *E, int32_t index, cmf_moments *out, int64_t cap, int64_t *n_out) {
  int rc = ens_check_index(E, index);
  if (rc != CMF_OK) return rc;
  if (!n_out || (cap > 0 && !out)) return fail(CMF_EINVAL, "NULL argument");
  if (cap < 0) return fail(CMF_EINVAL, "cap < 0");
  *n_out = 0;
  int64_t step = 0;
  rc = cmf_ensemble_get_step(E, &step);
  if (rc != CMF_OK) return rc;
  if (E->flags & CMF_FLAG_NO_STATS) {
    E->read_step[index] = step;
    return CMF_OK;
  }
  int64_t first = E->read_step[index];
  if (step - first > E->cap) first = step - E->cap;
  if (step - first > cap) first = step - cap;
  std::vector<double> ring((size_t)E->cap * kSeriesStride);
  if (step > first)
    HIP_TRY(hipMemcpy(ring.data(), E->series + (size_t)index * E->cap * kSeriesStride,
                      sizeof(double) * ring.size(), hipMemcpyDeviceToHost));
  bool bad = false;
  for (int64_t s = first; s < step; ++s) {
    const double *r = ring.data() + (s % E->cap) * kSeriesStride;
    cmf_moments &m = out[s - first];
    m.step = r[0];
    m.sum_rho = r[1];
    for (int a = 0; a < 3; ++a) {
      m.sum_j[a] = r[2 + a];
      m.sum_u[a] = r[5 + a];
      m.sum_u2[a] = r[8 + a];
    }
    m.nonfinite = r[11];
    if (m.nonfinite != 0.0) bad = true;
  }
  *n_out = step - first;
  E->read_step[index] = step;
  if (bad) return fail(CMF_ENONFINITE, "non-finite density or velocity in a recorded step");
  return CMF_OK;
}

}  // extern "C"
