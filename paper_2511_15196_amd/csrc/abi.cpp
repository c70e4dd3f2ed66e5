// C ABI of libphi4pmc: argument checks, workspace carving, handles and the
// native level loop.  Every compute step runs in the HIP kernels of this
// library; this file only validates, orders and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <algorithm>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"
#include "hmc.hpp"
#include "irmh.hpp"
#include "slice.hpp"

using namespace phi4;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_check(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(PHI4_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return PHI4_OK;
}

#define HIP_TRY(call)                                                                     \
  do {                                                                                    \
    const hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) return fail(PHI4_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;

// Sequential carving of a caller-provided workspace.
struct Carver {
  uintptr_t base;
  size_t off = 0;
  explicit Carver(void* p) : base(reinterpret_cast<uintptr_t>(p)) {}
  template <class T>
  T* take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
    return p;
  }
  size_t bytes() const { return (off + kAlign - 1) / kAlign * kAlign; }
};

double default_eps0(int d, double eps0) { return eps0 > 0 ? eps0 : 2.38 / std::sqrt((double)d); }

// HMC: d^(-1/4), the dimension scaling of leapfrog steps
double smc_eps0(const phi4_smc_config& c) {
  const int d = c.L * c.L;
  if (c.kernel == PHI4_KERNEL_HMC) return c.eps0 > 0 ? c.eps0 : std::pow((double)d, -0.25);
  return default_eps0(d, c.eps0);
}

// Scratch of the three-pass sweep for n particles.
LargeScratch take_large(Carver& cv, int n, int d) {
  if (n <= 0) return LargeScratch{nullptr, nullptr, nullptr, nullptr, nullptr};
  void* base = cv.take<char>(large_scratch_bytes(n, d));
  return cv.base ? large_scratch(base, n, d) : LargeScratch{nullptr, nullptr, nullptr, nullptr, nullptr};
}

// ------------------------------------------------------------------ SMC

struct SmcBufs {
  SmcState* st;
  float* alt_phi;
  float* alt_S;
  float* absM;
  float* obs_S;
  float* obs_absM;
  double* obs_mean;
  int32_t* anc;
  unsigned long long* cdf;
  int32_t* marks;
  double* w;
  float* part;
  double* sigma;
  double* A;
  float* Bt;
  LargeScratch large;
  int32_t* bstatus;
  double* bscr;
  IrmhScratch irmh;   // independence sampler only
  double* hvar;       // HMC only: site variances (d) and their partial sums
  double* hpart;
};

// Blocked-factor fields of FactorArgs from its carved scratch.
void set_blocked(FactorArgs& fa, int32_t* bstatus, double* bscr, int d) {
  if (blocked_attempts(d) == 0) return;   // d <= 64: one-workgroup factor
  fa.bstatus = bstatus;
  fa.attempts = blocked_attempts(d);
  fa.Aspec = bscr;
  fa.Winv = bscr + (size_t)(fa.attempts > 1 ? fa.attempts - 1 : 0) * d * d;
}

size_t smc_carve(const phi4_smc_config& c, void* ws, SmcBufs* b) {
  const int d = c.L * c.L, n = c.N;
  const CovPlan plan = cov_plan(n, d);
  Carver cv(ws);
  SmcBufs t;
  t.st = cv.take<SmcState>(1);
  t.alt_phi = cv.take<float>((size_t)n * d);
  t.alt_S = cv.take<float>(n);
  t.absM = cv.take<float>(n);
  t.obs_S = cv.take<float>(n);
  t.obs_absM = cv.take<float>(n);
  t.obs_mean = cv.take<double>(1);
  t.anc = cv.take<int32_t>(n);
  t.cdf = cv.take<unsigned long long>(n);
  t.marks = cv.take<int32_t>(n);
  t.w = cv.take<double>(n);
  t.part = cv.take<float>(cov_partial_floats(plan));
  t.sigma = cv.take<double>((size_t)d * d);
  t.A = cv.take<double>((size_t)d * d);
  t.Bt = cv.take<float>((size_t)d * d);
  t.large = take_large(cv, n, d);
  t.bstatus = cv.take<int32_t>(kJitterAttempts + 1);
  t.bscr = cv.take<double>(blocked_scratch_doubles(d));
  t.irmh = IrmhScratch{};
  t.hvar = t.hpart = nullptr;
  if (c.kernel == PHI4_KERNEL_HMC) {
    t.hvar = cv.take<double>(d);
    t.hpart = cv.take<double>((size_t)2 * site_var_chunks(n) * d);
  }
  if (c.kernel == PHI4_KERNEL_IRMH) {
    char* base = cv.take<char>(irmh_scratch_bytes(n, d));
    if (cv.base) t.irmh = irmh_scratch(base, n, d);
  }
  if (b) *b = t;
  return cv.bytes();
}

bool smc_valid(const phi4_smc_config* c, std::string* why) {
  if (!c) return *why = "config is NULL", false;
  const long long d = (long long)c->L * c->L;
  if (c->L < 1 || d > PHI4_MAX_SITES) return *why = "need 1 <= L and L*L <= 4096", false;
  if (c->N < 2 || c->N > (1 << 24)) return *why = "need 2 <= N <= 2^24", false;
  if (!(c->ess_frac > 0.0 && c->ess_frac <= 1.0)) return *why = "ess_frac must be in (0, 1]", false;
  if (c->n_steps < 0) return *why = "n_steps must be >= 0", false;
  if (!std::isfinite(c->m2) || !std::isfinite(c->lambda)) return *why = "couplings must be finite", false;
  if (!mutate_supported((int)d, c->precision)) return *why = "unsupported precision", false;
  if (c->kernel != PHI4_KERNEL_RW && c->kernel != PHI4_KERNEL_IRMH &&
      c->kernel != PHI4_KERNEL_HMC)
    return *why = "unknown inner kernel", false;
  if (c->kernel == PHI4_KERNEL_HMC && c->precision != PHI4_FP32)
    return *why = "the HMC kernel runs in float32 only", false;
  if (c->kernel == PHI4_KERNEL_HMC && (c->n_leapfrog < 0 || c->n_leapfrog > 1000))
    return *why = "n_leapfrog must be in [0, 1000]", false;
  if (c->kernel == PHI4_KERNEL_IRMH && c->precision != PHI4_FP32)
    return *why = "the independence sampler runs in float32 only", false;
  if (c->kernel == PHI4_KERNEL_IRMH && d > PHI4_IRMH_MAX_SITES)
    return *why = "the independence sampler needs L*L <= 1024", false;
  return true;
}

struct Handle {
  int kind;  // 0 SMC, 1 NS
  hipStream_t stream;
  float* phi;
  float* S;
  int L, d, n;
  float m2, lam;
  uint32_t seed, run;
  int precision;
  int n_steps;
  // SMC
  phi4_smc_config smc;
  SmcBufs sb;
  int sweep = PHI4_SWEEP_AUTO;
  int cur;          // 0: particles in phi/S, 1: in the workspace copy
  bool anc_pending; // resampling ancestors computed, not yet applied
  CovPlan plan;
  // NS
  phi4_ns_config ns;
  NsState* nst;
  float* absM;
  int32_t* dead;
  int32_t* surv;
  double* scratch;
  float* part;
  double* sigma;
  double* A;
  float* Bt;
  CovPlan nplan;
  LargeScratch nlarge;
  int32_t* nbstatus;
  double* nbscr;
  double* sone;      // slice refill: 1.0 (unit scale of the emitted factor)
  float* szero;      // slice refill: d zeros (base row of the direction product)
  // host mirrors
  void* pinned;      // two state copies
  void* pinned_dev;  // the same memory as the device addresses it
  hipEvent_t ev[2];
  // kernel timing
  bool timing;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> tev;  // event pool
  size_t tused;                                        // pairs recorded
};

// Times one mutation launch with a pair of events: the fused sweep records
// them on its own dispatch packet (attach), any other launch is bracketed by
// two event records on the stream (begin and the destructor).
struct TimedLaunch {
  Handle* h;
  hipEvent_t start = nullptr, stop = nullptr;
  bool attached = false;
  bool launched = true;   // attached pairs count only if the launch happened
  explicit TimedLaunch(Handle* hh) : h(hh) {
    if (!h->timing) return;
    if (h->tused == h->tev.size()) {
      std::pair<hipEvent_t, hipEvent_t> p{nullptr, nullptr};
      if (hipEventCreate(&p.first) != hipSuccess || hipEventCreate(&p.second) != hipSuccess) {
        h->timing = false;
        return;
      }
      h->tev.push_back(p);
    }
    start = h->tev[h->tused].first;
    stop = h->tev[h->tused].second;
  }
  // the fused sweep launches exactly when these hold (launch_mutate)
  void attach(MutateArgs& m) {
    if (!start || m.n <= 0 || m.n_steps < 0 || m.d > kFusedMaxSites || m.passes) return;
    m.ev_start = start;
    m.ev_stop = stop;
    attached = true;
  }
  void begin() {
    if (start && !attached) (void)hipEventRecord(start, h->stream);
  }
  ~TimedLaunch() {
    if (!stop) return;
    if (!attached) {
      (void)hipEventRecord(stop, h->stream);
      ++h->tused;
    } else if (launched) {
      ++h->tused;
    }
  }
};

int copy_state(Handle* h, void* host, size_t bytes, const void* dev) {
  HIP_TRY(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return PHI4_OK;
}

int state_error(int err) {
  if (err == PHI4_ECHOL) return fail(PHI4_ECHOL, "covariance not positive definite after jitter");
  if (err == PHI4_ENONFINITE) return fail(PHI4_ENONFINITE, "non-finite actions or weights");
  return fail(err, "device error");
}

float* cur_phi(Handle* h) { return h->cur ? h->sb.alt_phi : h->phi; }
float* cur_S(Handle* h) { return h->cur ? h->sb.alt_S : h->S; }
float* other_phi(Handle* h) { return h->cur ? h->phi : h->sb.alt_phi; }
float* other_S(Handle* h) { return h->cur ? h->S : h->sb.alt_S; }

// Applies pending resampling ancestors by a gather into the other buffer.
void materialize(Handle* h) {
  if (!h->anc_pending) return;
  launch_gather(cur_phi(h), cur_S(h), h->sb.anc, h->n, h->d, other_phi(h), other_S(h), nullptr,
                h->stream);
  h->cur ^= 1;
  h->anc_pending = false;
}

// Moves the particles back to the caller's phi / S if they sit in the workspace.
int settle(Handle* h) {
  if (h->anc_pending) materialize(h);
  if (!h->cur) return PHI4_OK;
  HIP_TRY(hipMemcpyAsync(h->phi, h->sb.alt_phi, sizeof(float) * (size_t)h->n * h->d,
                         hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(h->S, h->sb.alt_S, sizeof(float) * (size_t)h->n,
                         hipMemcpyDeviceToDevice, h->stream));
  h->cur = 0;
  return PHI4_OK;
}

// Reweighting, resampling ancestors, and the covariance factor of the
// resampled population (read through the ancestors; nothing is copied).
int enqueue_reweight(Handle* h, SmcState* mirror = nullptr) {
  SmcBufs& b = h->sb;
  materialize(h);
  ReweightArgs ra = {};
  ra.mirror = mirror;
  ra.S = cur_S(h);
  ra.n = h->n;
  ra.st = b.st;
  ra.w = b.w;
  ra.seed = h->seed;
  ra.run = h->run;
  ra.do_resample = 1;
  ra.cdf = b.cdf;
  ra.marks = b.marks;
  ra.anc = b.anc;
  launch_reweight(ra, h->stream);
  h->anc_pending = true;
  if (h->smc.kernel == PHI4_KERNEL_HMC) {
    // the diagonal mass needs the site variances only
    launch_site_variance(cur_phi(h), b.anc, h->n, h->d, b.hpart, b.hvar, &b.st->done, h->stream);
    return hip_check("smc_reweight_resample");
  }
  launch_cov_partials(cur_phi(h), b.anc, h->plan, b.part, &b.st->done, h->stream);
  FactorArgs fa = {};
  fa.part = b.part;
  fa.plan = h->plan;
  fa.sigma_out = b.sigma;
  fa.A = b.A;
  fa.Bt = b.Bt;
  fa.ldb = h->d;
  // the independence sampler proposes with L itself
  fa.eps_ptr = h->smc.kernel == PHI4_KERNEL_IRMH ? b.irmh.one : &b.st->eps;
  fa.tau_out = &b.st->tau;
  fa.err_out = &b.st->err;
  fa.done = &b.st->done;
  set_blocked(fa, b.bstatus, b.bscr, h->d);
  launch_factor(fa, h->stream);
  return hip_check("smc_reweight_resample");
}

// One sweep from the current particles (through pending ancestors) into the
// other buffer.
int enqueue_mutate(Handle* h) {
  SmcBufs& b = h->sb;
  MutateArgs m = {};
  m.src = cur_phi(h);
  m.src_rows = h->anc_pending ? b.anc : nullptr;
  m.dst = other_phi(h);
  m.rows = nullptr;
  m.n = h->n;
  m.L = h->L;
  m.d = h->d;
  m.m2 = h->m2;
  m.lam = h->lam;
  m.Bt = b.Bt;
  m.ldb = h->d;
  m.kind = 0;
  m.beta_ptr = &b.st->beta;
  m.seed = h->seed;
  m.run = h->run;
  m.level_ptr = &b.st->level;
  m.step0 = 0;
  m.n_steps = h->n_steps;
  m.zsign = 1.0f;
  m.done_ptr = &b.st->done;
  m.large = b.large;
  m.passes = h->sweep == PHI4_SWEEP_PASSES;
  m.S = other_S(h);
  m.absM = b.absM;
  m.acc_count = &b.st->acc;
  m.prop_count = &b.st->prop;
  int rc = PHI4_OK;
  {
    TimedLaunch tl(h);
    if (h->smc.kernel == PHI4_KERNEL_RW) tl.attach(m);
    tl.begin();
    if (h->smc.kernel == PHI4_KERNEL_IRMH) {
      rc = launch_irmh_sweep(m, b.A, b.irmh, h->stream);
    } else if (h->smc.kernel == PHI4_KERNEL_HMC) {
      HmcArgs ha = {};
      ha.src = m.src;
      ha.src_rows = m.src_rows;
      ha.dst = m.dst;
      ha.n = h->n;
      ha.L = h->L;
      ha.d = h->d;
      ha.m2 = h->m2;
      ha.lam = h->lam;
      ha.beta_ptr = &b.st->beta;
      ha.eps_ptr = &b.st->eps;
      ha.var = b.hvar;
      ha.n_leap = h->smc.n_leapfrog > 0 ? h->smc.n_leapfrog : 20;
      ha.n_steps = h->n_steps;
      ha.seed = h->seed;
      ha.run = h->run;
      ha.level_ptr = &b.st->level;
      ha.done = &b.st->done;
      ha.S = m.S;
      ha.absM = m.absM;
      ha.acc_count = m.acc_count;
      ha.prop_count = m.prop_count;
      launch_hmc_sweep(ha, h->stream);
    } else {
      rc = launch_mutate(m, h->precision, h->stream);
      tl.launched = rc == PHI4_OK;
    }
  }
  if (rc) return fail(rc, "smc_mutate: unsupported shape");
  h->cur ^= 1;
  h->anc_pending = false;
  return hip_check("smc_mutate");
}

Handle* as_handle(void* p, int kind) {
  Handle* h = static_cast<Handle*>(p);
  if (!h || h->kind != kind) return nullptr;
  return h;
}

int alloc_pinned(Handle* h, size_t bytes) {
  HIP_TRY(hipHostMalloc(&h->pinned, 2 * bytes, hipHostMallocDefault));
  HIP_TRY(hipHostGetDevicePointer(&h->pinned_dev, h->pinned, 0));
  HIP_TRY(hipEventCreateWithFlags(&h->ev[0], hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&h->ev[1], hipEventDisableTiming));
  return PHI4_OK;
}

// ------------------------------------------------------------------ NS

size_t ns_carve(const phi4_ns_config& c, void* ws, Handle* h) {
  const int d = c.L * c.L, n = c.n_live, k = c.k_delete;
  const CovPlan plan = cov_plan(n - k, d);
  Carver cv(ws);
  NsState* st = cv.take<NsState>(1);
  float* absM = cv.take<float>(n);
  int32_t* dead = cv.take<int32_t>(k);
  int32_t* surv = cv.take<int32_t>(n - k);
  double* scratch = cv.take<double>(2 * (size_t)k);
  float* part = cv.take<float>(cov_partial_floats(plan));
  double* sigma = cv.take<double>((size_t)d * d);
  double* A = cv.take<double>((size_t)d * d);
  float* Bt = cv.take<float>((size_t)d * d);
  const LargeScratch large = take_large(cv, k, d);
  int32_t* bstatus = cv.take<int32_t>(kJitterAttempts + 1);
  double* bscr = cv.take<double>(blocked_scratch_doubles(d));
  double* one = nullptr;
  float* zero = nullptr;
  if (c.kernel == PHI4_NS_SLICE) {
    one = cv.take<double>(1);
    zero = cv.take<float>(d);
  }
  if (h) {
    h->nlarge = large;
    h->sone = one;
    h->szero = zero;
    h->nbstatus = bstatus;
    h->nbscr = bscr;
    h->nst = st;
    h->absM = absM;
    h->dead = dead;
    h->surv = surv;
    h->scratch = scratch;
    h->part = part;
    h->sigma = sigma;
    h->A = A;
    h->Bt = Bt;
    h->nplan = plan;
  }
  return cv.bytes();
}

bool ns_valid(const phi4_ns_config* c, std::string* why) {
  if (!c) return *why = "config is NULL", false;
  const long long d = (long long)c->L * c->L;
  if (c->L < 1 || d > PHI4_MAX_SITES) return *why = "need 1 <= L and L*L <= 4096", false;
  if (c->n_live < 3 || c->n_live > 8192) return *why = "need 3 <= n_live <= 8192", false;
  if (c->k_delete < 1 || c->k_delete > c->n_live - 2) return *why = "need 1 <= k_delete <= n_live - 2", false;
  if (c->n_steps < 0) return *why = "n_steps must be >= 0", false;
  if (!(c->prior_var > 0.0) || !std::isfinite(c->prior_var)) return *why = "prior_var must be > 0", false;
  if (!(c->term_frac > 0.0 && c->term_frac < 1.0)) return *why = "term_frac must be in (0, 1)", false;
  if (!std::isfinite(c->m2) || !std::isfinite(c->lambda)) return *why = "couplings must be finite", false;
  if (!mutate_supported((int)d, c->precision)) return *why = "unsupported precision", false;
  if (c->kernel != PHI4_NS_RW && c->kernel != PHI4_NS_SLICE) return *why = "unknown refill kernel", false;
  if (c->kernel == PHI4_NS_SLICE && c->precision != PHI4_FP32)
    return *why = "the slice refill runs in float32 only", false;
  return true;
}

NsArgs ns_args(Handle* h) {
  NsArgs a = {};
  a.phi = h->phi;
  a.S = h->S;
  a.absM = h->absM;
  a.n = h->n;
  a.k = h->ns.k_delete;
  a.d = h->d;
  a.st = h->nst;
  a.seed = h->seed;
  a.run = h->run;
  a.dead_rows = h->dead;
  a.surv_rows = h->surv;
  a.scratch = h->scratch;
  a.term_frac = h->ns.term_frac;
  return a;
}

// step-level workspace
struct StepBufs {
  unsigned long long* cdf;
  int32_t* marks;
  int32_t* status;
  double* out;
  float* part;
  double* sigma;
  double* A;
  double* tau;
  LargeScratch large;
  double* bscr;
};

size_t step_carve(int n, int d, void* ws, StepBufs* b) {
  Carver cv(ws);
  StepBufs t;
  t.cdf = cv.take<unsigned long long>(n > 0 ? n : 1);
  t.marks = cv.take<int32_t>(n > 0 ? n : 1);
  t.status = cv.take<int32_t>(kJitterAttempts + 2);
  t.out = cv.take<double>(8);
  const int dd = d > 0 ? d : 1;
  t.part = cv.take<float>(cov_partial_floats(cov_plan(n > 1 ? n : 2, dd)));
  t.sigma = cv.take<double>((size_t)dd * dd);
  t.A = cv.take<double>((size_t)dd * dd);
  t.tau = cv.take<double>(1);
  t.large = take_large(cv, n, dd);
  t.bscr = cv.take<double>(blocked_scratch_doubles(dd));
  if (b) *b = t;
  return cv.bytes();
}

bool ws_ok(void* ws, size_t have, size_t need, std::string* why) {
  if (!ws) return *why = "workspace is NULL", false;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return *why = "workspace must be 256-byte aligned", false;
  if (have < need) return *why = "workspace too small: need " + std::to_string(need) + " bytes", false;
  return true;
}

}  // namespace

namespace {

// Resources of one batched call, released on every exit path.
struct BatchRes {
  std::vector<hipStream_t> branches;
  std::vector<hipEvent_t> events;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const SmcState** dptrs = nullptr;
  BatchStatus* dstat = nullptr;
  BatchStatus* hstat = nullptr;
  std::vector<std::pair<Handle*, hipStream_t>> saved_streams;
  std::vector<std::pair<Handle*, bool>> saved_timing;
  ~BatchRes() {
    for (auto& p : saved_streams) p.first->stream = p.second;
    for (auto& p : saved_timing) p.first->timing = p.second;
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    for (hipStream_t st : branches) (void)hipStreamDestroy(st);
    if (dptrs) (void)hipFree(dptrs);
    if (dstat) (void)hipFree(dstat);
    if (hstat) (void)hipHostFree(hstat);
  }
};

constexpr int kBatchBranches = 4;

}  // namespace

extern "C" {

const char* phi4_last_error(void) { return g_err.c_str(); }

size_t smc_workspace_bytes(const phi4_smc_config* cfg) {
  std::string why;
  if (!smc_valid(cfg, &why)) return 0;
  return smc_carve(*cfg, nullptr, nullptr);
}

int smc_init(const phi4_smc_config* cfg, float* phi, float* S, void* workspace,
             size_t workspace_bytes, void* stream, void** handle) {
  std::string why;
  if (!handle) return fail(PHI4_EINVAL, "handle is NULL");
  *handle = nullptr;
  if (!smc_valid(cfg, &why)) return fail(PHI4_EINVAL, "smc_init: " + why);
  if (!phi || !S) return fail(PHI4_EINVAL, "smc_init: phi / S is NULL");
  if (!ws_ok(workspace, workspace_bytes, smc_carve(*cfg, nullptr, nullptr), &why))
    return fail(PHI4_EINVAL, "smc_init: " + why);
  Handle* h = new (std::nothrow) Handle();
  if (!h) return fail(PHI4_EINVAL, "smc_init: out of host memory");
  h->kind = 0;
  h->stream = static_cast<hipStream_t>(stream);
  h->phi = phi;
  h->S = S;
  h->L = cfg->L;
  h->d = cfg->L * cfg->L;
  h->n = cfg->N;
  h->m2 = (float)cfg->m2;
  h->lam = (float)cfg->lambda;
  h->seed = cfg->seed;
  h->run = cfg->run;
  h->precision = cfg->precision;
  h->n_steps = cfg->n_steps;
  h->smc = *cfg;
  h->cur = 0;
  h->plan = cov_plan(h->n, h->d);
  smc_carve(*cfg, workspace, &h->sb);
  launch_cov_init(h->sb.part, h->plan, h->stream);
  launch_large_init(h->sb.large, h->n, h->stream);
  if (cfg->kernel == PHI4_KERNEL_IRMH) launch_irmh_init(h->sb.irmh, h->stream);
  int rc = alloc_pinned(h, sizeof(SmcState));
  if (rc) {
    delete h;
    return rc;
  }
  launch_smc_state_init(h->sb.st, smc_eps0(*cfg), cfg->acc_target, cfg->ess_frac,
                        h->stream);
  launch_init_fields(phi, S, h->sb.absM, h->n, h->L, h->m2, h->lam, 1.0f, h->seed, h->run,
                     h->stream);
  rc = hip_check("smc_init");
  if (rc) {
    phi4_destroy(h);
    return rc;
  }
  *handle = h;
  return PHI4_OK;
}

int smc_restart(void* handle, uint32_t seed, uint32_t run) {
  Handle* h = as_handle(handle, 0);
  if (!h) return fail(PHI4_EINVAL, "smc_restart: not an SMC handle");
  h->seed = seed;
  h->run = run;
  h->smc.seed = seed;
  h->smc.run = run;
  h->cur = 0;
  h->anc_pending = false;
  launch_smc_state_init(h->sb.st, smc_eps0(h->smc), h->smc.acc_target,
                        h->smc.ess_frac, h->stream);
  launch_init_fields(h->phi, h->S, h->sb.absM, h->n, h->L, h->m2, h->lam, 1.0f, seed, run,
                     h->stream);
  return hip_check("smc_restart");
}

int smc_reweight_resample(void* handle, double* beta_host) {
  Handle* h = as_handle(handle, 0);
  if (!h) return fail(PHI4_EINVAL, "smc_reweight_resample: not an SMC handle");
  int rc = enqueue_reweight(h);
  if (rc) return rc;
  if (!beta_host) return PHI4_OK;
  SmcState* s = static_cast<SmcState*>(h->pinned);
  rc = copy_state(h, s, sizeof(SmcState), h->sb.st);
  if (rc) return rc;
  if (s->err) return state_error(s->err);
  *beta_host = s->beta;
  return s->done ? PHI4_DONE : PHI4_OK;
}

int smc_mutate(void* handle, double* acc_host) {
  Handle* h = as_handle(handle, 0);
  if (!h) return fail(PHI4_EINVAL, "smc_mutate: not an SMC handle");
  int rc = enqueue_mutate(h);
  if (!rc) rc = settle(h);
  if (rc) return rc;
  if (!acc_host) return PHI4_OK;
  SmcState* s = static_cast<SmcState*>(h->pinned);
  rc = copy_state(h, s, sizeof(SmcState), h->sb.st);
  if (rc) return rc;
  if (s->err) return state_error(s->err);
  *acc_host = s->prop ? (double)s->acc / (double)s->prop : NAN;
  return s->done ? PHI4_DONE : PHI4_OK;
}

int smc_run(void* handle, int32_t max_levels, int32_t* levels_host) {
  Handle* h = as_handle(handle, 0);
  if (!h) return fail(PHI4_EINVAL, "smc_run: not an SMC handle");
  if (max_levels < 1) return fail(PHI4_EINVAL, "smc_run: max_levels must be >= 1");
  SmcState* slots = static_cast<SmcState*>(h->pinned);
  // Level t is enqueued before the state after level t-1 is inspected, so
  // the device always has the next level queued; the one level enqueued
  // after the final sweep finds beta = 1 and does nothing.
  int rc = PHI4_OK;
  bool finished = false;
  SmcState* slots_dev = static_cast<SmcState*>(h->pinned_dev);
  for (int t = 0; t < max_levels && !finished; ++t) {
    // the reweight kernel writes the state after its reweight into slot t & 1
    rc = enqueue_reweight(h, &slots_dev[t & 1]);
    if (!rc) rc = enqueue_mutate(h);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(h->ev[t & 1], h->stream));
    if (t >= 1) {
      HIP_TRY(hipEventSynchronize(h->ev[(t - 1) & 1]));
      const SmcState& s = slots[(t - 1) & 1];
      if (s.err) return state_error(s.err);
      if (s.beta >= 1.0) finished = true;
    }
  }
  rc = settle(h);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(h->stream));
  // the level enqueued after the final sweep did no work: drop its timing
  if (finished && h->timing && h->tused > 0) --h->tused;
  SmcState s;
  rc = copy_state(h, &slots[0], sizeof(SmcState), h->sb.st);
  if (rc) return rc;
  s = slots[0];
  if (s.err) return state_error(s.err);
  if (levels_host) *levels_host = s.level;
  return s.beta >= 1.0 ? PHI4_DONE : PHI4_OK;
}

// ------------------------------------------------------------------ batch


int smc_batch_run(void* const* handles, int32_t n_runs, int32_t max_levels, int32_t* levels_host,
                  void* stream) {
  if (!handles || n_runs < 1) return fail(PHI4_EINVAL, "smc_batch_run: need n_runs >= 1 handles");
  if (max_levels < 1) return fail(PHI4_EINVAL, "smc_batch_run: max_levels must be >= 1");
  std::vector<Handle*> hs((size_t)n_runs);
  for (int r = 0; r < n_runs; ++r) {
    hs[r] = as_handle(handles[r], 0);
    if (!hs[r]) return fail(PHI4_EINVAL, "smc_batch_run: handle " + std::to_string(r) +
                                             " is not an SMC handle");
    for (int q = 0; q < r; ++q)
      if (hs[q] == hs[r]) return fail(PHI4_EINVAL, "smc_batch_run: a handle appears twice");
  }
  hipStream_t caller = static_cast<hipStream_t>(stream);
  BatchRes res;
  // Level 1 of every run outside the graph, on the run's own stream: it
  // also settles pending ancestors and times the proposal-product tiles of
  // each shape (nothing can be timed during a capture).
  for (Handle* h : hs) {
    int rc = enqueue_reweight(h);
    if (!rc) rc = enqueue_mutate(h);
    if (rc) return rc;
  }
  for (Handle* h : hs) HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipStreamSynchronize(caller));
  // capture and replay on a private stream (the caller's may be the legacy
  // null stream, which cannot be captured)
  hipStream_t origin = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&origin, hipStreamNonBlocking));
  res.branches.push_back(origin);

  HIP_TRY(hipMalloc(&res.dptrs, sizeof(SmcState*) * (size_t)n_runs));
  HIP_TRY(hipMalloc(&res.dstat, sizeof(BatchStatus) * (size_t)n_runs));
  HIP_TRY(hipHostMalloc(&res.hstat, sizeof(BatchStatus) * (size_t)n_runs, hipHostMallocDefault));
  {
    std::vector<const SmcState*> ptrs((size_t)n_runs);
    for (int r = 0; r < n_runs; ++r) ptrs[r] = hs[r]->sb.st;
    HIP_TRY(hipMemcpy(res.dptrs, ptrs.data(), sizeof(SmcState*) * (size_t)n_runs,
                      hipMemcpyHostToDevice));
  }
  const int nb = std::min(kBatchBranches, n_runs);
  std::vector<hipStream_t> br;
  for (int k = 0; k < nb; ++k) {
    hipStream_t st = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    res.branches.push_back(st);
    br.push_back(st);
  }
  for (int k = 0; k < nb + 1; ++k) {
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    res.events.push_back(e);
  }
  // branches balanced by the work of one sweep (largest first)
  std::vector<int> order((size_t)n_runs);
  for (int r = 0; r < n_runs; ++r) order[r] = r;
  auto cost = [&](int r) {
    const double d = hs[r]->d;
    return (double)hs[r]->n * d * (d + 16.0) * std::max(hs[r]->n_steps, 1);
  };
  std::sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  std::vector<double> load((size_t)nb, 0.0);
  std::vector<int> branch_of((size_t)n_runs);
  for (int r : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    branch_of[r] = k;
    load[k] += cost(r);
  }
  // Two levels of every run per replay: each level flips the particle
  // buffers, so the captured pointers are valid for every replay; a run
  // that has finished makes its kernels return at once.
  for (Handle* h : hs) {
    res.saved_streams.push_back({h, h->stream});
    res.saved_timing.push_back({h, h->timing});
    h->timing = false;
  }
  // host-side buffer parity of every run; two captured levels leave it as
  // it was, and a capture that fails part-way must not change it either
  std::vector<std::pair<int, bool>> parity;
  for (Handle* h : hs) parity.push_back({h->cur, h->anc_pending});
  HIP_TRY(hipStreamBeginCapture(origin, hipStreamCaptureModeRelaxed));
  int rc = PHI4_OK;
  {
    bool ok = hipEventRecord(res.events[nb], origin) == hipSuccess;
    for (int k = 0; k < nb && ok; ++k)
      ok = hipStreamWaitEvent(br[k], res.events[nb], 0) == hipSuccess;
    for (int r = 0; r < n_runs && ok && !rc; ++r) {
      Handle* h = hs[r];
      h->stream = br[branch_of[r]];
      for (int lv = 0; lv < 2 && !rc; ++lv) {
        rc = enqueue_reweight(h);
        if (!rc) rc = enqueue_mutate(h);
      }
    }
    for (int k = 0; k < nb && ok; ++k) {
      ok = hipEventRecord(res.events[k], br[k]) == hipSuccess &&
           hipStreamWaitEvent(origin, res.events[k], 0) == hipSuccess;
    }
    if (ok) {
      launch_batch_status(res.dptrs, n_runs, res.dstat, origin);
      ok = hipMemcpyAsync(res.hstat, res.dstat, sizeof(BatchStatus) * (size_t)n_runs,
                          hipMemcpyDeviceToHost, origin) == hipSuccess;
    }
    const hipError_t ec = hipStreamEndCapture(origin, &res.graph);
    if (!rc && (!ok || ec != hipSuccess))
      rc = fail(PHI4_EHIP, "smc_batch_run: stream capture failed");
  }
  for (auto& p : res.saved_streams) p.first->stream = p.second;
  res.saved_streams.clear();
  for (int r = 0; r < n_runs; ++r) {
    hs[r]->cur = parity[r].first;
    hs[r]->anc_pending = parity[r].second;
  }
  if (rc) return rc;
  HIP_TRY(hipGraphInstantiate(&res.exec, res.graph, nullptr, nullptr, 0));
  bool all_done = false;
  int err = 0;
  for (int lv = 1; lv < max_levels && !all_done && !err; lv += 2) {
    HIP_TRY(hipGraphLaunch(res.exec, origin));
    HIP_TRY(hipStreamSynchronize(origin));
    all_done = true;
    for (int r = 0; r < n_runs; ++r) {
      if (res.hstat[r].err) err = res.hstat[r].err;
      if (res.hstat[r].beta < 1.0) all_done = false;
    }
  }
  if (max_levels == 1) {
    launch_batch_status(res.dptrs, n_runs, res.dstat, origin);
    HIP_TRY(hipMemcpyAsync(res.hstat, res.dstat, sizeof(BatchStatus) * (size_t)n_runs,
                           hipMemcpyDeviceToHost, origin));
    HIP_TRY(hipStreamSynchronize(origin));
    all_done = true;
    for (int r = 0; r < n_runs; ++r) {
      if (res.hstat[r].err) err = res.hstat[r].err;
      if (res.hstat[r].beta < 1.0) all_done = false;
    }
  }
  for (Handle* h : hs) {
    rc = settle(h);
    if (rc) return rc;
  }
  for (Handle* h : hs) HIP_TRY(hipStreamSynchronize(h->stream));
  if (levels_host)
    for (int r = 0; r < n_runs; ++r) levels_host[r] = res.hstat[r].level;
  if (err) return state_error(err);
  return all_done ? PHI4_DONE : PHI4_OK;
}

size_t ns_workspace_bytes(const phi4_ns_config* cfg) {
  std::string why;
  if (!ns_valid(cfg, &why)) return 0;
  return ns_carve(*cfg, nullptr, nullptr);
}

int ns_init(const phi4_ns_config* cfg, float* phi, float* S, void* workspace,
            size_t workspace_bytes, void* stream, void** handle) {
  std::string why;
  if (!handle) return fail(PHI4_EINVAL, "handle is NULL");
  *handle = nullptr;
  if (!ns_valid(cfg, &why)) return fail(PHI4_EINVAL, "ns_init: " + why);
  if (!phi || !S) return fail(PHI4_EINVAL, "ns_init: phi / S is NULL");
  if (!ws_ok(workspace, workspace_bytes, ns_carve(*cfg, nullptr, nullptr), &why))
    return fail(PHI4_EINVAL, "ns_init: " + why);
  Handle* h = new (std::nothrow) Handle();
  if (!h) return fail(PHI4_EINVAL, "ns_init: out of host memory");
  h->kind = 1;
  h->stream = static_cast<hipStream_t>(stream);
  h->phi = phi;
  h->S = S;
  h->L = cfg->L;
  h->d = cfg->L * cfg->L;
  h->n = cfg->n_live;
  h->m2 = (float)cfg->m2;
  h->lam = (float)cfg->lambda;
  h->seed = cfg->seed;
  h->run = cfg->run;
  h->precision = cfg->precision;
  h->n_steps = cfg->n_steps;
  h->ns = *cfg;
  ns_carve(*cfg, workspace, h);
  launch_cov_init(h->part, h->nplan, h->stream);
  launch_large_init(h->nlarge, cfg->k_delete, h->stream);
  if (cfg->kernel == PHI4_NS_SLICE) launch_slice_init(h->szero, h->d, h->sone, h->stream);
  int rc = alloc_pinned(h, sizeof(NsState));
  if (rc) {
    delete h;
    return rc;
  }
  launch_ns_state_init(h->nst, default_eps0(h->d, cfg->eps0), cfg->acc_target, h->stream);
  launch_init_fields(phi, S, h->absM, h->n, h->L, h->m2, h->lam, (float)std::sqrt(cfg->prior_var),
                     h->seed, h->run, h->stream);
  rc = hip_check("ns_init");
  if (rc) {
    phi4_destroy(h);
    return rc;
  }
  *handle = h;
  return PHI4_OK;
}

int ns_step(void* handle, int32_t* done_host) {
  Handle* h = as_handle(handle, 1);
  if (!h) return fail(PHI4_EINVAL, "ns_step: not a nested-sampling handle");
  const NsArgs a = ns_args(h);
  launch_ns_select(a, h->stream);
  launch_ns_seed_copy(a, h->stream);
  launch_cov_partials(h->phi, h->surv, h->nplan, h->part, &h->nst->done, h->stream);
  FactorArgs fa = {};
  fa.part = h->part;
  fa.plan = h->nplan;
  fa.sigma_out = h->sigma;
  fa.A = h->A;
  fa.Bt = h->Bt;
  fa.ldb = h->d;
  // the slice refill draws its directions from L itself
  fa.eps_ptr = h->ns.kernel == PHI4_NS_SLICE ? h->sone : &h->nst->eps;
  fa.tau_out = &h->nst->tau;
  fa.err_out = &h->nst->err;
  fa.done = &h->nst->done;
  set_blocked(fa, h->nbstatus, h->nbscr, h->d);
  launch_factor(fa, h->stream);
  MutateArgs m = {};
  m.src = h->phi;
  m.dst = h->phi;
  m.rows = h->dead;
  m.n = h->ns.k_delete;
  m.L = h->L;
  m.d = h->d;
  m.m2 = h->m2;
  m.lam = h->lam;
  m.Bt = h->Bt;
  m.ldb = h->d;
  m.kind = 1;
  m.sstar_ptr = &h->nst->s_star;
  m.inv_prior_var = (float)(1.0 / h->ns.prior_var);
  m.seed = h->seed;
  m.run = h->run;
  m.level_ptr = &h->nst->iter;
  m.step0 = 0;
  m.n_steps = h->n_steps;
  m.zsign = 1.0f;
  m.done_ptr = &h->nst->done;
  m.large = h->nlarge;
  m.passes = h->sweep == PHI4_SWEEP_PASSES;
  m.S = h->S;
  m.absM = h->absM;
  m.acc_count = &h->nst->acc;
  m.prop_count = &h->nst->prop;
  int rc;
  {
    TimedLaunch tl(h);
    if (h->ns.kernel != PHI4_NS_SLICE) tl.attach(m);
    tl.begin();
    rc = h->ns.kernel == PHI4_NS_SLICE ? launch_slice_sweep(m, h->szero, h->stream)
                                       : launch_mutate(m, h->precision, h->stream);
    tl.launched = rc == PHI4_OK;
  }
  if (rc) return fail(rc, "ns_step: unsupported shape");
  rc = hip_check("ns_step");
  if (rc) return rc;
  if (!done_host) return PHI4_OK;
  NsState* s = static_cast<NsState*>(h->pinned);
  rc = copy_state(h, s, sizeof(NsState), h->nst);
  if (rc) return rc;
  if (s->err) return state_error(s->err);
  *done_host = s->done;
  return s->done ? PHI4_DONE : PHI4_OK;
}

int logz(void* handle, double* logz_host, double* stderr_host) {
  Handle* h = static_cast<Handle*>(handle);
  if (!h || !logz_host) return fail(PHI4_EINVAL, "logz: NULL argument");
  if (h->kind == 0) {
    SmcState* s = static_cast<SmcState*>(h->pinned);
    const int rc = copy_state(h, s, sizeof(SmcState), h->sb.st);
    if (rc) return rc;
    if (s->err) return state_error(s->err);
    *logz_host = s->logz;
    if (stderr_host) *stderr_host = NAN;
    return PHI4_OK;
  }
  NsState* s = static_cast<NsState*>(h->pinned);
  const int rc = copy_state(h, s, sizeof(NsState), h->nst);
  if (rc) return rc;
  if (s->err) return state_error(s->err);
  *logz_host = s->logZ;
  if (stderr_host) *stderr_host = std::sqrt(std::fmax(s->H, 0.0) / h->n);
  return PHI4_OK;
}

int phi4_observables(void* handle, double* out) {
  Handle* h = static_cast<Handle*>(handle);
  if (!h || !out) return fail(PHI4_EINVAL, "phi4_observables: NULL argument");
  if (h->kind == 0) {
    SmcBufs& b = h->sb;
    materialize(h);
    launch_action(cur_phi(h), h->n, h->L, h->m2, h->lam, b.obs_S, b.obs_absM, h->stream);
    launch_mean_abs(b.obs_absM, h->n, &b.st->mean_abs_m, nullptr, h->stream);
    int rc = hip_check("phi4_observables");
    if (rc) return rc;
    SmcState* s = static_cast<SmcState*>(h->pinned);
    rc = copy_state(h, s, sizeof(SmcState), b.st);
    if (rc) return rc;
    out[0] = s->mean_abs_m;
    out[1] = s->beta;
    out[2] = s->last_acc;
    out[3] = s->eps;
    out[4] = s->level;
    out[5] = s->last_dbeta;
    out[6] = s->last_ess;
    out[7] = s->tau;
    out[8] = s->solve_iters;
    out[9] = s->done;
    return PHI4_OK;
  }
  NsState* s = static_cast<NsState*>(h->pinned);
  const int rc = copy_state(h, s, sizeof(NsState), h->nst);
  if (rc) return rc;
  out[0] = std::exp(s->logmz - s->logZ);
  out[1] = s->logX;
  out[2] = s->last_acc;
  out[3] = s->eps;
  out[4] = s->iter;
  out[5] = s->s_star;
  out[6] = s->H;
  out[7] = s->tau;
  out[8] = 0.0;
  out[9] = s->done;
  return PHI4_OK;
}

int phi4_tile_choice(int32_t n, int32_t d, int32_t precision, int32_t* rows_host,
                     int32_t* cols_host, int32_t* threads_host) {
  if (!rows_host || !cols_host || !threads_host)
    return fail(PHI4_EINVAL, "phi4_tile_choice: NULL output");
  int cols = 0, threads = 0;
  *rows_host = large_tile_choice(n, d, precision, &cols, &threads);
  *cols_host = cols;
  *threads_host = threads;
  return PHI4_OK;
}

int phi4_set_tile(int32_t n, int32_t d, int32_t precision, int32_t rows, int32_t cols,
                  int32_t threads) {
  if (n < 1 || d < 1 || d > PHI4_MAX_SITES || !mutate_supported(d, precision))
    return fail(PHI4_EINVAL, "phi4_set_tile: bad shape or precision");
  if (!large_set_tile(n, d, precision, rows, cols, threads))
    return fail(PHI4_EINVAL, "phi4_set_tile: tile must be 32x64, 64x64, 128x64 or 128x128 "
                             "with 256 threads, or 128x128 with 512");
  return PHI4_OK;
}

int phi4_set_sweep(void* handle, int32_t form) {
  Handle* h = static_cast<Handle*>(handle);
  if (!h) return fail(PHI4_EINVAL, "phi4_set_sweep: NULL handle");
  if (form < PHI4_SWEEP_AUTO || form > PHI4_SWEEP_PASSES ||
      (form == PHI4_SWEEP_FUSED && h->d > kFusedMaxSites))
    return fail(PHI4_EINVAL, "phi4_set_sweep: unknown form, or fused beyond d = 256");
  h->sweep = form;
  return PHI4_OK;
}

int phi4_set_timing(void* handle, int32_t enabled) {
  Handle* h = static_cast<Handle*>(handle);
  if (!h) return fail(PHI4_EINVAL, "phi4_set_timing: NULL handle");
  h->timing = enabled != 0;
  return PHI4_OK;
}

int phi4_kernel_time(void* handle, double* ms_host, int32_t* launches_host) {
  Handle* h = static_cast<Handle*>(handle);
  if (!h || !ms_host) return fail(PHI4_EINVAL, "phi4_kernel_time: NULL argument");
  HIP_TRY(hipStreamSynchronize(h->stream));
  double total = 0.0;
  for (size_t i = 0; i < h->tused; ++i) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, h->tev[i].first, h->tev[i].second));
    total += ms;
  }
  *ms_host = total;
  if (launches_host) *launches_host = (int32_t)h->tused;
  h->tused = 0;
  return PHI4_OK;
}

int phi4_destroy(void* handle) {
  Handle* h = static_cast<Handle*>(handle);
  if (!h) return PHI4_OK;
  for (auto& p : h->tev) {
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  if (h->pinned) (void)hipHostFree(h->pinned);
  if (h->ev[0]) (void)hipEventDestroy(h->ev[0]);
  if (h->ev[1]) (void)hipEventDestroy(h->ev[1]);
  delete h;
  return PHI4_OK;
}

// ------------------------------------------------------------ step level

size_t phi4_step_workspace_bytes(int32_t N, int32_t d) {
  if (N < 0 || d < 0 || d > PHI4_MAX_SITES) return 0;
  return step_carve(N, d, nullptr, nullptr);
}

int phi4_normals(uint32_t seed, uint32_t run, int32_t level, int32_t step, int32_t purpose,
                 const int32_t* rows, int32_t n, int32_t d, float* out, void* stream) {
  if (n < 0 || d < 1 || (n > 0 && !out)) return fail(PHI4_EINVAL, "phi4_normals: bad shape");
  if (level < 0 || level >= (1 << 24) || purpose < 0 || purpose > 255)
    return fail(PHI4_EINVAL, "phi4_normals: level / purpose out of range");
  launch_normals(seed, run, level, step, purpose, rows, n, d, out, static_cast<hipStream_t>(stream));
  return hip_check("phi4_normals");
}

int phi4_action(const float* phi, int32_t N, int32_t L, double m2, double lambda, float* S,
                float* absM, void* stream) {
  if (N < 0 || L < 1 || (long long)L * L > PHI4_MAX_SITES || (N > 0 && (!phi || !S)))
    return fail(PHI4_EINVAL, "phi4_action: bad shape");
  launch_action(phi, N, L, (float)m2, (float)lambda, S, absM, static_cast<hipStream_t>(stream));
  return hip_check("phi4_action");
}

int phi4_resample_systematic(const double* w, int32_t N, uint32_t U, int32_t* ancestors,
                             void* workspace, size_t workspace_bytes, void* stream) {
  std::string why;
  if (N < 0 || (N > 0 && (!w || !ancestors))) return fail(PHI4_EINVAL, "phi4_resample_systematic: bad shape");
  if (N == 0) return PHI4_OK;
  if (!ws_ok(workspace, workspace_bytes, step_carve(N, 1, nullptr, nullptr), &why))
    return fail(PHI4_EINVAL, "phi4_resample_systematic: " + why);
  StepBufs b;
  step_carve(N, 1, workspace, &b);
  hipStream_t s = static_cast<hipStream_t>(stream);
  launch_resample_weights(w, N, U, b.cdf, b.marks, ancestors, b.status, s);
  int rc = hip_check("phi4_resample_systematic");
  if (rc) return rc;
  int32_t status = 0;
  HIP_TRY(hipMemcpyAsync(&status, b.status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (status) return fail(status, "phi4_resample_systematic: weights must be finite, >= 0, max > 0");
  return PHI4_OK;
}

int phi4_reweight(const float* S, int32_t N, double beta, double ess_frac, double* w,
                  double* out_host, void* workspace, size_t workspace_bytes, void* stream) {
  std::string why;
  if (N < 1 || !S || !out_host) return fail(PHI4_EINVAL, "phi4_reweight: bad arguments");
  if (!(beta >= 0.0 && beta < 1.0) || !(ess_frac > 0.0 && ess_frac <= 1.0))
    return fail(PHI4_EINVAL, "phi4_reweight: need 0 <= beta < 1 and 0 < ess_frac <= 1");
  if (!ws_ok(workspace, workspace_bytes, step_carve(N, 1, nullptr, nullptr), &why))
    return fail(PHI4_EINVAL, "phi4_reweight: " + why);
  StepBufs b;
  step_carve(N, 1, workspace, &b);
  hipStream_t s = static_cast<hipStream_t>(stream);
  ReweightArgs ra = {};
  ra.S = S;
  ra.n = N;
  ra.st = nullptr;
  ra.beta_in = beta;
  ra.ess_frac_in = ess_frac;
  ra.out = b.out;
  ra.w = w;
  ra.do_resample = 0;
  launch_reweight(ra, s);
  int rc = hip_check("phi4_reweight");
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(out_host, b.out, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (!std::isfinite(out_host[0])) return fail(PHI4_ENONFINITE, "phi4_reweight: non-finite actions or stalled solve");
  return PHI4_OK;
}

int phi4_slice_move(float* phi, const int32_t* rows, const float* dirs, int32_t n, int32_t L,
                    double m2, double lambda, double s_star, double prior_var, uint32_t seed,
                    uint32_t run, int32_t level, int32_t step, float* S, float* absM,
                    void* stream) {
  const long long d = (long long)L * L;
  if (n < 0 || L < 1 || d > PHI4_MAX_SITES || !phi || !dirs || !S || !(prior_var > 0.0))
    return fail(PHI4_EINVAL, "phi4_slice_move: need phi, dirs, S, 1 <= L*L <= 4096, prior_var > 0");
  SliceArgs sa = {};
  sa.phi = phi;
  sa.rows = rows;
  sa.dirs = dirs;
  sa.n = n;
  sa.L = L;
  sa.d = (int)d;
  sa.m2 = (float)m2;
  sa.lam = (float)lambda;
  sa.s_star = (float)s_star;
  sa.inv_prior_var = (float)(1.0 / prior_var);
  sa.seed = seed;
  sa.run = run;
  sa.level = level;
  sa.step = (uint32_t)step;
  sa.S = S;
  sa.absM = absM;
  launch_slice_moves(sa, static_cast<hipStream_t>(stream));
  return hip_check("phi4_slice_move");
}

size_t phi4_whiten_workspace_bytes(int32_t N, int32_t d) {
  if (N < 1 || d < 1 || d > PHI4_IRMH_MAX_SITES) return 0;
  return irmh_scratch_bytes(N, d);
}

int phi4_whiten(const float* phi, const int32_t* rows, int32_t N, int32_t d, const double* L,
                float* r, float* mu, void* workspace, size_t workspace_bytes, void* stream) {
  std::string why;
  if (N < 1 || d < 1 || d > PHI4_IRMH_MAX_SITES || !phi || !L || !r)
    return fail(PHI4_EINVAL, "phi4_whiten: need N >= 1, 1 <= d <= 1024 and phi, L, r");
  if (!ws_ok(workspace, workspace_bytes, irmh_scratch_bytes(N, d), &why))
    return fail(PHI4_EINVAL, "phi4_whiten: " + why);
  IrmhScratch q = irmh_scratch(workspace, N, d);
  q.r = r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  launch_irmh_mean(phi, rows, N, d, q, nullptr, s);
  launch_irmh_inverse(L, d, q, nullptr, s);
  launch_irmh_whiten(phi, rows, N, d, q, nullptr, s);
  if (mu) HIP_TRY(hipMemcpyAsync(mu, q.mu, sizeof(float) * d, hipMemcpyDeviceToDevice, s));
  return hip_check("phi4_whiten");
}

int phi4_covariance(const float* phi, const int32_t* rows, int32_t N, int32_t d, double* sigma,
                    void* workspace, size_t workspace_bytes, void* stream) {
  std::string why;
  if (N < 2 || d < 1 || d > PHI4_MAX_SITES || !phi || !sigma)
    return fail(PHI4_EINVAL, "phi4_covariance: need N >= 2, 1 <= d <= 4096");
  if (!ws_ok(workspace, workspace_bytes, step_carve(N, d, nullptr, nullptr), &why))
    return fail(PHI4_EINVAL, "phi4_covariance: " + why);
  StepBufs b;
  step_carve(N, d, workspace, &b);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const CovPlan plan = cov_plan(N, d);
  launch_cov_init(b.part, plan, s);
  launch_cov_partials(phi, rows, plan, b.part, nullptr, s);
  FactorArgs fa = {};
  fa.part = b.part;
  fa.plan = plan;
  fa.sigma_out = sigma;
  fa.A = b.A;
  fa.cov_only = 1;
  launch_factor(fa, s);
  return hip_check("phi4_covariance");
}

int phi4_cholesky(const double* sigma, int32_t d, double* L, double* tau_host, void* workspace,
                  size_t workspace_bytes, void* stream) {
  std::string why;
  if (d < 1 || d > PHI4_MAX_SITES || !sigma || !L) return fail(PHI4_EINVAL, "phi4_cholesky: bad shape");
  if (!ws_ok(workspace, workspace_bytes, step_carve(2, d, nullptr, nullptr), &why))
    return fail(PHI4_EINVAL, "phi4_cholesky: " + why);
  StepBufs b;
  step_carve(2, d, workspace, &b);
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemsetAsync(b.status, 0, sizeof(int32_t), s));
  FactorArgs fa = {};
  fa.plan = cov_plan(2, d);
  fa.sigma_in = sigma;
  fa.sigma_out = b.sigma;
  fa.A = L;
  fa.tau_out = b.tau;
  fa.err_out = b.status;
  set_blocked(fa, b.status + 1, b.bscr, d);
  launch_factor(fa, s);
  int rc = hip_check("phi4_cholesky");
  if (rc) return rc;
  int32_t status = 0;
  double tau = 0;
  HIP_TRY(hipMemcpyAsync(&status, b.status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&tau, b.tau, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (status) return fail(status, "phi4_cholesky: not positive definite after jitter");
  if (tau_host) *tau_host = tau;
  return PHI4_OK;
}

int phi4_mutate(const float* src, float* dst, const int32_t* rows, int32_t n, int32_t L, double m2,
                double lambda, const float* Bt, int32_t kind, double beta, double s_star,
                double prior_var, uint32_t seed, uint32_t run, int32_t level, int32_t step0,
                int32_t n_steps, float zsign, int32_t precision, float* S, float* absM,
                unsigned long long* acc_count, uint8_t* acc_flags, float* prop, void* workspace,
                size_t workspace_bytes, void* stream) {
  const long long d = (long long)L * L;
  if (n < 0 || L < 1 || d > PHI4_MAX_SITES || n_steps < 0 || (kind != 0 && kind != 1))
    return fail(PHI4_EINVAL, "phi4_mutate: bad shape or kind");
  if (n > 0 && (!src || !dst || !Bt || !S)) return fail(PHI4_EINVAL, "phi4_mutate: NULL buffer");
  if (kind == 1 && !(prior_var > 0.0)) return fail(PHI4_EINVAL, "phi4_mutate: prior_var must be > 0");
  if (level < 0 || level >= (1 << 24)) return fail(PHI4_EINVAL, "phi4_mutate: level out of range");
  if (!mutate_supported((int)d, precision)) return fail(PHI4_EINVAL, "phi4_mutate: unsupported precision");
  MutateArgs m = {};
  m.src = src;
  m.dst = dst;
  m.rows = rows;
  m.n = n;
  m.L = L;
  m.d = (int)d;
  m.m2 = (float)m2;
  m.lam = (float)lambda;
  m.Bt = Bt;
  m.ldb = (int)d;
  m.kind = kind;
  m.beta = (float)beta;
  m.s_star = (float)s_star;
  m.inv_prior_var = kind == 1 ? (float)(1.0 / prior_var) : 0.f;
  m.seed = seed;
  m.run = run;
  m.level = level;
  m.step0 = step0;
  m.n_steps = n_steps;
  m.zsign = zsign;
  m.S = S;
  m.absM = absM;
  m.acc_count = acc_count;
  m.acc_flags = acc_flags;
  m.prop = prop;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (d > kFusedMaxSites && n > 0) {
    std::string why;
    if (!ws_ok(workspace, workspace_bytes, step_carve(n, (int)d, nullptr, nullptr), &why))
      return fail(PHI4_EINVAL, "phi4_mutate: " + why);
    StepBufs b;
    step_carve(n, (int)d, workspace, &b);
    m.large = b.large;
    launch_large_init(b.large, n, s);
  }
  const int rc = launch_mutate(m, precision, s);
  if (rc) return fail(rc, "phi4_mutate: unsupported shape");
  return hip_check("phi4_mutate");
}

}  // extern "C"
