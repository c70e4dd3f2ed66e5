// Reweighting between tempering levels (float64, one workgroup per run):
// ESS-adaptive increment of beta, log-sum-exp update of log Z and
// systematic resampling on an integer CDF.
//
// The tempering increment solves ESS(dbeta) = ess_frac * N with
// ESS = (sum w)^2 / sum w^2, w_i = exp(-dbeta (S_i - S_min)), by a
// bracketed float64 Newton iteration on g = log ESS - log target, started
// from a float32 Newton pre-solve; the returned increment is the lower end of
// a bracket of relative width <= 1e-13, so ESS(dbeta) >= target always holds
// (the adaptive SMC rule of App. A with the target ESS of the configuration).
//
// Systematic resampling (positions (i + U/2^32) / N of the normalised CDF)
// is evaluated on integer weights q_i = floor(2^k w_i / max w),
// k = 62 - 2 ceil(log2 N), so the ancestors do not depend on any
// floating-point summation order.  Ancestor j is taken by the particles
// i in [count(C_{j-1}), count(C_j)) where count(C) = #{i : T_i < C} =
// min(N, ceil((C N - off) / Q)) and T_i = floor((i Q + off) / N) with
// off = U (Q >> 32) + floor(U (Q mod 2^32) / 2^32); the ranges are
// scattered as marks and expanded by a prefix maximum.
#include "common.hpp"

namespace phi4 {

namespace {

constexpr int kRT = 512;                 // threads of the single-workgroup kernels
constexpr int kNW = kRT / 64;            // waves
constexpr int kSeg = 32;                 // particles per thread on the register path
constexpr int kRegN = kRT * kSeg;        // largest N on the register path (16384)

struct Sums {
  double a, b, da, db;  // sum e, sum e^2, d/dx sum e, d/dx sum e^2
};

// ---------------------------------------------------------------- scans

__device__ unsigned long long block_excl_scan_u64(unsigned long long v, unsigned long long* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  unsigned long long x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  unsigned long long off = 0;
#pragma unroll
  for (int w = 0; w < kNW; ++w)
    if (w < wid) off += sh[w];
  return off + x - v;
}

__device__ int block_excl_scan_max(int v, int* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x = max(x, y);
  }
  const int ex = __shfl_up(x, 1, 64);
  __syncthreads();
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  int off = 0;
#pragma unroll
  for (int w = 0; w < kNW; ++w)
    if (w < wid) off = max(off, sh[w]);
  return lane == 0 ? off : max(off, ex);
}

// #{i : T_i < C} = min(n, ceil((C n - off) / Q)) in exact integers: a
// float64 estimate of the quotient (relative error ~1e-16, so off by at most
// one for quotients below 2^52) corrected with exact products; every product
// stays below 2^63 because C <= Q <= n 2^k and n^2 2^k <= 2^62.
__device__ __forceinline__ long long count_below(unsigned long long C, unsigned long long Q,
                                                 unsigned long long off, int n) {
  const unsigned long long cn = C * (unsigned long long)n;
  if (cn <= off) return 0;
  const unsigned long long num = cn - off;
  unsigned long long c = (unsigned long long)ceil((double)num / (double)Q);
  if (c > (unsigned long long)n + 1) c = (unsigned long long)n + 1;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    if (c * Q < num) ++c;                       // too small
    else if (c > 0 && (c - 1) * Q >= num) --c;  // too large
  }
  return c < (unsigned long long)n ? (long long)c : (long long)n;
}

__device__ __forceinline__ int resample_bits(int n) {
  return n > 1 ? 62 - 2 * (32 - __clz((unsigned)(n - 1))) : 62;
}

// Systematic resampling of a register-resident segment: this thread holds
// the weights of particles [i0, i0 + cnt) (contiguous segments in thread
// order); wmax is the largest weight (> 0, all weights finite and >= 0).
// marks: LDS, n ints.  Writes anc.
__device__ void resample_seg(const double (&w)[kSeg], int cnt, int i0, int n, double wmax,
                             uint32_t U, int* marks, int32_t* __restrict__ anc,
                             unsigned long long* shu, int* shi) {
  __shared__ unsigned long long qsh;
  const int kb = resample_bits(n);
  unsigned long long c[kSeg];
  unsigned long long loc = 0;
#pragma unroll
  for (int k = 0; k < kSeg; ++k) {
    if (k < cnt) loc += (unsigned long long)floor(ldexp(w[k] / wmax, kb));
    c[k] = loc;
  }
  const unsigned long long ex = block_excl_scan_u64(loc, shu);
  for (int i = threadIdx.x; i < n; i += kRT) marks[i] = 0;
  if (cnt > 0 && i0 + cnt == n) qsh = ex + c[cnt - 1];   // Q = C_{n-1}
  __syncthreads();
  const unsigned long long Q = qsh;
  const unsigned long long uu = (unsigned long long)U;
  const unsigned long long off = uu * (Q >> 32) + ((uu * (Q & 0xFFFFFFFFull)) >> 32);
  long long lo = count_below(ex, Q, off, n);
#pragma unroll
  for (int k = 0; k < kSeg; ++k)
    if (k < cnt) {
      const long long hi = count_below(ex + c[k], Q, off, n);
      if (hi > lo) marks[lo] = i0 + k + 1;
      lo = hi;
    }
  __syncthreads();
  int mloc = 0;
#pragma unroll
  for (int k = 0; k < kSeg; ++k)
    if (k < cnt) mloc = max(mloc, marks[i0 + k]);
  int run = block_excl_scan_max(mloc, shi);
#pragma unroll
  for (int k = 0; k < kSeg; ++k)
    if (k < cnt) {
      run = max(run, marks[i0 + k]);
      anc[i0 + k] = run - 1;
    }
}

// Same on global memory for n > kRegN (weights w, scratch cdf and marks).
__device__ void resample_global(const double* __restrict__ w, int n, double wmax, uint32_t U,
                                unsigned long long* __restrict__ cdf, int32_t* __restrict__ marks,
                                int32_t* __restrict__ anc, unsigned long long* shu, int* shi) {
  const int kb = resample_bits(n);
  const int per = (n + kRT - 1) / kRT;
  const int i0 = min(n, (int)threadIdx.x * per), i1 = min(n, i0 + per);
  unsigned long long loc = 0;
  for (int i = i0; i < i1; ++i) {
    loc += (unsigned long long)floor(ldexp(w[i] / wmax, kb));
    cdf[i] = loc;
  }
  const unsigned long long ex = block_excl_scan_u64(loc, shu);
  for (int i = i0; i < i1; ++i) cdf[i] += ex;
  for (int i = threadIdx.x; i < n; i += kRT) marks[i] = 0;
  __syncthreads();
  const unsigned long long Q = cdf[n - 1];
  const unsigned long long uu = (unsigned long long)U;
  const unsigned long long off = uu * (Q >> 32) + ((uu * (Q & 0xFFFFFFFFull)) >> 32);
  for (int j = i0; j < i1; ++j) {
    const long long lo = count_below(j ? cdf[j - 1] : 0ull, Q, off, n);
    const long long hi = count_below(cdf[j], Q, off, n);
    if (hi > lo) marks[lo] = j + 1;
  }
  __syncthreads();
  int mloc = 0;
  for (int i = i0; i < i1; ++i) mloc = max(mloc, marks[i]);
  int run = block_excl_scan_max(mloc, shi);
  for (int i = i0; i < i1; ++i) {
    run = max(run, marks[i]);
    anc[i] = run - 1;
  }
}

// Resampling weight exp(l - lmax) with l = -dbeta S rounded to float64 on its
// own (no fused multiply-add), so l <= lmax exactly: every weight is <= 1 and
// the one at the smallest action is exactly 1.
__device__ __forceinline__ double tempered_weight(double dbeta, float s, double lmax) {
#pragma clang fp contract(off)
  const double l = -dbeta * (double)s;
  return exp(l - lmax);
}

// ------------------------------------------------------------ beta solve

// One float64 pass: e_i = exp(-x (S_i - smin)) and the derivatives in x.
template <class SGet>
__device__ Sums ess_sums(SGet sget, int n, double x, double smin, double* sh) {
  const double mx = -x * smin;
  double a = 0, b = 0, da = 0, db = 0;
  for (int i = threadIdx.x; i < n; i += kRT) {
    const double si = (double)sget(i);
    const double e = exp(-x * si - mx);
    const double sd = si - smin;
    a += e;
    b += e * e;
    da -= sd * e;
    db -= 2.0 * sd * e * e;
  }
  block_sum4<kNW>(a, b, da, db, sh);
  return Sums{a, b, da, db};
}

// Float32 Newton with the hardware exponential from x0 to a relative step of
// 1e-5: only a starting point for the float64 solve, which brackets afresh.
template <class SGet>
__device__ double presolve_f32(SGet sget, int n, double x0, double room, double ltarget,
                               double smin, double* sh) {
  double x = x0, lo = 0.0, hi = room;
  const float fsmin = (float)smin;
  for (int it = 0; it < 40; ++it) {
    const float xf = (float)x;
    float a = 0.f, b = 0.f, da = 0.f, db = 0.f;
    for (int i = threadIdx.x; i < n; i += kRT) {
      const float sd = sget(i) - fsmin;
      const float e = __expf(-xf * sd);
      a += e;
      b += e * e;
      da -= sd * e;
      db -= 2.f * sd * e * e;
    }
    double A = a, B = b, DA = da, DB = db;
    block_sum4<kNW>(A, B, DA, DB, sh);
    const double gval = 2.0 * log(A) - log(B) - ltarget;
    const double gder = 2.0 * DA / A - DB / B;
    if (gval >= 0.0) lo = x; else hi = x;
    double xn = x - gval / gder;
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    const bool fin = fabs(xn - x) <= 1e-5 * x;
    x = xn;
    if (fin) break;
  }
  return x;
}

// Tempering increment: ESS(dbeta) = target by bracketed float64 Newton on
// g = log ESS - log target; returns the lower end of the final bracket and
// the sums at it.
template <class SGet>
__device__ double solve_dbeta(SGet sget, int n, double room, double target, double smin,
                              double ssum, double ssq, double* sh, Sums& e, int& evals) {
  e = ess_sums(sget, n, room, smin, sh);
  evals = 1;
  if (e.a * e.a / e.b >= target) return room;
  const double ltarget = log(target);
  double lo = 0.0, hi = room;
  // second-order start: ESS / N ~ 1 / (1 + x^2 Var S), refined in float32
  const double mean = ssum / n, var = fmax(ssq / n - mean * mean, 0.0);
  double x = var > 0.0 ? sqrt(fmax(n / target - 1.0, 0.0) / var) : 0.5 * room;
  if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
  x = presolve_f32(sget, n, x, room, ltarget, smin, sh);
  if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    e = ess_sums(sget, n, x, smin, sh);
    ++evals;
    const double gval = 2.0 * log(e.a) - log(e.b) - ltarget;
    const double gder = 2.0 * e.da / e.a - e.db / e.b;
    if (gval >= 0.0) lo = x; else hi = x;
    if (hi - lo <= 1e-13 * hi) break;
    const double step = gval / gder;
    double xn = x - step;
    const double tol = 1e-14 * x;
    if (fabs(step) < tol) xn = gval >= 0.0 ? x + tol : x - tol;  // step across the root
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    x = xn;
  }
  if (lo > 0.0 && lo != x) {
    e = ess_sums(sget, n, lo, smin, sh);
    ++evals;
  }
  return lo;
}

// --------------------------------------------------------------- kernels

// Step-size adaptation of the finished sweep (App. A scaling steered to
// acc_target): log eps += acc - acc_target, clamped to [eps0/100, 10 eps0].
__device__ void adapt_eps(SmcState* st) {
  if (threadIdx.x == 0 && st->prop > 0) {
    const double abar = (double)st->acc / (double)st->prop;
    st->last_acc = abar;
    const double e = st->eps * exp(abar - st->acc_target);
    st->eps = fmin(fmax(e, st->eps0 / 100.0), 10.0 * st->eps0);
    st->acc = 0;
    st->prop = 0;
  }
}

__device__ void fail_reweight(const ReweightArgs& a, int code) {
  if (threadIdx.x == 0) {
    if (a.st) a.st->err = code;
    if (a.out) a.out[0] = a.out[1] = a.out[2] = a.out[3] = NAN;
  }
}

__device__ void finish_reweight(const ReweightArgs& a, int level, double dbeta, double new_beta,
                                double dlogz, double ess, int evals) {
  if (threadIdx.x != 0) return;
  if (SmcState* st = a.st) {
    st->logz += dlogz;
    st->beta = new_beta;
    st->level = level;
    st->last_dbeta = dbeta;
    st->last_ess = ess;
    st->solve_iters = evals;
  }
  if (a.out) {
    a.out[0] = dbeta;
    a.out[1] = new_beta;
    a.out[2] = dlogz;
    a.out[3] = ess;
  }
}

// Returns false if this launch has nothing more to do (run finished or failed).
__device__ bool reweight_prologue(const ReweightArgs& a, double& beta, double& ess_frac,
                                  int& level) {
  SmcState* st = a.st;
  if (!st) {
    beta = a.beta_in;
    ess_frac = a.ess_frac_in;
    level = 0;
    return true;
  }
  if (st->err) return false;
  adapt_eps(st);
  if (st->done || st->beta >= 1.0) {
    // the sweep at beta = 1 is finished: identity ancestors keep the
    // population in place through the gather that follows
    for (int i = threadIdx.x; i < a.n; i += kRT) a.anc[i] = i;
    __syncthreads();
    if (threadIdx.x == 0) st->done = 1;
    return false;
  }
  beta = st->beta;
  ess_frac = st->ess_frac;
  level = st->level + 1;
  return true;
}

__global__ __launch_bounds__(kRT) void reweight_kernel(ReweightArgs a) {
  __shared__ double shd[4 * kNW];
  __shared__ unsigned long long shu[kNW];
  __shared__ int shi[kNW];
  __shared__ int marks[kRegN];
  __shared__ float Sc[kRegN];
  double beta, ess_frac;
  int level;
  if (!reweight_prologue(a, beta, ess_frac, level)) return;
  const int n = a.n;
  // actions into LDS (exact float copies), all loads issued before use; a
  // non-finite action turns the minimum into -inf (one reduction)
  double smin = INFINITY;
  {
    float v[kSeg];
#pragma unroll
    for (int k = 0; k < kSeg; ++k) v[k] = a.S[min((int)threadIdx.x + k * kRT, n - 1)];
#pragma unroll
    for (int k = 0; k < kSeg; ++k) {
      const int i = threadIdx.x + k * kRT;
      if (i < n) {
        Sc[i] = v[k];
        smin = isfinite(v[k]) ? fmin(smin, (double)v[k]) : -INFINITY;
      }
    }
  }
  smin = block_reduce<kMin, kNW>(smin, shd);
  if (!isfinite(smin)) return fail_reweight(a, PHI4_ENONFINITE);
  const auto sget = [&](int i) { return Sc[i]; };
  double ssum = 0.0, ssq = 0.0, z0 = 0.0, z1 = 0.0;
  for (int i = threadIdx.x; i < n; i += kRT) {
    const double sd = (double)Sc[i] - smin;
    ssum += sd;
    ssq += sd * sd;
  }
  block_sum4<kNW>(ssum, ssq, z0, z1, shd);
  const double room = 1.0 - beta;
  Sums e;
  int evals = 0;
  const double dbeta = solve_dbeta(sget, n, room, ess_frac * n, smin, ssum, ssq, shd, e, evals);
  if (!(dbeta > 0.0)) return fail_reweight(a, PHI4_ENONFINITE);
  const double new_beta = dbeta == room ? 1.0 : fmin(1.0, beta + dbeta);
  const double dlogz = -dbeta * smin + log(e.a) - log((double)n);
  const double ess = e.a * e.a / e.b;
  // weights of this thread's contiguous segment; the largest is exactly 1
  const int per = (n + kRT - 1) / kRT;
  const int i0 = min(n, (int)threadIdx.x * per);
  const int cnt = max(0, min(n, i0 + per) - i0);
  const double lmax = -dbeta * smin;
  double w[kSeg];
#pragma unroll
  for (int k = 0; k < kSeg; ++k) w[k] = k < cnt ? tempered_weight(dbeta, Sc[i0 + k], lmax) : 0.0;
  if (a.w && !a.st) {
#pragma unroll
    for (int k = 0; k < kSeg; ++k)
      if (k < cnt) a.w[i0 + k] = w[k];
  }
  if (a.do_resample) {
    const uint32_t U = word0(0u, 0u, counter3((uint32_t)level, PHI4_RESAMPLE), a.seed, a.run);
    resample_seg(w, cnt, i0, n, 1.0, U, marks, a.anc, shu, shi);
  }
  __syncthreads();
  finish_reweight(a, level, dbeta, new_beta, dlogz, ess, evals);
}

// Large-N variant: actions and weights stay in global memory.
__global__ __launch_bounds__(kRT) void reweight_global_kernel(ReweightArgs a) {
  __shared__ double shd[4 * kNW];
  __shared__ unsigned long long shu[kNW];
  __shared__ int shi[kNW];
  double beta, ess_frac;
  int level;
  if (!reweight_prologue(a, beta, ess_frac, level)) return;
  const int n = a.n;
  double smin = INFINITY;
  for (int i = threadIdx.x; i < n; i += kRT) {
    const float v = a.S[i];
    smin = isfinite(v) ? fmin(smin, (double)v) : -INFINITY;
  }
  smin = block_reduce<kMin, kNW>(smin, shd);
  if (!isfinite(smin)) return fail_reweight(a, PHI4_ENONFINITE);
  const float* S = a.S;
  const auto sget = [&](int i) { return S[i]; };
  double ssum = 0.0, ssq = 0.0, z0 = 0.0, z1 = 0.0;
  for (int i = threadIdx.x; i < n; i += kRT) {
    const double sd = (double)S[i] - smin;
    ssum += sd;
    ssq += sd * sd;
  }
  block_sum4<kNW>(ssum, ssq, z0, z1, shd);
  const double room = 1.0 - beta;
  Sums e;
  int evals = 0;
  const double dbeta = solve_dbeta(sget, n, room, ess_frac * n, smin, ssum, ssq, shd, e, evals);
  if (!(dbeta > 0.0)) return fail_reweight(a, PHI4_ENONFINITE);
  const double new_beta = dbeta == room ? 1.0 : fmin(1.0, beta + dbeta);
  const double dlogz = -dbeta * smin + log(e.a) - log((double)n);
  const double ess = e.a * e.a / e.b;
  const double lmax = -dbeta * smin;
  if (a.w)
    for (int i = threadIdx.x; i < n; i += kRT) a.w[i] = tempered_weight(dbeta, S[i], lmax);
  __syncthreads();
  if (a.do_resample) {
    const uint32_t U = word0(0u, 0u, counter3((uint32_t)level, PHI4_RESAMPLE), a.seed, a.run);
    resample_global(a.w, n, 1.0, U, a.cdf, a.marks, a.anc, shu, shi);
  }
  __syncthreads();
  finish_reweight(a, level, dbeta, new_beta, dlogz, ess, evals);
}

// Stand-alone resampling of caller weights: checks them (finite, >= 0,
// max > 0) and resamples with the largest weight as the scale.
__global__ __launch_bounds__(kRT) void resample_kernel(const double* w, int n, uint32_t U,
                                                       unsigned long long* cdf, int32_t* marks,
                                                       int32_t* anc, int32_t* status) {
  __shared__ double shd[kNW];
  __shared__ unsigned long long shu[kNW];
  __shared__ int shi[kNW];
  __shared__ int mlds[kRegN];
  // one max-reduction decides validity: an invalid weight maps to +inf
  double wmax = -1.0;
  for (int i = threadIdx.x; i < n; i += kRT) {
    const double x = w[i];
    wmax = (x >= 0.0 && !isinf(x)) ? fmax(wmax, x) : INFINITY;
  }
  wmax = block_reduce<kMax, kNW>(wmax, shd);
  if (isinf(wmax) || !(wmax > 0.0)) {
    if (threadIdx.x == 0 && status) *status = PHI4_ENONFINITE;
    return;
  }
  if (n <= kRegN) {
    const int per = (n + kRT - 1) / kRT;
    const int i0 = min(n, (int)threadIdx.x * per);
    const int cnt = max(0, min(n, i0 + per) - i0);
    double wv[kSeg];
#pragma unroll
    for (int k = 0; k < kSeg; ++k) {
      const double v = w[min(i0 + k, n - 1)];   // valid address, masked
      wv[k] = k < cnt ? v : 0.0;
    }
    resample_seg(wv, cnt, i0, n, wmax, U, mlds, anc, shu, shi);
  } else {
    resample_global(w, n, wmax, U, cdf, marks, anc, shu, shi);
  }
  if (threadIdx.x == 0 && status) *status = 0;
}

__global__ void smc_state_init_kernel(SmcState* st, double eps0, double acc_target,
                                      double ess_frac) {
  SmcState s = {};
  s.beta = 0.0;
  s.logz = 0.0;
  s.eps = eps0;
  s.eps0 = eps0;
  s.acc_target = acc_target;
  s.ess_frac = ess_frac;
  s.last_acc = NAN;
  s.last_dbeta = NAN;
  s.last_ess = NAN;
  *st = s;
}

__global__ void ns_state_init_kernel(NsState* st, double eps0, double acc_target) {
  NsState s = {};
  s.logX = 0.0;
  s.logZ = -INFINITY;
  s.hsum = 0.0;
  s.logmz = -INFINITY;
  s.eps = eps0;
  s.eps0 = eps0;
  s.acc_target = acc_target;
  s.last_acc = NAN;
  *st = s;
}

__global__ __launch_bounds__(kRT) void mean_abs_kernel(const float* absM, int n, double* out) {
  __shared__ double shd[kNW];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kRT) s += (double)absM[i];
  s = block_reduce<kSum, kNW>(s, shd);
  if (threadIdx.x == 0) *out = s / n;
}

}  // namespace

void launch_reweight(const ReweightArgs& a, hipStream_t s) {
  if (a.n <= kRegN)
    reweight_kernel<<<1, kRT, 0, s>>>(a);
  else
    reweight_global_kernel<<<1, kRT, 0, s>>>(a);
}

void launch_resample_weights(const double* w, int n, uint32_t U, unsigned long long* cdf,
                             int32_t* marks, int32_t* anc, int32_t* status, hipStream_t s) {
  if (n <= 0) return;
  resample_kernel<<<1, kRT, 0, s>>>(w, n, U, cdf, marks, anc, status);
}

void launch_smc_state_init(SmcState* st, double eps0, double acc_target, double ess_frac,
                           hipStream_t s) {
  smc_state_init_kernel<<<1, 1, 0, s>>>(st, eps0, acc_target, ess_frac);
}

void launch_ns_state_init(NsState* st, double eps0, double acc_target, hipStream_t s) {
  ns_state_init_kernel<<<1, 1, 0, s>>>(st, eps0, acc_target);
}

void launch_mean_abs(const float* absM, int n, double* out, const int32_t* done, hipStream_t s) {
  (void)done;
  if (n <= 0) return;
  mean_abs_kernel<<<1, kRT, 0, s>>>(absM, n, out);
}

}  // namespace phi4
