// Reweighting between tempering levels (float64, one workgroup per run):
// ESS-adaptive increment of beta, log-sum-exp update of log Z and
// systematic resampling on an integer CDF.
//
// The tempering increment solves ESS(dbeta) = ess_frac * N with
// ESS = (sum w)^2 / sum w^2, w_i = exp(-dbeta (S_i - S_min)), by a
// bracketed Newton iteration on g = log ESS - log target; the returned
// increment is the lower end of a bracket of relative width <= 1e-13, so
// ESS(dbeta) >= target always holds (the adaptive SMC rule of App. A with
// the target ESS of the configuration).
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

constexpr int kRT = 1024;  // threads of the single-workgroup kernels

struct Sums {
  double a, b, da, db;  // sum e, sum e^2, d/dx sum e, d/dx sum e^2
};

// e_i = exp(l_i - max l) with l_i = -x S_i and max l = -x smin
__device__ Sums ess_sums(const float* __restrict__ S, int n, double x, double smin, double* sh) {
  const double mx = -x * smin;
  double a = 0, b = 0, da = 0, db = 0;
  for (int i = threadIdx.x; i < n; i += kRT) {
    const double si = (double)S[i];
    const double e = exp(-x * si - mx);
    const double sd = si - smin;
    a += e;
    b += e * e;
    da -= sd * e;
    db -= 2.0 * sd * e * e;
  }
  block_sum4(a, b, da, db, sh);
  return Sums{a, b, da, db};
}

__device__ unsigned long long block_excl_scan_u64(unsigned long long v, unsigned long long* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
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
  for (int w = 0; w < wid; ++w) off += sh[w];
  (void)nw;
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
  for (int w = 0; w < wid; ++w) off = max(off, sh[w]);
  return lane == 0 ? off : max(off, ex);
}

__device__ __forceinline__ long long count_below(unsigned long long C, unsigned long long Q,
                                                 unsigned long long off, int n) {
  const unsigned long long cn = C * (unsigned long long)n;
  if (cn <= off) return 0;
  const unsigned long long c = (cn - off + Q - 1) / Q;
  return c < (unsigned long long)n ? (long long)c : (long long)n;
}

// Systematic resampling of w[0..n) (finite, >= 0, max > 0) with offset word
// U.  Scratch: cdf[n] (uint64), marks[n] (int).  Writes anc[n].  Returns
// 0, or PHI4_ENONFINITE for invalid weights (uniform across the block).
__device__ int resample_block(const double* __restrict__ w, int n, uint32_t U,
                              unsigned long long* __restrict__ cdf, int32_t* __restrict__ marks,
                              int32_t* __restrict__ anc, double* shd,
                              unsigned long long* shu, int* shi) {
  // validity and max
  double wmax = -1.0, bad = 0.0;
  for (int i = threadIdx.x; i < n; i += kRT) {
    const double x = w[i];
    if (!(x >= 0.0) || isinf(x)) bad = 1.0;
    wmax = fmax(wmax, x);
  }
  bad = block_reduce<kMax>(bad, shd);
  wmax = block_reduce<kMax>(wmax, shd);
  if (bad != 0.0 || !(wmax > 0.0)) return PHI4_ENONFINITE;
  const int k = n > 1 ? 62 - 2 * (32 - __clz((unsigned)(n - 1))) : 62;
  // contiguous segment per thread
  const int per = (n + kRT - 1) / kRT;
  const int i0 = min(n, (int)threadIdx.x * per), i1 = min(n, i0 + per);
  unsigned long long loc = 0;
  for (int i = i0; i < i1; ++i) {
    const unsigned long long q = (unsigned long long)floor(ldexp(w[i] / wmax, k));
    loc += q;
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
    const unsigned long long cprev = j ? cdf[j - 1] : 0ull;
    const long long lo = count_below(cprev, Q, off, n);
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
  __syncthreads();
  return 0;
}

constexpr int kSeg = 16;                 // particles per thread on the register path
constexpr int kRegN = kRT * kSeg;        // largest N on the register path (16384)

// Systematic resampling of a register-resident segment: thread t holds the
// weights of particles [i0, i0 + cnt).  marks: LDS, n ints.  Writes anc.
__device__ int resample_seg(const double (&w)[kSeg], int cnt, int i0, int n, uint32_t U,
                            int* marks, int32_t* __restrict__ anc, double* shd,
                            unsigned long long* shu, int* shi) {
  double wmax = -1.0, bad = 0.0;
#pragma unroll
  for (int k = 0; k < kSeg; ++k)
    if (k < cnt) {
      if (!(w[k] >= 0.0) || isinf(w[k])) bad = 1.0;
      wmax = fmax(wmax, w[k]);
    }
  bad = block_reduce<kMax>(bad, shd);
  wmax = block_reduce<kMax>(wmax, shd);
  if (bad != 0.0 || !(wmax > 0.0)) return PHI4_ENONFINITE;
  const int kb = n > 1 ? 62 - 2 * (32 - __clz((unsigned)(n - 1))) : 62;
  unsigned long long c[kSeg];
  unsigned long long loc = 0;
#pragma unroll
  for (int k = 0; k < kSeg; ++k) {
    if (k < cnt) loc += (unsigned long long)floor(ldexp(w[k] / wmax, kb));
    c[k] = loc;
  }
  const unsigned long long ex = block_excl_scan_u64(loc, shu);
  for (int i = threadIdx.x; i < n; i += kRT) marks[i] = 0;
  // Q = C_{n-1}: the inclusive total, broadcast through LDS
  __shared__ unsigned long long qsh;
  if (cnt > 0 && i0 + cnt == n) qsh = ex + c[cnt - 1];
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
  return 0;
}

__device__ Sums ess_sums_lds(const float* Sc, int n, double x, double smin, double* sh) {
  const double mx = -x * smin;
  double a = 0, b = 0, da = 0, db = 0;
  for (int i = threadIdx.x; i < n; i += kRT) {
    const double si = (double)Sc[i];
    const double e = exp(-x * si - mx);
    const double sd = si - smin;
    a += e;
    b += e * e;
    da -= sd * e;
    db -= 2.0 * sd * e * e;
  }
  block_sum4(a, b, da, db, sh);
  return Sums{a, b, da, db};
}

// Float32 Newton on g(x) = log ESS(x) - log target with the hardware
// exponential, from x0 to a relative step of 1e-5; only a starting point for
// the float64 solve, which re-brackets from [0, room].
__device__ double presolve_f32(const float* Sc, int n, double x0, double room, double ltarget,
                               double smin, double* sh) {
  double x = x0, lo = 0.0, hi = room;
  const float fsmin = (float)smin;
  for (int it = 0; it < 40; ++it) {
    const float xf = (float)x;
    float a = 0.f, b = 0.f, da = 0.f, db = 0.f;
    for (int i = threadIdx.x; i < n; i += kRT) {
      const float sd = Sc[i] - fsmin;
      const float e = __expf(-xf * sd);
      a += e;
      b += e * e;
      da -= sd * e;
      db -= 2.f * sd * e * e;
    }
    double A = a, B = b, DA = da, DB = db;
    block_sum4(A, B, DA, DB, sh);
    const double gval = 2.0 * log(A) - log(B) - ltarget;
    const double gder = 2.0 * DA / A - DB / B;
    if (gval >= 0.0) lo = x; else hi = x;
    const double step = gval / gder;
    double xn = x - step;
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    const bool fin = fabs(xn - x) <= 1e-5 * x;
    x = xn;
    if (fin) break;
  }
  return x;
}

// Tempering increment: ESS(dbeta) = target by bracketed Newton on
// g = log ESS - log target; returns the lower end of the final bracket.
template <class Eval, class Guess>
__device__ double solve_dbeta(Eval eval, Guess guess, double room, double target, int n,
                              double ssum, double ssq, Sums& e, int& evals) {
  e = eval(room);
  evals = 1;
  if (e.a * e.a / e.b >= target) return room;
  const double ltarget = log(target);
  double lo = 0.0, hi = room;
  // second-order start: ESS / N ~ 1 / (1 + x^2 Var S), refined by `guess`
  const double mean = ssum / n, var = fmax(ssq / n - mean * mean, 0.0);
  double x = var > 0.0 ? sqrt(fmax(n / target - 1.0, 0.0) / var) : 0.5 * room;
  if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
  x = guess(x, room, ltarget);
  if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    e = eval(x);
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
  if (lo > 0.0) {
    e = eval(lo);
    ++evals;
  }
  return lo;
}

__global__ __launch_bounds__(kRT) void reweight_kernel(ReweightArgs a) {
  __shared__ double shd[4 * (kRT / 64)];
  __shared__ unsigned long long shu[kRT / 64];
  __shared__ int shi[kRT / 64];
  __shared__ int marks[kRegN];
  __shared__ float Sc[kRegN];
  SmcState* st = a.st;
  const int n = a.n;
  double beta, ess_frac;
  int level = 0;
  if (st) {
    if (st->err) return;
    // step-size adaptation of the finished sweep (App. A scaling steered to
    // acc_target): log eps += acc - acc_target, clamped to [eps0/100, 10 eps0]
    if (threadIdx.x == 0 && st->prop > 0) {
      const double abar = (double)st->acc / (double)st->prop;
      st->last_acc = abar;
      const double e = st->eps * exp(abar - st->acc_target);
      st->eps = fmin(fmax(e, st->eps0 / 100.0), 10.0 * st->eps0);
      st->acc = 0;
      st->prop = 0;
    }
    if (st->done || st->beta >= 1.0) {
      // the sweep at beta = 1 is finished: identity ancestors keep the
      // population in place through the gather that follows
      for (int i = threadIdx.x; i < n; i += kRT) a.anc[i] = i;
      __syncthreads();
      if (threadIdx.x == 0) st->done = 1;
      return;
    }
    beta = st->beta;
    ess_frac = st->ess_frac;
    level = st->level + 1;
  } else {
    beta = a.beta_in;
    ess_frac = a.ess_frac_in;
  }
  // actions in LDS (exact float copies); all loads issued before use
  double smin = INFINITY, bad = 0.0;
  {
    float v[kSeg];
#pragma unroll
    for (int k = 0; k < kSeg; ++k) v[k] = a.S[min((int)threadIdx.x + k * kRT, n - 1)];
#pragma unroll
    for (int k = 0; k < kSeg; ++k) {
      const int i = threadIdx.x + k * kRT;
      if (i < n) {
        Sc[i] = v[k];
        if (!isfinite(v[k])) bad = 1.0;
        smin = fmin(smin, (double)v[k]);
      }
    }
  }
  bad = block_reduce<kMax>(bad, shd);
  smin = block_reduce<kMin>(smin, shd);
  if (bad != 0.0) {
    if (threadIdx.x == 0) {
      if (st) st->err = PHI4_ENONFINITE;
      if (a.out) a.out[0] = a.out[1] = a.out[2] = a.out[3] = NAN;
    }
    return;
  }
  double ssum = 0.0, ssq = 0.0, z0 = 0.0, z1 = 0.0;
  for (int i = threadIdx.x; i < n; i += kRT) {
    const double sd = (double)Sc[i] - smin;
    ssum += sd;
    ssq += sd * sd;
  }
  block_sum4(ssum, ssq, z0, z1, shd);
  const double room = 1.0 - beta;
  const double target = ess_frac * n;
  Sums e;
  int evals = 0;
  const double dbeta = solve_dbeta(
      [&](double x) { return ess_sums_lds(Sc, n, x, smin, shd); },
      [&](double x0, double rm, double lt) { return presolve_f32(Sc, n, x0, rm, lt, smin, shd); },
      room, target, n, ssum, ssq, e, evals);
  if (!(dbeta > 0.0)) {
    if (threadIdx.x == 0) {
      if (st) st->err = PHI4_ENONFINITE;
      if (a.out) a.out[0] = a.out[1] = a.out[2] = a.out[3] = NAN;
    }
    return;
  }
  const double new_beta = dbeta == room ? 1.0 : fmin(1.0, beta + dbeta);
  const double dlogz = -dbeta * smin + log(e.a) - log((double)n);
  const double ess = e.a * e.a / e.b;
  // weights exp(l_i - max l), l_i = -dbeta S_i, for this thread's contiguous segment
  const int per = (n + kRT - 1) / kRT;
  const int i0 = min(n, (int)threadIdx.x * per);
  const int cnt = max(0, min(n, i0 + per) - i0);
  double w[kSeg];
  const double mx = -dbeta * smin;
#pragma unroll
  for (int k = 0; k < kSeg; ++k) {
    w[k] = k < cnt ? exp(-dbeta * (double)Sc[i0 + k] - mx) : 0.0;
    if (a.w && k < cnt) a.w[i0 + k] = w[k];
  }
  int rc = 0;
  if (a.do_resample) {
    const uint32_t U = word0(0u, 0u, counter3((uint32_t)level, PHI4_RESAMPLE), a.seed, a.run);
    rc = resample_seg(w, cnt, i0, n, U, marks, a.anc, shd, shu, shi);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (st) {
      if (rc) {
        st->err = rc;
      } else {
        st->logz += dlogz;
        st->beta = new_beta;
        st->level = level;
        st->last_dbeta = dbeta;
        st->last_ess = ess;
        st->solve_iters = evals;
      }
    }
    if (a.out) {
      a.out[0] = dbeta;
      a.out[1] = new_beta;
      a.out[2] = dlogz;
      a.out[3] = ess;
    }
  }
}

// Large-N variant: actions and weights stay in global memory.
__global__ __launch_bounds__(kRT) void reweight_global_kernel(ReweightArgs a) {
  __shared__ double shd[4 * (kRT / 64)];
  __shared__ unsigned long long shu[kRT / 64];
  __shared__ int shi[kRT / 64];
  SmcState* st = a.st;
  const int n = a.n;
  double beta, ess_frac;
  int level = 0;
  if (st) {
    if (st->err) return;
    if (threadIdx.x == 0 && st->prop > 0) {
      const double abar = (double)st->acc / (double)st->prop;
      st->last_acc = abar;
      const double e = st->eps * exp(abar - st->acc_target);
      st->eps = fmin(fmax(e, st->eps0 / 100.0), 10.0 * st->eps0);
      st->acc = 0;
      st->prop = 0;
    }
    if (st->done || st->beta >= 1.0) {
      for (int i = threadIdx.x; i < n; i += kRT) a.anc[i] = i;
      __syncthreads();
      if (threadIdx.x == 0) st->done = 1;
      return;
    }
    beta = st->beta;
    ess_frac = st->ess_frac;
    level = st->level + 1;
  } else {
    beta = a.beta_in;
    ess_frac = a.ess_frac_in;
  }
  double smin = INFINITY, bad = 0.0;
  for (int i = threadIdx.x; i < n; i += kRT) {
    const double si = (double)a.S[i];
    if (!isfinite(si)) bad = 1.0;
    smin = fmin(smin, si);
  }
  bad = block_reduce<kMax>(bad, shd);
  smin = block_reduce<kMin>(smin, shd);
  if (bad != 0.0) {
    if (threadIdx.x == 0) {
      if (st) st->err = PHI4_ENONFINITE;
      if (a.out) a.out[0] = a.out[1] = a.out[2] = a.out[3] = NAN;
    }
    return;
  }
  double ssum = 0.0, ssq = 0.0, z0 = 0.0, z1 = 0.0;
  for (int i = threadIdx.x; i < n; i += kRT) {
    const double sd = (double)a.S[i] - smin;
    ssum += sd;
    ssq += sd * sd;
  }
  block_sum4(ssum, ssq, z0, z1, shd);
  const double room = 1.0 - beta;
  Sums e;
  int evals = 0;
  const double dbeta = solve_dbeta(
      [&](double x) { return ess_sums(a.S, n, x, smin, shd); },
      [](double x0, double, double) { return x0; }, room, ess_frac * n, n, ssum, ssq, e, evals);
  if (!(dbeta > 0.0)) {
    if (threadIdx.x == 0) {
      if (st) st->err = PHI4_ENONFINITE;
      if (a.out) a.out[0] = a.out[1] = a.out[2] = a.out[3] = NAN;
    }
    return;
  }
  const double new_beta = dbeta == room ? 1.0 : fmin(1.0, beta + dbeta);
  const double dlogz = -dbeta * smin + log(e.a) - log((double)n);
  const double ess = e.a * e.a / e.b;
  if (a.w) {
    const double mx = -dbeta * smin;
    for (int i = threadIdx.x; i < n; i += kRT) a.w[i] = exp(-dbeta * (double)a.S[i] - mx);
  }
  __syncthreads();
  int rc = 0;
  if (a.do_resample) {
    const uint32_t U = word0(0u, 0u, counter3((uint32_t)level, PHI4_RESAMPLE), a.seed, a.run);
    rc = resample_block(a.w, n, U, a.cdf, a.marks, a.anc, shd, shu, shi);
  }
  if (threadIdx.x == 0) {
    if (st) {
      if (rc) {
        st->err = rc;
      } else {
        st->logz += dlogz;
        st->beta = new_beta;
        st->level = level;
        st->last_dbeta = dbeta;
        st->last_ess = ess;
        st->solve_iters = evals;
      }
    }
    if (a.out) {
      a.out[0] = dbeta;
      a.out[1] = new_beta;
      a.out[2] = dlogz;
      a.out[3] = ess;
    }
  }
}

__global__ __launch_bounds__(kRT) void resample_kernel(const double* w, int n, uint32_t U,
                                                       unsigned long long* cdf, int32_t* marks,
                                                       int32_t* anc, int32_t* status) {
  __shared__ double shd[4 * (kRT / 64)];
  __shared__ unsigned long long shu[kRT / 64];
  __shared__ int shi[kRT / 64];
  __shared__ int mlds[kRegN];
  int rc;
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
    rc = resample_seg(wv, cnt, i0, n, U, mlds, anc, shd, shu, shi);
  } else {
    rc = resample_block(w, n, U, cdf, marks, anc, shd, shu, shi);
  }
  if (threadIdx.x == 0 && status) *status = rc;
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

__global__ __launch_bounds__(kRT) void mean_abs_kernel(const float* absM, int n, double* out,
                                                       const int32_t* done) {
  __shared__ double shd[kRT / 64];
  (void)done;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kRT) s += (double)absM[i];
  s = block_reduce<kSum>(s, shd);
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
  if (n <= 0) return;
  mean_abs_kernel<<<1, kRT, 0, s>>>(absM, n, out, done);
}

}  // namespace phi4
