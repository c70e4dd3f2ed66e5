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

// ------------------------------------------------------------ reductions

// Workgroup reductions of NV values at once with a single barrier: the
// per-wave results go to one of two LDS slots that alternate between calls
// (a thread can only reach a slot again after every thread has passed the
// barrier of the call in between, i.e. finished reading it).  The first NMIN
// values are min-reduced, the rest summed; fixed order, every thread gets
// the same bits.
template <class T>
struct BlockRed {
  T* sh;      // 2 * kMaxV * kNW
  int slot;
  static constexpr int kMaxV = 4;
  template <int NV, int NMIN = 0>
  __device__ __forceinline__ void run(T (&x)[NV]) {
    static_assert(NV <= kMaxV, "too many values");
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] = wave_op(x[v], v < NMIN);
    T* s = sh + slot * (kMaxV * kNW);
    slot ^= 1;
    if (lane == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) s[v * kNW + wid] = x[v];
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      T r = s[v * kNW];
#pragma unroll
      for (int w = 1; w < kNW; ++w) r = v < NMIN ? fmin(r, s[v * kNW + w]) : r + s[v * kNW + w];
      x[v] = r;
    }
  }
  __device__ __forceinline__ static double wave_op(double v, bool mn) {
    return mn ? wave_red<kMin>(v) : wave_red<kSum>(v);
  }
  __device__ __forceinline__ static float wave_op(float v, bool) { return wave_sum_f(v); }
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

// ---------------------------------------------------------- resampling

__device__ __forceinline__ int resample_bits(int n) {
  return n > 1 ? 62 - 2 * (32 - __clz((unsigned)(n - 1))) : 62;
}

// Shared constants of one systematic resampling pass.
struct Grid {
  unsigned long long Q, off;
  double invQ;
  int n;
};

__device__ __forceinline__ Grid make_grid(unsigned long long Q, uint32_t U, int n) {
  const unsigned long long uu = (unsigned long long)U;
  Grid g;
  g.Q = Q;
  g.off = uu * (Q >> 32) + ((uu * (Q & 0xFFFFFFFFull)) >> 32);
  g.invQ = 1.0 / (double)Q;
  g.n = n;
  return g;
}

// #{i : T_i < C} = min(n, ceil((C n - off) / Q)) in exact integers: a
// float64 estimate of the quotient (within 1e-11 of it, as the quotient is
// at most n) fixed by one exact comparison each way.  C n < 2^63 because
// C <= Q <= n 2^k and n^2 2^k <= 2^62.
// Branch-free (selects only), so that independent calls overlap.
__device__ __forceinline__ int count_below(unsigned long long C, const Grid& g) {
  const unsigned long long cn = C * (unsigned long long)g.n;
  const bool pos = cn > g.off;
  const unsigned long long num = pos ? cn - g.off : 0ull;
  const double est = ceil((double)num * g.invQ);
  unsigned long long c = est < (double)g.n + 2.0 ? (unsigned long long)est : g.n + 2ull;
  const unsigned long long cq = c * g.Q;
  const bool small = cq < num;                        // estimate one too small
  const bool large = !small && c > 0 && cq - g.Q >= num;   // estimate one too large
  c = small ? c + 1 : (large ? c - 1 : c);
  c = pos ? c : 0ull;
  return c < (unsigned long long)g.n ? (int)c : g.n;
}

// Systematic resampling of a register-resident segment: this thread holds
// the weights of particles [i0, i0 + cnt) (contiguous segments in thread
// order); wmax is the largest weight (> 0, all weights finite and >= 0).
// Every particle writes its own ancestor range [count(C_{j-1}), count(C_j))
// of anc directly.
template <int SEG>
__device__ void resample_seg(const double (&w)[SEG], int cnt, int i0, int n, double wmax,
                             uint32_t U, int32_t* __restrict__ anc, unsigned long long* shu) {
  __shared__ unsigned long long qsh;
  const int kb = resample_bits(n);
  unsigned long long c[SEG];
  unsigned long long loc = 0;
#pragma unroll
  for (int k = 0; k < SEG; ++k) {
    if (k < cnt) loc += (unsigned long long)floor(ldexp(w[k] / wmax, kb));
    c[k] = loc;
  }
  const unsigned long long ex = block_excl_scan_u64(loc, shu);
  if (cnt > 0 && i0 + cnt == n) qsh = ex + loc;   // Q = C_{n-1}
  __syncthreads();
  const Grid g = make_grid(qsh, U, n);
  // every range end first (independent), then the writes; past cnt the
  // running sums stop growing, so those ranges are empty
  int hi[SEG];
#pragma unroll
  for (int k = 0; k < SEG; ++k) hi[k] = count_below(ex + c[k], g);
  int lo = count_below(ex, g);
#pragma unroll
  for (int k = 0; k < SEG; ++k) {
    for (int p = lo; p < hi[k]; ++p) anc[p] = i0 + k;
    lo = hi[k];
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
  const Grid g = make_grid(cdf[n - 1], U, n);
  for (int j = i0; j < i1; ++j) {
    const int lo = count_below(j ? cdf[j - 1] : 0ull, g);
    const int hi = count_below(cdf[j], g);
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

// g(x) = log ESS(x) - log target from the sums: log of A^2 / (target B)
// and its derivative 2 A'/A - B'/B.
__device__ __forceinline__ void ess_newton(const Sums& e, double target, double& g, double& gd) {
  g = log(e.a * e.a / (target * e.b));
  gd = (2.0 * e.da * e.b - e.db * e.a) / (e.a * e.b);
}

// ------------------------------------------------------------ beta solve
//
// Register-path solve over the thread's segment s[0..cnt) of actions.
// Float32 Newton pre-solve, then float64 Newton: an exact exponential pass
// e0 = exp(-x0 sd) at the pre-solved x0, and every further evaluation at x
// near the previous point x0 as e0 exp(-(x - x0) sd) with the exponential of
// the small argument u = (x - x0) sd, |u| <= 2e-3, summed to degree 5
// (truncation below 1e-19 relative); a point farther away gets a fresh
// exact pass.  The bracket
// and the lower end returned follow the float64 Newton of the global path.
template <int SEG>
struct SegSolver {
  const float (&s)[SEG];
  int cnt, n;
  double smin, smax;
  BlockRed<double>& rd;
  BlockRed<float>& rf;
  double e0[SEG];
  double x0;

  // Sums at x; leaves e0 = exp(-x sd) and x0 = x for the next call.
  __device__ Sums eval(double x, bool first) {
    const double dx = x - x0;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (first || !(fabs(dx) * (smax - smin) <= 2e-3)) {
      const double mx = -x * smin;
#pragma unroll
      for (int k = 0; k < SEG; ++k) {
        const double si = (double)s[k];
        const double e = k < cnt ? exp(-x * si - mx) : 0.0;
        const double sd = si - smin;
        e0[k] = e;
        v[0] += e;
        v[1] += e * e;
        v[2] -= sd * e;
        v[3] -= 2.0 * sd * e * e;
        if ((k & 7) == 7) __builtin_amdgcn_sched_barrier(0);   // bound the exp interleave
      }
    } else {
#pragma unroll
      for (int k = 0; k < SEG; ++k) {
        const double sd = (double)s[k] - smin;
        const double u = dx * sd;
        // exp(-u) to degree 5
        const double p =
            1.0 - u * (1.0 - u * (0.5 - u * (1.0 / 6 - u * (1.0 / 24 - u * (1.0 / 120)))));
        const double e = e0[k] * p;
        e0[k] = e;
        v[0] += e;
        v[1] += e * e;
        v[2] -= sd * e;
        v[3] -= 2.0 * sd * e * e;
      }
    }
    x0 = x;
    rd.template run<4>(v);
    return Sums{v[0], v[1], v[2], v[3]};
  }

  // Float32 Newton with the hardware exponential from xs to a relative step
  // of 1e-5; room counts as reached when g(room) >= 0 in float32.
  __device__ double presolve(double xs, double room, double target) {
    const float lt = __logf((float)target);
    const float fsmin = (float)smin;
    float sdf[SEG];
#pragma unroll
    for (int k = 0; k < SEG; ++k) sdf[k] = k < cnt ? s[k] - fsmin : INFINITY;
    double x = xs, lo = 0.0, hi = room;
#pragma unroll 1
    for (int it = 0; it < 40; ++it) {
      const float xf = (float)x;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < SEG; ++k) {
        const float e = __expf(-xf * sdf[k]);   // 0 beyond the segment
        const float sd = k < cnt ? sdf[k] : 0.f;
        v[0] += e;
        v[1] += e * e;
        v[2] -= sd * e;
        v[3] -= 2.f * sd * e * e;
      }
      rf.template run<4>(v);
      const double g = (double)(2.f * __logf(v[0]) - __logf(v[1]) - lt);
      const double gd = (double)(2.f * v[2] / v[0] - v[3] / v[1]);
      if (g >= 0.0) lo = x; else hi = x;
      if (x == room && g >= 0.0) break;
      double xn = x - g / gd;
      if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
      const bool fin = fabs(xn - x) <= 1e-5 * x;
      x = xn;
      if (fin) break;
    }
    return x;
  }

  // Tempering increment: room when g(room) >= 0, else the lower end of a
  // bracket of relative width <= 1e-13 around the root of g; e holds the
  // sums at the returned point.  Room is evaluated whenever the bracket
  // closes against it (or the pre-solve lands on it).
  __device__ double solve(double room, double target, double var, Sums& e, int& evals) {
    // second-order start: ESS / N ~ 1 / (1 + x^2 Var S)
    double xs = var > 0.0 ? sqrt(fmax(n / target - 1.0, 0.0) / var) : room;
    if (!(xs > 0.0) || xs > room) xs = room;
    double x = presolve(xs, room, target);
    if (!(x > 0.0 && x <= room)) x = 0.5 * room;
    double lo = 0.0, hi = room;
    bool room_seen = false, have_lo = false;
    Sums elo = {};
    evals = 0;
#pragma unroll 1
    for (int it = 0; it < 200; ++it) {
      e = eval(x, evals == 0);
      ++evals;
      if (x == room) room_seen = true;
      double g, gd;
      ess_newton(e, target, g, gd);
      if (g >= 0.0) {
        if (x == room) return room;
        lo = x;
        elo = e;
        have_lo = true;
      } else {
        hi = x;
      }
      if (hi - lo <= 1e-13 * hi) {
        if (hi == room && !room_seen) {
          x = room;
          continue;
        }
        break;
      }
      const double step = g / gd;
      double xn = x - step;
      const double tol = 1e-14 * x;
      if (fabs(step) < tol) xn = g >= 0.0 ? x + tol : x - tol;  // step across the root
      if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
      x = xn;
    }
    if (!have_lo) return 0.0;   // no feasible point: the caller reports the failure
    e = elo;
    return lo;
  }
};

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

// Register path, n <= 512 SEG: thread t holds the actions of particles
// [t per, t per + per), per = ceil(n / 512), for the whole launch.
template <int SEG>
__device__ __forceinline__ void reweight_impl(const ReweightArgs& a) {
  __shared__ double shd[2 * 4 * kNW];
  __shared__ float shf[2 * 4 * kNW];
  __shared__ unsigned long long shu[kNW];
  const int n = a.n;
  const int per = (n + kRT - 1) / kRT;
  const int i0 = min(n, (int)threadIdx.x * per);
  const int cnt = max(0, min(n, i0 + per) - i0);
  // action loads first (clamped valid addresses), then the state
  float s[SEG];
#pragma unroll
  for (int k = 0; k < SEG; ++k) s[k] = a.S[min(i0 + k, n - 1)];
  const float c0 = a.S[0];
  double beta, ess_frac;
  int level;
  if (!reweight_prologue(a, beta, ess_frac, level)) return;
  BlockRed<double> rd{shd, 0};
  BlockRed<float> rf{shf, 0};
  // min, max and the first two moments about S_0 in one reduction; a
  // non-finite action turns the minimum into -inf
  double m[4] = {INFINITY, INFINITY, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < SEG; ++k)
    if (k < cnt) {
      const double v = (double)s[k];
      if (isfinite(s[k])) {
        m[0] = fmin(m[0], v);
        m[1] = fmin(m[1], -v);
        const double dv = v - (double)c0;
        m[2] += dv;
        m[3] += dv * dv;
      } else {
        m[0] = -INFINITY;
      }
    }
  rd.template run<4, 2>(m);
  if (!isfinite(m[0])) return fail_reweight(a, PHI4_ENONFINITE);
  const double smin = m[0], smax = -m[1];
  const double mean = m[2] / n, var = fmax(m[3] / n - mean * mean, 0.0);
  const double room = 1.0 - beta;
  const double target = ess_frac * n;
  SegSolver<SEG> sv{s, cnt, n, smin, smax, rd, rf};
  Sums e;
  int evals = 0;
  const double dbeta = sv.solve(room, target, var, e, evals);
  if (!(dbeta > 0.0)) return fail_reweight(a, PHI4_ENONFINITE);
  const double new_beta = dbeta == room ? 1.0 : fmin(1.0, beta + dbeta);
  const double dlogz = -dbeta * smin + log(e.a) - log((double)n);
  const double ess = e.a * e.a / e.b;
  // weights of this thread's segment; the largest is exactly 1
  const double lmax = -dbeta * smin;
  double w[SEG];
#pragma unroll
  for (int k = 0; k < SEG; ++k) {
    w[k] = k < cnt ? tempered_weight(dbeta, s[k], lmax) : 0.0;
    if ((k & 7) == 7) __builtin_amdgcn_sched_barrier(0);
  }
  if (a.w && !a.st) {
#pragma unroll
    for (int k = 0; k < SEG; ++k)
      if (k < cnt) a.w[i0 + k] = w[k];
  }
  if (a.do_resample) {
    const uint32_t U = word0(0u, 0u, counter3((uint32_t)level, PHI4_RESAMPLE), a.seed, a.run);
    resample_seg<SEG>(w, cnt, i0, n, 1.0, U, a.anc, shu);
  }
  finish_reweight(a, level, dbeta, new_beta, dlogz, ess, evals);
}

// Float64 Newton of the global path: one exact pass per evaluation.
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

template <class SGet>
__device__ double solve_dbeta(SGet sget, int n, double room, double target, double smin,
                              double ssum, double ssq, double* sh, Sums& e, int& evals) {
  e = ess_sums(sget, n, room, smin, sh);
  evals = 1;
  if (e.a * e.a / e.b >= target) return room;
  double lo = 0.0, hi = room;
  const double mean = ssum / n, var = fmax(ssq / n - mean * mean, 0.0);
  double x = var > 0.0 ? sqrt(fmax(n / target - 1.0, 0.0) / var) : 0.5 * room;
  if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    e = ess_sums(sget, n, x, smin, sh);
    ++evals;
    double g, gd;
    ess_newton(e, target, g, gd);
    if (g >= 0.0) lo = x; else hi = x;
    if (hi - lo <= 1e-13 * hi) break;
    const double step = g / gd;
    double xn = x - step;
    const double tol = 1e-14 * x;
    if (fabs(step) < tol) xn = g >= 0.0 ? x + tol : x - tol;  // step across the root
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    x = xn;
  }
  if (lo > 0.0 && lo != x) {
    e = ess_sums(sget, n, lo, smin, sh);
    ++evals;
  }
  return lo;
}

// Large-N variant: actions and weights stay in global memory.
__device__ __forceinline__ void reweight_global_impl(const ReweightArgs& a) {
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
template <int SEG>
__global__ __launch_bounds__(kRT) void resample_kernel(const double* w, int n, uint32_t U,
                                                       unsigned long long* cdf, int32_t* marks,
                                                       int32_t* anc, int32_t* status) {
  __shared__ double shd[kNW];
  __shared__ unsigned long long shu[kNW];
  __shared__ int shi[kNW];
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
  if (n <= kRT * SEG) {
    const int per = (n + kRT - 1) / kRT;
    const int i0 = min(n, (int)threadIdx.x * per);
    const int cnt = max(0, min(n, i0 + per) - i0);
    double wv[SEG];
#pragma unroll
    for (int k = 0; k < SEG; ++k) {
      const double v = w[min(i0 + k, n - 1)];   // valid address, masked
      wv[k] = k < cnt ? v : 0.0;
    }
    resample_seg<SEG>(wv, cnt, i0, n, wmax, U, anc, shu);
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

// Level, beta and error of many SMC runs gathered into one array (the
// status word of a batched launch).
__global__ __launch_bounds__(64) void batch_status_kernel(const SmcState* const* __restrict__ st,
                                                          int runs,
                                                          BatchStatus* __restrict__ out) {
  const int r = blockIdx.x * 64 + threadIdx.x;
  if (r >= runs) return;
  const SmcState* s = st[r];
  BatchStatus b;
  b.beta = s->beta;
  b.level = s->level;
  b.done = s->done;
  b.err = s->err;
  b.pad = 0;
  out[r] = b;
}

// Thread 0 wrote every field of the run state, so it can publish the state
// to the host mirror right after the reweight without a barrier.
__device__ __forceinline__ void publish_state(const ReweightArgs& a) {
  if (a.mirror && a.st && threadIdx.x == 0) *a.mirror = *a.st;
}

template <int SEG>
__global__ __launch_bounds__(kRT) void reweight_kernel(ReweightArgs a) {
  reweight_impl<SEG>(a);
  publish_state(a);
}

__global__ __launch_bounds__(kRT) void reweight_global_kernel(ReweightArgs a) {
  reweight_global_impl(a);
  publish_state(a);
}

}  // namespace

void launch_reweight(const ReweightArgs& a, hipStream_t s) {
  if (a.n <= kRT * 8)
    reweight_kernel<8><<<1, kRT, 0, s>>>(a);
  else if (a.n <= kRT * 16)
    reweight_kernel<16><<<1, kRT, 0, s>>>(a);
  else if (a.n <= kRegN)
    reweight_kernel<kSeg><<<1, kRT, 0, s>>>(a);
  else
    reweight_global_kernel<<<1, kRT, 0, s>>>(a);
}

void launch_resample_weights(const double* w, int n, uint32_t U, unsigned long long* cdf,
                             int32_t* marks, int32_t* anc, int32_t* status, hipStream_t s) {
  if (n <= 0) return;
  if (n <= kRT * 8)
    resample_kernel<8><<<1, kRT, 0, s>>>(w, n, U, cdf, marks, anc, status);
  else
    resample_kernel<kSeg><<<1, kRT, 0, s>>>(w, n, U, cdf, marks, anc, status);
}

void launch_smc_state_init(SmcState* st, double eps0, double acc_target, double ess_frac,
                           hipStream_t s) {
  smc_state_init_kernel<<<1, 1, 0, s>>>(st, eps0, acc_target, ess_frac);
}

void launch_ns_state_init(NsState* st, double eps0, double acc_target, hipStream_t s) {
  ns_state_init_kernel<<<1, 1, 0, s>>>(st, eps0, acc_target);
}

void launch_batch_status(const SmcState* const* st, int runs, BatchStatus* out, hipStream_t s) {
  if (runs > 0) batch_status_kernel<<<(runs + 63) / 64, 64, 0, s>>>(st, runs, out);
}

void launch_mean_abs(const float* absM, int n, double* out, const int32_t* done, hipStream_t s) {
  (void)done;
  if (n <= 0) return;
  mean_abs_kernel<<<1, kRT, 0, s>>>(absM, n, out);
}

}  // namespace phi4
