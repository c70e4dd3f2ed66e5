// Nested-sampling iteration kernels (Sec. 2 (iv); App. A: delete a fraction
// of the live points, refill under the likelihood constraint).
//
// select: termination test, deletion of the k lowest-likelihood points
//   (log L = -S; ascending (log L, row) by a bitonic sort of 64-bit keys in
//   LDS), float64 bookkeeping of the prior volume (expected log shrinkage
//   sum_{m<=j} 1/(n-m) for the j-th deletion) and the evidence
//   (w_j = L_j (X_{j-1} - X_j), log-sum-exp accumulation), the information
//   H and the posterior-weighted |M|; it also lists the rows to refill and
//   the survivors in deletion order.
// seed copy: new point j copies survivor floor(U_j (n-k) / 2^32) (U_j the
//   NS_PICK word of j).
// The covariance of the survivors and the constrained sweep reuse the SMC
// kernels with row lists.
#include "common.hpp"

namespace phi4 {

namespace {

constexpr int kNT = 1024;
constexpr int kMaxLive = 8192;

__device__ __forceinline__ uint32_t order_bits(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ double block_excl_scan_d(double v, double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  double off = 0.0;
  for (int w = 0; w < wid; ++w) off += sh[w];
  return off + x - v;
}

__device__ __forceinline__ double lse2(double a, double b) {
  const double m = fmax(a, b);
  if (m == -INFINITY) return -INFINITY;
  return m + log(exp(a - m) + exp(b - m));
}

// Adds the live points (each with weight X / n * L_i) and sets done.
__device__ void ns_add_live(const NsArgs& a, double* shd) {
  NsState* st = a.st;
  const int n = a.n;
  const double logX = st->logX, logZ0 = st->logZ;
  double lmax = -INFINITY, mmax = -INFINITY;
  for (int i = threadIdx.x; i < n; i += kNT) {
    const double lw = logX - log((double)n) - (double)a.S[i];
    lmax = fmax(lmax, lw);
    mmax = fmax(mmax, lw + log((double)a.absM[i]));
  }
  lmax = block_reduce<kMax, 16>(lmax, shd);
  mmax = block_reduce<kMax, 16>(mmax, shd);
  double sw = 0.0, sm = 0.0;
  for (int i = threadIdx.x; i < n; i += kNT) {
    const double lw = logX - log((double)n) - (double)a.S[i];
    sw += exp(lw - lmax);
    if (mmax > -INFINITY) sm += exp(lw + log((double)a.absM[i]) - mmax);
  }
  sw = block_reduce<kSum, 16>(sw, shd);
  sm = block_reduce<kSum, 16>(sm, shd);
  const double lz_live = lmax + log(sw);
  const double logZ = lse2(logZ0, lz_live);
  double hs = 0.0;
  for (int i = threadIdx.x; i < n; i += kNT) {
    const double lw = logX - log((double)n) - (double)a.S[i];
    hs += exp(lw - logZ) * (-(double)a.S[i]);
  }
  hs = block_reduce<kSum, 16>(hs, shd);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double hsum = (logZ0 > -INFINITY ? st->hsum * exp(logZ0 - logZ) : 0.0) + hs;
    st->hsum = hsum;
    st->logZ = logZ;
    st->H = hsum - logZ;
    if (mmax > -INFINITY) st->logmz = lse2(st->logmz, mmax + log(sm));
    st->done = 1;
  }
}

__global__ __launch_bounds__(kNT) void ns_select_kernel(NsArgs a) {
  __shared__ unsigned long long keys[kMaxLive];
  __shared__ double shd[kNT / 64];
  NsState* st = a.st;
  if (st->done || st->err) return;
  const int n = a.n, k = a.k;
  // ---- step-size adaptation of the previous refill
  __syncthreads();
  if (threadIdx.x == 0 && st->prop > 0) {
    const double abar = (double)st->acc / (double)st->prop;
    st->last_acc = abar;
    const double e = st->eps * exp(abar - st->acc_target);
    st->eps = fmin(fmax(e, st->eps0 / 100.0), 10.0 * st->eps0);
    st->acc = 0;
    st->prop = 0;
  }
  // ---- termination test: live evidence fraction
  if (st->logZ > -INFINITY) {
    double lmax = -INFINITY;
    for (int i = threadIdx.x; i < n; i += kNT) lmax = fmax(lmax, -(double)a.S[i]);
    lmax = block_reduce<kMax, 16>(lmax, shd);
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kNT) s += exp(-(double)a.S[i] - lmax);
    s = block_reduce<kSum, 16>(s, shd);
    const double live = st->logX + lmax + log(s) - log((double)n);
    if (live - st->logZ < log(a.term_frac)) {
      ns_add_live(a, shd);
      return;
    }
  }
  // ---- deletion order: ascending (log L, row)
  int npad = 1;
  while (npad < n) npad <<= 1;
  for (int i = threadIdx.x; i < npad; i += kNT)
    keys[i] = i < n ? ((unsigned long long)order_bits(-a.S[i]) << 32) | (unsigned)i : ~0ull;
  __syncthreads();
  for (int size = 2; size <= npad; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < npad; i += kNT) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const unsigned long long x = keys[i], y = keys[j];
          if ((x > y) == up) {
            keys[i] = y;
            keys[j] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  // ---- bookkeeping of the k deletions
  const int per = (k + kNT - 1) / kNT;
  const int j0 = min(k, (int)threadIdx.x * per), j1 = min(k, j0 + per);
  double loc = 0.0;
  for (int j = j0; j < j1; ++j) loc += 1.0 / (double)(n - j);
  double run = block_excl_scan_d(loc, shd);
  const double logX = st->logX, logZ0 = st->logZ;
  double* xs = a.scratch;              // log X_j
  for (int j = j0; j < j1; ++j) {
    run += 1.0 / (double)(n - j);
    xs[j] = logX - run;
  }
  __syncthreads();
  double lmax = -INFINITY, mmax = -INFINITY;
  double* lw = a.scratch + k;          // log w_j
  for (int j = threadIdx.x; j < k; j += kNT) {
    const int r = (int)(keys[j] & 0xFFFFFFFFull);
    const double prev = j ? xs[j - 1] : logX;
    const double v = -(double)a.S[r] + prev + log(-expm1(xs[j] - prev));
    lw[j] = v;
    lmax = fmax(lmax, v);
    mmax = fmax(mmax, v + log((double)a.absM[r]));
  }
  lmax = block_reduce<kMax, 16>(lmax, shd);
  mmax = block_reduce<kMax, 16>(mmax, shd);
  double sw = 0.0, sm = 0.0;
  for (int j = threadIdx.x; j < k; j += kNT) {
    const int r = (int)(keys[j] & 0xFFFFFFFFull);
    sw += exp(lw[j] - lmax);
    if (mmax > -INFINITY) sm += exp(lw[j] + log((double)a.absM[r]) - mmax);
  }
  sw = block_reduce<kSum, 16>(sw, shd);
  sm = block_reduce<kSum, 16>(sm, shd);
  const double logZ = lse2(logZ0, lmax + log(sw));
  double hs = 0.0;
  for (int j = threadIdx.x; j < k; j += kNT) {
    const int r = (int)(keys[j] & 0xFFFFFFFFull);
    hs += exp(lw[j] - logZ) * (-(double)a.S[r]);
  }
  hs = block_reduce<kSum, 16>(hs, shd);
  // ---- row lists
  for (int j = threadIdx.x; j < n; j += kNT) {
    const int r = (int)(keys[j] & 0xFFFFFFFFull);
    if (j < k) a.dead_rows[j] = r;
    else a.surv_rows[j - k] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st->hsum = (logZ0 > -INFINITY ? st->hsum * exp(logZ0 - logZ) : 0.0) + hs;
    st->logZ = logZ;
    st->H = st->hsum - logZ;
    if (mmax > -INFINITY) st->logmz = lse2(st->logmz, mmax + log(sm));
    st->logX = xs[k - 1];
    st->s_star = a.S[(int)(keys[k - 1] & 0xFFFFFFFFull)];
    st->iter += 1;
  }
}

__global__ __launch_bounds__(256) void ns_seed_copy_kernel(NsArgs a) {
  NsState* st = a.st;
  if (st->done || st->err) return;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= a.k) return;
  const uint32_t w = word0((uint32_t)j, 0u, counter3((uint32_t)st->iter, PHI4_NS_PICK), a.seed,
                           a.run);
  const int m = (int)(((unsigned long long)w * (unsigned long long)(a.n - a.k)) >> 32);
  const int src = a.surv_rows[m], dst = a.dead_rows[j];
  const int d = a.d;
  for (int x = threadIdx.x & 63; x < d; x += 64) a.phi[(size_t)dst * d + x] = a.phi[(size_t)src * d + x];
  if ((threadIdx.x & 63) == 0) {
    a.S[dst] = a.S[src];
    a.absM[dst] = a.absM[src];
  }
}

}  // namespace

void launch_ns_select(const NsArgs& a, hipStream_t s) {
  ns_select_kernel<<<1, kNT, 0, s>>>(a);
}

void launch_ns_seed_copy(const NsArgs& a, hipStream_t s) {
  if (a.k <= 0) return;
  ns_seed_copy_kernel<<<(a.k + 3) / 4, 256, 0, s>>>(a);
}

}  // namespace phi4
