// Particle covariance and its jittered float64 Cholesky factor (App. A:
// the single data-driven covariance that preconditions every inner kernel).
//
// Covariance: the sample covariance with divisor N - 1 of the rows given,
// accumulated on the matrix cores as float32 products of rows shifted by the
// first row c (one wave per 16 x 16 output block and particle chunk),
// combined in float64 as
//   Sigma = (sum (phi - c)(phi - c)^T - m1 m1^T / N) / (N - 1),
//   m1 = sum (phi - c),
// which equals the centred form exactly in real arithmetic and keeps
// float32 products at the scale of the spread.
//
// Factor: tau = 1e-10 tr(Sigma) / d is added to the diagonal and multiplied
// by 100 after each failed factorisation (at most five retries).  For
// d <= 64 one workgroup forms Sigma from the chunk sums and factorises it
// right-looking in 16-column panels (cov_factor_kernel); larger d is
// factorised right-looking in 64-column panels: the diagonal block in LDS in
// outer-product form, the panel below it solved row by row and the trailing
// matrix updated from LDS.  The scaled factor is emitted
// transposed in float32 for the mutation kernel: Bt[k*d + c] = eps * L[c][k].
#include <utility>

#include "common.hpp"

namespace phi4 {

namespace {

constexpr int kTile = 64;
constexpr int kFT = 1024;    // threads of the large-d factor kernel
constexpr int kPanelRows = 128;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxChunks = 32;   // particle chunks per covariance block (at most)

__device__ __forceinline__ int blk_of(int bi, int bj) { return bi * (bi + 1) / 2 + bj; }

// One wave: the 16 x 16 block (bi, bj), bi >= bj, of sum_k (x_k - c)(x_k - c)^T
// over the particles of one chunk, on MFMA (16x16x4, four particles per
// instruction); diagonal blocks also sum the shifted rows (first moments).
__global__ __launch_bounds__(64) void cov_partial_kernel(const float* __restrict__ phi,
                                                         const int32_t* __restrict__ rows,
                                                         CovPlan p, float* __restrict__ part,
                                                         const int32_t* __restrict__ done) {
  if (done && *done) return;
  const int blk = blockIdx.x, chunk = blockIdx.y;
  int bi = 0;
  while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
  const int bj = blk - bi * (bi + 1) / 2;
  const int lane = threadIdx.x, i = lane & 15, g = lane >> 4;
  const int d = p.d;
  const int sr = 16 * bi + i, sc = 16 * bj + i;   // sites of this lane's A and B values
  const bool vr = sr < d, vc = sc < d;
  const size_t row0 = (size_t)(rows ? rows[0] : 0) * d;
  // loads always read a valid address and are masked afterwards, so that the
  // compiler issues them without branches
  const int src_ = min(sr, d - 1), scc_ = min(sc, d - 1);
  const float cr0 = phi[row0 + src_], cc0 = phi[row0 + scc_];
  const float cr = vr ? cr0 : 0.f, cc = vc ? cc0 : 0.f;
  const int k_begin = chunk * p.chunk, k_end = min(p.n, k_begin + p.chunk);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  float m1 = 0.f;
  // 32 MFMA steps (128 particles) per batch: the row indices of a batch, then
  // all its field loads, are issued before the matrix instructions consume
  // them (two memory round trips per batch)
  constexpr int kU = 32;
  for (int k0 = k_begin; k0 < k_end; k0 += 4 * kU) {
    int rk[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = k0 + 4 * u + g;
      const int kc = min(k, k_end - 1);
      const int r = rows ? rows[kc] : kc;
      rk[u] = k < k_end ? r : -1;
    }
    float av[kU], bv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const size_t rb = (size_t)(rk[u] < 0 ? 0 : rk[u]) * d;
      const float va = phi[rb + src_], vb = phi[rb + scc_];
      av[u] = (rk[u] >= 0 && vr) ? va : cr;
      bv[u] = (rk[u] >= 0 && vc) ? vb : cc;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const float a = av[u] - cr, b = bv[u] - cc;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
      m1 += a;
    }
  }
  const CovWork w = cov_work(part, p);
  float* out = w.part + ((size_t)chunk * p.blocks + blk) * 256;
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) out[(4 * g + jj) * 16 + i] = acc[jj];
  if (bi == bj) {
    m1 += __shfl_xor(m1, 16, 64);
    m1 += __shfl_xor(m1, 32, 64);
    if (g == 0) w.part1[(size_t)chunk * p.nb * 16 + sr] = m1;
  }
}

// Sums each block's partials over the chunks in chunk order (float64) into
// fin / fin1.  A kernel of its own: summing in the last-arriving chunk
// workgroup needs an agent-scope fence per workgroup, which on a chip of
// several L2 caches costs more than this launch.
__global__ __launch_bounds__(64) void cov_sum_kernel(CovPlan p, float* __restrict__ part,
                                                     const int32_t* __restrict__ done) {
  if (done && *done) return;
  const int blk = blockIdx.x, lane = threadIdx.x;
  int bi = 0;
  while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
  const int bj = blk - bi * (bi + 1) / 2;
  const CovWork w = cov_work(part, p);
  {
    // every partial of the block in flight at once (one round trip)
    float x[4][kMaxChunks];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int c = 0; c < kMaxChunks; ++c)
        x[t][c] = w.part[((size_t)min(c, p.chunks - 1) * p.blocks + blk) * 256 + lane + 64 * t];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      double m2 = 0.0;
#pragma unroll
      for (int c = 0; c < kMaxChunks; ++c) m2 += c < p.chunks ? (double)x[t][c] : 0.0;
      w.fin[(size_t)blk * 256 + lane + 64 * t] = m2;
    }
  }
  if (bi == bj && lane < 16) {
    float x[kMaxChunks];
#pragma unroll
    for (int c = 0; c < kMaxChunks; ++c)
      x[c] = w.part1[(size_t)min(c, p.chunks - 1) * p.nb * 16 + 16 * bi + lane];
    double m = 0.0;
#pragma unroll
    for (int c = 0; c < kMaxChunks; ++c) m += c < p.chunks ? (double)x[c] : 0.0;
    w.fin1[16 * bi + lane] = m;
  }
}

__global__ void cov_init_kernel(int32_t* cnt, int blocks) {
  for (int i = threadIdx.x; i < blocks; i += blockDim.x) cnt[i] = 0;
}

// Sigma from the chunk sums: one thread per lower entry (i, j),
// Sigma = (M2 - m1_i m1_j / N) / (N - 1), written symmetric.
__global__ __launch_bounds__(256) void cov_reduce_kernel(const float* __restrict__ part, CovPlan p,
                                                        double* __restrict__ sigma,
                                                        const int32_t* __restrict__ done) {
  if (done && *done) return;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= p.blocks * 256) return;
  const int blk = e >> 8, r = (e >> 4) & 15, cc = e & 15;
  int bi = 0;
  while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
  const int bj = blk - bi * (bi + 1) / 2;
  const int i = 16 * bi + r, j = 16 * bj + cc;
  const int d = p.d;
  if (i >= d || j >= d || j > i) return;
  const CovWork w = cov_work(part, p);
  const double v = (w.fin[e] - w.fin1[i] * w.fin1[j] / p.n) / (p.n - 1);
  sigma[(size_t)i * d + j] = v;
  sigma[(size_t)j * d + i] = v;
}

// Covariance entry (i, j), i >= j, from the partials: float64 sums over the
// chunks in a fixed order.
__device__ __forceinline__ const float* partial_entry(const float* part, const CovPlan& p, int i,
                                                      int j) {
  return part + (size_t)blk_of(i >> 4, j >> 4) * 256 + (i & 15) * 16 + (j & 15);
}

// Outer-product Cholesky of the nb x nb block in LDS (lower part used):
// after the call D[i][j] (j <= i) holds L[i][j].  Returns false if a pivot
// is not positive and finite (uniform across the block).
__device__ bool chol_block(double (*D)[kTile + 1], int nb, int* flag) {
  // thread -> fixed (i, j) slots of the nb x nb block, lower part only
  for (int k = 0; k < nb; ++k) {
    const double dkk = D[k][k];
    if (!(dkk > 0.0) || isinf(dkk)) return false;
    const double inv = 1.0 / dkk;
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
      const int i = e / nb, j = e - (e / nb) * nb;
      if (j > k && j <= i) D[i][j] -= D[i][k] * D[j][k] * inv;
    }
    __syncthreads();
  }
  // scale: L[i][k] = D[i][k] / sqrt(D[k][k])
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int i = e / nb, k = e % nb;
    if (k < i) D[i][k] /= sqrt(D[k][k]);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nb; k += blockDim.x) D[k][k] = sqrt(D[k][k]);
  __syncthreads();
  (void)flag;
  return true;
}

// Right-looking blocked Cholesky of A (d x d row-major, lower used).
__device__ bool chol_full(double* __restrict__ A, int d, double (*D)[kTile + 1],
                          double (*P)[kTile + 1], int* flag) {
  for (int kb = 0; kb < d; kb += kTile) {
    const int nb = min(kTile, d - kb);
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
      const int i = e / nb, j = e % nb;
      D[i][j] = j <= i ? A[(size_t)(kb + i) * d + kb + j] : 0.0;
    }
    __syncthreads();
    if (!chol_block(D, nb, flag)) return false;
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
      const int i = e / nb, j = e % nb;
      if (j <= i) A[(size_t)(kb + i) * d + kb + j] = D[i][j];
    }
    const int rest = d - kb - nb;
    for (int pr = 0; pr < rest; pr += kPanelRows) {
      const int nr = min(kPanelRows, rest - pr);
      const int rbase = kb + nb + pr;
      __syncthreads();
      for (int e = threadIdx.x; e < nr * nb; e += blockDim.x) {
        const int i = e / nb, j = e % nb;
        P[i][j] = A[(size_t)(rbase + i) * d + kb + j];
      }
      __syncthreads();
      // panel solve: X L11^T = A21, one row per thread
      if ((int)threadIdx.x < nr) {
        const int i = threadIdx.x;
        for (int m = 0; m < nb; ++m) {
          double s = P[i][m];
          for (int l = 0; l < m; ++l) s -= P[i][l] * D[m][l];
          P[i][m] = s / D[m][m];
        }
      }
      __syncthreads();
      for (int e = threadIdx.x; e < nr * nb; e += blockDim.x) {
        const int i = e / nb, j = e % nb;
        A[(size_t)(rbase + i) * d + kb + j] = P[i][j];
      }
    }
    __syncthreads();
    // trailing update A22 -= X X^T (lower part), X read back from A
    for (int e = threadIdx.x; e < rest * rest; e += blockDim.x) {
      const int i = e / rest, j = e % rest;
      if (j > i) continue;
      const double* xi = A + (size_t)(kb + nb + i) * d + kb;
      const double* xj = A + (size_t)(kb + nb + j) * d + kb;
      double s = 0.0;
      for (int m = 0; m < nb; ++m) s += xi[m] * xj[m];
      A[(size_t)(kb + nb + i) * d + kb + nb + j] -= s;
    }
    __syncthreads();
  }
  return true;
}

__global__ __launch_bounds__(kFT) void factor_kernel(FactorArgs a) {
  if (a.done && *a.done) return;
  // behind the blocked factor this kernel only continues the jitter
  // escalation after every attempt that ran there failed
  if (a.bstatus && a.bstatus[kJitterAttempts] == 0) return;
  const int first = a.bstatus ? a.attempts : 0;
  __shared__ double D[kTile][kTile + 1];
  __shared__ double P[kPanelRows][kTile + 1];
  __shared__ double shd[kFT / 64];
  __shared__ int flag;
  const CovPlan& p = a.plan;
  const int d = p.d;
  double* sig = a.sigma_out;  // the covariance (kept for retries)
  // ---- covariance (already reduced into sig, or given)
  if (a.sigma_in) {
    for (int e = threadIdx.x; e < d * d; e += kFT) sig[e] = a.sigma_in[e];
  }
  __syncthreads();
  if (a.cov_only) return;
  double tr = 0.0;
  for (int i = threadIdx.x; i < d; i += kFT) tr += sig[(size_t)i * d + i];
  tr = block_reduce<kSum, 16>(tr, shd);
  double tau = 1e-10 * tr / d;
  for (int q = 0; q < first; ++q) tau *= 100.0;
  bool ok = false;
  for (int attempt = first; attempt < kJitterAttempts && !ok; ++attempt) {
    if (attempt > first) tau *= 100.0;
    for (int e = threadIdx.x; e < d * d; e += kFT) {
      const int i = e / d, j = e % d;
      a.A[e] = sig[e] + (i == j ? tau : 0.0);
    }
    __syncthreads();
    ok = chol_full(a.A, d, D, P, &flag);
    __syncthreads();
  }
  if (!ok) {
    if (threadIdx.x == 0 && a.err_out) *a.err_out = PHI4_ECHOL;
    return;
  }
  // zero the strict upper part and emit the scaled transposed factor
  for (int e = threadIdx.x; e < d * d; e += kFT) {
    const int i = e / d, j = e % d;
    if (j > i) a.A[e] = 0.0;
  }
  if (a.Bt) {
    const double eps = *a.eps_ptr;
    for (int e = threadIdx.x; e < d * d; e += kFT) {
      const int k = e / d, c = e % d;
      a.Bt[(size_t)k * a.ldb + c] = k <= c ? (float)(eps * a.A[(size_t)c * d + k]) : 0.f;
    }
  }
  if (threadIdx.x == 0 && a.tau_out) *a.tau_out = tau;
}

constexpr int kSmallD = 64;

// One-wave Cholesky for d <= D (D = 16, 32 or 64): lane i keeps row i of the
// matrix in registers, padded to D x D with the identity (the padding stays
// the identity and factors to itself).  Right-looking outer-product form: at
// step k every lane publishes its entry of column k through LDS, and lane i
// applies D[i][j] -= (D[i][k] / D[k][k]) D[j][k] for j > k, then keeps
// L[i][k] = D[i][k] / sqrt(D[k][k]) (sqrt(D[k][k]) on the diagonal, 0 above
// it).  Column k + 1 is updated and published first so that its LDS round
// trip overlaps the rest of step k.  Entries above the diagonal are carried
// along unused until their own step zeroes them.
// 1 / p in float64: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double recip_f64(double p) {
  double r = __builtin_amdgcn_rcp(p);
  double e = fma(-p, r, 1.0);
  r = fma(r, e, r);
  e = fma(-p, r, 1.0);
  return fma(r, e, r);
}

// ------------------------------------------------ fused small-d kernel

constexpr int kCF = 512;   // threads of the fused covariance + factor kernel

// Orders LDS traffic among the lanes of one wave (its LDS operations are
// processed in order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Step K of a 16-column panel sweep by one wave: lane i holds D[i][c0 + q]
// in v[q], rp = 1 / D[c0+K][c0+K] and cn[j] = D[c0+j][c0+K] for j >= K + 2
// (read from LDS one step ahead).  Column K + 1 is updated first, published
// through LDS and read back at once for the next step, and its pivot comes
// from its lane's register, so the LDS round trip and the next reciprocal
// overlap the remaining updates of this step.
template <int K>
__device__ __forceinline__ void panel_step(double (&v)[16], double (&cn)[16], double* col, int i,
                                           int c0, double& rp, double& pown, bool& bad) {
  const double f = v[K] * rp;
  double nx[16];
  if constexpr (K + 1 < 16) {
    v[K + 1] = fma(-f, readlane64(v[K], c0 + K + 1), v[K + 1]);
    col[i] = v[K + 1];                         // publish column c0 + K + 1
#pragma unroll
    for (int j = K + 3; j < 16; ++j) nx[j] = col[c0 + j];   // in order after the write
    pown = i == c0 + K + 1 ? v[K + 1] : pown;  // its pivot's lane keeps it
    const double pn = readlane64(v[K + 1], c0 + K + 1);
    bad |= !(pn > 0.0) | isinf(pn);
    rp = recip_f64(pn);
  }
#pragma unroll
  for (int j = K + 2; j < 16; ++j) v[j] = fma(-f, cn[j], v[j]);
#pragma unroll
  for (int j = K + 3; j < 16; ++j) cn[j] = nx[j];
  __builtin_amdgcn_sched_barrier(0);   // keep the next step's uses after this step's work
}

template <int... K>
__device__ __forceinline__ void panel_sweep(double (&v)[16], double (&cn)[16], double* col,
                                            int i, int c0, double& rp, double& pown, bool& bad,
                                            std::integer_sequence<int, K...>) {
  (panel_step<K>(v, cn, col, i, c0, rp, pown, bad), ...);
}

// Right-looking Cholesky of the D x D matrix in LDS (lower part in, L out;
// entries above the diagonal are scratch), D = 16, 32 or 64, by 512
// threads: wave 0 sweeps each 16-column panel in registers (lane = row,
// outer-product steps, columns broadcast through LDS one step ahead, pivots
// read from their lanes' registers), then the waves apply the rank-16
// update of the trailing lower triangle on FP64 MFMA, one 16 x 16 tile
// each.  Returns false (uniformly) if a pivot is not positive and finite.
template <int D>
__device__ bool chol_lds(double (*M)[D + 1], double* col, double* rs, int* flag) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) *flag = 0;
  __syncthreads();
    for (int c0 = 0; c0 < D; c0 += 16) {
      if (wv == 0) {
        const int ir = min(lane, D - 1);        // lanes beyond D mirror row D - 1, unused
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = M[ir][c0 + q];
        double cn[16];
        col[lane] = v[0];
#pragma unroll
        for (int j = 2; j < 16; ++j) cn[j] = col[c0 + j];
        const double p0 = readlane64(v[0], c0);
        bool bad = !(p0 > 0.0) | isinf(p0);
        double rp = recip_f64(p0);
        double pown = lane == c0 ? v[0] : 1.0;
        panel_sweep(v, cn, col, lane, c0, rp, pown, bad, std::make_integer_sequence<int, 16>{});
        // L[i][c0+q] = D[i][c0+q] / sqrt(pivot q) below the diagonal
        const double sq = sqrt(pown);
        if (lane >= c0 && lane < c0 + 16) rs[lane] = 1.0 / sq;
        wave_sync();
        if (lane >= c0 && lane < D) {
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const int j = c0 + q;
            if (lane > j) M[lane][j] = v[q] * rs[j];
            else if (lane == j) M[lane][j] = sq;
          }
        }
        if (bad && lane == 0) *flag = 1;
      }
      __syncthreads();
      if (*flag) break;
      // rank-16 update of the trailing lower triangle: tile (I, J), J <= I,
      // of 16 x 16 gets -= L[I rows][panel] L[J rows][panel]^T (FP64 MFMA,
      // K = 4 per instruction; operand lane p + 16k holds A[p][k] / B[k][p],
      // result item r of lane (p, g) is row g + 4r, column p)
      {
        const int t0 = c0 + 16, nt = (D - t0) / 16;
        int I = 0, J = wv;
        while (J > I) J -= ++I;                 // wave wv -> tile (I, J) in row order
        if (I < nt) {
          const int pl = lane & 15, gl = lane >> 4;
          const int r0 = t0 + 16 * I, s0 = t0 + 16 * J;
          f64x4 acc;
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[r] = M[r0 + gl + 4 * r][s0 + pl];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const double av = -M[r0 + pl][c0 + 4 * kk + gl];   // A[i][k]: row i = pl
            const double bv = M[s0 + pl][c0 + 4 * kk + gl];    // B[k][j]: column j = pl
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) M[r0 + gl + 4 * r][s0 + pl] = acc[r];
        }
      }
      __syncthreads();
    }
  const bool ok = *flag == 0;
  __syncthreads();
  return ok;
}

// Covariance from the chunk sums and its jittered Cholesky factor in one
// workgroup, for d <= D (D = 16, 32, 64; the matrix is padded to D x D with
// the identity): Sigma = (M2 - m1_i m1_j / N) / (N - 1) into LDS (and
// sigma_out).  The factor is right-looking in 16-column panels: wave 0
// sweeps a panel in registers (lane = row, outer-product steps, columns
// broadcast through LDS one step ahead, pivots read from their lanes'
// registers), then the waves
// apply the rank-16 update of the trailing lower triangle on FP64 MFMA,
// one 16 x 16 tile each.
template <int D>
__global__ __launch_bounds__(kCF) void cov_factor_kernel(FactorArgs a) {
  if (a.done && *a.done) return;
  __shared__ double M[D][D + 1];
  __shared__ double Ms[D][D + 1];   // the covariance again, for retries
  __shared__ double col[64];        // column broadcast of the panel sweep
  __shared__ double m1s[64];
  __shared__ double rs[64];
  __shared__ int flag;
  const CovPlan& p = a.plan;
  const int d = p.d, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double eps = a.Bt ? *a.eps_ptr : 0.0;      // issued early, used at the end
  double* sig = a.sigma_out;
  constexpr int NBD = D / 16, BLKS = NBD * (NBD + 1) / 2;
  constexpr int EPT = (BLKS * 256 + kCF - 1) / kCF;   // padded entries per thread

  // ---- covariance into M
  auto load_padded = [&](const double* src) {
    for (int e = tid; e < D * D; e += kCF) {
      const int r = e / D, c = e % D;
      const double x = src[(size_t)min(r, d - 1) * d + min(c, d - 1)];
      M[r][c] = (r < d && c < d) ? x : (r == c ? 1.0 : 0.0);
    }
  };
  if (a.sigma_in) {
    load_padded(a.sigma_in);
    __syncthreads();
    for (int e = tid; e < d * d; e += kCF) sig[e] = M[e / d][e % d];
  } else {
    const CovWork w = cov_work(a.part, p);
    if (tid < 64) m1s[tid] = w.fin1[min(tid, d - 1)];
    double x[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = min(tid + q * kCF, BLKS * 256 - 1);
      const int blk = min(e >> 8, p.blocks - 1);
      x[q] = w.fin[(size_t)blk * 256 + (e & 255)];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + q * kCF;
      if (e >= BLKS * 256) break;
      const int blk = e >> 8, r = (e >> 4) & 15, cc = e & 15;
      int bi = 0;
      while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
      const int bj = blk - bi * (bi + 1) / 2;
      const int i = 16 * bi + r, j = 16 * bj + cc;
      if (j > i) continue;                      // its mirror entry writes both
      double v;
      if (i < d && j < d) {
        v = (x[q] - m1s[i] * m1s[j] / p.n) / (p.n - 1);
        sig[(size_t)i * d + j] = v;
        sig[(size_t)j * d + i] = v;
      } else {
        v = i == j ? 1.0 : 0.0;
      }
      M[i][j] = v;
      M[j][i] = v;
    }
  }
  __syncthreads();
  for (int e = tid; e < D * D; e += kCF) Ms[e / D][e % D] = M[e / D][e % D];

  // ---- jitter: tau = 1e-10 tr / d, x100 per failed attempt (five retries)
  const double tr = wave_red<kSum>(lane < d ? M[min(lane, D - 1)][min(lane, D - 1)] : 0.0);
  double tau = 1e-10 * tr / d;
  bool ok = false;
  for (int attempt = 0; attempt < 6 && !ok; ++attempt) {
    if (attempt) {
      tau *= 100.0;
      for (int e = tid; e < D * D; e += kCF) M[e / D][e % D] = Ms[e / D][e % D];
      __syncthreads();
    }
    if (tid < d) M[tid][tid] += tau;
    __syncthreads();
    ok = chol_lds<D>(M, col, rs, &flag);
    __syncthreads();
  }
  if (!ok) {
    if (tid == 0 && a.err_out) *a.err_out = PHI4_ECHOL;
    return;
  }
  // ---- outputs: the float64 factor (zero above the diagonal) and
  // Bt[k][c] = eps L[c][k] in float32, both coalesced
  for (int e = tid; e < d * d; e += kCF) {
    const int i = e / d, j = e - i * d;
    if (a.A) a.A[e] = j <= i ? M[i][j] : 0.0;
    if (a.Bt) {
      const int k = i, c = j;   // Bt row k, column c
      a.Bt[(size_t)k * a.ldb + c] = c >= k ? (float)(eps * M[c][k]) : 0.f;
    }
  }
  if (tid == 0 && a.tau_out) *a.tau_out = tau;
}

// ------------------------------------------------------ blocked factor
//
// For d > 64: right-looking Cholesky of Sigma + tau_j I in 64-column panels,
// two kernels per stage: the panel kernel factors the 64 x 64 diagonal block
// (chol_lds) and its inverse in every workgroup and forms the panel below it
// as the product A21 L11^-T on FP64 MFMA; the rank-64 update of the trailing
// lower tiles runs on FP64 MFMA.  The jitter attempts tau_j = tau0 100^j (j < attempts) run
// side by side in gridDim.y, each on its own copy of the matrix: the
// sequence of attempts is decided by data the host never sees, and running
// them together costs one factorisation's latency instead of up to six.  A
// pivot failure sets that attempt's status and its later stages return at
// once; the emit stage takes the first attempt that succeeded, as the
// sequential rule would.  If every attempt fails and fewer than six ran, the
// single-workgroup factor_kernel continues the escalation.


__device__ inline double* attempt_matrix(double* A, double* Aspec, int j, int d) {
  return j == 0 ? A : Aspec + (size_t)(j - 1) * d * d;
}

__global__ __launch_bounds__(1024) void bf_init_kernel(const double* __restrict__ src, int d,
                                                       double* __restrict__ tau,
                                                       int32_t* __restrict__ status,
                                                       int attempts,
                                                       const int32_t* __restrict__ done) {
  if (done && *done) return;
  __shared__ double shd[16];
  double t = 0.0;
  for (int i = threadIdx.x; i < d; i += 1024) t += src[(size_t)i * d + i];
  t = block_reduce<kSum, 16>(t, shd);
  if (threadIdx.x == 0) *tau = 1e-10 * t / d;
  if (threadIdx.x < attempts) status[threadIdx.x] = 0;
  if (threadIdx.x == 0) status[kJitterAttempts] = 1;   // cleared by a successful emit
}

__device__ inline double attempt_tau(double tau0, int j) {
  double t = tau0;
  for (int q = 0; q < j; ++q) t *= 100.0;
  return t;
}

// A_j (lower part) = src + tau_j I
__global__ __launch_bounds__(256) void bf_copy_kernel(const double* __restrict__ src,
                                                      double* __restrict__ A,
                                                      double* __restrict__ Aspec, int d,
                                                      const double* __restrict__ tau,
                                                      const int32_t* __restrict__ done) {
  if (done && *done) return;
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long long)d * d) return;
  double* Aj = attempt_matrix(A, Aspec, blockIdx.y, d);
  const int i = (int)(e / d), j = (int)(e - (long long)i * d);
  if (j <= i) Aj[e] = src[e] + (i == j ? attempt_tau(*tau, blockIdx.y) : 0.0);
}

// Loads the diagonal block kb of Aj into M (padded with the identity past d)
// and factors it in LDS.  Returns false if a pivot fails (uniform).
__device__ bool diag_factor(const double* Aj, int d, int kb, double (*M)[65], double* col,
                            double* rs, int* flag) {
  const int nb = min(64, d - kb);
  for (int e = threadIdx.x; e < 64 * 64; e += kCF) {
    const int r = e >> 6, c = e & 63;
    double v = r == c ? 1.0 : 0.0;
    if (r < nb && c <= r) v = Aj[(size_t)(kb + r) * d + kb + c];
    M[r][c] = v;
  }
  __syncthreads();
  return chol_lds<64>(M, col, rs, flag);
}

// W = L^-1 of the factored block in M, by 16 x 16 blocks: the diagonal
// blocks W_bb = L_bb^-1 by forward substitution (lane 16 b + c owns column c
// of block b), then W_ij = -W_ii sum_{j <= k < i} L_ik W_kj for i > j, one
// block distance i - j at a time (every block it needs is then known).
__device__ void diag_inverse(const double (*M)[65], double (*Wl)[65], double (*Tt)[16][17]) {
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += kCF) Wl[e >> 6][e & 63] = 0.0;
  __syncthreads();
  if (tid < 64) {
    const int o = 16 * (tid >> 4), c = tid & 15;
    double w[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      double t = i == c ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) t = fma(-M[o + i][o + k], w[k], t);
      w[i] = i >= c ? t / M[o + i][o + i] : 0.0;
      Wl[o + i][o + c] = w[i];
    }
  }
  __syncthreads();
  for (int dist = 1; dist < 4; ++dist) {
    const int work = (4 - dist) * 256;
    for (int e = tid; e < work; e += kCF) {
      const int j = e >> 8, r = (e >> 4) & 15, c = e & 15, i = j + dist;
      double t = 0.0;
      for (int k = 16 * j; k < 16 * i; ++k) t = fma(M[16 * i + r][k], Wl[k][16 * j + c], t);
      Tt[j][r][c] = t;
    }
    __syncthreads();
    for (int e = tid; e < work; e += kCF) {
      const int j = e >> 8, r = (e >> 4) & 15, c = e & 15, i = j + dist;
      double t = 0.0;
#pragma unroll
      for (int m = 0; m < 16; ++m) t = fma(Wl[16 * i + r][16 * i + m], Tt[j][m][c], t);
      Wl[16 * i + r][16 * j + c] = -t;
    }
    __syncthreads();
  }
}

// Last diagonal block (no rows below it): factor in LDS and write back.
__global__ __launch_bounds__(kCF) void bf_diag_kernel(double* __restrict__ A,
                                                      double* __restrict__ Aspec, int d, int kb,
                                                      int32_t* __restrict__ status,
                                                      const int32_t* __restrict__ done) {
  const int at = blockIdx.y;
  if ((done && *done) || status[at]) return;
  double* Aj = attempt_matrix(A, Aspec, at, d);
  __shared__ double M[64][65];
  __shared__ double col[64];
  __shared__ double rs[64];
  __shared__ int flag;
  if (!diag_factor(Aj, d, kb, M, col, rs, &flag)) {
    if (threadIdx.x == 0) status[at] = 1;
    return;
  }
  const int nb = min(64, d - kb);
  for (int e = threadIdx.x; e < 64 * 64; e += kCF) {
    const int r = e >> 6, c = e & 63;
    if (r < nb && c <= r) Aj[(size_t)(kb + r) * d + kb + c] = M[r][c];
  }
}

// Stage kb with rows below it, one kernel: every workgroup factors the
// diagonal block and forms its inverse W = L11^-1 in LDS (the same
// arithmetic in each, so all agree on failure), then solves its 128 panel
// rows X = A21 L11^-T = A21 W^T on FP64 MFMA (wave v: rows 16v..16v+15 as
// four 16 x 16 tiles).  The factored block goes to Dfac (workgroup 0): the
// block itself is still being read by the other workgroups, so the trailing
// update kernel that follows copies it into place.
constexpr int kPR = 128;   // panel rows per workgroup

__global__ __launch_bounds__(kCF) void bf_panel_kernel(double* __restrict__ A,
                                                       double* __restrict__ Aspec,
                                                       double* __restrict__ Dfac, int d, int kb,
                                                       int32_t* __restrict__ status,
                                                       const int32_t* __restrict__ done) {
  const int at = blockIdx.y;
  if ((done && *done) || status[at]) return;
  double* Aj = attempt_matrix(A, Aspec, at, d);
  __shared__ double M[64][65];
  __shared__ double Wl[64][65];
  __shared__ double Tt[3][16][17];
  __shared__ double Xs[kPR][65];
  __shared__ double col[64];
  __shared__ double rs[64];
  __shared__ int flag;
  const int tid = threadIdx.x;
  const int r0 = kb + 64 + blockIdx.x * kPR;
  // panel rows first (independent of the factor), then the diagonal block
  for (int e = tid; e < kPR * 64; e += kCF) {
    const int r = e >> 6, c = e & 63;
    const double v = Aj[(size_t)min(r0 + r, d - 1) * d + kb + c];
    Xs[r][c] = r0 + r < d ? v : 0.0;
  }
  if (!diag_factor(Aj, d, kb, M, col, rs, &flag)) {
    if (tid == 0 && blockIdx.x == 0) status[at] = 1;
    return;
  }
  if (blockIdx.x == 0) {
    double* D = Dfac + (size_t)at * 4096;
    for (int e = tid; e < 64 * 64; e += kCF) D[e] = M[e >> 6][e & 63];
  }
  diag_inverse(M, Wl, Tt);
  const int lane = tid & 63, wv = tid >> 6;
  const int pl = lane & 15, gl = lane >> 4;
  f64x4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const double av = Xs[16 * wv + pl][4 * kk + gl];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const double bv = Wl[16 * b + pl][4 * kk + gl];   // W^T[k][col] = W[col][k]
      acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = r0 + 16 * wv + gl + 4 * r;
      if (row < d) Aj[(size_t)row * d + kb + 16 * b + pl] = acc[b][r];
    }
}

// Trailing update A[I][J] -= X_I X_J^T for the 64 x 64 tiles (I, J), J <= I,
// below block kb; X is the solved panel.  Wave w computes a 32 x 32 quarter
// as 2 x 2 FP64 MFMA tiles (K = 4 per instruction).
__global__ __launch_bounds__(256) void bf_syrk_kernel(double* __restrict__ A,
                                                      double* __restrict__ Aspec,
                                                      const double* __restrict__ Dfac, int d,
                                                      int kb, const int32_t* __restrict__ status,
                                                      const int32_t* __restrict__ done) {
  const int at = blockIdx.y;
  if ((done && *done) || status[at]) return;
  double* Aj = attempt_matrix(A, Aspec, at, d);
  if (blockIdx.x == 0) {
    // the stage's factored diagonal block into place (lower part; rows below
    // it exist, so the block is full)
    const double* D = Dfac + (size_t)at * 4096;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
      const int r = e >> 6, c = e & 63;
      if (c <= r) Aj[(size_t)(kb + r) * d + kb + c] = D[e];
    }
  }
  __shared__ double Xi[64][65];
  __shared__ double Xj[64][65];
  int I = 0, J = blockIdx.x;
  while (J > I) J -= ++I;                       // block -> tile (I, J) in row order
  const int t0 = kb + 64;
  const int r0 = t0 + 64 * I, s0 = t0 + 64 * J;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    const int ri = min(r0 + r, d - 1), rj = min(s0 + r, d - 1);
    const double vi = Aj[(size_t)ri * d + kb + c], vj = Aj[(size_t)rj * d + kb + c];
    Xi[r][c] = r0 + r < d ? vi : 0.0;
    Xj[r][c] = s0 + r < d ? vj : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int pl = lane & 15, gl = lane >> 4;
  const int wr = wv >> 1, wc = wv & 1;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + 32 * wr + 16 * a + gl + 4 * r, c = s0 + 32 * wc + 16 * b + pl;
        acc[a][b][r] = Aj[(size_t)min(row, d - 1) * d + min(c, d - 1)];
      }
#pragma unroll
  for (int kk = 0; kk < 16; ++kk)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const double av = -Xi[32 * wr + 16 * a + pl][4 * kk + gl];
        const double bv = Xj[32 * wc + 16 * b + pl][4 * kk + gl];
        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[a][b], 0, 0, 0);
      }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + 32 * wr + 16 * a + gl + 4 * r, c = s0 + 32 * wc + 16 * b + pl;
        if (row < d && c < d && c <= row) Aj[(size_t)row * d + c] = acc[a][b][r];
      }
}

// Outputs from the first attempt that succeeded: its factor copied into A
// with the upper part zeroed, Bt[k][c] = eps L[c][k] in float32, and tau.
__global__ __launch_bounds__(256) void bf_emit_kernel(double* __restrict__ A,
                                                      double* __restrict__ Aspec, int d,
                                                      float* __restrict__ Bt, int ldb,
                                                      const double* __restrict__ eps_ptr,
                                                      double* __restrict__ tau,
                                                      int32_t* __restrict__ status, int attempts,
                                                      int32_t* __restrict__ err_out,
                                                      const int32_t* __restrict__ done) {
  if (done && *done) return;
  int j = 0;
  while (j < attempts && status[j]) ++j;
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (j == attempts) {
    // no attempt succeeded: the escalation ends here after six attempts,
    // else the single-workgroup kernel continues it
    if (e == 0) {
      if (attempts >= kJitterAttempts) {
        status[kJitterAttempts] = 0;
        if (err_out) *err_out = PHI4_ECHOL;
      }
    }
    return;
  }
  const double* Aj = attempt_matrix(A, Aspec, j, d);
  if (e < (long long)d * d) {
    const int i = (int)(e / d), c = (int)(e - (long long)i * d);
    if (j > 0 || c > i) A[e] = c <= i ? Aj[e] : 0.0;
    if (Bt) {
      const int k = i;   // Bt row k, column c
      Bt[(size_t)k * ldb + c] = c >= k ? (float)(*eps_ptr * Aj[(size_t)c * d + k]) : 0.f;
    }
  }
  // block 0 alone touches tau and the summary word (no block reads either)
  if (e == 0) {
    *tau = attempt_tau(*tau, j);
    status[kJitterAttempts] = 0;
  }
}

}  // namespace

CovPlan cov_plan(int n, int d) {
  CovPlan p;
  p.d = d;
  p.n = n;
  p.nb = (d + 15) / 16;
  p.blocks = p.nb * (p.nb + 1) / 2;
  // about 4096 waves, at most 32 partials per block (cov_sum_kernel sums
  // them in one round trip), at least 64 particles per chunk
  int chunks = (4096 + p.blocks - 1) / p.blocks;
  if (chunks > kMaxChunks) chunks = kMaxChunks;
  const int max_chunks = (n + 63) / 64;
  if (chunks > max_chunks) chunks = max_chunks;
  if (chunks < 1) chunks = 1;
  int chunk = (n + chunks - 1) / chunks;
  chunk = (chunk + 3) / 4 * 4;
  p.chunk = chunk > 0 ? chunk : 4;
  p.chunks = (n + p.chunk - 1) / p.chunk;
  if (p.chunks < 1) p.chunks = 1;
  return p;
}

int blocked_attempts(int d) { return d <= kSmallD ? 0 : kJitterAttempts; }

size_t blocked_scratch_doubles(int d) {
  const int P = blocked_attempts(d);
  if (P == 0) return 0;
  return (size_t)(P - 1) * d * d + (size_t)P * 4096;
}

size_t cov_partial_floats(const CovPlan& p) {
  size_t o = (size_t)p.chunks * p.blocks * 256 + (size_t)p.chunks * p.nb * 16;
  o = (o + 1) & ~(size_t)1;
  return o + 2 * (size_t)p.blocks * 256 + 2 * (size_t)p.nb * 16 + (size_t)p.blocks;
}

void launch_cov_init(float* part, const CovPlan& p, hipStream_t s) {
  cov_init_kernel<<<1, 256, 0, s>>>(cov_work(part, p).cnt, p.blocks);
}

void launch_cov_partials(const float* phi, const int32_t* rows, const CovPlan& p, float* part,
                         const int32_t* done, hipStream_t s) {
  cov_partial_kernel<<<dim3(p.blocks, p.chunks), 64, 0, s>>>(phi, rows, p, part, done);
  cov_sum_kernel<<<p.blocks, 64, 0, s>>>(p, part, done);
}

void launch_factor(const FactorArgs& a, hipStream_t s) {
  const int d = a.plan.d;
  if (!a.cov_only && d <= kSmallD && a.plan.chunks <= kMaxChunks) {
    // covariance reduction and factor in one workgroup
    if (d <= 16)
      cov_factor_kernel<16><<<1, kCF, 0, s>>>(a);
    else if (d <= 32)
      cov_factor_kernel<32><<<1, kCF, 0, s>>>(a);
    else
      cov_factor_kernel<kSmallD><<<1, kCF, 0, s>>>(a);
    return;
  }
  if (!a.sigma_in) {
    const int entries = a.plan.blocks * 256;
    cov_reduce_kernel<<<(entries + 255) / 256, 256, 0, s>>>(a.part, a.plan, a.sigma_out, a.done);
  }
  if (a.cov_only) return;
  if (a.bstatus && d > kSmallD) {
    // blocked factor, the jitter attempts side by side; the single-workgroup
    // kernel below only runs if all of them failed and fewer than six ran
    const int P = a.attempts;
    const double* src = a.sigma_in ? a.sigma_in : a.sigma_out;
    const unsigned nel = (unsigned)(((long long)d * d + 255) / 256);
    bf_init_kernel<<<1, 1024, 0, s>>>(src, d, a.tau_out, a.bstatus, P, a.done);
    bf_copy_kernel<<<dim3(nel, P), 256, 0, s>>>(src, a.A, a.Aspec, d, a.tau_out, a.done);
    for (int kb = 0; kb < d; kb += 64) {
      const int below = d - kb - 64;
      if (below > 0) {
        const int nt = (below + 63) / 64;
        bf_panel_kernel<<<dim3((below + kPR - 1) / kPR, P), kCF, 0, s>>>(
            a.A, a.Aspec, a.Winv, d, kb, a.bstatus, a.done);
        bf_syrk_kernel<<<dim3(nt * (nt + 1) / 2, P), 256, 0, s>>>(a.A, a.Aspec, a.Winv, d, kb,
                                                                  a.bstatus, a.done);
      } else {
        bf_diag_kernel<<<dim3(1, P), kCF, 0, s>>>(a.A, a.Aspec, d, kb, a.bstatus, a.done);
      }
    }
    bf_emit_kernel<<<nel, 256, 0, s>>>(a.A, a.Aspec, d, a.Bt, a.ldb, a.eps_ptr, a.tau_out,
                                       a.bstatus, P, a.err_out, a.done);
    if (P >= kJitterAttempts) return;
  }
  factor_kernel<<<1, kFT, 0, s>>>(a);
}

}  // namespace phi4
