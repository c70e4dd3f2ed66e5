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
// by 100 after each failed factorisation (at most five retries).  The
// factorisation is right-looking in 64-column panels: the diagonal block is
// factorised in LDS in outer-product form (one barrier per column), the panel
// below it is solved row by row and the trailing matrix updated from LDS.
// The scaled factor is emitted transposed in float32 for the mutation
// kernel: Bt[k*d + c] = eps * L[c][k].
#include "common.hpp"

namespace phi4 {

namespace {

constexpr int kTile = 64;
constexpr int kFT = 1024;    // threads of the large-d factor kernel
constexpr int kPanelRows = 128;

typedef float f32x4 __attribute__((ext_vector_type(4)));

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
  // 8 MFMA steps (32 particles) per batch: all loads of a batch are issued
  // before the matrix instructions consume them
  constexpr int kU = 8;
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
  float* out = part + ((size_t)chunk * p.blocks + blk) * 256;
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) out[(4 * g + jj) * 16 + i] = acc[jj];
  if (bi == bj) {
    m1 += __shfl_xor(m1, 16, 64);
    m1 += __shfl_xor(m1, 32, 64);
    if (g == 0) part[(size_t)p.chunks * p.blocks * 256 + (size_t)chunk * p.nb * 16 + sr] = m1;
  }
}

// Sigma from the partials: one thread per lower entry (i, j); the chunk
// partials of M2 and of the first moments are summed in float64 in a fixed
// order, Sigma = (M2 - m1_i m1_j / N) / (N - 1), written symmetric.
constexpr int kMaxChunks = 32;
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
  const float* part1 = part + (size_t)p.chunks * p.blocks * 256;
  float v2[kMaxChunks], vi[kMaxChunks], vj[kMaxChunks];
#pragma unroll
  for (int c = 0; c < kMaxChunks; ++c) {
    const int cl = min(c, p.chunks - 1);   // valid address, masked below
    v2[c] = part[(size_t)cl * p.blocks * 256 + e];
    vi[c] = part1[(size_t)cl * p.nb * 16 + i];
    vj[c] = part1[(size_t)cl * p.nb * 16 + j];
  }
#pragma unroll
  for (int c = 0; c < kMaxChunks; ++c)
    if (c >= p.chunks) v2[c] = vi[c] = vj[c] = 0.f;
  double m2 = 0.0, mi = 0.0, mj = 0.0;
#pragma unroll
  for (int c = 0; c < kMaxChunks; ++c) {
    m2 += (double)v2[c];
    mi += (double)vi[c];
    mj += (double)vj[c];
  }
  const double v = (m2 - mi * mj / p.n) / (p.n - 1);
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
  tr = block_reduce<kSum>(tr, shd);
  double tau = 1e-10 * tr / d;
  bool ok = false;
  for (int attempt = 0; attempt < 6 && !ok; ++attempt) {
    if (attempt) tau *= 100.0;
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

// Owner-computes Cholesky for d <= 64 with 256 threads: thread t owns column
// j = t mod 64 and rows i = t / 64 + 4q (q < 16) of the matrix, in registers.
// Outer-product form without square roots during the sweep: at step k the
// current column k is broadcast through LDS (double buffered) and every
// owner applies D[i][j] -= D[i][k] D[j][k] / D[k][k] for k < j <= i;
// afterwards L[i][j] = D[i][j] / sqrt(D[j][j]).  One barrier per column.
__global__ __launch_bounds__(256) void factor_small_kernel(FactorArgs a) {
  if (a.done && *a.done) return;
  __shared__ double col[2][kSmallD];
  __shared__ double piv[kSmallD];
  __shared__ double shd[64];
  const CovPlan& p = a.plan;
  const int d = p.d, tid = threadIdx.x;
  const int j = tid & 63, i0 = tid >> 6;
  double* sig = a.sigma_out;
  const double* src = a.sigma_in ? a.sigma_in : sig;
  const bool jv = j < d;
  double v[16];
  auto load = [&]() {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i = i0 + 4 * q;
      const double x = src[(size_t)min(i, d - 1) * d + min(j, d - 1)];   // valid address
      v[q] = (jv && i < d) ? x : 0.0;
    }
  };
  load();
  if (a.sigma_in) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i = i0 + 4 * q;
      if (jv && i < d) sig[(size_t)i * d + j] = v[q];
    }
  }
  if (a.cov_only) return;
  double tr = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q)
    if (jv && i0 + 4 * q == j) tr += v[q];
  block_sum4(tr, z1, z2, z3, shd);
  double tau = 1e-10 * tr / d;
  bool ok = false;
  for (int attempt = 0; attempt < 6 && !ok; ++attempt) {
    if (attempt) {
      tau *= 100.0;
      load();
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i = i0 + 4 * q;
      if (jv && i == j) v[q] += tau;
      if (j == 0 && i < d) col[0][i] = v[q];
    }
    __syncthreads();
    ok = true;
    for (int k = 0; k < d; ++k) {
      const int cb = k & 1;
      const double dkk = col[cb][k];
      if (!(dkk > 0.0) || isinf(dkk)) {
        ok = false;
        break;
      }
      if (tid == 0) piv[k] = dkk;
      if (jv && j > k) {
        const double cj = col[cb][j] / dkk;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int i = i0 + 4 * q;
          if (i >= j && i < d) v[q] -= col[cb][i] * cj;
        }
        if (j == k + 1) {
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const int i = i0 + 4 * q;
            if (i >= j && i < d) col[cb ^ 1][i] = v[q];   // next column, final now
          }
        }
      }
      __syncthreads();
    }
    __syncthreads();
  }
  if (!ok) {
    if (tid == 0 && a.err_out) *a.err_out = PHI4_ECHOL;
    return;
  }
  if (!jv) return;
  const double eps = a.Bt ? *a.eps_ptr : 0.0;
  const double rj = 1.0 / sqrt(piv[j]);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int i = i0 + 4 * q;
    if (i >= d) continue;
    double l = 0.0;
    if (j < i) l = v[q] * rj;
    else if (j == i) l = sqrt(piv[i]);
    a.A[(size_t)i * d + j] = l;
    // Bt[k][c] = eps L[c][k]: this entry is L[i][j] -> Bt[j][i]
    if (a.Bt) a.Bt[(size_t)j * a.ldb + i] = (j <= i) ? (float)(eps * l) : 0.f;
  }
  if (tid == 0 && a.tau_out) *a.tau_out = tau;
}

}  // namespace

CovPlan cov_plan(int n, int d) {
  CovPlan p;
  p.d = d;
  p.n = n;
  p.nb = (d + 15) / 16;
  p.blocks = p.nb * (p.nb + 1) / 2;
  // about 1024 waves, at most 32 partials per block (the reduction is one
  // workgroup), at least 64 particles per chunk
  int chunks = (1024 + p.blocks - 1) / p.blocks;
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

size_t cov_partial_floats(const CovPlan& p) {
  return (size_t)p.chunks * p.blocks * 256 + (size_t)p.chunks * p.nb * 16;
}

void launch_cov_partials(const float* phi, const int32_t* rows, const CovPlan& p, float* part,
                         const int32_t* done, hipStream_t s) {
  cov_partial_kernel<<<dim3(p.blocks, p.chunks), 64, 0, s>>>(phi, rows, p, part, done);
}

void launch_factor(const FactorArgs& a, hipStream_t s) {
  if (!a.sigma_in) {
    const int entries = a.plan.blocks * 256;
    cov_reduce_kernel<<<(entries + 255) / 256, 256, 0, s>>>(a.part, a.plan, a.sigma_out, a.done);
  }
  if (a.cov_only) return;
  if (a.plan.d <= kSmallD)
    factor_small_kernel<<<1, 256, 0, s>>>(a);
  else
    factor_kernel<<<1, kFT, 0, s>>>(a);
}

}  // namespace phi4
