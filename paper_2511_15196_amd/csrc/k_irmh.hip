// Per-level set-up of the independent Metropolis-Hastings inner kernel
// (SMC-IRMH, Sec. 2 (ii); App. A).  The proposal is phi' = mu + L z with mu
// the mean and L the jittered Cholesky factor of the resampled particles,
// so log q(phi') = -|z|^2 / 2 + const; the current particle needs its
// whitened residual r = |L^{-1}(phi - mu)|^2 once per level.  A resampled
// cloud can be nearly degenerate (condition numbers of 1e6 .. 1e10 at a few
// particles per site), so r is formed in float64 throughout:
//
//   mean:     column sums in float64, chunks of 64 rows, then the chunks
//             by one wave per column in a fixed order (deterministic);
//   inverse:  column j of L^{-1} by forward substitution in float64, one
//             wave per column, the column's entries in registers (lane m % 64,
//             slot m / 64) and the rows of L prefetched several rows ahead;
//   whiten:   (phi - mu) L^{-T} in 64 x 64 float64 tiles staged through LDS
//             (only K <= the tile's last column), squared and summed per
//             particle over the tile's columns, then over the column tiles
//             in a fixed order;
//   row sums of squares (|z|^2 of a step's normals), one wave per row.
#include "irmh.hpp"

namespace phi4 {

namespace {

constexpr int kMeanRows = 64;
constexpr int kWT = 64;   // whitening tile: particles x columns
constexpr int kWK = 16;   // K chunk

__global__ void irmh_init_kernel(double* one) {
  if (threadIdx.x == 0) *one = 1.0;
}

__global__ __launch_bounds__(256) void mean_partial_kernel(const float* __restrict__ phi,
                                                           const int32_t* __restrict__ rows, int n,
                                                           int d, double* __restrict__ part,
                                                           const int32_t* __restrict__ done) {
  if (done && *done) return;
  __shared__ double sh[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const int r0 = blockIdx.y * kMeanRows, r1 = min(n, r0 + kMeanRows);
  double s = 0.0;
  if (c < d)
#pragma unroll 4
    for (int i = r0 + wv; i < r1; i += 4) {
      const int r = rows ? rows[i] : i;
      s += (double)phi[(size_t)r * d + c];
    }
  sh[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && c < d)
    part[(size_t)blockIdx.y * d + c] = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
}

__global__ __launch_bounds__(256) void mean_final_kernel(const double* __restrict__ part,
                                                         int chunks, int n, int d,
                                                         float* __restrict__ mu,
                                                         double* __restrict__ mu64,
                                                         const int32_t* __restrict__ done) {
  if (done && *done) return;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= d) return;   // whole waves
  double s = 0.0;
  for (int b = lane; b < chunks; b += 64) s += part[(size_t)b * d + c];
  s = wave_sum(s);
  if (lane == 0) {
    mu64[c] = s / n;
    mu[c] = (float)(s / n);
  }
}

// Column j of L^{-1}: x_0 = 1 / L[j][j], x_m = -(sum_{k < m} L[j+m][j+k] x_k)
// / L[j+m][j+m].  Entry x_m sits in lane m % 64, register slot m / 64
// (PL = ceil(d / 64) slots); rows of L are loaded PF rows ahead of their
// use, every load unconditional with a clamped address.  Writes row j of
// the transposed inverse, linv[j][j + m] = x_m.
template <int PL, int PF>
__global__ __launch_bounds__(64) void linv_kernel(const double* __restrict__ A, int d,
                                                  double* __restrict__ linv,
                                                  const int32_t* __restrict__ done) {
  if (done && *done) return;
  const int j = blockIdx.x, lane = threadIdx.x;
  const int len = d - j;   // entries on and below the diagonal
  double x[PL];
#pragma unroll
  for (int t = 0; t < PL; ++t) x[t] = 0.0;
  if (lane == 0) x[0] = 1.0 / A[(size_t)j * d + j];
  double ring[PF][PL], rdg[PF];
  auto load = [&](double(&v)[PL], double& dg, int m) __attribute__((always_inline)) {
    const int i = j + min(m, len - 1);
    const double* row = A + (size_t)i * d + j;
#pragma unroll
    for (int t = 0; t < PL; ++t) v[t] = row[min(lane + 64 * t, len - 1)];
    dg = row[i - j];
  };
#pragma unroll
  for (int u = 0; u < PF; ++u) load(ring[u], rdg[u], 1 + u);
  for (int m0 = 1; m0 < len; m0 += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int mi = m0 + u;
      if (mi < len) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < PL; ++t)
          if (lane + 64 * t < mi) s = fma(ring[u][t], x[t], s);
        s = wave_sum(s);
        const double xi = -s / rdg[u];
#pragma unroll
        for (int t = 0; t < PL; ++t)
          if (lane + 64 * t == mi) x[t] = xi;
      }
      load(ring[u], rdg[u], mi + PF);
    }
  }
  double* out = linv + (size_t)j * d + j;
#pragma unroll
  for (int t = 0; t < PL; ++t)
    if (lane + 64 * t < len) out[lane + 64 * t] = x[t];
}

// Workgroup (column tile x, particle tile y): W[p][c] = sum_{k <= c}
// (phi[rows[p]][k] - mu[k]) linv[k][c] for 64 particles and 64 columns,
// 16 x 16 threads with 4 x 4 outputs each (rows ty + 16 i, columns
// tx + 16 j); then part[x][p] = sum over the tile's columns of W^2.
__global__ __launch_bounds__(256) void whiten_kernel(const float* __restrict__ phi,
                                                     const int32_t* __restrict__ rows,
                                                     const double* __restrict__ mu,
                                                     const double* __restrict__ linv, int n,
                                                     int d, double* __restrict__ part,
                                                     const int32_t* __restrict__ done) {
  if (done && *done) return;
  __shared__ double xs[kWK][kWT + 1];
  __shared__ double bs[kWK][kWT + 1];
  __shared__ double red[16][kWT];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int c0 = blockIdx.x * kWT, p0 = blockIdx.y * kWT;
  const int kend = min(d, c0 + kWT);
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k0 = 0; k0 < kend; k0 += kWK) {
#pragma unroll
    for (int u = 0; u < kWT * kWK / 256; ++u) {
      const int e = tid + 256 * u;
      const int pp = e / kWK, kk = e % kWK;   // particle tile row, K column
      const int p = p0 + pp, k = k0 + kk;
      double v = 0.0;
      if (p < n && k < d) v = (double)phi[(size_t)(rows ? rows[p] : p) * d + k] - mu[k];
      xs[kk][pp] = v;
      const int kb = e / kWT, cc = e % kWT;   // K row, column
      const int kr = k0 + kb, c = c0 + cc;
      bs[kb][cc] = (kr < d && c < d && kr <= c) ? linv[(size_t)kr * d + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kWK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = xs[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) s = fma(acc[i][j], acc[i][j], s);   // columns >= d are zero
    red[tx][ty + 16 * i] = s;
  }
  __syncthreads();
  if (tid < kWT && p0 + tid < n) {
    double s = 0.0;
    for (int t = 0; t < 16; ++t) s += red[t][tid];
    part[(size_t)blockIdx.x * n + p0 + tid] = s;
  }
}

__global__ __launch_bounds__(256) void whiten_sum_kernel(const double* __restrict__ part,
                                                         int tiles, int n, float* __restrict__ r,
                                                         const int32_t* __restrict__ done) {
  if (done && *done) return;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  double s = 0.0;
  for (int t = 0; t < tiles; ++t) s += part[(size_t)t * n + p];
  r[p] = (float)s;
}

__global__ __launch_bounds__(256) void rowsq_kernel(const float* __restrict__ x, int ld, int n,
                                                    int d, float* __restrict__ out,
                                                    const int32_t* __restrict__ done) {
  if (done && *done) return;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (p >= n) return;   // whole waves
  const float* row = x + (size_t)p * ld;
  float s = 0.f;
  for (int k = lane; k < d; k += 64) s = fmaf(row[k], row[k], s);
  s = wave_sum_f(s);
  if (lane == 0) out[p] = s;
}

}  // namespace

int irmh_mean_chunks(int n) { return (n + kMeanRows - 1) / kMeanRows; }

size_t irmh_scratch_bytes(int n, int d) {
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t tiles = (size_t)(d + kWT - 1) / kWT;
  return up(sizeof(float) * d) + up(sizeof(double) * d) +
         up(sizeof(double) * (size_t)irmh_mean_chunks(n) * d) + up(sizeof(double) * (size_t)d * d) +
         up(sizeof(double) * tiles * n) + up(sizeof(float) * n) + up(sizeof(float) * 2 * n) +
         up(sizeof(double));
}

IrmhScratch irmh_scratch(void* base, int n, int d) {
  IrmhScratch q;
  char* p = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) / 256 * 256;
    return r;
  };
  const size_t tiles = (size_t)(d + kWT - 1) / kWT;
  q.mu = reinterpret_cast<float*>(take(sizeof(float) * d));
  q.mu64 = reinterpret_cast<double*>(take(sizeof(double) * d));
  q.mpart = reinterpret_cast<double*>(take(sizeof(double) * (size_t)irmh_mean_chunks(n) * d));
  q.linv = reinterpret_cast<double*>(take(sizeof(double) * (size_t)d * d));
  q.wpart = reinterpret_cast<double*>(take(sizeof(double) * tiles * n));
  q.r = reinterpret_cast<float*>(take(sizeof(float) * n));
  q.zz = reinterpret_cast<float*>(take(sizeof(float) * 2 * n));
  q.one = reinterpret_cast<double*>(take(sizeof(double)));
  return q;
}

void launch_irmh_init(const IrmhScratch& q, hipStream_t s) {
  irmh_init_kernel<<<1, 64, 0, s>>>(q.one);
}

void launch_irmh_mean(const float* phi, const int32_t* rows, int n, int d, const IrmhScratch& q,
                      const int32_t* done, hipStream_t s) {
  const int chunks = irmh_mean_chunks(n);
  mean_partial_kernel<<<dim3((unsigned)((d + 63) / 64), (unsigned)chunks), 256, 0, s>>>(
      phi, rows, n, d, q.mpart, done);
  mean_final_kernel<<<(d + 3) / 4, 256, 0, s>>>(q.mpart, chunks, n, d, q.mu, q.mu64, done);
}

void launch_irmh_inverse(const double* A, int d, const IrmhScratch& q, const int32_t* done,
                         hipStream_t s) {
  const int pl = (d + 63) / 64;
  if (pl <= 1)
    linv_kernel<1, 16><<<d, 64, 0, s>>>(A, d, q.linv, done);
  else if (pl <= 2)
    linv_kernel<2, 8><<<d, 64, 0, s>>>(A, d, q.linv, done);
  else if (pl <= 4)
    linv_kernel<4, 4><<<d, 64, 0, s>>>(A, d, q.linv, done);
  else if (pl <= 8)
    linv_kernel<8, 4><<<d, 64, 0, s>>>(A, d, q.linv, done);
  else
    linv_kernel<16, 2><<<d, 64, 0, s>>>(A, d, q.linv, done);
}

void launch_irmh_whiten(const float* phi, const int32_t* rows, int n, int d, const IrmhScratch& q,
                        const int32_t* done, hipStream_t s) {
  const int tiles = (d + kWT - 1) / kWT;
  whiten_kernel<<<dim3((unsigned)tiles, (unsigned)((n + kWT - 1) / kWT)), 256, 0, s>>>(
      phi, rows, q.mu64, q.linv, n, d, q.wpart, done);
  whiten_sum_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(q.wpart, tiles, n, q.r, done);
}

void launch_rowsq(const float* x, int ld, int n, int d, float* out, const int32_t* done,
                  hipStream_t s) {
  rowsq_kernel<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(x, ld, n, d, out, done);
}

}  // namespace phi4
