// Field kernels: initial draws, the action of Sec. 2 Eq. (1), raw normal
// streams and the ancestor gather of resampling.
#include "common.hpp"

namespace phi4 {

namespace {

constexpr int kRowThreads = 64;

// Action terms of one row held in LDS: s_x = 1/2 [(phi_{x+e1} - phi_x)^2 +
// (phi_{x+e0} - phi_x)^2] + 1/2 m2 phi_x^2 + lam phi_x^4 with periodic
// wrap; e1 = +1 inside the row of L sites, e0 = +L modulo d.  Returns
// (sum s_x, sum phi_x) reduced over the 64 threads of the row.
__device__ __forceinline__ float2 row_action(const float* row, int L, int d, float m2, float lam) {
  float s = 0.f, m = 0.f;
  for (int x = threadIdx.x; x < d; x += kRowThreads) {
    const int x1 = x % L;
    const int y1 = x - x1 + (x1 + 1 == L ? 0 : x1 + 1);
    const int y0 = x + L < d ? x + L : x + L - d;
    const float f = row[x];
    const float a1 = row[y1] - f, a0 = row[y0] - f;
    const float f2 = f * f;
    s += 0.5f * (a1 * a1 + a0 * a0) + 0.5f * m2 * f2 + lam * (f2 * f2);
    m += f;
  }
  return make_float2(wave_sum_f(s), wave_sum_f(m));
}

__global__ __launch_bounds__(kRowThreads) void init_fields_kernel(
    float* __restrict__ phi, float* __restrict__ S, float* __restrict__ absM, int n, int L,
    float m2, float lam, float scale, uint32_t seed, uint32_t run) {
  __shared__ float row[PHI4_MAX_SITES + 4];
  const int i = blockIdx.x;
  const int d = L * L;
  const int groups = (d + 3) >> 2;
  for (int g = threadIdx.x; g < groups; g += kRowThreads) {
    const float4 z = normals4(g, i, 0, counter3(0, PHI4_INIT), seed, run);
    const int x = 4 * g;
    row[x] = scale * z.x;
    if (x + 1 < d) row[x + 1] = scale * z.y;
    if (x + 2 < d) row[x + 2] = scale * z.z;
    if (x + 3 < d) row[x + 3] = scale * z.w;
  }
  __syncthreads();
  for (int x = threadIdx.x; x < d; x += kRowThreads) phi[(size_t)i * d + x] = row[x];
  const float2 r = row_action(row, L, d, m2, lam);
  if (threadIdx.x == 0) {
    S[i] = r.x;
    if (absM) absM[i] = fabsf(r.y / d);
  }
}

__global__ __launch_bounds__(kRowThreads) void action_kernel(const float* __restrict__ phi,
                                                             int n, int L, float m2, float lam,
                                                             float* __restrict__ S,
                                                             float* __restrict__ absM) {
  __shared__ float row[PHI4_MAX_SITES + 4];
  const int i = blockIdx.x;
  const int d = L * L;
  for (int x = threadIdx.x; x < d; x += kRowThreads) row[x] = phi[(size_t)i * d + x];
  __syncthreads();
  const float2 r = row_action(row, L, d, m2, lam);
  if (threadIdx.x == 0) {
    S[i] = r.x;
    if (absM) absM[i] = fabsf(r.y / d);
  }
}

__global__ void normals_kernel(uint32_t seed, uint32_t run, int level, int step, int purpose,
                               const int32_t* __restrict__ rows, int n, int d,
                               float* __restrict__ out) {
  const int groups = (d + 3) >> 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * groups) return;
  const int i = (int)(t / groups), g = (int)(t % groups);
  const uint32_t p = rows ? (uint32_t)rows[i] : (uint32_t)i;
  const float4 z = normals4(g, p, step, counter3(level, purpose), seed, run);
  float* o = out + (size_t)i * d + 4 * g;
  o[0] = z.x;
  if (4 * g + 1 < d) o[1] = z.y;
  if (4 * g + 2 < d) o[2] = z.z;
  if (4 * g + 3 < d) o[3] = z.w;
}

__global__ __launch_bounds__(256) void gather_kernel(const float* __restrict__ src,
                                                     const float* __restrict__ srcS,
                                                     const int32_t* __restrict__ anc, int n,
                                                     int d, float* __restrict__ dst,
                                                     float* __restrict__ dstS,
                                                     const int32_t* __restrict__ done) {
  if (done && *done) return;
  const int rows_per_block = blockDim.x / 64;
  const int i = blockIdx.x * rows_per_block + (threadIdx.x >> 6);
  if (i >= n) return;
  const int a = anc[i];
  const float* s = src + (size_t)a * d;
  float* o = dst + (size_t)i * d;
  for (int x = threadIdx.x & 63; x < d; x += 64) o[x] = s[x];
  if ((threadIdx.x & 63) == 0) dstS[i] = srcS[a];
}

}  // namespace

void launch_init_fields(float* phi, float* S, float* absM, int n, int L, float m2, float lam,
                        float scale, uint32_t seed, uint32_t run, hipStream_t s) {
  if (n <= 0) return;
  init_fields_kernel<<<n, kRowThreads, 0, s>>>(phi, S, absM, n, L, m2, lam, scale, seed, run);
}

void launch_action(const float* phi, int n, int L, float m2, float lam, float* S, float* absM,
                   hipStream_t s) {
  if (n <= 0) return;
  action_kernel<<<n, kRowThreads, 0, s>>>(phi, n, L, m2, lam, S, absM);
}

void launch_normals(uint32_t seed, uint32_t run, int level, int step, int purpose,
                    const int32_t* rows, int n, int d, float* out, hipStream_t s) {
  const long long total = (long long)n * ((d + 3) / 4);
  if (total <= 0) return;
  const int bs = 256;
  normals_kernel<<<(unsigned)((total + bs - 1) / bs), bs, 0, s>>>(seed, run, level, step,
                                                                  purpose, rows, n, d, out);
}

void launch_gather(const float* src, const float* srcS, const int32_t* anc, int n, int d,
                   float* dst, float* dstS, const int32_t* done, hipStream_t s) {
  if (n <= 0) return;
  gather_kernel<<<(n + 3) / 4, 256, 0, s>>>(src, srcS, anc, n, d, dst, dstS, done);
}

}  // namespace phi4
