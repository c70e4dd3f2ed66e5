// Hamiltonian Monte Carlo inner kernel of tempered SMC (SMC-HMC, Sec. 2
// (iii); App. A): per particle, n_steps trajectories of n_leap leapfrog steps
// on the potential V = U0 + beta S of the tempered target, with the diagonal
// mass M = diag(1 / v_x), v_x the variance of site x over the particles.
//
// One workgroup per particle keeps the particle's field, momentum, gradient
// and per-site potential terms in registers for the whole sweep; each
// gradient evaluation exchanges the field through LDS once (the four
// periodic neighbours of Sec. 2 Eq. (1)):
//   dV/dphi_x = phi_x + beta [(4 + m^2) phi_x - sum of neighbours
//                             + 4 lambda phi_x^3].
// The momenta are drawn from the PROPOSE stream (p = z / sqrt(v)), quads of
// sites cooperatively into LDS; the energy change is summed per site
// (potential terms of the end point minus those of the start, plus the
// kinetic terms), so float32 does not cancel at |S| ~ 1e3.  A trajectory
// that diverges ends with a non-finite energy and is rejected.
#include "hmc.hpp"

namespace phi4 {

namespace {

template <int NT, int PER>   // threads per particle, sites per thread (NT * PER >= d)
__global__ __launch_bounds__(NT) void hmc_kernel(HmcArgs a) {
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) float xs[];   // d floats: field exchange, normals
  __shared__ float red[NW][3];
  const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int d = a.d, L = a.L;
  const int srow = a.src_rows ? a.src_rows[p] : p;
  const bool frozen = a.done && *a.done;
  const int steps = frozen ? 0 : a.n_steps;
  const float beta = (float)*a.beta_ptr;
  const float eps = (float)*a.eps_ptr;
  const uint32_t level = (uint32_t)*a.level_ptr;
  const float m2 = a.m2, lam = a.lam, c4 = 4.f + m2;

  bool ok[PER];
  int xi[PER], n1[PER], n2[PER], n3[PER], n4[PER];   // site, x+e1, x-e1, x+e0, x-e0
  float f0[PER], var[PER], sd[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int x = tid + NT * i;
    ok[i] = x < d;
    const int xc = min(x, d - 1);
    const int r0 = xc / L, c1 = xc - r0 * L;
    xi[i] = xc;
    n1[i] = r0 * L + (c1 + 1 == L ? 0 : c1 + 1);
    n2[i] = r0 * L + (c1 == 0 ? L - 1 : c1 - 1);
    n3[i] = xc + L < d ? xc + L : xc + L - d;
    n4[i] = xc >= L ? xc - L : xc - L + d;
    f0[i] = a.src[(size_t)srow * d + xc];
    var[i] = (float)a.var[xc];
    sd[i] = sqrtf(var[i]);
  }

  // gradient of V at f into g; with `terms`, also the per-site action terms
  // s_x (st) and potential terms phi^2/2 + beta s_x (vt), zero off the lattice
  auto eval = [&](const float(&f)[PER], float(&g)[PER], float(&vt)[PER], float(&st)[PER],
                  bool terms) __attribute__((always_inline)) {
    __syncthreads();   // earlier readers of xs are done
#pragma unroll
    for (int i = 0; i < PER; ++i)
      if (ok[i]) xs[xi[i]] = f[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const float c = f[i];
      const float b1 = xs[n1[i]], b2 = xs[n2[i]], b3 = xs[n3[i]], b4 = xs[n4[i]];
      g[i] = c + beta * (c4 * c - ((b1 + b2) + (b3 + b4)) + 4.f * lam * c * c * c);
      if (terms) {
        const float e1 = b1 - c, e3 = b3 - c, c2 = c * c;
        const float s = 0.5f * (e1 * e1 + e3 * e3) + 0.5f * m2 * c2 + lam * c2 * c2;
        st[i] = ok[i] ? s : 0.f;
        vt[i] = ok[i] ? 0.5f * c2 + beta * s : 0.f;
      }
    }
  };
  // block sums of three values, identical on every thread (fixed order)
  auto reduce3 = [&](float(&v)[3]) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < 3; ++q) v[q] = wave_sum_f(v[q]);
    __syncthreads();   // earlier readers of red are done
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 3; ++q) red[wv][q] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      float t = red[0][q];
      for (int w = 1; w < NW; ++w) t += red[w][q];
      v[q] = t;
    }
  };

  float g0[PER], vt0[PER], st[PER];
  eval(f0, g0, vt0, st, true);
  float s_cur, m_cur;
  {
    float r[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      r[0] += st[i];
      r[1] += ok[i] ? f0[i] : 0.f;
    }
    reduce3(r);
    s_cur = r[0];
    m_cur = r[1];
  }

  const uint32_t c3p = counter3(level, PHI4_PROPOSE), c3a = counter3(level, PHI4_ACCEPT);
  const int nq = (d + 3) / 4;
  int nacc = 0;
  for (int s = 0; s < steps; ++s) {
    const uint32_t step = (uint32_t)s;
    __syncthreads();   // earlier readers of xs are done
    for (int q = tid; q < nq; q += NT) {
      const float4 z = normals4((uint32_t)q, (uint32_t)p, step, c3p, a.seed, a.run);
      const int x = 4 * q;
      xs[x] = z.x;
      if (x + 1 < d) xs[x + 1] = z.y;
      if (x + 2 < d) xs[x + 2] = z.z;
      if (x + 3 < d) xs[x + 3] = z.w;
    }
    __syncthreads();
    float mom[PER], f1[PER], g1[PER], vt1[PER], kin0[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const float z = ok[i] ? xs[xi[i]] : 0.f;
      kin0[i] = 0.5f * z * z;
      mom[i] = ok[i] ? z / sd[i] : 0.f;
      mom[i] -= 0.5f * eps * g0[i];
      f1[i] = f0[i];
    }
    for (int l = 0; l < a.n_leap; ++l) {
      const bool last = l == a.n_leap - 1;
#pragma unroll
      for (int i = 0; i < PER; ++i) f1[i] += eps * var[i] * mom[i];
      eval(f1, g1, vt1, st, last);
      const float h = last ? 0.5f * eps : eps;
#pragma unroll
      for (int i = 0; i < PER; ++i) mom[i] -= h * g1[i];
    }
    float r[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (ok[i]) {
        r[0] += (vt1[i] - vt0[i]) + (0.5f * var[i] * mom[i] * mom[i] - kin0[i]);
        r[1] += st[i];
        r[2] += f1[i];
      }
    }
    reduce3(r);
    const float lu = __logf(u01(word0((uint32_t)p, step, c3a, a.seed, a.run)));
    if (lu < -r[0]) {   // a non-finite energy change compares false and rejects
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        f0[i] = f1[i];
        g0[i] = g1[i];
        vt0[i] = vt1[i];
      }
      s_cur = r[1];
      m_cur = r[2];
      ++nacc;
    }
  }
#pragma unroll
  for (int i = 0; i < PER; ++i)
    if (ok[i]) a.dst[(size_t)p * d + xi[i]] = f0[i];
  if (tid == 0) {
    a.S[p] = s_cur;
    if (a.absM) a.absM[p] = fabsf(m_cur / d);
    if (a.acc_count && nacc) atomicAdd(a.acc_count, (unsigned long long)nacc);
    if (a.prop_count && p == 0 && steps)
      atomicAdd(a.prop_count, (unsigned long long)a.n * (unsigned long long)steps);
  }
}

constexpr int kVarRows = 64;

// Column tile x (64 sites) and row chunk y: sums of (phi - c) and
// (phi - c)^2 over the chunk's rows, c the first row's value (float64).
__global__ __launch_bounds__(256) void var_partial_kernel(const float* __restrict__ phi,
                                                          const int32_t* __restrict__ rows, int n,
                                                          int d, double* __restrict__ part,
                                                          const int32_t* __restrict__ done) {
  if (done && *done) return;
  __shared__ double sh[2][4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x = blockIdx.x * 64 + lane, xc = min(x, d - 1);
  const int r0 = blockIdx.y * kVarRows, r1 = min(n, r0 + kVarRows);
  const double c = (double)phi[(size_t)(rows ? rows[0] : 0) * d + xc];
  double s1 = 0.0, s2 = 0.0;
#pragma unroll 4
  for (int i = r0 + wv; i < r1; i += 4) {
    const double y = (double)phi[(size_t)(rows ? rows[i] : i) * d + xc] - c;
    s1 += y;
    s2 += y * y;
  }
  sh[0][wv][lane] = s1;
  sh[1][wv][lane] = s2;
  __syncthreads();
  if (wv == 0 && x < d) {
    const size_t o = (size_t)blockIdx.y * d + x, half = (size_t)gridDim.y * d;
    part[o] = (sh[0][0][lane] + sh[0][1][lane]) + (sh[0][2][lane] + sh[0][3][lane]);
    part[half + o] = (sh[1][0][lane] + sh[1][1][lane]) + (sh[1][2][lane] + sh[1][3][lane]);
  }
}

// One wave per site: lanes take the chunks lane, lane + 64, ..., then a
// fixed-order wave sum.
__global__ __launch_bounds__(256) void var_final_kernel(const double* __restrict__ part, int chunks,
                                                        int n, int d, double* __restrict__ var,
                                                        const int32_t* __restrict__ done) {
  if (done && *done) return;
  const int x = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (x >= d) return;   // whole waves
  double s1 = 0.0, s2 = 0.0;
  for (int b = lane; b < chunks; b += 64) {
    s1 += part[(size_t)b * d + x];
    s2 += part[(size_t)(chunks + b) * d + x];
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (lane == 0) var[x] = (s2 - s1 * s1 / n) / (n - 1);
}

}  // namespace

int site_var_chunks(int n) { return (n + kVarRows - 1) / kVarRows; }

void launch_site_variance(const float* phi, const int32_t* rows, int n, int d, double* part,
                          double* var, const int32_t* done, hipStream_t s) {
  const int chunks = site_var_chunks(n);
  var_partial_kernel<<<dim3((unsigned)((d + 63) / 64), (unsigned)chunks), 256, 0, s>>>(
      phi, rows, n, d, part, done);
  var_final_kernel<<<(unsigned)((d + 3) / 4), 256, 0, s>>>(part, chunks, n, d, var, done);
}

void launch_hmc_sweep(const HmcArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  const size_t lds = sizeof(float) * (size_t)a.d;
  const unsigned g = (unsigned)a.n;
  if (a.d <= 64)
    hmc_kernel<64, 1><<<g, 64, lds, s>>>(a);
  else if (a.d <= 128)
    hmc_kernel<128, 1><<<g, 128, lds, s>>>(a);
  else if (a.d <= 256)
    hmc_kernel<256, 1><<<g, 256, lds, s>>>(a);
  else if (a.d <= 512)
    hmc_kernel<512, 1><<<g, 512, lds, s>>>(a);
  else if (a.d <= 1024)
    hmc_kernel<1024, 1><<<g, 1024, lds, s>>>(a);
  else if (a.d <= 2048)
    hmc_kernel<1024, 2><<<g, 1024, lds, s>>>(a);
  else
    hmc_kernel<1024, 4><<<g, 1024, lds, s>>>(a);
}

}  // namespace phi4
