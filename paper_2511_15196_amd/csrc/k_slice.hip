// Slice-sampling refill of nested sampling (Sec. 2 (iv); App. A: the
// paper's own NS kernel).  A move of one refilled point phi along its
// direction u (drawn from the survivors' covariance by the proposal-product
// pass) samples t from the slice of
//   t -> N(phi + t u; 0, prior_var I) * [S(phi + t u) < S*]
// at the level log y = log prior(phi) + log U0, with Neal's stepping-out
// (width w, at most m - 1 expansions split J / K by a uniform) and
// shrinkage toward t = 0 (Neal, "Slice sampling", Ann. Statist. 2003).  If
// every shrinkage draw misses, the point stays.
//
// One workgroup per point keeps phi and u in registers; each evaluation at t
// writes phi + t u to LDS once, forms the action of Sec. 2 Eq. (1) per site
// from the forward neighbours, and reduces S, |x|^2 and sum x over the
// workgroup in a fixed order.  Every thread takes the same decisions (the
// sums and the uniforms are identical on all of them), so the data-dependent
// bracketing and shrinkage loops stay uniform across the workgroup.  The
// uniforms come from the SLICE stream: the j-th is word j mod 4 of the call
// (j / 4, row, step, level << 8 | SLICE).
#include "slice.hpp"

namespace phi4 {

namespace {

template <int NT, int PER>   // threads per point, sites per thread (NT * PER >= d)
__global__ __launch_bounds__(NT) void slice_kernel(SliceArgs a) {
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) float xs[];   // d floats: the evaluated field
  __shared__ float red[NW][3];
  if (a.done && *a.done) return;                // whole workgroup
  const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int d = a.d, L = a.L;
  const int row = a.rows ? a.rows[p] : p;
  const float m2 = a.m2, lam = a.lam, ipv = a.inv_prior_var;
  bool ok[PER];
  int xi[PER], n1[PER], n3[PER];   // site, x + e1, x + e0
  float f[PER], u[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int x = tid + NT * i;
    ok[i] = x < d;
    const int xc = min(x, d - 1);
    const int r0 = xc / L, c1 = xc - r0 * L;
    xi[i] = xc;
    n1[i] = r0 * L + (c1 + 1 == L ? 0 : c1 + 1);
    n3[i] = xc + L < d ? xc + L : xc + L - d;
    f[i] = a.phi[(size_t)row * d + xc];
    u[i] = a.dirs[(size_t)p * d + xc];
  }
  const float sstar = a.sstar_ptr ? *a.sstar_ptr : a.s_star;
  const uint32_t c3 = counter3((uint32_t)(a.level_ptr ? *a.level_ptr : a.level), PHI4_SLICE);
  uint4 wq = make_uint4(0u, 0u, 0u, 0u);
  int gq = -1;
  auto unif = [&](int j) __attribute__((always_inline)) {
    const int g = j >> 2;
    if (g != gq) {
      wq = philox4x32_10(make_uint4((uint32_t)g, (uint32_t)row, a.step, c3), a.seed, a.run);
      gq = g;
    }
    const int k = j & 3;
    return u01(k == 0 ? wq.x : k == 1 ? wq.y : k == 2 ? wq.z : wq.w);
  };
  // S, |x|^2 and sum x at x = phi + t u, identical on every thread
  float v[3];
  auto eval = [&](float t) __attribute__((always_inline)) {
    float xv[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) xv[i] = f[i] + t * u[i];
    __syncthreads();   // earlier readers of xs / red are done
#pragma unroll
    for (int i = 0; i < PER; ++i)
      if (ok[i]) xs[xi[i]] = xv[i];
    __syncthreads();
    float s = 0.f, q = 0.f, m = 0.f;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (ok[i]) {
        const float c = xv[i];
        const float e1 = xs[n1[i]] - c, e3 = xs[n3[i]] - c, c2 = c * c;
        s += 0.5f * (e1 * e1 + e3 * e3) + 0.5f * m2 * c2 + lam * c2 * c2;
        q += c2;
        m += c;
      }
    }
    v[0] = wave_sum_f(s);
    v[1] = wave_sum_f(q);
    v[2] = wave_sum_f(m);
    if (lane == 0) {
      red[wv][0] = v[0];
      red[wv][1] = v[1];
      red[wv][2] = v[2];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float t2 = red[0][k];
      for (int w = 1; w < NW; ++w) t2 += red[w][k];
      v[k] = t2;
    }
  };
  eval(0.f);
  const float log_y = -0.5f * v[1] * ipv + __logf(unif(0));
  auto in_slice = [&](float t) __attribute__((always_inline)) {
    eval(t);
    return (-0.5f * v[1] * ipv > log_y) && (v[0] < sstar);
  };
  float lo = -kSliceWidth * unif(1);
  float hi = lo + kSliceWidth;
  int J = (int)floorf((float)kSliceMaxSteps * unif(2));
  int K = kSliceMaxSteps - 1 - J;
  while (J > 0 && in_slice(lo)) {
    lo -= kSliceWidth;
    --J;
  }
  while (K > 0 && in_slice(hi)) {
    hi += kSliceWidth;
    --K;
  }
  bool moved = false;
  float tm = 0.f, sm = 0.f, mm = 0.f;
  for (int i = 0; i < kSliceMaxShrink; ++i) {
    const float t = lo + unif(3 + i) * (hi - lo);
    if (in_slice(t)) {
      moved = true;
      tm = t;
      sm = v[0];
      mm = v[2];
      break;
    }
    if (t < 0.f)
      lo = t;
    else
      hi = t;
  }
  if (moved) {
#pragma unroll
    for (int i = 0; i < PER; ++i)
      if (ok[i]) a.phi[(size_t)row * d + xi[i]] = f[i] + tm * u[i];
    if (tid == 0) {
      a.S[row] = sm;
      if (a.absM) a.absM[row] = fabsf(mm / d);
      if (a.accp) a.accp[p] += 1;
    }
  }
}

__global__ void slice_init_kernel(float* zero, int d, double* one) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < d) zero[i] = 0.f;
  if (i == 0) *one = 1.0;
}

}  // namespace

void launch_slice_moves(const SliceArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  const size_t lds = sizeof(float) * (size_t)a.d;
  const unsigned g = (unsigned)a.n;
  if (a.d <= 64)
    slice_kernel<64, 1><<<g, 64, lds, s>>>(a);
  else if (a.d <= 128)
    slice_kernel<128, 1><<<g, 128, lds, s>>>(a);
  else if (a.d <= 256)
    slice_kernel<256, 1><<<g, 256, lds, s>>>(a);
  else if (a.d <= 512)
    slice_kernel<512, 1><<<g, 512, lds, s>>>(a);
  else if (a.d <= 1024)
    slice_kernel<1024, 1><<<g, 1024, lds, s>>>(a);
  else if (a.d <= 2048)
    slice_kernel<1024, 2><<<g, 1024, lds, s>>>(a);
  else
    slice_kernel<1024, 4><<<g, 1024, lds, s>>>(a);
}

void launch_slice_init(float* zero, int d, double* one, hipStream_t s) {
  slice_init_kernel<<<(d + 255) / 256, 256, 0, s>>>(zero, d, one);
}

}  // namespace phi4
