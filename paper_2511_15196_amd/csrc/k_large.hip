// Random-walk Metropolis sweep for large lattices (d > 256): one step is
// three passes over the particles instead of the register-resident fused
// sweep, whose per-workgroup factor no longer fits on chip.
//
//   1. normals:  z[p][k] from the PROPOSE stream (App. A random-walk
//      kernel), float32 or rounded to bfloat16 / float16, materialised in
//      HBM (z is shared by every column tile of the product);
//   2. proposal: phi'[p][c] = phi[p][c] + sum_{k <= c} z[p][k] Bt[k][c] on the
//      matrix cores, 64 x 64 output tiles staged through LDS, only the
//      K range on or above the diagonal of the triangular factor; the
//      16-bit forms take (M(z) - M(-z)) / 2 so that the increment is odd
//      in z (exactly symmetric proposal, no Hastings term);
//   3. accept: one workgroup per particle stages phi and phi' in LDS, forms
//      S(phi), S(phi') and dS as a sum of per-site differences (Sec. 2
//      Eq. (1)), dU0 = (|phi'|^2 - |phi|^2) / 2, tests the tempered
//      (log u < -dU0 - beta dS) or likelihood-constrained (S' < S* and
//      log u < -dU0 / prior_var) condition and writes phi' over phi when
//      accepted.
//
// Acceptances are counted per particle (no contended atomics) and summed
// once at the end of the sweep.
#include <type_traits>

#include "common.hpp"

namespace phi4 {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int kTM = 64, kTN = 64, kTK = 32;   // GEMM tile: particles x columns x K
constexpr int kGT = 256;                       // GEMM threads (4 waves, 32 x 32 each)
constexpr int kAT = 256;                       // accept threads per particle

__device__ __forceinline__ unsigned short to16(float x, int prec) {
  if (prec == PHI4_BF16) {
    uint32_t b = __float_as_uint(x);
    b += 0x7FFFu + ((b >> 16) & 1u);   // round to nearest even (finite inputs)
    return (unsigned short)(b >> 16);
  }
  return __builtin_bit_cast(unsigned short, (_Float16)x);
}

// ------------------------------------------------------------------ normals

// z[p][k], k < dz (multiple of 4; zero beyond d), one Philox call per quad.
template <int PREC>
__global__ __launch_bounds__(256) void z_kernel(float* __restrict__ z, int n, int d, int dz,
                                                const int32_t* __restrict__ rows, uint32_t step,
                                                int level, const int32_t* __restrict__ level_ptr,
                                                uint32_t seed, uint32_t run, float zsign,
                                                const int32_t* __restrict__ done) {
  if (done && *done) return;
  const uint32_t c3 = counter3((uint32_t)(level_ptr ? *level_ptr : level), PHI4_PROPOSE);
  const int nq = dz / 4;
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long long)n * nq) return;
  const int p = (int)(e / nq), q = (int)(e - (long long)p * nq);
  const uint32_t prow = (uint32_t)(rows ? rows[p] : p);
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (4 * q < d) {
    v = normals4((uint32_t)q, prow, step, c3, seed, run);
    v.x *= zsign;
    v.y *= zsign;
    v.z *= zsign;
    v.w *= zsign;
  }
  if constexpr (PREC == PHI4_FP32) {
    *reinterpret_cast<float4*>(z + (size_t)p * dz + 4 * q) = v;
  } else {
    unsigned short* zh = reinterpret_cast<unsigned short*>(z);
    ushort4 h;
    h.x = to16(v.x, PREC);
    h.y = to16(v.y, PREC);
    h.z = to16(v.z, PREC);
    h.w = to16(v.w, PREC);
    *reinterpret_cast<ushort4*>(zh + (size_t)p * dz + 4 * q) = h;
  }
}

// ------------------------------------------------------------------ proposal

// phi'[p][c] = phi[irow(p)][c] + (z Bt)[p][c] for a 64 x 64 tile.  LDS holds
// the z tile as As[row][k] and the factor tile transposed as Bs[col][k]
// (k contiguous), so that each lane reads its MFMA operands with vector
// loads; the next K tile is loaded into registers while the current one is
// multiplied.
template <int PREC>
__global__ __launch_bounds__(kGT) void proposal_kernel(const float* __restrict__ zin,
                                                       const float* __restrict__ Bt, int ldb,
                                                       const float* __restrict__ phi,
                                                       const int32_t* __restrict__ irows,
                                                       float* __restrict__ prop, int n, int d,
                                                       int dz, const int32_t* __restrict__ done) {
  if (done && *done) return;
  constexpr bool F32 = PREC == PHI4_FP32;
  using T = typename std::conditional<F32, float, unsigned short>::type;
  constexpr int KS = kTK + (F32 ? 4 : 8);   // LDS row stride (elements)
  __shared__ __align__(16) T As[2][kTM * KS];
  __shared__ __align__(16) T Bs[2][kTN * KS];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int pl = lane & 15, gl = lane >> 4;
  const int p0 = blockIdx.y * kTM, c0 = blockIdx.x * kTN;
  const int wr = wv >> 1, wc = wv & 1;         // this wave's 32 x 32 sub-tile
  const int kend = min(d, c0 + kTN);           // Bt[k][c] = 0 for k > c
  const int nkt = (kend + kTK - 1) / kTK;

  // staging assignments: A: 64 rows x 32 k; B: 32 k x 64 columns (float32 source)
  const int ar = tid >> 2, aq = tid & 3;       // A row, 8-element quarter of the k range
  const int bk = tid >> 3, bc = (tid & 7) * 8; // B row k, 8 consecutive columns
  const T* zt = reinterpret_cast<const T*>(zin);
  const int arow = min(p0 + ar, n - 1);        // valid address; rows beyond n unused
  T ra[8];
  float rb[8];
  auto load_tile = [&](int kt) {
    const int k0 = kt * kTK;
    const T* src = zt + (size_t)arow * dz + k0 + 8 * aq;   // dz >= k0 + 32 (padded)
    if constexpr (F32) {
      const float4 x0 = *reinterpret_cast<const float4*>(src);
      const float4 x1 = *reinterpret_cast<const float4*>(src + 4);
      ra[0] = x0.x; ra[1] = x0.y; ra[2] = x0.z; ra[3] = x0.w;
      ra[4] = x1.x; ra[5] = x1.y; ra[6] = x1.z; ra[7] = x1.w;
    } else {
      const u16x8 x = *reinterpret_cast<const u16x8*>(src);
#pragma unroll
      for (int e = 0; e < 8; ++e) ra[e] = x[e];
    }
    const int k = k0 + bk;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = c0 + bc + e;
      const float v = Bt[(size_t)min(k, d - 1) * ldb + min(c, d - 1)];
      rb[e] = (k < d && c < d) ? v : 0.f;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) As[buf][ar * KS + 8 * aq + e] = ra[e];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      if constexpr (F32)
        Bs[buf][(bc + e) * KS + bk] = rb[e];
      else
        Bs[buf][(bc + e) * KS + bk] = to16(rb[e], PREC);
    }
  };

  f32x4 acc[2][2], accn[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = accn[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  if (nkt > 0) {
    load_tile(0);
    store_tile(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nkt; ++kt) {
    const int cb = kt & 1;
    if (kt + 1 < nkt) load_tile(kt + 1);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int row = 32 * wr + 16 * i + pl;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = 32 * wc + 16 * j + pl;
        if constexpr (F32) {
          // lane (p, g) supplies A[p][k] and B[k][p] for k = 4 m + g
#pragma unroll
          for (int m = 0; m < kTK / 4; ++m) {
            const float av = As[cb][row * KS + 4 * m + gl];
            const float bv = Bs[cb][col * KS + 4 * m + gl];
            if (m & 1)
              accn[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, accn[i][j], 0, 0, 0);
            else
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[i][j], 0, 0, 0);
          }
        } else {
          // lane (p, g) supplies A[p][8g .. 8g+7] and B[8g .. 8g+7][p]
          const u16x8 za = *reinterpret_cast<const u16x8*>(&As[cb][row * KS + 8 * gl]);
          const u16x8 zn = za ^ (unsigned short)0x8000u;   // -z, exact
          const u16x8 b = *reinterpret_cast<const u16x8*>(&Bs[cb][col * KS + 8 * gl]);
          if constexpr (PREC == PHI4_BF16) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(bf16x8, za), __builtin_bit_cast(bf16x8, b), acc[i][j], 0, 0, 0);
            accn[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(bf16x8, zn), __builtin_bit_cast(bf16x8, b), accn[i][j], 0, 0, 0);
          } else {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                __builtin_bit_cast(f16x8, za), __builtin_bit_cast(f16x8, b), acc[i][j], 0, 0, 0);
            accn[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                __builtin_bit_cast(f16x8, zn), __builtin_bit_cast(f16x8, b), accn[i][j], 0, 0, 0);
          }
        }
      }
    }
    if (kt + 1 < nkt) store_tile(cb ^ 1);
    __syncthreads();
  }
  // epilogue: result item r of lane (p, g) is row 4g + r, column p
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = c0 + 32 * wc + 16 * j + pl;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = p0 + 32 * wr + 16 * i + 4 * gl + r;
        if (p < n && c < d) {
          const float inc = F32 ? acc[i][j][r] + accn[i][j][r]
                                : 0.5f * (acc[i][j][r] - accn[i][j][r]);
          const int ir = irows ? irows[p] : p;
          prop[(size_t)p * d + c] = phi[(size_t)ir * d + c] + inc;
        }
      }
    }
}

// ------------------------------------------------------------------ accept

struct AcceptArgs {
  const float* cur;          // current fields (rows crow(p))
  const int32_t* crows;      // row of slot p in cur (NULL: p)
  const float* prop;         // proposals, slot-major [n][d]
  float* dst;                // output fields (rows orow(p))
  const int32_t* orows;      // row of slot p in dst / S / absM (NULL: p)
  bool copy_rejected;        // dst != cur: rejected rows are copied too
  bool reject_all;           // a sweep of zero steps: move the rows only
  const int32_t* done;       // finished run: move the rows only
  int n, L, d;
  float m2, lam;
  float beta;
  const double* beta_ptr;
  float s_star;
  const float* sstar_ptr;
  float inv_prior_var;
  uint32_t seed, run, step;
  int level;
  const int32_t* level_ptr;
  float* S;
  float* absM;
  int32_t* accp;             // per-slot acceptance counts
  uint8_t* acc_flags;        // optional, per slot (this step)
};

// Site terms of Sec. 2 Eq. (1) for site x of a row staged in LDS.
__device__ __forceinline__ float site_term(const float* f, int x, int L, int d, float m2,
                                           float lam, float& f2) {
  const int x1 = x % L;
  const int y1 = x - x1 + (x1 + 1 == L ? 0 : x1 + 1);
  const int y0 = x + L < d ? x + L : x + L - d;
  const float v = f[x];
  const float a1 = f[y1] - v, a0 = f[y0] - v;
  f2 = v * v;
  return 0.5f * (a1 * a1 + a0 * a0) + 0.5f * m2 * f2 + lam * f2 * f2;
}

template <bool CONSTRAINED>
__global__ __launch_bounds__(kAT) void accept_kernel(AcceptArgs a) {
  extern __shared__ float rowbuf[];   // 2 d floats: phi, phi'
  __shared__ float red[kAT / 64][6];
  __shared__ int dec;
  const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int d = a.d, L = a.L;
  const int cr = a.crows ? a.crows[p] : p;
  const int orw = a.orows ? a.orows[p] : p;
  float* fo = rowbuf;
  float* fn = rowbuf + d;
  for (int x = tid; x < d; x += kAT) {
    fo[x] = a.cur[(size_t)cr * d + x];
    fn[x] = a.prop[(size_t)p * d + x];
  }
  __syncthreads();
  // S(phi), S(phi'), sum of per-site differences, dU0, M(phi), M(phi')
  float so = 0.f, sn = 0.f, ds = 0.f, du = 0.f, mo = 0.f, mn = 0.f;
  for (int x = tid; x < d; x += kAT) {
    float f2o, f2n;
    const float to = site_term(fo, x, L, d, a.m2, a.lam, f2o);
    const float tn = site_term(fn, x, L, d, a.m2, a.lam, f2n);
    so += to;
    sn += tn;
    ds += tn - to;
    du += 0.5f * (f2n - f2o);
    mo += fo[x];
    mn += fn[x];
  }
  float v[6] = {so, sn, ds, du, mo, mn};
#pragma unroll
  for (int q = 0; q < 6; ++q) v[q] = wave_sum_f(v[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < 6; ++q) red[wv][q] = v[q];
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      float t = red[0][q];
      for (int w = 1; w < kAT / 64; ++w) t += red[w][q];
      v[q] = t;
    }
    const bool frozen = a.reject_all || (a.done && *a.done);
    const uint32_t c3a = counter3((uint32_t)(a.level_ptr ? *a.level_ptr : a.level), PHI4_ACCEPT);
    const float lu = __logf(u01(word0((uint32_t)orw, a.step, c3a, a.seed, a.run)));
    int acc;
    if constexpr (!CONSTRAINED) {
      const float beta = a.beta_ptr ? (float)(*a.beta_ptr) : a.beta;
      acc = lu < -v[3] - beta * v[2];
    } else {
      const float sstar = a.sstar_ptr ? *a.sstar_ptr : a.s_star;
      acc = (v[1] < sstar) && (lu < -v[3] * a.inv_prior_var);
    }
    if (frozen) acc = 0;
    dec = acc;
    a.S[orw] = acc ? v[1] : v[0];
    if (a.absM) a.absM[orw] = fabsf((acc ? v[5] : v[4]) / d);
    if (a.accp && !frozen) a.accp[p] += acc;
    if (a.acc_flags) a.acc_flags[p] = (uint8_t)acc;
  }
  __syncthreads();
  if (dec || a.copy_rejected) {
    const float* srow = dec ? fn : fo;
    for (int x = tid; x < d; x += kAT) a.dst[(size_t)orw * d + x] = srow[x];
  }
}

// Sums the per-slot acceptance counts into the run's counters and clears them.
__global__ __launch_bounds__(1024) void acc_sum_kernel(int32_t* accp, int n, int nsteps,
                                                       unsigned long long* acc_count,
                                                       unsigned long long* prop_count,
                                                       const int32_t* done) {
  if (done && *done) nsteps = 0;
  __shared__ double shd[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    s += (double)accp[i];
    accp[i] = 0;
  }
  s = block_reduce<kSum, 16>(s, shd);
  if (threadIdx.x == 0) {
    if (acc_count) atomicAdd(acc_count, (unsigned long long)s);
    if (prop_count) atomicAdd(prop_count, (unsigned long long)n * nsteps);
  }
}

__global__ void clear_i32_kernel(int32_t* x, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] = 0;
}

template <int PREC>
void enqueue_step(const MutateArgs& a, const LargeScratch& w, int s, bool first, hipStream_t st) {
  const int n = a.n, d = a.d, dz = large_dz(d);
  const uint32_t step = (uint32_t)(a.step0 + s);
  const long long nz = (long long)n * (dz / 4);
  z_kernel<PREC><<<(unsigned)((nz + 255) / 256), 256, 0, st>>>(w.z, n, d, dz, a.rows, step,
                                                               a.level, a.level_ptr, a.seed,
                                                               a.run, a.zsign, a.done_ptr);
  // current fields: the step-0 source (through its row maps) or the output
  const float* cur = first ? a.src : a.dst;
  const int32_t* crows = first ? (a.src_rows ? a.src_rows : a.rows) : a.rows;
  const dim3 grid((unsigned)((d + kTN - 1) / kTN), (unsigned)((n + kTM - 1) / kTM));
  proposal_kernel<PREC><<<grid, kGT, 0, st>>>(w.z, a.Bt, a.ldb, cur, crows, w.prop, n, d, dz,
                                               a.done_ptr);
  AcceptArgs aa = {};
  aa.cur = cur;
  aa.crows = crows;
  aa.prop = w.prop;
  aa.dst = a.dst;
  aa.orows = a.rows;
  aa.copy_rejected = first && (a.src != a.dst || a.src_rows != nullptr);
  aa.reject_all = a.n_steps == 0;
  aa.done = a.done_ptr;
  aa.n = n;
  aa.L = a.L;
  aa.d = d;
  aa.m2 = a.m2;
  aa.lam = a.lam;
  aa.beta = a.beta;
  aa.beta_ptr = a.beta_ptr;
  aa.s_star = a.s_star;
  aa.sstar_ptr = a.sstar_ptr;
  aa.inv_prior_var = a.inv_prior_var;
  aa.seed = a.seed;
  aa.run = a.run;
  aa.level = a.level;
  aa.level_ptr = a.level_ptr;
  aa.step = step;
  aa.S = a.S;
  aa.absM = a.absM;
  aa.accp = w.accp;
  aa.acc_flags = (s == a.n_steps - 1) ? a.acc_flags : nullptr;
  const size_t lds = 2 * (size_t)d * sizeof(float);
  if (a.kind == 1)
    accept_kernel<true><<<n, kAT, lds, st>>>(aa);
  else
    accept_kernel<false><<<n, kAT, lds, st>>>(aa);
}

}  // namespace

int large_dz(int d) { return (d + 63) / 64 * 64; }

size_t large_scratch_bytes(int n, int d) {
  return (size_t)n * large_dz(d) * sizeof(float) + (size_t)n * d * sizeof(float) +
         (size_t)n * sizeof(int32_t) + 3 * 256;
}

LargeScratch large_scratch(void* base, int n, int d) {
  LargeScratch w;
  char* p = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) / 256 * 256;
    return r;
  };
  w.z = reinterpret_cast<float*>(take((size_t)n * large_dz(d) * sizeof(float)));
  w.prop = reinterpret_cast<float*>(take((size_t)n * d * sizeof(float)));
  w.accp = reinterpret_cast<int32_t*>(take((size_t)n * sizeof(int32_t)));
  return w;
}

void launch_large_init(const LargeScratch& w, int n, hipStream_t s) {
  if (n > 0 && w.accp) clear_i32_kernel<<<(n + 255) / 256, 256, 0, s>>>(w.accp, n);
}

// One sweep: n_steps steps of normals, proposal and accept.  A sweep of zero
// steps (or of a finished run) only moves the rows when dst differs from src.
int launch_mutate_large(const MutateArgs& a, const LargeScratch& w, int precision, hipStream_t s) {
  if (a.n <= 0) return PHI4_OK;
  const bool moves = a.src != a.dst || a.src_rows != nullptr;
  if (a.n_steps == 0 && !moves) return PHI4_OK;
  const int steps = a.n_steps > 0 ? a.n_steps : 1;
  for (int t = 0; t < steps; ++t) {
    switch (precision) {
      case PHI4_FP32: enqueue_step<PHI4_FP32>(a, w, t, t == 0, s); break;
      case PHI4_BF16: enqueue_step<PHI4_BF16>(a, w, t, t == 0, s); break;
      case PHI4_FP16: enqueue_step<PHI4_FP16>(a, w, t, t == 0, s); break;
      default: return PHI4_EINVAL;
    }
  }
  if (a.prop && a.n_steps > 0) {
    const hipError_t e = hipMemcpyAsync(a.prop, w.prop, sizeof(float) * (size_t)a.n * a.d,
                                        hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return PHI4_EHIP;
  }
  acc_sum_kernel<<<1, 1024, 0, s>>>(w.accp, a.n, a.n_steps, a.acc_count, a.prop_count, a.done_ptr);
  return PHI4_OK;
}

}  // namespace phi4
