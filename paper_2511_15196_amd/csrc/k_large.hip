// Random-walk Metropolis sweep for large lattices (d > 256): one step is
// three passes over the particles instead of the register-resident fused
// sweep, whose per-workgroup factor no longer fits on chip.
//
//   1. normals:  z[p][k] from the PROPOSE stream (App. A random-walk
//      kernel), float32 or rounded to bfloat16 / float16, materialised in
//      HBM (z is shared by every column tile of the product); drawn by a
//      pass of their own for the first step of a sweep and by the accept
//      pass of the step before for the others (its ALUs are idle while its
//      row loads are in flight);
//   2. proposal: phi'[p][c] = phi[p][c] + sum_{k <= c} z[p][k] Bt[k][c] on the
//      matrix cores, output tiles staged through LDS (XCD-aware tile order),
//      only the K range on or above the diagonal of the triangular factor; the
//      16-bit forms take s M(s z) with s the sign of the row's first
//      normal, so that the increment is odd in z (exactly symmetric
//      proposal, no Hastings term) at the cost of one product;
//   3. accept: one workgroup per particle stages phi and phi' in LDS, forms
//      S(phi), S(phi') and dS as a sum of per-site differences (Sec. 2
//      Eq. (1)), dU0 = (|phi'|^2 - |phi|^2) / 2, tests the tempered
//      (log u < -dU0 - beta dS) or likelihood-constrained (S' < S* and
//      log u < -dU0 / prior_var) condition and writes phi' over phi when
//      accepted.
//
// Acceptances are counted per particle (no contended atomics) and summed
// once at the end of the sweep.
#include <map>
#include <mutex>
#include <type_traits>

#include "common.hpp"
#include "irmh.hpp"
#include "slice.hpp"

namespace phi4 {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

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
                                                unsigned short* __restrict__ zsgn,
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
    if (q == 0) zsgn[p] = h.x & 0x8000u;   // sign bit of the row's first normal
  }
}

// ------------------------------------------------------------------ proposal

// Lp[c][k] = Bt[k][c] = eps L[c][k] for k <= c < d and zero elsewhere, as a
// dz x dz array with k contiguous (float32, or rounded to bfloat16 /
// float16): the factor in the same row layout as z, so that both operands
// of the product load as contiguous 16-byte vectors.  Built once per sweep
// through 32 x 32 LDS tiles (coalesced on both sides).
template <int PREC>
__global__ __launch_bounds__(256) void lp_kernel(const float* __restrict__ Bt, int ldb, int d,
                                                 int dz, void* __restrict__ lp,
                                                 const int32_t* __restrict__ done) {
  if (done && *done) return;
  __shared__ float t[32][33];
  const int k0 = blockIdx.y * 32, c0 = blockIdx.x * 32;   // Bt rows k, columns c
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int k = k0 + r, c = c0 + tx;
    float v = 0.f;
    if (k < d && c < d && k <= c) v = Bt[(size_t)k * ldb + c];
    t[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int c = c0 + r, k = k0 + tx;   // Lp row c, column k
    const float v = t[tx][r];
    if constexpr (PREC == PHI4_FP32)
      static_cast<float*>(lp)[(size_t)c * dz + k] = v;
    else
      static_cast<unsigned short*>(lp)[(size_t)c * dz + k] = to16(v, PREC);
  }
}

// phi'[p][c] = phi[irow(p)][c] + sum_{k <= c} z[p][k] Lp[c][k]; the base rows
// are ldphi floats apart (0: one row for every particle, the independence
// sampler's mean).
//
// Workgroup tile BM particles x BN columns, 4 waves as 2 x 2 (each
// BM/2 x BN/2 as 16 x 16 MFMA fragments), K in tiles of 64 through
// double-buffered LDS (row stride padded by one 16-byte vector); global
// loads run S K tiles ahead in S register stages, so that a load has S tiles
// of MFMA work to land (S = 4 for the 16-bit 128 x 128 tile, whose K tiles
// are short in MFMA time, else 2).  Column tiles are taken in pairs (x, J - 1 - x): tile j of the
// triangular product has j + 1 K tiles, so every pair costs the same.
//
// float32 form: lane (p, g) of 16x16x4 step m supplies A[p][k], B[k][p] with
// k = 16 kc + 4 g + m (one 16-byte LDS read feeds four steps; the order of
// the sum is a permutation of k).  16-bit forms: 16x16x32 with
// A[p][8g .. 8g+7] per lane; row p of z enters with its sign flipped when
// the row's first normal is negative (s = -1, an exact bit flip) and the
// result is multiplied by s: the increment s M(s z) is odd in z bit for bit
// (negating z flips s), which the rounding inside the 16-bit dot products
// alone does not guarantee.
template <int PREC, int BM, int BN, int S, int NT = 256>
__global__ __launch_bounds__(NT) void gemm_kernel(const void* __restrict__ zin,
                                                   const unsigned short* __restrict__ zsgn,
                                                   const void* __restrict__ lpin,
                                                   const float* __restrict__ phi,
                                                   const int32_t* __restrict__ irows,
                                                   float* __restrict__ prop, int n, int d,
                                                   int dz, int ldphi,
                                                   const int32_t* __restrict__ done) {
  if (done && *done) return;
  constexpr bool F32 = PREC == PHI4_FP32;
  using T = typename std::conditional<F32, float, unsigned short>::type;
  constexpr int BK = 64;
  constexpr int EPV = 16 / (int)sizeof(T);     // elements per 16-byte vector
  constexpr int VPR = BK / EPV;                // vectors per tile row
  constexpr int KS = BK + EPV;                 // LDS row stride (elements)
  constexpr int WC = NT / 128;                 // waves: 2 rows x WC columns
  constexpr int AV = BM * VPR / NT, BV = BN * VPR / NT;
  static_assert(AV >= 1 && BV >= 1 && BM * VPR % NT == 0 && BN * VPR % NT == 0,
                "tile too small for the thread count");
  constexpr int WM = BM / 2, WN = BN / WC;     // wave tile
  constexpr int FM = WM / 16, FN = WN / 16;    // fragments per wave
  __shared__ __align__(16) T As[2][BM * KS];
  __shared__ __align__(16) T Bs[2][BN * KS];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int pl = lane & 15, gl = lane >> 4;
  const int wr = wv / WC, wc = wv % WC;
  // XCD-aware order: workgroups go round-robin to the 8 XCDs, so the
  // dispatch index i is remapped to the tile (i mod 8) G/8 + i div 8: each
  // XCD takes a contiguous run of tiles (column pairs of one particle tile,
  // then the next), and the workgroups resident on one XCD share their z
  // rows and factor columns in that XCD's L2
  const int G = gridDim.x * gridDim.y;
  const int lin = blockIdx.y * gridDim.x + blockIdx.x;
  const int tile = (G & 7) ? lin : (lin & 7) * (G >> 3) + (lin >> 3);
  const int p0 = (tile / gridDim.x) * BM;
  const int J = (d + BN - 1) / BN;
  const int x = tile % gridDim.x;
  const int ntile = (J - 1 - x > x) ? 2 : 1;
  const T* z = static_cast<const T*>(zin);
  const T* lp = static_cast<const T*>(lpin);

  static_assert(S % 2 == 0, "register stages pair with the two LDS buffers");
  u32x4 ra[S][AV], rb[S][BV];   // register stages: tile t waits in stage t % S
  // 16-bit forms: sign masks of this thread's A rows (both halves of a word)
  unsigned int amask[AV];
#pragma unroll
  for (int i = 0; i < AV; ++i) {
    const int row = (tid + NT * i) / VPR;
    const unsigned int m = F32 ? 0u : (unsigned int)zsgn[min(p0 + row, n - 1)];
    amask[i] = m | (m << 16);
  }
  auto gload = [&](u32x4(&ra)[AV], u32x4(&rb)[BV], int c0, int kt) __attribute__((always_inline)) {
    const int k0 = kt * BK;
#pragma unroll
    for (int i = 0; i < AV; ++i) {
      const int v = tid + NT * i, row = v / VPR, vc = v % VPR;
      ra[i] = *reinterpret_cast<const u32x4*>(z + (size_t)min(p0 + row, n - 1) * dz + k0 +
                                              vc * EPV);
    }
#pragma unroll
    for (int i = 0; i < BV; ++i) {
      const int v = tid + NT * i, row = v / VPR, vc = v % VPR;
      rb[i] = *reinterpret_cast<const u32x4*>(lp + (size_t)min(c0 + row, dz - 1) * dz + k0 +
                                              vc * EPV);
    }
  };
  auto sstore = [&](const u32x4(&ra)[AV], const u32x4(&rb)[BV], int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < AV; ++i) {
      const int v = tid + NT * i, row = v / VPR, vc = v % VPR;
      *reinterpret_cast<u32x4*>(&As[buf][row * KS + vc * EPV]) = F32 ? ra[i] : (ra[i] ^ amask[i]);
    }
#pragma unroll
    for (int i = 0; i < BV; ++i) {
      const int v = tid + NT * i, row = v / VPR, vc = v % VPR;
      *reinterpret_cast<u32x4*>(&Bs[buf][row * KS + vc * EPV]) = rb[i];
    }
  };

  f32x4 acc[FM][FN];
  auto compute = [&](int buf) __attribute__((always_inline)) {
    if constexpr (F32) {
#pragma unroll
      for (int kc = 0; kc < BK / 16; ++kc) {
        float4 af[FM], bf[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
          af[i] = *reinterpret_cast<const float4*>(
              &As[buf][(wr * WM + 16 * i + pl) * KS + 16 * kc + 4 * gl]);
#pragma unroll
        for (int j = 0; j < FN; ++j)
          bf[j] = *reinterpret_cast<const float4*>(
              &Bs[buf][(wc * WN + 16 * j + pl) * KS + 16 * kc + 4 * gl]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i].x, bf[j].x, acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i].y, bf[j].y, acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i].z, bf[j].z, acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i].w, bf[j].w, acc[i][j], 0, 0, 0);
          }
      }
    } else {
#pragma unroll
      for (int kc = 0; kc < BK / 32; ++kc) {
        u16x8 af[FM], bf[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
          af[i] = *reinterpret_cast<const u16x8*>(
              &As[buf][(wr * WM + 16 * i + pl) * KS + 32 * kc + 8 * gl]);
#pragma unroll
        for (int j = 0; j < FN; ++j)
          bf[j] = *reinterpret_cast<const u16x8*>(
              &Bs[buf][(wc * WN + 16 * j + pl) * KS + 32 * kc + 8 * gl]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            if constexpr (PREC == PHI4_BF16)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                  __builtin_bit_cast(bf16x8, af[i]), __builtin_bit_cast(bf16x8, bf[j]), acc[i][j],
                  0, 0, 0);
            else
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                  __builtin_bit_cast(f16x8, af[i]), __builtin_bit_cast(f16x8, bf[j]), acc[i][j],
                  0, 0, 0);
          }
      }
    }
  };

  for (int tt = 0; tt < ntile; ++tt) {
    const int c0 = (tt ? J - 1 - x : x) * BN;
    const int nkt = (min(d, c0 + BN) + BK - 1) / BK;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // tile 0 into LDS buffer 0, tiles 1 .. S in flight (tile S reuses stage 0)
    gload(ra[0], rb[0], c0, 0);
    sstore(ra[0], rb[0], 0);
#pragma unroll
    for (int u = 1; u <= S; ++u)
      if (u < nkt) gload(ra[u % S], rb[u % S], c0, u);
    __syncthreads();
    // tile kt is multiplied from LDS buffer kt & 1 while tiles kt+1 .. kt+S
    // are in flight; a load has S tiles of work to land.  The steady-state
    // loop issues every load unconditionally, so that the wait before each
    // store counts only the loads it needs (a conditional load makes the
    // compiler wait for all of them); the tail handles the last tiles.
    int kt0 = 0;
    for (; kt0 + 2 * S < nkt; kt0 += S) {
#pragma unroll
      for (int u = 0; u < S; ++u) {
        const int kt = kt0 + u;
        compute(u & 1);
        sstore(ra[(u + 1) % S], rb[(u + 1) % S], (u + 1) & 1);
        __syncthreads();
        gload(ra[(u + 1) % S], rb[(u + 1) % S], c0, kt + 1 + S);
        __builtin_amdgcn_sched_barrier(0);   // issue the loads here, not after the next tile
      }
    }
    for (; kt0 < nkt; kt0 += S) {
#pragma unroll
      for (int u = 0; u < S; ++u) {
        const int kt = kt0 + u;
        if (kt < nkt) {
          compute(u & 1);
          if (kt + 1 < nkt) sstore(ra[(u + 1) % S], rb[(u + 1) % S], (u + 1) & 1);
          __syncthreads();
          if (kt + 1 + S < nkt) gload(ra[(u + 1) % S], rb[(u + 1) % S], c0, kt + 1 + S);
        }
      }
    }
    // epilogue: result item r of lane (p, g) is row 4g + r, column p.  All
    // loads first (clamped addresses, no branches), so that they overlap;
    // then the masked stores.
    int irw[FM][4];
    bool neg[FM][4];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pc = min(p0 + wr * WM + 16 * i + 4 * gl + r, n - 1);
        irw[i][r] = irows ? irows[pc] : pc;
        neg[i][r] = !F32 && zsgn[pc] != 0;
      }
    float old[FM][FN][4];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int cc = min(c0 + wc * WN + 16 * j + pl, d - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) old[i][j][r] = phi[(size_t)irw[i][r] * ldphi + cc];
      }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int c = c0 + wc * WN + 16 * j + pl;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int p = p0 + wr * WM + 16 * i + 4 * gl + r;
          if (p < n && c < d)
            prop[(size_t)p * d + c] = old[i][j][r] + (neg[i][r] ? -acc[i][j][r] : acc[i][j][r]);
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
  // optional: the normals of the next step for this slot, drawn while the
  // row loads are in flight (the same values the normals pass would write)
  float* znext;              // z of the next step, layout of z_kernel (NULL: none)
  unsigned short* zsgn;      // 16-bit forms: sign bit of each row's first normal
  int dz, zprec;
  float zsign;
  // independence sampler: log alpha gains (|z|^2 - r) / 2 with r the
  // whitened residual of the slot's current field (replaced by |z|^2 on
  // acceptance); |z|^2 of the next step's normals is summed while drawing them
  float* r;
  const float* zz_in;
  float* zz_out;
};

// VEC (d a multiple of 4, PER >= 4): each thread loads its sites as float4
// quads of consecutive sites (quad tid + kAT j) instead of single floats.
template <bool CONSTRAINED, int PER, bool IND = false, bool VEC = false>   // PER >= d / kAT
__global__ __launch_bounds__(kAT) void accept_kernel(AcceptArgs a) {
  constexpr int NV = IND ? 7 : 6;   // reduced sums
  extern __shared__ __align__(16) float rowbuf[];   // d pairs (phi, phi')
  __shared__ float red[kAT / 64][NV];
  __shared__ int dec;
  const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int d = a.d, L = a.L;
  const int cr = a.crows ? a.crows[p] : p;
  const int orw = a.orows ? a.orows[p] : p;
  float2* f = reinterpret_cast<float2*>(rowbuf);
  float zq = 0.f;   // |z|^2 of this thread's share of the next step's normals
  {
    // every load of this thread in flight before the first LDS store
    const float* cp = a.cur + (size_t)cr * d;
    const float* pp = a.prop + (size_t)p * d;
    float vo[PER], vn[PER];
    if constexpr (VEC) {
      static_assert(PER % 4 == 0, "quads of sites");
      const int nq4 = d / 4;
#pragma unroll
      for (int j = 0; j < PER / 4; ++j) {
        const int q = min(tid + j * kAT, nq4 - 1);
        const float4 o = reinterpret_cast<const float4*>(cp)[q];
        const float4 w = reinterpret_cast<const float4*>(pp)[q];
        vo[4 * j] = o.x;
        vo[4 * j + 1] = o.y;
        vo[4 * j + 2] = o.z;
        vo[4 * j + 3] = o.w;
        vn[4 * j] = w.x;
        vn[4 * j + 1] = w.y;
        vn[4 * j + 2] = w.z;
        vn[4 * j + 3] = w.w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int x = min(tid + i * kAT, d - 1);
        vo[i] = cp[x];
        vn[i] = pp[x];
      }
    }
    if (a.znext && !(a.done && *a.done)) {
      const uint32_t c3p =
          counter3((uint32_t)(a.level_ptr ? *a.level_ptr : a.level), PHI4_PROPOSE);
      const int nq = a.dz / 4;
      for (int q = tid; q < nq; q += kAT) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (4 * q < d) {
          v = normals4((uint32_t)q, (uint32_t)orw, a.step + 1, c3p, a.seed, a.run);
          v.x *= a.zsign;
          v.y *= a.zsign;
          v.z *= a.zsign;
          v.w *= a.zsign;
        }
        if constexpr (IND) zq += (v.x * v.x + v.y * v.y) + (v.z * v.z + v.w * v.w);
        if (a.zprec == PHI4_FP32) {
          *reinterpret_cast<float4*>(a.znext + (size_t)p * a.dz + 4 * q) = v;
        } else {
          ushort4 h;
          h.x = to16(v.x, a.zprec);
          h.y = to16(v.y, a.zprec);
          h.z = to16(v.z, a.zprec);
          h.w = to16(v.w, a.zprec);
          *reinterpret_cast<ushort4*>(reinterpret_cast<unsigned short*>(a.znext) +
                                      (size_t)p * a.dz + 4 * q) = h;
          if (q == 0) a.zsgn[p] = h.x & 0x8000u;
        }
      }
    }
    if constexpr (VEC) {
#pragma unroll
      for (int j = 0; j < PER / 4; ++j) {
        const int q = tid + j * kAT;
        if (q < d / 4) {
          float4* f4 = reinterpret_cast<float4*>(f + 4 * q);
          f4[0] = make_float4(vo[4 * j], vn[4 * j], vo[4 * j + 1], vn[4 * j + 1]);
          f4[1] = make_float4(vo[4 * j + 2], vn[4 * j + 2], vo[4 * j + 3], vn[4 * j + 3]);
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < PER; ++i)
        if (tid + i * kAT < d) f[tid + i * kAT] = make_float2(vo[i], vn[i]);
    }
  }
  __syncthreads();
  // S(phi), S(phi'), sum of per-site differences, dU0, M(phi), M(phi');
  // neighbours x + e1 (wrapping within the row) and x + e0 (wrapping over
  // the lattice), one 8-byte LDS read per site for both fields
  float so = 0.f, sn = 0.f, ds = 0.f, du = 0.f, mo = 0.f, mn = 0.f;
  const int cstep = kAT % L;
  int col = tid % L;
  const float hm2 = 0.5f * a.m2, lam = a.lam;
  for (int x = tid; x < d; x += kAT) {
    const int y1 = col + 1 == L ? x + 1 - L : x + 1;
    const int y0 = x + L < d ? x + L : x + L - d;
    const float2 v = f[x], r1 = f[y1], r0 = f[y0];
    const float a1o = r1.x - v.x, a0o = r0.x - v.x, f2o = v.x * v.x;
    const float a1n = r1.y - v.y, a0n = r0.y - v.y, f2n = v.y * v.y;
    const float to = 0.5f * (a1o * a1o + a0o * a0o) + hm2 * f2o + lam * f2o * f2o;
    const float tn = 0.5f * (a1n * a1n + a0n * a0n) + hm2 * f2n + lam * f2n * f2n;
    so += to;
    sn += tn;
    ds += tn - to;
    du += 0.5f * (f2n - f2o);
    mo += v.x;
    mn += v.y;
    col += cstep;
    if (col >= L) col -= L;
  }
  float v[NV];
  v[0] = so;
  v[1] = sn;
  v[2] = ds;
  v[3] = du;
  v[4] = mo;
  v[5] = mn;
  if constexpr (IND) v[6] = zq;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum_f(v[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) red[wv][q] = v[q];
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
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
      if constexpr (IND)
        acc = lu < -v[3] - beta * v[2] + 0.5f * (a.zz_in[p] - a.r[p]);
      else
        acc = lu < -v[3] - beta * v[2];
    } else {
      const float sstar = a.sstar_ptr ? *a.sstar_ptr : a.s_star;
      acc = (v[1] < sstar) && (lu < -v[3] * a.inv_prior_var);
    }
    if (frozen) acc = 0;
    if constexpr (IND) {
      if (acc) a.r[p] = a.zz_in[p];
      if (a.znext) a.zz_out[p] = v[6];
    }
    dec = acc;
    a.S[orw] = acc ? v[1] : v[0];
    if (a.absM) a.absM[orw] = fabsf((acc ? v[5] : v[4]) / d);
    if (a.accp && !frozen) a.accp[p] += acc;
    if (a.acc_flags) a.acc_flags[p] = (uint8_t)acc;
  }
  __syncthreads();
  if (dec || a.copy_rejected) {
    const bool take_new = dec;
    for (int x = tid; x < d; x += kAT) a.dst[(size_t)orw * d + x] = take_new ? f[x].y : f[x].x;
  }
}

// The same accept for d <= 512: one wave per particle, four particles per
// workgroup (a 256-thread workgroup per particle leaves most lanes idle at
// these sizes).  Every lane of a wave forms the same sums (DPP reduction)
// and takes the same decision; lane 0 writes the per-particle outputs.
constexpr int kAW = 4;   // particles (waves) per workgroup

template <bool CONSTRAINED, int PER, bool IND>   // PER >= d / 64 sites per lane
__global__ __launch_bounds__(64 * kAW) void accept_wave_kernel(AcceptArgs a) {
  constexpr int NV = IND ? 7 : 6;
  extern __shared__ __align__(16) float rowbuf[];   // kAW x d pairs (phi, phi')
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int p = blockIdx.x * kAW + wv;
  const bool live = p < a.n;                      // uniform per wave
  const int pc = live ? p : a.n - 1;
  const int d = a.d, L = a.L;
  const int cr = a.crows ? a.crows[pc] : pc;
  const int orw = a.orows ? a.orows[pc] : pc;
  float2* f = reinterpret_cast<float2*>(rowbuf) + (size_t)wv * d;
  float zq = 0.f;
  {
    const float* cp = a.cur + (size_t)cr * d;
    const float* pp = a.prop + (size_t)pc * d;
    float vo[PER], vn[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int x = min(lane + i * 64, d - 1);
      vo[i] = cp[x];
      vn[i] = pp[x];
    }
    if (live && a.znext && !(a.done && *a.done)) {
      const uint32_t c3p =
          counter3((uint32_t)(a.level_ptr ? *a.level_ptr : a.level), PHI4_PROPOSE);
      const int nq = a.dz / 4;
      for (int q = lane; q < nq; q += 64) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (4 * q < d) {
          v = normals4((uint32_t)q, (uint32_t)orw, a.step + 1, c3p, a.seed, a.run);
          v.x *= a.zsign;
          v.y *= a.zsign;
          v.z *= a.zsign;
          v.w *= a.zsign;
        }
        if constexpr (IND) zq += (v.x * v.x + v.y * v.y) + (v.z * v.z + v.w * v.w);
        if (a.zprec == PHI4_FP32) {
          *reinterpret_cast<float4*>(a.znext + (size_t)p * a.dz + 4 * q) = v;
        } else {
          ushort4 h;
          h.x = to16(v.x, a.zprec);
          h.y = to16(v.y, a.zprec);
          h.z = to16(v.z, a.zprec);
          h.w = to16(v.w, a.zprec);
          *reinterpret_cast<ushort4*>(reinterpret_cast<unsigned short*>(a.znext) +
                                      (size_t)p * a.dz + 4 * q) = h;
          if (q == 0) a.zsgn[p] = h.x & 0x8000u;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < PER; ++i)
      if (lane + i * 64 < d) f[lane + i * 64] = make_float2(vo[i], vn[i]);
  }
  __syncthreads();
  float so = 0.f, sn = 0.f, ds = 0.f, du = 0.f, mo = 0.f, mn = 0.f;
  const int cstep = 64 % L;
  int col = lane % L;
  const float hm2 = 0.5f * a.m2, lam = a.lam;
  for (int x = lane; x < d; x += 64) {
    const int y1 = col + 1 == L ? x + 1 - L : x + 1;
    const int y0 = x + L < d ? x + L : x + L - d;
    const float2 v = f[x], r1 = f[y1], r0 = f[y0];
    const float a1o = r1.x - v.x, a0o = r0.x - v.x, f2o = v.x * v.x;
    const float a1n = r1.y - v.y, a0n = r0.y - v.y, f2n = v.y * v.y;
    const float to = 0.5f * (a1o * a1o + a0o * a0o) + hm2 * f2o + lam * f2o * f2o;
    const float tn = 0.5f * (a1n * a1n + a0n * a0n) + hm2 * f2n + lam * f2n * f2n;
    so += to;
    sn += tn;
    ds += tn - to;
    du += 0.5f * (f2n - f2o);
    mo += v.x;
    mn += v.y;
    col += cstep;
    if (col >= L) col -= L;
  }
  float v[NV];
  v[0] = so;
  v[1] = sn;
  v[2] = ds;
  v[3] = du;
  v[4] = mo;
  v[5] = mn;
  if constexpr (IND) v[6] = zq;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum_f(v[q]);
  const bool frozen = a.reject_all || (a.done && *a.done);
  const uint32_t c3a = counter3((uint32_t)(a.level_ptr ? *a.level_ptr : a.level), PHI4_ACCEPT);
  const float lu = __logf(u01(word0((uint32_t)orw, a.step, c3a, a.seed, a.run)));
  int acc;
  if constexpr (!CONSTRAINED) {
    const float beta = a.beta_ptr ? (float)(*a.beta_ptr) : a.beta;
    if constexpr (IND)
      acc = lu < -v[3] - beta * v[2] + 0.5f * (a.zz_in[pc] - a.r[pc]);
    else
      acc = lu < -v[3] - beta * v[2];
  } else {
    const float sstar = a.sstar_ptr ? *a.sstar_ptr : a.s_star;
    acc = (v[1] < sstar) && (lu < -v[3] * a.inv_prior_var);
  }
  if (frozen) acc = 0;
  if (live && lane == 0) {
    if constexpr (IND) {
      if (acc) a.r[p] = a.zz_in[p];
      if (a.znext) a.zz_out[p] = v[6];
    }
    a.S[orw] = acc ? v[1] : v[0];
    if (a.absM) a.absM[orw] = fabsf((acc ? v[5] : v[4]) / d);
    if (a.accp && !frozen) a.accp[p] += acc;
    if (a.acc_flags) a.acc_flags[p] = (uint8_t)acc;
  }
  if (live && (acc || a.copy_rejected))
    for (int x = lane; x < d; x += 64) a.dst[(size_t)orw * d + x] = acc ? f[x].y : f[x].x;
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

// Proposal-product tiles the tuner chooses from (particles x columns x
// threads): the last runs eight waves (2 x 4) for two waves per SIMD.
constexpr int kNumTiles = 5;
constexpr int kTiles[kNumTiles][3] = {
    {32, 64, 256}, {64, 64, 256}, {128, 64, 256}, {128, 128, 256}, {128, 128, 512}};

template <int PREC>
void launch_gemm(int tile, const LargeScratch& w, const float* cur, const int32_t* crows, int n,
                 int d, const int32_t* done, hipStream_t st, int ldphi = -1) {
  if (ldphi < 0) ldphi = d;
  const int dz = large_dz(d);
  const int bm = kTiles[tile][0], bn = kTiles[tile][1];
  const int J = (d + bn - 1) / bn;
  const dim3 grid((unsigned)((J + 1) / 2), (unsigned)((n + bm - 1) / bm));
  switch (tile) {
    case 0:
      gemm_kernel<PREC, 32, 64, 2><<<grid, 256, 0, st>>>(w.z, w.zsgn, w.lp, cur, crows, w.prop, n, d,
                                                      dz, ldphi, done);
      break;
    case 2:
      gemm_kernel<PREC, 128, 64, 2><<<grid, 256, 0, st>>>(w.z, w.zsgn, w.lp, cur, crows, w.prop, n, d,
                                                       dz, ldphi, done);
      break;
    case 3:
      gemm_kernel<PREC, 128, 128, PREC == PHI4_FP32 ? 2 : 4><<<grid, 256, 0, st>>>(
          w.z, w.zsgn, w.lp, cur, crows, w.prop, n, d, dz, ldphi, done);
      break;
    case 4:
      gemm_kernel<PREC, 128, 128, 2, 512><<<grid, 512, 0, st>>>(
          w.z, w.zsgn, w.lp, cur, crows, w.prop, n, d, dz, ldphi, done);
      break;
    default:
      gemm_kernel<PREC, 64, 64, 2><<<grid, 256, 0, st>>>(w.z, w.zsgn, w.lp, cur, crows, w.prop, n, d,
                                                      dz, ldphi, done);
      break;
  }
}

template <bool CONSTRAINED, bool IND = false>
void launch_accept(int per, int n, size_t lds, const AcceptArgs& aa, hipStream_t st) {
  static_assert(PHI4_MAX_SITES <= 16 * kAT, "accept stages at most 16 sites per thread");
  if (aa.d <= 512) {   // one wave per particle
    const unsigned g = (unsigned)((n + kAW - 1) / kAW);
    const size_t wl = kAW * 2 * (size_t)aa.d * sizeof(float);
    if (aa.d <= 64)
      accept_wave_kernel<CONSTRAINED, 1, IND><<<g, 64 * kAW, wl, st>>>(aa);
    else if (aa.d <= 128)
      accept_wave_kernel<CONSTRAINED, 2, IND><<<g, 64 * kAW, wl, st>>>(aa);
    else if (aa.d <= 256)
      accept_wave_kernel<CONSTRAINED, 4, IND><<<g, 64 * kAW, wl, st>>>(aa);
    else
      accept_wave_kernel<CONSTRAINED, 8, IND><<<g, 64 * kAW, wl, st>>>(aa);
    return;
  }
  const bool vec = aa.d % 4 == 0;   // rows 16-byte aligned: quad loads
  if (per <= 4)   // d > 512 here, so per >= 3
    vec ? accept_kernel<CONSTRAINED, 4, IND, true><<<n, kAT, lds, st>>>(aa)
        : accept_kernel<CONSTRAINED, 4, IND><<<n, kAT, lds, st>>>(aa);
  else if (per <= 8)
    vec ? accept_kernel<CONSTRAINED, 8, IND, true><<<n, kAT, lds, st>>>(aa)
        : accept_kernel<CONSTRAINED, 8, IND><<<n, kAT, lds, st>>>(aa);
  else
    vec ? accept_kernel<CONSTRAINED, 16, IND, true><<<n, kAT, lds, st>>>(aa)
        : accept_kernel<CONSTRAINED, 16, IND><<<n, kAT, lds, st>>>(aa);
}

// One step.  With q (independence sampler, float32): the proposal is
// mu + z L^T (one base row), |z|^2 of the first step's normals is summed
// by its own pass and the accept adds the proposal-density ratio.
template <int PREC>
void enqueue_step(const MutateArgs& a, const LargeScratch& w, int tile, int s, bool first,
                  hipStream_t st, const IrmhScratch* q = nullptr) {
  const int n = a.n, d = a.d, dz = large_dz(d);
  const uint32_t step = (uint32_t)(a.step0 + s);
  // the normals of the first step; each later step's are drawn by the
  // accept pass of the step before
  if (first) {
    const long long nz = (long long)n * (dz / 4);
    z_kernel<PREC><<<(unsigned)((nz + 255) / 256), 256, 0, st>>>(w.z, n, d, dz, a.rows, step,
                                                                 a.level, a.level_ptr, a.seed,
                                                                 a.run, a.zsign, w.zsgn,
                                                                 a.done_ptr);
    if (q) launch_rowsq(w.z, dz, n, d, q->zz, a.done_ptr, st);
  }
  // current fields: the step-0 source (through its row maps) or the output
  const float* cur = first ? a.src : a.dst;
  const int32_t* crows = first ? (a.src_rows ? a.src_rows : a.rows) : a.rows;
  if (q)
    launch_gemm<PREC>(tile, w, q->mu, nullptr, n, d, a.done_ptr, st, 0);
  else
    launch_gemm<PREC>(tile, w, cur, crows, n, d, a.done_ptr, st);
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
  if (s + 1 < a.n_steps) {
    aa.znext = w.z;
    aa.zsgn = w.zsgn;
    aa.dz = dz;
    aa.zprec = PREC;
    aa.zsign = a.zsign;
  }
  const size_t lds = 2 * (size_t)d * sizeof(float);
  const int per = (d + kAT - 1) / kAT;
  if (q) {
    aa.r = q->r;
    aa.zz_in = q->zz + (size_t)(s & 1) * n;
    aa.zz_out = q->zz + (size_t)((s + 1) & 1) * n;
    launch_accept<false, true>(per, n, lds, aa, st);
  } else if (a.kind == 1)
    launch_accept<true>(per, n, lds, aa, st);
  else
    launch_accept<false>(per, n, lds, aa, st);
}

// Proposal-product tile per (device, n, d, precision): timed once per shape
// on the caller's stream (hipEvents, three launches of each choice after one
// warm-up) and kept for the process.  Inside a stream capture nothing can be
// timed; the choice is then the largest tile that still gives every compute
// unit two workgroups, and it is not kept.
struct TileKey {
  int dev, n, d, prec;
  bool operator<(const TileKey& o) const {
    if (dev != o.dev) return dev < o.dev;
    if (n != o.n) return n < o.n;
    if (d != o.d) return d < o.d;
    return prec < o.prec;
  }
};
std::mutex g_tile_mu;
std::map<TileKey, int> g_tiles;

int heuristic_tile(int n, int d) {
  for (int t = 3; t > 0; --t) {   // 256-thread tiles only
    const int bm = kTiles[t][0], bn = kTiles[t][1];
    const long long wgs = (long long)(((d + bn - 1) / bn + 1) / 2) * ((n + bm - 1) / bm);
    if (wgs >= 512) return t;
  }
  return 0;
}

template <int PREC>
int tune_tile(const LargeScratch& w, int n, int d, hipStream_t st) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return heuristic_tile(n, d);
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return heuristic_tile(n, d);
  }
  int best = heuristic_tile(n, d);
  float best_ms = 1e30f;
  for (int t = 0; t < kNumTiles; ++t) {
    // operands: whatever the scratch holds (timing only); prop doubles as phi
    launch_gemm<PREC>(t, w, w.prop, nullptr, n, d, nullptr, st);
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < 3; ++r) launch_gemm<PREC>(t, w, w.prop, nullptr, n, d, nullptr, st);
    (void)hipEventRecord(e1, st);
    float ms = 0.f;
    if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
        ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

int gemm_tile(const LargeScratch& w, int n, int d, int prec, hipStream_t st) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const TileKey key{dev, n, d, prec};
  {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    auto it = g_tiles.find(key);
    if (it != g_tiles.end()) return it->second;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return heuristic_tile(n, d);
  int tile;
  switch (prec) {
    case PHI4_BF16: tile = tune_tile<PHI4_BF16>(w, n, d, st); break;
    case PHI4_FP16: tile = tune_tile<PHI4_FP16>(w, n, d, st); break;
    default: tile = tune_tile<PHI4_FP32>(w, n, d, st); break;
  }
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tiles[key] = tile;
  return tile;
}

}  // namespace

int large_dz(int d) { return (d + 63) / 64 * 64; }

size_t large_scratch_bytes(int n, int d) {
  const size_t dz = (size_t)large_dz(d);
  return (size_t)n * dz * sizeof(float) + (size_t)n * d * sizeof(float) +
         (size_t)n * sizeof(int32_t) + dz * dz * sizeof(float) +
         (size_t)n * sizeof(unsigned short) + 5 * 256;
}

LargeScratch large_scratch(void* base, int n, int d) {
  LargeScratch w;
  char* p = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) / 256 * 256;
    return r;
  };
  const size_t dz = (size_t)large_dz(d);
  w.z = reinterpret_cast<float*>(take((size_t)n * dz * sizeof(float)));
  w.prop = reinterpret_cast<float*>(take((size_t)n * d * sizeof(float)));
  w.accp = reinterpret_cast<int32_t*>(take((size_t)n * sizeof(int32_t)));
  w.lp = take(dz * dz * sizeof(float));
  w.zsgn = reinterpret_cast<unsigned short*>(take((size_t)n * sizeof(unsigned short)));
  return w;
}

void launch_large_init(const LargeScratch& w, int n, hipStream_t s) {
  if (n > 0 && w.accp) clear_i32_kernel<<<(n + 255) / 256, 256, 0, s>>>(w.accp, n);
}

bool large_set_tile(int n, int d, int precision, int rows, int cols, int threads) {
  for (int t = 0; t < kNumTiles; ++t) {
    if (kTiles[t][0] == rows && kTiles[t][1] == cols && kTiles[t][2] == threads) {
      int dev = 0;
      (void)hipGetDevice(&dev);
      std::lock_guard<std::mutex> lk(g_tile_mu);
      g_tiles[TileKey{dev, n, d, precision}] = t;
      return true;
    }
  }
  return false;
}

int large_tile_choice(int n, int d, int precision, int* cols, int* threads) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_tile_mu);
  auto it = g_tiles.find(TileKey{dev, n, d, precision});
  if (it == g_tiles.end()) {
    *cols = *threads = 0;
    return 0;
  }
  *cols = kTiles[it->second][1];
  *threads = kTiles[it->second][2];
  return kTiles[it->second][0];
}

// One sweep: n_steps steps of normals, proposal and accept.  A sweep of zero
// steps (or of a finished run) only moves the rows when dst differs from src.
int launch_mutate_large(const MutateArgs& a, const LargeScratch& w, int precision, hipStream_t s) {
  if (a.n <= 0) return PHI4_OK;
  const bool moves = a.src != a.dst || a.src_rows != nullptr;
  if (a.n_steps == 0 && !moves) return PHI4_OK;
  const int steps = a.n_steps > 0 ? a.n_steps : 1;
  if (precision != PHI4_FP32 && precision != PHI4_BF16 && precision != PHI4_FP16)
    return PHI4_EINVAL;
  const int tile = gemm_tile(w, a.n, a.d, precision, s);
  {
    const int dz = large_dz(a.d);
    const dim3 g((unsigned)(dz / 32), (unsigned)(dz / 32));
    if (precision == PHI4_FP32)
      lp_kernel<PHI4_FP32><<<g, 256, 0, s>>>(a.Bt, a.ldb, a.d, dz, w.lp, a.done_ptr);
    else if (precision == PHI4_BF16)
      lp_kernel<PHI4_BF16><<<g, 256, 0, s>>>(a.Bt, a.ldb, a.d, dz, w.lp, a.done_ptr);
    else
      lp_kernel<PHI4_FP16><<<g, 256, 0, s>>>(a.Bt, a.ldb, a.d, dz, w.lp, a.done_ptr);
  }
  for (int t = 0; t < steps; ++t) {
    switch (precision) {
      case PHI4_FP32: enqueue_step<PHI4_FP32>(a, w, tile, t, t == 0, s); break;
      case PHI4_BF16: enqueue_step<PHI4_BF16>(a, w, tile, t, t == 0, s); break;
      default: enqueue_step<PHI4_FP16>(a, w, tile, t, t == 0, s); break;
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

// One sweep of the independence sampler (float32 steps): the mean, the
// inverse factor and the whitened residuals r = |(phi - mu) L^{-T}|^2 of
// the particles src[src_rows] (float64), then n_steps steps of normals,
// proposal mu + z L^T and accept.  A sweep of zero steps only moves the rows.
int launch_irmh_sweep(const MutateArgs& a, const double* A, const IrmhScratch& q,
                      hipStream_t s) {
  if (a.n <= 0) return PHI4_OK;
  if (a.n_steps == 0) return launch_mutate_large(a, a.large, PHI4_FP32, s);
  const int n = a.n, d = a.d, dz = large_dz(d);
  const LargeScratch& w = a.large;
  const int32_t* srows = a.src_rows ? a.src_rows : a.rows;
  const int tile = gemm_tile(w, n, d, PHI4_FP32, s);
  const dim3 g((unsigned)(dz / 32), (unsigned)(dz / 32));
  launch_irmh_mean(a.src, srows, n, d, q, a.done_ptr, s);
  launch_irmh_inverse(A, d, q, a.done_ptr, s);
  launch_irmh_whiten(a.src, srows, n, d, q, a.done_ptr, s);
  lp_kernel<PHI4_FP32><<<g, 256, 0, s>>>(a.Bt, a.ldb, d, dz, w.lp, a.done_ptr);
  for (int t = 0; t < a.n_steps; ++t) enqueue_step<PHI4_FP32>(a, w, tile, t, t == 0, s, &q);
  if (a.prop) {
    const hipError_t e = hipMemcpyAsync(a.prop, w.prop, sizeof(float) * (size_t)n * d,
                                        hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return PHI4_EHIP;
  }
  acc_sum_kernel<<<1, 1024, 0, s>>>(w.accp, n, a.n_steps, a.acc_count, a.prop_count, a.done_ptr);
  return PHI4_OK;
}

// n_steps slice moves of the rows a.rows of a.dst (a.Bt = L^T unscaled):
// per step the normals of the PROPOSE stream, the directions z L^T on the
// proposal-product kernel with a zero base row, then one slice move per
// point; moves are counted per slot and summed once at the end.
int launch_slice_sweep(const MutateArgs& a, const float* zero, hipStream_t s) {
  if (a.n <= 0 || a.n_steps <= 0) return PHI4_OK;
  const int n = a.n, d = a.d, dz = large_dz(d);
  const LargeScratch& w = a.large;
  const int tile = gemm_tile(w, n, d, PHI4_FP32, s);
  const dim3 g((unsigned)(dz / 32), (unsigned)(dz / 32));
  lp_kernel<PHI4_FP32><<<g, 256, 0, s>>>(a.Bt, a.ldb, d, dz, w.lp, a.done_ptr);
  const long long nz = (long long)n * (dz / 4);
  for (int t = 0; t < a.n_steps; ++t) {
    const uint32_t step = (uint32_t)(a.step0 + t);
    z_kernel<PHI4_FP32><<<(unsigned)((nz + 255) / 256), 256, 0, s>>>(
        w.z, n, d, dz, a.rows, step, a.level, a.level_ptr, a.seed, a.run, 1.0f, w.zsgn,
        a.done_ptr);
    launch_gemm<PHI4_FP32>(tile, w, zero, nullptr, n, d, a.done_ptr, s, 0);
    SliceArgs sa = {};
    sa.phi = a.dst;
    sa.rows = a.rows;
    sa.dirs = w.prop;
    sa.n = n;
    sa.L = a.L;
    sa.d = d;
    sa.m2 = a.m2;
    sa.lam = a.lam;
    sa.sstar_ptr = a.sstar_ptr;
    sa.inv_prior_var = a.inv_prior_var;
    sa.seed = a.seed;
    sa.run = a.run;
    sa.level_ptr = a.level_ptr;
    sa.step = step;
    sa.done = a.done_ptr;
    sa.S = a.S;
    sa.absM = a.absM;
    sa.accp = w.accp;
    launch_slice_moves(sa, s);
  }
  acc_sum_kernel<<<1, 1024, 0, s>>>(w.accp, n, a.n_steps, a.acc_count, a.prop_count, a.done_ptr);
  return PHI4_OK;
}

}  // namespace phi4
