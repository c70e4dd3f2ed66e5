// Fused random-walk Metropolis sweep: n_steps steps of a 16-particle tile
// per workgroup with the fields resident in registers across steps.
//
// One step (App. A random-walk kernel; Sec. 2 tempered family):
//   z ~ N(0, I) from the PROPOSE stream, phi' = phi + Bt^T z on MFMA
//   (Bt = (eps L)^T upper triangular; only blocks on or above the diagonal
//   are multiplied), the periodic stencil of Sec. 2 Eq. (1) on phi and phi'
//   through LDS, then the tempered (log alpha = -dU0 - beta dS) or
//   likelihood-constrained (S' < S* and log u < -dU0 / prior_var)
//   Metropolis test with u from the ACCEPT stream.
//
// Work split: the tile is 16 particles x DP sites (DP = d rounded up to a
// multiple of 16), on W x H waves.  The waves generate the 16 x DP normals
// together into LDS; column-block set c (of W) holds the 16-column blocks nb
// with nb % 2W in {c, 2W-1-c} (a snake that balances the triangular MFMA
// work).  Each of the set's H waves keeps the set's B fragments in
// registers for the whole sweep and forms the set's whole product, whose
// MFMA output layout gives lane (p, g) rows 4g..4g+3 of column 16 nb + p;
// of these the wave owns 4 / H rows, whose fields it holds and whose
// stencil and Metropolis terms it evaluates.  H = 2 at d <= 64 doubles the
// waves of a tile (8 instead of 4 at d = 64), so that at N = 4096 every
// SIMD holds two waves to hide each other's latency (the per-site sums and
// every result are unchanged, bit for bit).  dS is accumulated from per-site
// differences so that float32 does not cancel |S|.
//
// Pipelining: the normals do not depend on the fields, so the tile's
// normals for step s+1 are drawn into the second LDS buffer while the
// matrix cores work on step s; a step needs two workgroup barriers.
//
// Symmetry: the float32 product (four MFMA chains over interleaved K, added
// at the end) is odd in z by IEEE rounding.  The 16-bit matrix instructions
// round their internal sums in a way that is not odd, so the 16-bit
// increment is formed as s M(s z), with s the sign of the particle's first
// normal (row p enters with its sign bits flipped when s = -1, exactly):
// negating z flips s, so the increment is odd in z bit for bit at the cost
// of one product; with the symmetric normals the proposal law is exactly
// symmetric, so the Metropolis ratio needs no Hastings term.
#include <hip/hip_ext.h>

#include <type_traits>

#include "common.hpp"

namespace phi4 {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// Metropolis log-uniforms are drawn for kAccChunk steps at a time.
constexpr int kAccChunk = 32;

// float32 -> bfloat16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  uint32_t b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (unsigned short)(b >> 16);
}
// float32 -> float16 bits, round to nearest even.
__device__ __forceinline__ unsigned short f16_bits(float x) {
  const _Float16 h = (_Float16)x;
  return __builtin_bit_cast(unsigned short, h);
}

// Sum over the 16 lanes of a DPP row; every lane of the row gets the same
// bits (pairs: xor 1, xor 2, mirror within 8, mirror within 16).
__device__ __forceinline__ float row16_sum(float v) {
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x140, 0xF, 0xF, false));
  return v;
}

template <int DP_, int W_, int PREC_, int KIND_, int H_ = 1>
struct Cfg {
  static constexpr int DP = DP_;
  static constexpr int W = W_;
  static constexpr int H = H_;          // waves per column block (row split)
  static constexpr int JJ = 4 / H_;     // tile rows per lane
  static constexpr int NT = 64 * W_ * H_;
  static constexpr int PREC = PREC_;
  static constexpr bool CONSTRAINED = KIND_ == 1;   // likelihood-constrained (else tempered)
  static constexpr bool F32 = PREC_ == PHI4_FP32;
  static constexpr int NB = DP / 16;
  static constexpr int NBW = NB / W;
  static_assert(NB % W == 0, "W must divide the number of column blocks");
  static constexpr int DPZ = F32 ? DP : (DP < 32 ? 32 : DP);  // z columns (16-bit K = 32)
  static constexpr int ZS = F32 ? DPZ + 4 : DPZ + 8;         // z row stride, elements
  static constexpr int XS = DP + 4;                          // exchange row stride
  // static bound on the K-group index t for slot j (column block nb < (j+1) W)
  static constexpr int TB(int j) { return F32 ? (j + 1) * W : ((j + 1) * W - 1) / 2 + 1; }
  static constexpr int OFF(int j) {  // offset of slot j's fragments
    int o = 0;
    for (int i = 0; i < j; ++i) o += TB(i);
    return o;
  }
  static constexpr int NFRAG = OFF(NBW);
};

template <class C>
__global__ __launch_bounds__(C::NT) void mutate_kernel(MutateArgs a) {
  constexpr int W = C::W, NBW = C::NBW, ZS = C::ZS, XS = C::XS, DPZ = C::DPZ;
  constexpr int JJ = C::JJ, NT = C::NT;
  constexpr bool F32 = C::F32;
  using ZT = typename std::conditional<F32, float, unsigned short>::type;
  using FragT = typename std::conditional<F32, f32x4, u16x8>::type;

  // a finished run does no steps; an out-of-place call still moves its rows
  const bool finished = a.done_ptr && *a.done_ptr;
  if (finished && a.dst == a.src) return;

  __shared__ __align__(16) ZT zs[2][16 * ZS];     // normals of steps s (cur) and s+1
  __shared__ __align__(16) float xo[16 * XS];
  __shared__ __align__(16) float xn[16 * XS];
  __shared__ float red0[W * 16];
  __shared__ float red1[W * 16];
  __shared__ float lus[2][kAccChunk][16];         // log u, kAccChunk steps per buffer

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int p = lane & 15, g = lane >> 4;
  // wave wv works on column-block set cw and, of each lane's four MFMA
  // output rows 4g .. 4g+3, on rows 4g + jb .. 4g + jb + JJ - 1.  Both waves
  // of a set form its whole product (the triangular MFMA work grows with
  // the block index); the second half of the waves takes the sets in reverse
  // order, so that waves wv and wv + W, which share a SIMD when the waves of
  // a workgroup are placed round-robin, carry equal MFMA work together.
  const int hh = C::H == 1 ? 0 : wv / W;
  const int cw = (hh & 1) ? W - 1 - wv % W : wv % W, jb = hh * JJ;
  const int base = blockIdx.x * 16;
  const int n = a.n, d = a.d, L = a.L;

  const float beta = a.beta_ptr ? (float)(*a.beta_ptr) : a.beta;
  const float sstar = a.sstar_ptr ? *a.sstar_ptr : a.s_star;
  const int level = a.level_ptr ? *a.level_ptr : a.level;
  const uint32_t c3p = counter3((uint32_t)level, PHI4_PROPOSE);
  const uint32_t c3a = counter3((uint32_t)level, PHI4_ACCEPT);
  constexpr bool constrained = C::CONSTRAINED;
  const int nsteps = finished ? 0 : a.n_steps;

  // rows of this lane's output particles (tile slots 4g + jj) and of the
  // fields they start from
  int orow[JJ], irow[JJ];
  bool oval[JJ];
#pragma unroll
  for (int jj = 0; jj < JJ; ++jj) {
    const int i = base + 4 * g + jb + jj;
    oval[jj] = i < n;
    const int ic = min(i, n - 1);              // valid index, masked below
    const int r = a.rows ? a.rows[ic] : ic;
    orow[jj] = oval[jj] ? r : 0;
    const int ri = a.src_rows ? a.src_rows[ic] : r;
    irow[jj] = oval[jj] ? ri : 0;
  }

  // owned column blocks, columns and periodic neighbours
  int col[NBW], y1[NBW], y0[NBW], nbs[NBW];
  bool cval[NBW];
#pragma unroll
  for (int j = 0; j < NBW; ++j) {
    nbs[j] = j * W + ((j & 1) ? (W - 1 - cw) : cw);
    const int x = 16 * nbs[j] + p;
    col[j] = x;
    cval[j] = x < d;
    const int xx = cval[j] ? x : 0;
    const int x1 = xx % L;
    y1[j] = xx - x1 + (x1 + 1 == L ? 0 : x1 + 1);
    y0[j] = xx + L < d ? xx + L : xx + L - d;
  }

  // B fragments, register resident for the sweep: slot j, K-group t.
  // float32: element w4 of group t is Bt[16t + 4g + w4][col];
  // 16-bit: element e of group t is Bt[32t + 8g + e][col].
  FragT bfr[C::NFRAG];
#pragma unroll
  for (int j = 0; j < NBW; ++j) {
    const int c = col[j];
#pragma unroll
    for (int t = 0; t < C::TB(j); ++t) {
      FragT f;
      if constexpr (F32) {
#pragma unroll
        for (int w4 = 0; w4 < 4; ++w4) {
          const int k = 16 * t + 4 * g + w4;
          const float v = a.Bt[(size_t)min(k, d - 1) * a.ldb + min(c, d - 1)];
          f[w4] = (k < d && c < d && k <= c) ? v : 0.f;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = 32 * t + 8 * g + e;
          const float v0 = a.Bt[(size_t)min(k, d - 1) * a.ldb + min(c, d - 1)];
          const float v = (k < d && c < d && k <= c) ? v0 : 0.f;
          f[e] = C::PREC == PHI4_BF16 ? bf16_bits(v) : f16_bits(v);
        }
      }
      bfr[C::OFF(j) + t] = f;
    }
  }

  // fields of the owned columns
  float ph[NBW][JJ], pn[NBW][JJ];
#pragma unroll
  for (int j = 0; j < NBW; ++j)
#pragma unroll
    for (int jj = 0; jj < JJ; ++jj)
    {
      const float v = a.src[(size_t)irow[jj] * d + min(col[j], d - 1)];
      ph[j][jj] = (oval[jj] && cval[j]) ? v : 0.f;
    }

  // 16-bit K = 32 needs z columns DP..31 of a 16-column tile to be zero
  if constexpr (DPZ > C::DP) {
    for (int e = tid; e < 2 * 16 * (DPZ - C::DP); e += NT) {
      const int b = e / (16 * (DPZ - C::DP)), r = e % (16 * (DPZ - C::DP));
      zs[b][(r / (DPZ - C::DP)) * ZS + C::DP + r % (DPZ - C::DP)] = 0;
    }
  }

  // physical rows of the Z-phase calls (fixed over the sweep): 4 DP calls
  // of four normals per step, ZC per thread
  constexpr int NZC = 4 * C::DP, ZC = (NZC + NT - 1) / NT;
  int zrow[ZC];
  bool zval[ZC];
#pragma unroll
  for (int i = 0; i < ZC; ++i) {
    const int c = tid + NT * i;
    const int ps = c & 15, q = c >> 4;
    const int ti = base + ps;
    zval[i] = c < NZC && ti < n && 4 * q < d;
    const int tc = min(ti, n - 1);
    const int r = a.rows ? a.rows[tc] : tc;
    zrow[i] = zval[i] ? r : 0;
  }

  // normals of one step into zs[buf]: NBW Philox calls per lane
  auto draw_normals = [&](int buf, uint32_t step) {
#pragma unroll
    for (int i = 0; i < ZC; ++i) {
      const int c = tid + NT * i;
      if (NZC % NT != 0 && c >= NZC) break;   // whole waves
      const int ps = c & 15, q = c >> 4;
      float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
      if (zval[i]) {
        z = normals4((uint32_t)q, (uint32_t)zrow[i], step, c3p, a.seed, a.run);
        z.x *= a.zsign;
        z.y *= a.zsign;
        z.z *= a.zsign;
        z.w *= a.zsign;
      }
      if constexpr (F32) {
        *reinterpret_cast<float4*>(&zs[buf][ps * ZS + 4 * q]) = z;
      } else {
        u16x4 h;
        if constexpr (C::PREC == PHI4_BF16) {
          h[0] = bf16_bits(z.x); h[1] = bf16_bits(z.y); h[2] = bf16_bits(z.z); h[3] = bf16_bits(z.w);
        } else {
          h[0] = f16_bits(z.x); h[1] = f16_bits(z.y); h[2] = f16_bits(z.z); h[3] = f16_bits(z.w);
        }
        *reinterpret_cast<u16x4*>(&zs[buf][ps * ZS + 4 * q]) = h;
      }
    }
  };
  // log-uniforms of the ACCEPT stream for steps s0 .. s0 + kAccChunk - 1
  auto draw_uniforms = [&](int s0) {
    const int lb = (s0 / kAccChunk) & 1;
    for (int e = tid; e < 16 * kAccChunk; e += NT) {
      const int sl = e & 15, ss = e >> 4;
      const int ti = base + sl;
      float lu = 0.f;
      if (ti < n && s0 + ss < nsteps) {
        const uint32_t prow = (uint32_t)(a.rows ? a.rows[ti] : ti);
        lu = __logf(u01(word0(prow, (uint32_t)(a.step0 + s0 + ss), c3a, a.seed, a.run)));
      }
      lus[lb][ss][sl] = lu;
    }
  };

  unsigned long long nacc = 0;
  if (nsteps > 0) {
    draw_uniforms(0);
    draw_normals(0, (uint32_t)a.step0);
  }
  __syncthreads();

  for (int s = 0; s < nsteps; ++s) {
    const int cb = s & 1;
    // ---- proposal phi' = phi + Bt^T z for the owned column blocks (MFMA)
    f32x4 acc[NBW], accn[NBW], acc2[NBW], acc3[NBW];  // float32: four independent chains
    // 16-bit forms: sign bit of the first normal of this lane's A row
    unsigned short rsgn = 0;
    if constexpr (!F32)
      rsgn = reinterpret_cast<const unsigned short*>(&zs[cb][p * ZS])[0] & 0x8000u;
#pragma unroll
    for (int j = 0; j < NBW; ++j) {
      const int nb = nbs[j];
      acc[j] = accn[j] = acc2[j] = acc3[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < C::TB(j); ++t) {
        if constexpr (F32) {
          if (t <= nb) {
            const float4 zq = *reinterpret_cast<const float4*>(&zs[cb][p * ZS + 16 * t + 4 * g]);
            const f32x4 b = bfr[C::OFF(j) + t];
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(zq.x, b[0], acc[j], 0, 0, 0);
            accn[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(zq.y, b[1], accn[j], 0, 0, 0);
            acc2[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(zq.z, b[2], acc2[j], 0, 0, 0);
            acc3[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(zq.w, b[3], acc3[j], 0, 0, 0);
          }
        } else {
          if (2 * t <= nb) {
            const u16x8 za =
                *reinterpret_cast<const u16x8*>(&zs[cb][p * ZS + 32 * t + 8 * g]) ^ rsgn;
            const FragT b = bfr[C::OFF(j) + t];
            if constexpr (C::PREC == PHI4_BF16)
              acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, za),
                                                               __builtin_bit_cast(bf16x8, b),
                                                               acc[j], 0, 0, 0);
            else
              acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, za),
                                                              __builtin_bit_cast(f16x8, b),
                                                              acc[j], 0, 0, 0);
          }
        }
      }
    }

    // ---- randomness of the next step while the matrix cores work (the
    // buffer written was last read before the previous step's barriers)
    if (s + 1 < nsteps) {
      if ((s + 1) % kAccChunk == 0) draw_uniforms(s + 1);
      draw_normals(cb ^ 1, (uint32_t)(a.step0 + s + 1));
    }

    // 16-bit forms: signs of the rows of this lane's outputs (rows 4g + jj)
    bool oneg[JJ];
#pragma unroll
    for (int jj = 0; jj < JJ; ++jj) oneg[jj] = false;
    if constexpr (!F32) {
#pragma unroll
      for (int jj = 0; jj < JJ; ++jj)
        oneg[jj] =
            reinterpret_cast<const unsigned short*>(&zs[cb][(4 * g + jb + jj) * ZS])[0] & 0x8000u;
    }
    if constexpr (JJ == 4) {
#pragma unroll
      for (int j = 0; j < NBW; ++j)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const float inc = F32 ? (acc[j][jj] + accn[j][jj]) + (acc2[j][jj] + acc3[j][jj])
                                : (oneg[jj] ? -acc[j][jj] : acc[j][jj]);
          pn[j][jj] = ph[j][jj] + inc;
        }
    } else {
#pragma unroll
      for (int j = 0; j < NBW; ++j) {
        float o[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
          o[r] = F32 ? (acc[j][r] + accn[j][r]) + (acc2[j][r] + acc3[j][r]) : acc[j][r];
#pragma unroll
        for (int jj = 0; jj < JJ; ++jj) {
          // output row jb + jj of the lane (jb is wave-uniform: selects, no
          // indexed register access)
          float v = o[0];
#pragma unroll
          for (int r = 1; r < 4; ++r)
            if (r == jb + jj) v = o[r];
          pn[j][jj] = ph[j][jj] + (F32 ? v : (oneg[jj] ? -v : v));
        }
      }
    }

    // ---- exchange old and new fields for the stencil
#pragma unroll
    for (int j = 0; j < NBW; ++j)
#pragma unroll
      for (int jj = 0; jj < JJ; ++jj) {
        xo[(4 * g + jb + jj) * XS + col[j]] = ph[j][jj];
        xn[(4 * g + jb + jj) * XS + col[j]] = pn[j][jj];
      }

    __syncthreads();

    // ---- per-site terms: tempered -> (dS, dU0); constrained -> (S', dU0).
    // Neighbour values of all owned sites are read first (one LDS round
    // trip); columns beyond d contribute zero.
    float r0[JJ], r1[JJ];
#pragma unroll
    for (int jj = 0; jj < JJ; ++jj) r0[jj] = r1[jj] = 0.f;
    {
      float n1n[NBW][JJ], n0n[NBW][JJ], n1o[NBW][JJ], n0o[NBW][JJ];
#pragma unroll
      for (int j = 0; j < NBW; ++j)
#pragma unroll
        for (int jj = 0; jj < JJ; ++jj) {
          const int rb = (4 * g + jb + jj) * XS;
          n1n[j][jj] = xn[rb + y1[j]];
          n0n[j][jj] = xn[rb + y0[j]];
          if constexpr (!constrained) {
            n1o[j][jj] = xo[rb + y1[j]];
            n0o[j][jj] = xo[rb + y0[j]];
          }
        }
#pragma unroll
      for (int j = 0; j < NBW; ++j)
#pragma unroll
        for (int jj = 0; jj < JJ; ++jj) {
          const float f = ph[j][jj], fn = pn[j][jj];
          const float a1n = n1n[j][jj] - fn, a0n = n0n[j][jj] - fn;
          const float ds = (fn - f) * (fn + f);
          float t0;
          if constexpr (!constrained) {
            const float a1o = n1o[j][jj] - f, a0o = n0o[j][jj] - f;
            const float dk = (a1n - a1o) * (a1n + a1o) + (a0n - a0o) * (a0n + a0o);
            t0 = 0.5f * dk + 0.5f * a.m2 * ds + a.lam * ds * (fn * fn + f * f);
          } else {
            const float fn2 = fn * fn;
            t0 = 0.5f * (a1n * a1n + a0n * a0n) + 0.5f * a.m2 * fn2 + a.lam * (fn2 * fn2);
          }
          r0[jj] += cval[j] ? t0 : 0.f;
          r1[jj] += cval[j] ? 0.5f * ds : 0.f;
        }
    }
#pragma unroll
    for (int jj = 0; jj < JJ; ++jj) {
      r0[jj] = row16_sum(r0[jj]);
      r1[jj] = row16_sum(r1[jj]);
    }
    if (p == 0) {
#pragma unroll
      for (int jj = 0; jj < JJ; ++jj) {
        red0[cw * 16 + 4 * g + jb + jj] = r0[jj];
        red1[cw * 16 + 4 * g + jb + jj] = r1[jj];
      }
    }
    __syncthreads();

    // ---- Metropolis test (every wave evaluates the 16 decisions)
    int accept = 0;
    if (lane < 16) {
      float q0 = 0.f, q1 = 0.f;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        q0 += red0[w * 16 + lane];
        q1 += red1[w * 16 + lane];
      }
      const int ti = base + lane;
      if (ti < n) {
        const float lu = lus[(s / kAccChunk) & 1][s % kAccChunk][lane];
        if constexpr (!constrained) {
          const float la = -q1 - beta * q0;
          accept = lu < la;
        } else {
          const float la = -q1 * a.inv_prior_var;
          accept = (q0 < sstar) && (lu < la);
        }
        if (s == nsteps - 1 && wv == 0 && a.acc_flags) a.acc_flags[ti] = (uint8_t)accept;
      }
    }
    const unsigned long long mask = __ballot(accept);
    if (s == nsteps - 1 && a.prop) {
#pragma unroll
      for (int j = 0; j < NBW; ++j)
#pragma unroll
        for (int jj = 0; jj < JJ; ++jj) {
          const int ti = base + 4 * g + jb + jj;
          if (oval[jj] && cval[j]) a.prop[(size_t)ti * d + col[j]] = pn[j][jj];
        }
    }
#pragma unroll
    for (int j = 0; j < NBW; ++j)
#pragma unroll
      for (int jj = 0; jj < JJ; ++jj)
        if ((mask >> (4 * g + jb + jj)) & 1ull) ph[j][jj] = pn[j][jj];
    nacc += __popcll(mask);
  }

  // ---- action and magnetisation of the final fields
#pragma unroll
  for (int j = 0; j < NBW; ++j)
#pragma unroll
    for (int jj = 0; jj < JJ; ++jj) xo[(4 * g + jb + jj) * XS + col[j]] = ph[j][jj];
  __syncthreads();
  float r0[JJ], r1[JJ];
#pragma unroll
  for (int jj = 0; jj < JJ; ++jj) r0[jj] = r1[jj] = 0.f;
#pragma unroll
  for (int j = 0; j < NBW; ++j) {
    if (!cval[j]) continue;
#pragma unroll
    for (int jj = 0; jj < JJ; ++jj) {
      const int rb = (4 * g + jb + jj) * XS;
      const float f = ph[j][jj];
      const float a1 = xo[rb + y1[j]] - f, a0 = xo[rb + y0[j]] - f;
      const float f2 = f * f;
      r0[jj] += 0.5f * (a1 * a1 + a0 * a0) + 0.5f * a.m2 * f2 + a.lam * (f2 * f2);
      r1[jj] += f;
    }
  }
#pragma unroll
  for (int jj = 0; jj < JJ; ++jj) {
    r0[jj] = row16_sum(r0[jj]);
    r1[jj] = row16_sum(r1[jj]);
  }
  if (p == 0) {
#pragma unroll
    for (int jj = 0; jj < JJ; ++jj) {
      red0[cw * 16 + 4 * g + jb + jj] = r0[jj];
      red1[cw * 16 + 4 * g + jb + jj] = r1[jj];
    }
  }
  // field write-back
#pragma unroll
  for (int j = 0; j < NBW; ++j)
#pragma unroll
    for (int jj = 0; jj < JJ; ++jj)
      if (oval[jj] && cval[j]) a.dst[(size_t)orow[jj] * d + col[j]] = ph[j][jj];
  __syncthreads();
  if (wv == 0 && lane < 16) {
    const int ti = base + lane;
    if (ti < n) {
      float q0 = 0.f, q1 = 0.f;
      for (int w = 0; w < W; ++w) {
        q0 += red0[w * 16 + lane];
        q1 += red1[w * 16 + lane];
      }
      const int prow = a.rows ? a.rows[ti] : ti;
      a.S[prow] = q0;
      if (a.absM) a.absM[prow] = fabsf(q1 / d);
    }
  }
  if (tid == 0) {
    const int valid = min(16, n - base);
    if (a.acc_count) atomicAdd(a.acc_count, nacc);
    if (a.prop_count) atomicAdd(a.prop_count, (unsigned long long)valid * nsteps);
  }
}

// One launch; with timing events they ride on the dispatch packet itself.
template <class C>
void launch_cfg(const MutateArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.n + 15) / 16)), block(C::NT);
  if (a.ev_start)
    hipExtLaunchKernelGGL(mutate_kernel<C>, grid, block, 0, s, a.ev_start, a.ev_stop, 0, a);
  else
    mutate_kernel<C><<<grid, block, 0, s>>>(a);
}

template <int DP, int W, int KIND, int H>
int launch_kind(const MutateArgs& a, int precision, hipStream_t s) {
  switch (precision) {
    case PHI4_FP32:
      launch_cfg<Cfg<DP, W, PHI4_FP32, KIND, H>>(a, s);
      break;
    case PHI4_BF16:
      launch_cfg<Cfg<DP, W, PHI4_BF16, KIND, H>>(a, s);
      break;
    case PHI4_FP16:
      launch_cfg<Cfg<DP, W, PHI4_FP16, KIND, H>>(a, s);
      break;
    default:
      return PHI4_EINVAL;
  }
  return PHI4_OK;
}

template <int DP, int W, int H = 2>
int launch_dp(const MutateArgs& a, int precision, hipStream_t s) {
  return a.kind == 1 ? launch_kind<DP, W, 1, H>(a, precision, s)
                     : launch_kind<DP, W, 0, H>(a, precision, s);
}

}  // namespace

int mutate_supported(int d, int precision) {
  return d >= 1 && d <= PHI4_MAX_SITES && precision >= PHI4_FP32 && precision <= PHI4_FP16;
}

int launch_mutate(const MutateArgs& a, int precision, hipStream_t s) {
  if (!mutate_supported(a.d, precision) || a.n < 0 || a.n_steps < 0) return PHI4_EINVAL;
  if (a.n == 0) return PHI4_OK;
  if (a.d > kFusedMaxSites || a.passes) {
    if (!a.large.z || !a.large.prop || !a.large.accp) return PHI4_EINVAL;
    return launch_mutate_large(a, a.large, precision, s);
  }
  const int dp = (a.d + 15) / 16 * 16;
  if (dp <= 16) return launch_dp<16, 1>(a, precision, s);
  if (dp <= 32) return launch_dp<32, 2>(a, precision, s);
  if (dp <= 64) return launch_dp<64, 4>(a, precision, s);
  // d > 64: each wave forms two or more column blocks' float32 products, and
  // splitting the rows would repeat that MFMA work in both waves of a set
  if (dp <= 128) return launch_dp<128, 4, 1>(a, precision, s);
  return launch_dp<256, 8, 1>(a, precision, s);   // 1024 threads would cap a wave at 128 VGPRs
}

}  // namespace phi4
