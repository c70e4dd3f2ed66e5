// Shared device helpers and internal launch interfaces of libphi4pmc.
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) written from its
// published definition; stream map (key = (seed, run), counter = (group,
// particle, step, level << 8 | purpose)) as stated in include/phi4pmc.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phi4pmc.h"

namespace phi4 {

// ------------------------------------------------------------------ Philox

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c.x;   // one 32x32 -> 64 multiply each
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
                   (uint32_t)p0);
  }
  return c;
}

__device__ __forceinline__ uint32_t counter3(uint32_t level, uint32_t purpose) {
  return (level << 8) | purpose;
}

// ((w >> 9) + 1/2) * 2^-23: odd multiples of 2^-24 inside (0, 1), exact in float32.
__device__ __forceinline__ float u01(uint32_t w) {
  return (static_cast<float>(w >> 9) + 0.5f) * 0x1p-23f;
}

// Box-Muller in float32: r = sqrt(-2 ln ua); (r cos 2 pi ub, r sin 2 pi ub).
// The hardware sine / cosine take their argument in revolutions, so 2 pi ub
// is never formed.  Angles in the second half-turn are folded onto the first
// (ub - 1/2, exact) with the sign carried by r: the pair (za, zb) and its
// negation then come from the two grid points ub and ub +- 1/2 through the
// same arithmetic, so the law of the float32 normals is exactly symmetric.
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& za, float& zb) {
  float r = __builtin_sqrtf(-2.0f * __logf(u01(wa)));
  float t = u01(wb);
  if (t >= 0.5f) {
    t -= 0.5f;
    r = -r;
  }
  za = r * __builtin_amdgcn_cosf(t);
  zb = r * __builtin_amdgcn_sinf(t);
}

// Four normals for sites 4*group .. 4*group+3 of one particle.
__device__ __forceinline__ float4 normals4(uint32_t group, uint32_t particle, uint32_t step,
                                           uint32_t c3, uint32_t seed, uint32_t run) {
  const uint4 w = philox4x32_10(make_uint4(group, particle, step, c3), seed, run);
  float4 z;
  box_muller(w.x, w.y, z.x, z.y);
  box_muller(w.z, w.w, z.z, z.w);
  return z;
}

// Word 0 of the call (0, particle, step, c3).
__device__ __forceinline__ uint32_t word0(uint32_t particle, uint32_t step, uint32_t c3,
                                          uint32_t seed, uint32_t run) {
  return philox4x32_10(make_uint4(0u, particle, step, c3), seed, run).x;
}

// ------------------------------------------------------------ reductions
//
// Fixed-order reductions: DPP inside each row of 16 lanes (pairs xor 1,
// xor 2, mirror in 8, mirror in 16 -- every lane of the row ends with the
// same bits), readlane of lanes 0, 16, 32, 48 for the four rows, and for a
// workgroup one partial per wave reduced again the same way.  Results are
// identical on every lane and deterministic for a fixed blockDim.

enum RedOp { kSum = 0, kMin = 1, kMax = 2 };

template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ double readlane64(double v, int lane) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_readlane(hi, lane), __builtin_amdgcn_readlane(lo, lane));
}

template <int OP>
__device__ __forceinline__ double red_op(double a, double b) {
  return OP == kSum ? a + b : OP == kMin ? fmin(a, b) : fmax(a, b);
}

template <int OP>
__device__ __forceinline__ double wave_red(double v) {
  v = red_op<OP>(v, dpp64<0xB1>(v));
  v = red_op<OP>(v, dpp64<0x4E>(v));
  v = red_op<OP>(v, dpp64<0x141>(v));
  v = red_op<OP>(v, dpp64<0x140>(v));
  const double r0 = readlane64(v, 0), r1 = readlane64(v, 16);
  const double r2 = readlane64(v, 32), r3 = readlane64(v, 48);
  return red_op<OP>(red_op<OP>(r0, r1), red_op<OP>(r2, r3));
}

template <int OP>
__device__ __forceinline__ double red_identity() {
  return OP == kSum ? 0.0 : OP == kMin ? INFINITY : -INFINITY;
}

__device__ __forceinline__ double wave_sum(double v) { return wave_red<kSum>(v); }
__device__ __forceinline__ double wave_min(double v) { return wave_red<kMin>(v); }
__device__ __forceinline__ double wave_max(double v) { return wave_red<kMax>(v); }
__device__ __forceinline__ double wave_sum_dpp(double v) { return wave_red<kSum>(v); }

// float sum over a wave (fixed order, every lane gets the same bits)
__device__ __forceinline__ float wave_sum_f(float v) {
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x140, 0xF, 0xF, false));
  const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0));
  const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16));
  const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
  const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48));
  return (r0 + r1) + (r2 + r3);
}

// Workgroup reductions for NW waves (blockDim = 64 NW).  The per-wave
// results go through LDS; with at most 8 waves every thread sums them in
// wave order, otherwise they are reduced once more like a wave.  `sh` needs
// NW doubles (block_reduce) or 4 NW doubles (block_sum4).  Every thread gets
// the result.
template <int OP, int NW>
__device__ __forceinline__ double block_reduce(double v, double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = wave_red<OP>(v);
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  if constexpr (NW <= 8) {
    double r = sh[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) r = red_op<OP>(r, sh[w]);
    return r;
  } else {
    const double x = lane < NW ? sh[lane] : red_identity<OP>();
    return wave_red<OP>(x);
  }
}

template <int NW>
__device__ __forceinline__ void block_sum4(double& a, double& b, double& c, double& e,
                                           double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  a = wave_red<kSum>(a);
  b = wave_red<kSum>(b);
  c = wave_red<kSum>(c);
  e = wave_red<kSum>(e);
  __syncthreads();
  if (lane == 0) {
    sh[wid] = a;
    sh[NW + wid] = b;
    sh[2 * NW + wid] = c;
    sh[3 * NW + wid] = e;
  }
  __syncthreads();
  if constexpr (NW <= 8) {
    a = sh[0];
    b = sh[NW];
    c = sh[2 * NW];
    e = sh[3 * NW];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      a += sh[w];
      b += sh[NW + w];
      c += sh[2 * NW + w];
      e += sh[3 * NW + w];
    }
  } else {
    const bool in = lane < NW;
    a = wave_red<kSum>(in ? sh[lane] : 0.0);
    b = wave_red<kSum>(in ? sh[NW + lane] : 0.0);
    c = wave_red<kSum>(in ? sh[2 * NW + lane] : 0.0);
    e = wave_red<kSum>(in ? sh[3 * NW + lane] : 0.0);
  }
}

// --------------------------------------------------------------- states

// Device-resident state of one SMC run (in the caller's workspace).
struct SmcState {
  double beta;         // inverse temperature after the last reweight
  double logz;         // running log Z estimate
  double eps;          // step scale of the next sweep
  double eps0;
  double acc_target;
  double ess_frac;
  double last_dbeta;
  double last_ess;
  double last_acc;     // acceptance of the last finished sweep
  double tau;          // jitter of the last factorisation
  double mean_abs_m;   // filled by the observables kernel
  int32_t level;       // reweights done (the Philox level of the current sweep)
  int32_t done;        // 1 once the sweep at beta = 1 has finished
  int32_t err;         // sticky device error (PHI4_E*)
  int32_t solve_iters; // Newton evaluations of the last beta solve
  unsigned long long acc;   // accepted proposals of the current sweep
  unsigned long long prop;  // proposals of the current sweep
};

// Device-resident state of one nested-sampling run.
struct NsState {
  double logX;         // log prior volume enclosed by the current constraint
  double logZ;         // running log evidence (-inf before the first deletion)
  double hsum;         // sum_j exp(log w_j - logZ) log L_j
  double logmz;        // log sum_j w_j |M_j|
  double eps;
  double eps0;
  double acc_target;
  double last_acc;
  double tau;
  double H;            // information, set when done
  float s_star;        // action of the last deleted point (constraint S < s_star)
  int32_t iter;        // iterations done (the Philox level of the current refill)
  int32_t done;
  int32_t err;
  unsigned long long acc;
  unsigned long long prop;
};

// ------------------------------------------------------ kernel interfaces

// Scratch of the large-lattice sweep (k_large.hip) for n particles: normals
// (n x large_dz(d) floats), proposals (n x d floats), per-particle
// acceptance counts (n int32, zero between sweeps), the factor in the
// operand layout of the proposal product (large_dz(d)^2 floats) and the sign
// bit of each row's first normal (n uint16, 16-bit forms).
struct LargeScratch {
  float* z;
  float* prop;
  int32_t* accp;
  void* lp;
  unsigned short* zsgn;
};

struct MutateArgs {
  const float* src;        // input rows
  float* dst;              // output rows (may equal src unless src_rows is set)
  const int32_t* rows;     // physical row of tile slot i (NULL: i)
  const int32_t* src_rows; // source row of slot i's initial field (NULL: its own row);
                           // the resampling ancestors, dst != src
  int32_t n;               // rows processed
  int32_t L, d;
  float m2, lam;
  const float* Bt;         // Bt[k * ldb + c] = eps L[c][k]
  int32_t ldb;
  int32_t kind;            // 0 tempered, 1 constrained
  float beta;              // used if beta_ptr == NULL
  const double* beta_ptr;  // device beta (SMC state)
  float s_star;            // used if sstar_ptr == NULL
  const float* sstar_ptr;
  float inv_prior_var;
  uint32_t seed, run;
  int32_t level;           // used if level_ptr == NULL
  const int32_t* level_ptr;
  int32_t step0, n_steps;
  float zsign;
  const int32_t* done_ptr; // if *done_ptr != 0: no Metropolis steps; rows are still
                           // copied (with their action) when dst != src
  float* S;                // out: action of final rows (indexed by row)
  float* absM;             // out (optional)
  unsigned long long* acc_count;
  unsigned long long* prop_count;
  uint8_t* acc_flags;      // test output (optional), indexed by tile slot
  float* prop;             // test output (optional), indexed by tile slot
  LargeScratch large;      // scratch of the three-pass sweep
  int32_t passes;          // 1: three passes per step even for d <= kFusedMaxSites
  hipEvent_t ev_start;     // if set: timing events recorded by the fused sweep's own
  hipEvent_t ev_stop;      // dispatch (no separate event packets on the stream)
};

// k_mutate.hip (fused sweep, d <= kFusedMaxSites; larger d goes to k_large.hip)
constexpr int kFusedMaxSites = 256;
int launch_mutate(const MutateArgs& a, int precision, hipStream_t s);
int mutate_supported(int d, int precision);

// k_large.hip: per-step passes for d > kFusedMaxSites (scratch: LargeScratch).
int large_dz(int d);
size_t large_scratch_bytes(int n, int d);
LargeScratch large_scratch(void* base, int n, int d);
void launch_large_init(const LargeScratch& w, int n, hipStream_t s);
// Tile (particles; columns and threads into *cols, *threads) the proposal
// product uses at this shape on the current device once it has been timed
// (0 before).
int large_tile_choice(int n, int d, int precision, int* cols, int* threads);
// Pins the tile of a shape on the current device (false: not a tile choice).
bool large_set_tile(int n, int d, int precision, int rows, int cols, int threads);
int launch_mutate_large(const MutateArgs& a, const LargeScratch& w, int precision, hipStream_t s);

// k_field.hip
void launch_init_fields(float* phi, float* S, float* absM, int n, int L, float m2, float lam,
                        float scale, uint32_t seed, uint32_t run, hipStream_t s);
void launch_action(const float* phi, int n, int L, float m2, float lam, float* S, float* absM,
                   hipStream_t s);
void launch_normals(uint32_t seed, uint32_t run, int level, int step, int purpose,
                    const int32_t* rows, int n, int d, float* out, hipStream_t s);
void launch_gather(const float* src, const float* srcS, const int32_t* anc, int n, int d,
                   float* dst, float* dstS, const int32_t* done, hipStream_t s);

// k_reweight.hip
struct ReweightArgs {
  const float* S;
  int32_t n;
  SmcState* st;            // SMC state (NULL: stand-alone mode below)
  double beta_in, ess_frac_in;
  double* out;             // stand-alone outputs [4]: dbeta, new beta, dlogz, ess
  double* w;               // optional weights out
  // resampling
  uint32_t seed, run;
  int32_t do_resample;
  unsigned long long* cdf; // n
  int32_t* marks;          // n
  int32_t* anc;            // n
  SmcState* mirror;        // optional host-mapped copy of the state after the reweight
};
void launch_reweight(const ReweightArgs& a, hipStream_t s);
void launch_resample_weights(const double* w, int n, uint32_t U, unsigned long long* cdf,
                             int32_t* marks, int32_t* anc, int32_t* status, hipStream_t s);

// k_factor.hip
struct CovPlan {
  int d, n;
  int nb;       // 16-site blocks: ceil(d / 16)
  int blocks;   // lower-triangular 16 x 16 output blocks: nb (nb + 1) / 2
  int chunks;   // particle chunks (one partial per chunk and block)
  int chunk;    // particles per chunk (multiple of 4)
};
CovPlan cov_plan(int n, int d);
// Covariance work area (one float buffer): per-chunk float32 partials of
// M2 and of the first moments, their float64 sums over the chunks, and one
// arrival counter per block (zero between launches, see launch_cov_init).
struct CovWork {
  float* part;    // chunks * blocks * 256
  float* part1;   // chunks * nb * 16
  double* fin;    // blocks * 256: M2 summed over the chunks
  double* fin1;   // nb * 16: first moments summed over the chunks
  int32_t* cnt;   // blocks
};
__host__ __device__ inline CovWork cov_work(const float* base, const CovPlan& p) {
  float* b = const_cast<float*>(base);
  CovWork w;
  size_t o = (size_t)p.chunks * p.blocks * 256;
  w.part = b;
  w.part1 = b + o;
  o += (size_t)p.chunks * p.nb * 16;
  o = (o + 1) & ~(size_t)1;                 // 8-byte alignment for the sums
  w.fin = reinterpret_cast<double*>(b + o);
  o += 2 * (size_t)p.blocks * 256;
  w.fin1 = reinterpret_cast<double*>(b + o);
  o += 2 * (size_t)p.nb * 16;
  w.cnt = reinterpret_cast<int32_t*>(b + o);
  return w;
}
size_t cov_partial_floats(const CovPlan& p);
// Zeroes the arrival counters (once per work area; the reducing workgroup of
// each launch leaves them at zero again).
void launch_cov_init(float* part, const CovPlan& p, hipStream_t s);
void launch_cov_partials(const float* phi, const int32_t* rows, const CovPlan& p, float* part,
                         const int32_t* done, hipStream_t s);
// Reduces the partials, forms sigma (d*d doubles, written if sigma_out),
// factorises with jitter into Lw (d*d doubles) and, if Bt, emits
// Bt[k*ldb+c] = eps * L[c][k] (float32) with eps read from eps_ptr.
struct FactorArgs {
  const float* part;
  CovPlan plan;
  double* sigma_out;       // optional: the covariance
  const double* sigma_in;  // optional: factorise this instead of the partials
  double* A;               // d*d scratch / the factor (lower)
  float* Bt;
  int32_t ldb;
  const double* eps_ptr;
  double* tau_out;
  int32_t* err_out;
  const int32_t* done;
  int32_t cov_only;        // stop after writing sigma_out
  int32_t* bstatus;        // blocked factor (d > 64): kJitterAttempts + 1 ints of status
  double* Aspec;           // blocked factor: matrices of attempts 1 .. attempts-1, then
  double* Winv;            //   attempts 64 x 64 factored diagonal blocks (staging)
  int32_t attempts;        // jitter attempts run side by side (blocked_attempts(d))
};
// Jitter attempts of the factorisation (tau0, then five times x100).
constexpr int kJitterAttempts = 6;
// Attempts the blocked factor runs side by side at size d (0 for d <= 64),
// and the float64 scratch it needs besides A: blocked_scratch_doubles(d),
// to be split as Aspec = base, Winv = base + (attempts - 1) d d.
int blocked_attempts(int d);
size_t blocked_scratch_doubles(int d);
void launch_factor(const FactorArgs& a, hipStream_t s);

// k_ns.hip
struct NsArgs {
  float* phi;        // fields, updated in place
  float* S;
  float* absM;
  int32_t n, k, d;
  NsState* st;
  uint32_t seed, run;
  unsigned long long* keys;  // n sort keys
  int32_t* dead_rows;        // k rows to refill (output)
  int32_t* surv_rows;        // n-k survivors in deletion order (output)
  double* scratch;           // 2k doubles: log X_j, log w_j
  double term_frac;
};
void launch_ns_select(const NsArgs& a, hipStream_t s);
void launch_ns_seed_copy(const NsArgs& a, hipStream_t s);

// small state kernels (k_reweight.hip)
void launch_smc_state_init(SmcState* st, double eps0, double acc_target, double ess_frac,
                           hipStream_t s);
void launch_ns_state_init(NsState* st, double eps0, double acc_target, hipStream_t s);
void launch_mean_abs(const float* absM, int n, double* out, const int32_t* done, hipStream_t s);
struct BatchStatus {
  double beta;
  int32_t level, done, err, pad;
};
void launch_batch_status(const SmcState* const* st, int runs, BatchStatus* out, hipStream_t s);

}  // namespace phi4
