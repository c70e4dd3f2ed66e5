/*
 * phi4pmc -- particle Monte Carlo samplers for 2D lattice phi^4 on MI355X (gfx950).
 *
 * C ABI of the hot path of "Particle Monte Carlo methods for Lattice Field
 * Theory" (arXiv 2511.15196): the batched covariance-preconditioned
 * random-walk Metropolis mutation of adaptive tempered SMC and of nested
 * sampling, with the reweighting, log Z, systematic resampling and
 * covariance / Cholesky re-estimate between mutation sweeps.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named *_host are host memory; every other array pointer is
 *   device memory on the current HIP device.  The library never allocates
 *   or frees device memory: the caller owns all buffers, including the
 *   workspace, and keeps them alive until the handle is destroyed.
 * - Particle fields are float32 rows of d = L*L sites, row-major, site
 *   (x0, x1) at x0*L + x1 (x1 fastest); particle i starts at phi + i*d.
 * - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *   stream-ordered; calls that fill a *_host output synchronise `stream`,
 *   the others return as soon as the work is enqueued.
 * - Return value: PHI4_OK (0), PHI4_DONE (1: beta reached 1 / nested
 *   sampling terminated) or a negative error code; phi4_last_error() gives a
 *   thread-local message.  No C++ exception crosses this boundary.
 *   Rejected or non-finite proposals are not errors (they are rejected).
 * - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key
 *   (seed, run) and counter (group, particle, step, level << 8 | purpose);
 *   the normal for site x is word x%4 of the call with group x/4 via
 *   Box-Muller on words (0,1) and (2,3); uniforms are
 *   ((w >> 9) + 1/2) * 2^-23.  A fixed seed on the same GPU and build gives
 *   bitwise-identical results.
 */
#ifndef PHI4PMC_H
#define PHI4PMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PHI4_OK = 0,
  PHI4_DONE = 1,
  PHI4_EINVAL = -1,     /* bad argument or shape */
  PHI4_EHIP = -2,       /* a HIP runtime call failed */
  PHI4_ECHOL = -3,      /* covariance not factorisable after jitter escalation */
  PHI4_ENONFINITE = -4  /* non-finite actions / weights or a stalled beta solve */
};

/* Precision of the proposal product eps * L * z (operands; accumulation is
 * always float32).  Reduced precision rounds z and L to nearest-even, which
 * keeps the increment an odd function of z and the proposal symmetric. */
enum { PHI4_FP32 = 0, PHI4_BF16 = 1, PHI4_FP16 = 2 };

/* Philox stream purposes (low byte of counter word 3). */
enum { PHI4_INIT = 1, PHI4_PROPOSE = 2, PHI4_ACCEPT = 3, PHI4_RESAMPLE = 4, PHI4_NS_PICK = 5,
       PHI4_SLICE = 6 };

/* Largest lattice, d = L*L sites: the register-resident fused sweep covers
 * d <= 256, the three-pass sweep the rest. */
#define PHI4_MAX_SITES 4096

/* Inner (rejuvenation) kernels of SMC.
 * PHI4_KERNEL_RW: random-walk Metropolis, phi' = phi + eps L z (Sec. 2 (i);
 *   App. A), eps adapted per level toward acc_target.
 * PHI4_KERNEL_IRMH: independent Metropolis-Hastings (Sec. 2 (ii); App. A),
 *   phi' = mu + L z with mu and L L^T the mean and the jittered covariance
 *   of the resampled particles, log alpha = -dU0 - beta dS + (|z|^2 - r) / 2
 *   with r = |L^{-1}(phi - mu)|^2 of the current particle.  float32 only,
 *   d <= PHI4_IRMH_MAX_SITES; eps0 and acc_target are unused (the eps that
 *   phi4_observables reports is then meaningless).
 * PHI4_KERNEL_HMC: Hamiltonian Monte Carlo (Sec. 2 (iii); App. A),
 *   n_leapfrog leapfrog steps per trajectory on V = U0 + beta S with the
 *   diagonal mass diag(1 / v), v the site variances of the resampled
 *   particles; momentum p = z / sqrt(v) with z from the PROPOSE stream;
 *   accept iff log u < -(H' - H).  eps0 <= 0 selects d^(-1/4); eps is
 *   steered to acc_target like the random walk's.  float32 only; each
 *   level forms the site variances only (no covariance, no factor). */
enum { PHI4_KERNEL_RW = 0, PHI4_KERNEL_IRMH = 1, PHI4_KERNEL_HMC = 2 };
#define PHI4_IRMH_MAX_SITES 1024

/* One adaptive tempered SMC run (Sec. 2 "Particle-based Monte Carlo
 * methods" (i) - (iii); App. A).  Target p_beta ~ exp(-[U0 + beta S]) with
 * U0 = |phi|^2 / 2 and S the action of Sec. 2 Eq. (1); log Z estimates
 * log E_{phi ~ N(0, I)}[exp(-S(phi))]. */
typedef struct phi4_smc_config {
  int32_t L;            /* lattice side, d = L*L in [1, PHI4_MAX_SITES] */
  int32_t N;            /* particles, >= 2 */
  double m2;            /* bare mass squared m0^2 */
  double lambda;        /* quartic coupling */
  double ess_frac;      /* target ESS / N for the next beta, in (0, 1] */
  int32_t n_steps;      /* Metropolis steps per tempering level, >= 0 */
  double acc_target;    /* acceptance the step size is steered to (e.g. 0.3) */
  double eps0;          /* initial step scale; <= 0 selects 2.38 / sqrt(d) (App. A) */
  uint32_t seed;        /* Philox key word 0 */
  uint32_t run;         /* Philox key word 1 */
  int32_t precision;    /* PHI4_FP32 / PHI4_BF16 / PHI4_FP16 */
  int32_t kernel;       /* inner kernel: PHI4_KERNEL_RW (0), _IRMH (1) or _HMC (2) */
  int32_t n_leapfrog;   /* HMC: leapfrog steps per trajectory, 0 selects 20 (App. A), <= 1000 */
} phi4_smc_config;

/* One nested-sampling run (Sec. 2 (iv); App. A) with a likelihood-
 * constrained random-walk refill.  Prior N(0, prior_var I), likelihood
 * exp(-S); log Z estimates log E_{phi ~ N(0, prior_var I)}[exp(-S(phi))]. */
typedef struct phi4_ns_config {
  int32_t L;            /* lattice side, d = L*L in [1, PHI4_MAX_SITES] */
  int32_t n_live;       /* live points n, >= 3 */
  int32_t k_delete;     /* points deleted and refilled per iteration, 0 < k < n-1 */
  int32_t n_steps;      /* constrained Metropolis steps per refill */
  double m2;
  double lambda;
  double prior_var;     /* prior variance per site (e.g. 4.0) */
  double term_frac;     /* stop when the live evidence fraction drops below this */
  double acc_target;
  double eps0;          /* <= 0 selects 2.38 / sqrt(d) */
  uint32_t seed;
  uint32_t run;
  int32_t precision;
  int32_t kernel;       /* refill: PHI4_NS_RW (0) or PHI4_NS_SLICE (1) */
} phi4_ns_config;

/* Refill kernels of nested sampling.
 * PHI4_NS_RW: n_steps likelihood-constrained random-walk Metropolis steps,
 *   phi' = phi + eps L z, eps steered to acc_target.
 * PHI4_NS_SLICE: n_steps hit-and-run slice moves (the paper's NS kernel,
 *   Sec. 2 (iv); App. A) of the prior restricted to S < S*, along directions
 *   L z (L the factor of the survivors' covariance, z from the PROPOSE
 *   stream), Neal's stepping-out (w = 1, at most 31 expansions) and
 *   shrinkage (at most 64 draws, else the point stays); uniforms from the
 *   SLICE stream, the j-th being word j mod 4 of the call (j / 4, row,
 *   step, iteration << 8 | PHI4_SLICE).  float32 only; eps0 and acc_target
 *   are unused, the acceptance reported is the fraction of moves. */
enum { PHI4_NS_RW = 0, PHI4_NS_SLICE = 1 };

/* ------------------------------------------------------------------ SMC */

/* Bytes of device workspace smc_init needs for this configuration
 * (0 if the configuration is invalid). */
size_t smc_workspace_bytes(const phi4_smc_config* cfg);

/* Starts a run: draws phi_i ~ N(0, I) from the INIT stream into phi
 * (N*d floats), writes S(phi_i) into S (N floats), sets beta = 0,
 * log Z = 0, eps = eps0.  phi, S and workspace (>= smc_workspace_bytes,
 * 256-byte aligned) stay owned by the caller; *handle receives host
 * metadata only.  After smc_init, smc_mutate and smc_run the current
 * particles are in phi / S; smc_reweight_resample leaves them there and
 * keeps the resampling ancestors in the workspace, and the next smc_mutate
 * starts particle i from ancestor anc[i] (inside smc_run the particles
 * alternate between phi / S and a workspace copy and are back in phi / S
 * when it returns). */
int smc_init(const phi4_smc_config* cfg, float* phi, float* S, void* workspace,
             size_t workspace_bytes, void* stream, void** handle);

/* Restarts the run of `handle` with Philox key (seed, run): redraws the
 * initial particles into the same buffers and resets beta, log Z and eps,
 * exactly as smc_init does, without any allocation. */
int smc_restart(void* handle, uint32_t seed, uint32_t run);

/* One reweighting step (Sec. 2 tempered family; App. A adaptive target
 * ESS): finishes the step-size adaptation of the previous sweep
 * (log eps += acceptance - acc_target, clamped to [eps0/100, 10 eps0]),
 * picks dbeta so that ESS(-dbeta S) = ess_frac * N (dbeta = 1 - beta if
 * that already suffices), adds LSE(-dbeta S) - log N to log Z (float64),
 * resamples systematically on the integer CDF (RESAMPLE word of this
 * level), re-estimates the particle covariance over the resampled
 * particles and its jittered float64 Cholesky factor L, and prepares
 * eps * L for the next sweep.  *beta_host (optional) receives the new
 * beta.  Returns PHI4_DONE without work once the run is complete. */
int smc_reweight_resample(void* handle, double* beta_host);

/* n_steps random-walk Metropolis steps of every particle at the current
 * beta, proposal phi' = phi + eps * L z (App. A: particle covariance
 * scaled by 2.38^2 / V), accepted iff log u < -(U0(phi') - U0(phi))
 * - beta (S(phi') - S(phi)).  The first sweep after a reweight reads the
 * resampled population.  *acc_host (optional) receives the acceptance
 * rate of this sweep. */
int smc_mutate(void* handle, double* acc_host);

/* Native driver: alternates smc_reweight_resample and smc_mutate until the
 * sweep at beta = 1 is done (at most max_levels levels).  *levels_host
 * (optional) receives the number of levels. */
int smc_run(void* handle, int32_t max_levels, int32_t* levels_host);

/* Batched form (Sec. 2 tempered SMC, many independent runs): advances the
 * n_runs SMC handles together until every run has finished its sweep at
 * beta = 1 or max_levels levels have run (levels go in pairs after the first,
 * so a run may take max_levels + 1).  The first level of every run is
 * enqueued on the run's own stream; then two levels of all runs are captured
 * into one hipGraph (independent runs on separate branches, parameters read
 * from device memory, finished runs' kernels return at once) and the graph
 * is replayed on a private stream, with the runs' levels, beta and errors
 * gathered into one status read after each replay.  `stream` is the caller's
 * stream: it and the runs' streams are synchronised before the first level,
 * and the call returns with all work complete.  The runs' shapes, couplings and
 * precisions may all differ; each handle keeps its own buffers.  On return
 * the particles of every run are in its phi / S, levels_host[r] (may be
 * NULL) holds run r's level count, and logz / phi4_observables report each
 * run.  Returns PHI4_DONE when every run finished, PHI4_OK when max_levels
 * came first, or the first device error.  Allocates a few small buffers,
 * streams and the graph for the duration of the call; the handles must not
 * be used concurrently by other calls. */
int smc_batch_run(void* const* handles, int32_t n_runs, int32_t max_levels, int32_t* levels_host,
                  void* stream);

/* ------------------------------------------------------- nested sampling */

size_t ns_workspace_bytes(const phi4_ns_config* cfg);

/* Draws n_live points phi_i ~ N(0, prior_var I) (INIT stream) into phi
 * (n_live*d floats) with their actions in S; log X = 0, log Z = -inf. */
int ns_init(const phi4_ns_config* cfg, float* phi, float* S, void* workspace,
            size_t workspace_bytes, void* stream, void** handle);

/* One nested-sampling iteration: termination test
 * (log X + LSE(log L_live) - log n - log Z < log term_frac), then deletion
 * of the k_delete lowest-likelihood points (ties by row index), float64
 * prior-volume and evidence bookkeeping
 * (log X_j = log X - sum_{m<=j} 1/(n-m), w_j = L_j (X_{j-1} - X_j)),
 * seeds drawn uniformly from the survivors (NS_PICK stream), covariance of
 * the survivors, and n_steps constrained steps of the new points
 * (accept iff S(phi') < S* and log u < -(|phi'|^2 - |phi|^2) / (2 prior_var)).
 * *done_host (optional) receives 1 once the run has terminated; the final
 * live points are then already added to log Z. */
int ns_step(void* handle, int32_t* done_host);

/* --------------------------------------------------------- both samplers */

/* Current log Z (float64).  *stderr_host: nested sampling sqrt(H / n);
 * SMC has no single-run error bar and gets NaN. */
int logz(void* handle, double* logz_host, double* stderr_host);

/* Observables of the current population, synchronous:
 * out_host[0] = <|M|> (SMC: mean over the current particles; NS: posterior
 *               weighted over dead and live points once done, else the
 *               dead points so far),
 * out_host[1] = beta (SMC) or log X (NS),
 * out_host[2] = acceptance rate of the last sweep,
 * out_host[3] = eps of the next sweep,
 * out_host[4] = number of levels / iterations done,
 * out_host[5] = last dbeta (SMC) or S* (NS),
 * out_host[6] = ESS of the last reweight (SMC) or information H (NS),
 * out_host[7] = jitter tau of the last factorisation,
 * out_host[8] = evaluations of the last beta solve (SMC) or 0 (NS),
 * out_host[9] = 1 once the run is complete, else 0. */
int phi4_observables(void* handle, double* out_host);

/* Form of the Metropolis sweep of smc_mutate / smc_run / ns_step:
 * PHI4_SWEEP_AUTO (default) runs the fused register-resident sweep for
 * d <= 256 and three passes per step (normals, proposal product, accept)
 * above; PHI4_SWEEP_FUSED and PHI4_SWEEP_PASSES force one form
 * (PHI4_SWEEP_FUSED only for d <= 256).  Both forms draw the same Philox
 * streams and take the same decisions up to float32 rounding. */
#define PHI4_SWEEP_AUTO 0
#define PHI4_SWEEP_FUSED 1
#define PHI4_SWEEP_PASSES 2
int phi4_set_sweep(void* handle, int32_t form);

/* Tile of the three-pass proposal product (autotuned).  The first sweep of a
 * shape (n particles, d sites, precision) on a device times each workgroup
 * tile (particles x columns x threads: 32 x 64, 64 x 64, 128 x 64 and
 * 128 x 128 with 256 threads, 128 x 128 with 512) on the caller's stream and
 * keeps the fastest for the process.  *rows_host, *cols_host and
 * *threads_host receive the tile chosen for the current device, or 0 if that
 * shape has not run yet.  Host-only, never fails for valid pointers. */
int phi4_tile_choice(int32_t n, int32_t d, int32_t precision, int32_t* rows_host,
                     int32_t* cols_host, int32_t* threads_host);

/* Pins the proposal-product tile of a shape on the current device instead of
 * timing it (one of the tiles above): for reproducible launches and for
 * tests of every tile.  PHI4_EINVAL for another tile or a bad shape.
 * Host-only. */
int phi4_set_tile(int32_t n, int32_t d, int32_t precision, int32_t rows, int32_t cols,
                  int32_t threads);

/* Kernel timing: while enabled, every mutation launch of
 * smc_mutate / smc_run / ns_step is timed by a pair of HIP events on the
 * handle's stream: the fused random-walk sweep (d <= 256) records them on its
 * own dispatch packet, every other mutation launch is bracketed by two event
 * records (the no-op launch smc_run enqueues after the final sweep is not
 * counted). */
int phi4_set_timing(void* handle, int32_t enabled);

/* Synchronises the handle's stream and returns the summed duration (ms) and
 * the number of the mutation launches recorded since the previous call. */
int phi4_kernel_time(void* handle, double* ms_host, int32_t* launches_host);

/* Releases the host metadata.  Caller memory is untouched. */
int phi4_destroy(void* handle);

/* Thread-local description of the last error ("" if none). */
const char* phi4_last_error(void);

/* ------------------------------------------ step-level entry points
 * The same kernels the samplers use, on caller-supplied inputs, for
 * parity checks and microbenchmarks. */

/* out[i*d + x] = normal of site x of particle rows[i] (rows NULL: i) at
 * (level, step, purpose) under key (seed, run), float32. */
int phi4_normals(uint32_t seed, uint32_t run, int32_t level, int32_t step, int32_t purpose,
                 const int32_t* rows, int32_t n, int32_t d, float* out, void* stream);

/* Action of Sec. 2 Eq. (1) per particle: S[i] = sum_x s_x(phi_i) and
 * absM[i] = |(1/d) sum_x phi_ix| (absM may be NULL), float32. */
int phi4_action(const float* phi, int32_t N, int32_t L, double m2, double lambda,
                float* S, float* absM, void* stream);

/* Systematic resampling on the integer CDF of float64 weights w[0..N)
 * (w >= 0, finite, max > 0): q_i = floor(2^k w_i / max w) with
 * k = 62 - 2 ceil(log2 N); ancestors[i] = min{ j : C_j > T_i },
 * T_i = floor((i Q + U Q / 2^32) / N) in exact integers.  Needs
 * phi4_step_workspace_bytes(N, 0) bytes of workspace. */
int phi4_resample_systematic(const double* w, int32_t N, uint32_t U, int32_t* ancestors,
                             void* workspace, size_t workspace_bytes, void* stream);

/* Reweighting of one SMC level on caller-given actions S[0..N) at
 * inverse temperature beta: out_host[0] = dbeta, [1] = new beta,
 * [2] = log Z increment, [3] = ESS; w (optional, N doubles) receives
 * exp(l_i - max l) with l_i = -dbeta S_i.  Synchronous. */
int phi4_reweight(const float* S, int32_t N, double beta, double ess_frac, double* w,
                  double* out_host, void* workspace, size_t workspace_bytes, void* stream);

/* Particle covariance (divisor N - 1) of the rows phi[rows[i]] (rows NULL:
 * all N rows), float32 accumulation of shifted products combined in
 * float64: sigma (d*d doubles, row-major, full symmetric). */
int phi4_covariance(const float* phi, const int32_t* rows, int32_t N, int32_t d, double* sigma,
                    void* workspace, size_t workspace_bytes, void* stream);

/* Jittered float64 Cholesky factor of sigma (d*d, symmetric): L lower
 * (d*d row-major, upper part zeroed) of sigma + tau I with
 * tau = 1e-10 tr(sigma)/d, multiplied by 100 after each failure, at most
 * five retries (PHI4_ECHOL after that).  *tau_host (optional) receives tau.
 * Synchronous. */
int phi4_cholesky(const double* sigma, int32_t d, double* L, double* tau_host,
                  void* workspace, size_t workspace_bytes, void* stream);

/* Workspace bytes the step-level entry points need for N particles of d sites. */
size_t phi4_step_workspace_bytes(int32_t N, int32_t d);

/* Whitened residuals of the independence sampler's current particles
 * (Sec. 2 (ii); App. A: the proposal density N(mu, L L^T) at phi is
 * proportional to exp(-r / 2)): mu = mean of the rows phi[rows[i]] (rows
 * NULL: rows 0..N-1) and r[i] = |L^{-1}(phi[rows[i]] - mu)|^2 for the lower
 * factor L (float64, d*d row-major, nonzero diagonal; the upper part is not
 * read), all arithmetic in float64.  r (N floats) and mu (optional, d floats)
 * receive the results rounded to float32.  Needs 1 <= N, 1 <= d <=
 * PHI4_IRMH_MAX_SITES and workspace >= phi4_whiten_workspace_bytes(N, d)
 * (256-byte aligned); returns PHI4_EINVAL otherwise.  Asynchronous on
 * stream. */
size_t phi4_whiten_workspace_bytes(int32_t N, int32_t d);
int phi4_whiten(const float* phi, const int32_t* rows, int32_t N, int32_t d, const double* L,
                float* r, float* mu, void* workspace, size_t workspace_bytes, void* stream);

/* n_steps fused Metropolis steps of the rows of src selected by rows
 * (rows NULL: rows 0..n-1), written to the same rows of dst (dst may equal
 * src).  Bt is the scaled factor transposed, Bt[k*d + c] = eps * L[c][k]
 * (float32, d*d, upper triangular incl. diagonal); the proposal is
 * phi' = phi + zsign * Bt^T z with z from the PROPOSE stream at
 * (level, step0 + s).  kind 0 (tempered): log alpha = -dU0 - beta dS;
 * kind 1 (constrained): accept iff S(phi') < s_star and
 * log u < -(|phi'|^2 - |phi|^2) / (2 prior_var).  S (N floats, per row)
 * and absM (optional) receive the action and |M| of the final rows.
 * acc_count (optional, device uint64) is incremented by the number of
 * accepted proposals.  Test outputs (optional): acc_flags[i] (uint8) = 1
 * if the last step accepted row i's proposal; prop[i*d..] = the last
 * step's proposal of row i.  precision: PHI4_FP32 / PHI4_BF16 / PHI4_FP16.
 * workspace (>= phi4_step_workspace_bytes(n, d), 256-byte aligned) is
 * scratch for d > 256, where a step is three passes (normals, proposal
 * product, accept) instead of the fused register-resident sweep; it may be
 * NULL for d <= 256. */
int phi4_mutate(const float* src, float* dst, const int32_t* rows, int32_t n, int32_t L,
                double m2, double lambda, const float* Bt, int32_t kind, double beta,
                double s_star, double prior_var, uint32_t seed, uint32_t run, int32_t level,
                int32_t step0, int32_t n_steps, float zsign, int32_t precision, float* S,
                float* absM, unsigned long long* acc_count, uint8_t* acc_flags, float* prop,
                void* workspace, size_t workspace_bytes, void* stream);

/* One slice move of each row phi[rows[i]] (rows NULL: i), i < n, along the
 * direction dirs[i*d ..] (float32, caller-given): the move the slice refill
 * of nested sampling makes (PHI4_NS_SLICE: prior N(0, prior_var I)
 * restricted to S < s_star, Neal's stepping-out and shrinkage, uniforms of
 * the SLICE stream at (level, step) with the row as particle).  S[row]
 * must hold the row's action on entry; rows that move get their new field,
 * S and (absM optional) |M|.  Rows must be distinct.  Asynchronous on
 * stream; no workspace. */
int phi4_slice_move(float* phi, const int32_t* rows, const float* dirs, int32_t n, int32_t L,
                    double m2, double lambda, double s_star, double prior_var, uint32_t seed,
                    uint32_t run, int32_t level, int32_t step, float* S, float* absM,
                    void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PHI4PMC_H */
