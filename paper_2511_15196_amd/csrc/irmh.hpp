// Internal interfaces of the independent Metropolis-Hastings inner kernel
// (SMC-IRMH, Sec. 2 (ii); App. A): proposal N(mu, L L^T) from the mean and
// the jittered Cholesky factor of the resampled particles.
#pragma once

#include "common.hpp"

namespace phi4 {

// Scratch of the independence sampler for n particles of d sites.
struct IrmhScratch {
  float* mu;       // d: mean field of the resampled particles (float32 base row)
  double* mu64;    // d: the same mean in float64 (whitening)
  double* mpart;   // irmh_mean_chunks(n) x d partial column sums of the mean
  double* linv;    // d x d: linv[k][c] = Linv[c][k] for k <= c (transposed inverse)
  double* wpart;   // ceil(d / 64) x n partial sums of squares of the whitening
  float* r;        // n: |L^{-1}(phi - mu)|^2 of each slot's current field
  float* zz;       // 2 n: |z|^2 of this step's and the next step's normals
  double* one;     // 1.0: scale of the emitted factor (no random-walk step size)
};

int irmh_mean_chunks(int n);
size_t irmh_scratch_bytes(int n, int d);
IrmhScratch irmh_scratch(void* base, int n, int d);
// Sets `one`; once per handle.
void launch_irmh_init(const IrmhScratch& q, hipStream_t s);
// Mean of the rows phi[rows[i]] (rows NULL: i) into q.mu and q.mu64.
void launch_irmh_mean(const float* phi, const int32_t* rows, int n, int d, const IrmhScratch& q,
                      const int32_t* done, hipStream_t s);
// q.linv from the float64 lower factor A (row-major d x d).
void launch_irmh_inverse(const double* A, int d, const IrmhScratch& q, const int32_t* done,
                         hipStream_t s);
// q.r[p] = |L^{-1}(phi[rows[p]] - mu)|^2, float64 throughout.
void launch_irmh_whiten(const float* phi, const int32_t* rows, int n, int d, const IrmhScratch& q,
                        const int32_t* done, hipStream_t s);
// out[p] = sum_{k < d} x[p][k]^2 (row stride ld).
void launch_rowsq(const float* x, int ld, int n, int d, float* out, const int32_t* done,
                  hipStream_t s);

// k_large.hip: one sweep of n_steps independence-sampler steps.  a.Bt holds
// L^T (unscaled), A the float64 factor; the mean and the whitening factor
// of the particles a.src[a.src_rows] are formed first.
int launch_irmh_sweep(const MutateArgs& a, const double* A, const IrmhScratch& q,
                      hipStream_t s);

}  // namespace phi4
