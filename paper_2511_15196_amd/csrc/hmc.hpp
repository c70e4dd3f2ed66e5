// Internal interface of the Hamiltonian Monte Carlo inner kernel (SMC-HMC,
// Sec. 2 (iii); App. A).
#pragma once

#include "common.hpp"

namespace phi4 {

struct HmcArgs {
  const float* src;         // current fields, rows src_rows[p] (NULL: p)
  const int32_t* src_rows;  // resampling ancestors of slot p
  float* dst;               // output fields, row p (dst != src when src_rows is set)
  int32_t n, L, d;
  float m2, lam;
  const double* beta_ptr;   // inverse temperature (device)
  const double* eps_ptr;    // leapfrog step (device)
  const double* var;        // d site variances of the particles (float64): the inverse mass
  int32_t n_leap;           // leapfrog steps per trajectory
  int32_t n_steps;          // trajectories per sweep
  uint32_t seed, run;
  const int32_t* level_ptr;
  const int32_t* done;      // if *done: no trajectories, rows are only moved
  float* S;                 // out: action of the final rows (row p)
  float* absM;              // out (optional): |M| of the final rows
  unsigned long long* acc_count;
  unsigned long long* prop_count;
};

// One sweep: n_steps HMC steps of every particle, one workgroup per particle,
// the fields resident across the sweep.  d <= PHI4_MAX_SITES.
void launch_hmc_sweep(const HmcArgs& a, hipStream_t s);

// Site variances (divisor n - 1) of the rows phi[rows[i]] (rows NULL: i),
// float64, shifted by the first row as the covariance is: var[x] =
// (sum (phi - c)^2 - (sum (phi - c))^2 / n) / (n - 1).  part holds
// 2 * site_var_chunks(n) * d doubles.
int site_var_chunks(int n);
void launch_site_variance(const float* phi, const int32_t* rows, int n, int d, double* part,
                          double* var, const int32_t* done, hipStream_t s);

}  // namespace phi4
