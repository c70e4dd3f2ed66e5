// Internal interface of the slice-sampling refill of nested sampling
// (Sec. 2 (iv); App. A): hit-and-run slice moves of the prior restricted to
// the likelihood constraint, Neal's stepping-out and shrinkage.
#pragma once

#include "common.hpp"

namespace phi4 {

constexpr float kSliceWidth = 1.0f;   // w, in units of the direction L z
constexpr int kSliceMaxSteps = 32;    // m: at most m - 1 expansions in total
constexpr int kSliceMaxShrink = 64;   // shrinkage draws; if all miss, the point stays

struct SliceArgs {
  float* phi;               // fields, rows rows[p], updated in place
  const int32_t* rows;      // row of slot p
  const float* dirs;        // directions, slot-major [n][d] (float32)
  int32_t n, L, d;
  float m2, lam;
  const float* sstar_ptr;   // likelihood constraint S < S* (NULL: s_star)
  float s_star;
  float inv_prior_var;      // 1 / prior variance
  uint32_t seed, run;
  const int32_t* level_ptr; // NS iteration (NULL: level)
  int32_t level;
  uint32_t step;
  const int32_t* done;
  float* S;                 // action of each row (read, and written when it moves)
  float* absM;              // |M| of each row (written when it moves)
  int32_t* accp;            // per-slot count of moves (optional)
};

// One slice move of every slot (one workgroup per slot).
void launch_slice_moves(const SliceArgs& a, hipStream_t s);
// zero[0..d) = 0, *one = 1 (the base row of the direction product and the
// unit scale of the emitted factor); once per handle.
void launch_slice_init(float* zero, int d, double* one, hipStream_t s);

// k_large.hip: n_steps slice moves of the rows a.rows of a.dst: per step the
// normals, the directions z L^T (a.Bt = L^T) on the proposal-product kernel
// with the zero base row, and the moves.
int launch_slice_sweep(const MutateArgs& a, const float* zero, hipStream_t s);

}  // namespace phi4
