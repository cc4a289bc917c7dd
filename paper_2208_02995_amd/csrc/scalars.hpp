// CG scalars of Alg. 3 formed on the device by the kernel that consumes a
// reduction: every block sums the producer's per-block partials (the same
// order in every block, so all agree bitwise) and block 0 records them.
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace emin {

// Scalars after <Y, Y_hat> of iteration k (Alg. 3): delta is reduced from
// the masked product's partials by every block; alpha = gamma_k / delta,
// dE_k = gamma_k alpha (Sec. 3.3, eq. CG_dEa), the energy-monitor stop
// (eq. relRed) and breakdown when delta <= 0.  Block 0 records them.  Returns
// the stop code (0: apply the update) and alpha.
__device__ __forceinline__ int scalars_after_delta(const UpdArgs& a, double* alpha_out) {
  DevState* st = a.st;
  const int k = a.k;
  const double delta = sum_partials(a.part_in, a.np_in);
  const double gk = a.hist.gamma[k - 1];
  int stop = 0;
  double alpha = 0.0, dE = 0.0, dE1 = 0.0;
  if (!(delta > 0.0)) {
    stop = kBreakdown;
  } else {
    alpha = gk / delta;
    dE = gk * alpha;
    dE1 = (k == 1) ? dE : st->dE1;
    if (st->tau > 0.0 && dE < st->tau * dE1) stop = kTauStop;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->delta = delta;
    st->k = k;
    a.hist.delta[k - 1] = delta;
    a.hist.alpha[k - 1] = alpha;
    st->alpha = alpha;
    if (k == 1) st->dE1 = dE;
    if (stop) st->done = stop;
  }
  *alpha_out = alpha;
  return stop;
}

// Scalars after <R, Z> (gamma of iteration k + 1): reduced from the update
// kernel's partials by every block; relative floor (converged), negative
// (breakdown), beta = gamma_{k+1} / gamma_k.  Block 0 records them.
__device__ __forceinline__ int scalars_after_gamma(const UpdArgs& a, bool first, double* beta_out) {
  DevState* st = a.st;
  const int k = a.k;
  const double gamma = sum_partials(a.part_in, a.np_in);
  const double g1 = first ? gamma : st->gamma1;
  int stop = 0;
  double beta = 0.0;
  if (gamma < 0.0 || gamma != gamma) stop = kBreakdown;
  else if (gamma <= a.gamma_floor * g1) stop = kConverged;
  else if (!first) beta = gamma / a.hist.gamma[k - 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->iterations = k;
    if (first) st->gamma1 = gamma;
    st->gamma = gamma;
    st->beta = beta;
    if (k < a.k_max) {
      a.hist.gamma[k] = gamma;
      a.hist.beta[k] = beta;
    }
    if (stop) st->done = stop;
  }
  *beta_out = beta;
  return stop;
}

}  // namespace emin
