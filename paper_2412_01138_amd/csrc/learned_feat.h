// Learned coarse correction: device helpers shared by the training-row and
// correction kernels (network inputs of one slice and mode).
#pragma once

#include "pe_internal.h"

namespace pe {

// ---------------------------------------------------------------- learned G
// Orthonormal polynomial basis of the eight forcing sample times of a slice
// (points t_j = (j - 3.5)/3.5): q[j * 8 + i] = q_i(t_j).  Built on the host.
struct SampleBasis {
  double q[PE_MLP_SAMPLES * PE_MLP_SAMPLES];
};
SampleBasis sample_basis();

// Cp[n][i][m] = sum_j q_i(t_j) amp_m tau_m(t0 + n dT + j dT / 7): the
// polynomial coefficients of the forcing samples of slice n are
// c_i = sum_m Cp[n][i][m] prod_a spec_a[m][k_a] (the forcing is a sum of
// separable terms, so its spectral samples are too).
size_t learned_coef_bytes(pe_grid g, int N);
pe_status learned_coefs(pe_grid g, int N, double t0, double dT, double *Cp, hipStream_t st);

// z-features [ln z / 8, e^{-z}, phi_1(-z), 2 phi_2(-z)] in FP64 (series
// below z = 1e-3, where the closed forms cancel).
__device__ inline void z_features(double z, float *x) {
  const double e = exp(-z);
  double p1, p2;
  if (z < 1e-3) {
    p1 = 1.0 - z / 2 + z * z / 6 - z * z * z / 24;
    p2 = 0.5 - z / 6 + z * z / 24 - z * z * z / 120;
  } else {
    p1 = -expm1(-z) / z;
    p2 = (z - 1.0 + e) / (z * z);
  }
  x[0] = float(log(z) / 8.0);
  x[1] = float(e);
  x[2] = float(p1);
  x[3] = float(2.0 * p2);
}

// Sample features x[4..11] and the output scale s from the polynomial
// coefficients c[8] of the samples (|g| = |c|: the basis is orthonormal).
__device__ inline void coeff_features(const double *c, float *x, double &s) {
  double gn = 0.0, hn = 0.0;
  for (int i = 0; i < PE_MLP_SAMPLES; ++i) gn += c[i] * c[i];
  for (int i = 4; i < PE_MLP_SAMPLES; ++i) hn += c[i] * c[i];
  gn = sqrt(gn);
  s = sqrt(hn);
  const double ig = gn > 0.0 ? 1.0 / gn : 0.0, ih = s > 0.0 ? 1.0 / s : 0.0;
  for (int i = 0; i < 4; ++i) x[4 + i] = float(c[i] * ig);
  for (int i = 4; i < PE_MLP_SAMPLES; ++i) x[4 + i] = float(c[i] * ih);
}

// Eigenvalue sum lambda_k of natural mode index k (last axis fastest).
__device__ inline double mode_lambda(int d, int n1, int n2, const double *l0, const double *l1,
                                     const double *l2, int64_t k) {
  if (d == 1) return l0[k];
  if (d == 2) return l0[k / n1] + l1[k % n1];
  const int64_t k2 = k % n2, r = k / n2;
  return l0[r / n1] + l1[r % n1] + l2[k2];
}

}  // namespace pe
