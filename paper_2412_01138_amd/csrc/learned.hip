// Learned coarse correction: forcing samples, training rows.
//
// The network input of slice n and mode k uses the spectral forcing at the
// eight times T_n + j dT / 7 (j = 0..7), expanded in orthonormal polynomials
// of those times.  The forcing is a sum of separable terms, so these
// coefficients come from the per-axis term spectra and a small per-slice
// table (learned_coefs) with no field transform.  pe_learned_samples still
// produces the samples themselves like the stage fields of a fine pass
// (quadrature + transform).  Training rows pair the inputs with the target
// (R_n - r_n)_k / (s dT), R_n = F^J(0) and r_n = G(0) of the same slice, s the
// size of the samples' part of degree >= 4; rows where it vanishes carry no
// information and are skipped (ordered, deterministic compaction).
#include <algorithm>
#include <cmath>

#include "learned_feat.h"

namespace pe {

// out[f][k] = sigma_k G[f][pos(k)] for `count` fields (natural mode order)
template <typename T>
__global__ void k_compact_fields(int d, int n0, int n1, int n2, int np0, int np1, int np2, int Kh0,
                                 int Kh1, int Kh2, const double *s0, const double *s1,
                                 const double *s2, const T *G, T *out, int64_t count, int64_t dof,
                                 int64_t dofp) {
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < count * dof;
       idx += int64_t(gridDim.x) * blockDim.x) {
    const int64_t f = idx / dof, k = idx - f * dof;
    int kk[3] = {0, 0, 0};
    int64_t r = k;
    const int n[3] = {n0, n1, n2};
    for (int a = d - 1; a >= 0; --a) {
      kk[a] = int(r % n[a]);
      r /= n[a];
    }
    const int np[3] = {np0, np1, np2}, Kh[3] = {Kh0, Kh1, Kh2};
    int64_t p = 0;
    for (int a = 0; a < d; ++a) p = p * np[a] + fold_pos(kk[a], Kh[a]);
    double sg = s0[kk[0]];
    if (d > 1) sg *= s1[kk[1]];
    if (d > 2) sg *= s2[kk[2]];
    out[idx] = T(sg * double(G[f * dofp + p]));
  }
}

// Gram-Schmidt (modified, applied twice) of the monomials 1, t, .., t^7 at
// t_j = (j - 3.5)/3.5.  Each q_i gets a positive leading coefficient.
SampleBasis sample_basis() {
  constexpr int S = PE_MLP_SAMPLES;
  SampleBasis B{};
  for (int i = 0; i < S; ++i) {
    double v[S];
    for (int j = 0; j < S; ++j) v[j] = std::pow((j - 3.5) / 3.5, i);
    for (int pass = 0; pass < 2; ++pass)
      for (int m = 0; m < i; ++m) {
        double d = 0.0;
        for (int j = 0; j < S; ++j) d += B.q[j * S + m] * v[j];
        for (int j = 0; j < S; ++j) v[j] -= d * B.q[j * S + m];
      }
    double nrm = 0.0;
    for (int j = 0; j < S; ++j) nrm += v[j] * v[j];
    nrm = std::sqrt(nrm);
    for (int j = 0; j < S; ++j) B.q[j * S + i] = v[j] / nrm;
  }
  return B;
}

static unsigned nblk(int64_t n) {
  int64_t b = (n + 255) / 256;
  return unsigned(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

static size_t sample_field_bytes(pe_grid g) {
  return 2 * field_bytes(g) + sizeof(double) * size_t(std::max(g->n_terms, 1));
}

// ---------------------------------------------------- sample coefficients
__global__ void k_learned_coefs(int N, double t0, double dT, const DevTerm *terms, int M,
                                SampleBasis B, double *Cp) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(N) * PE_MLP_SAMPLES * M) return;
  const int m = int(idx % M);
  const int i = int((idx / M) % PE_MLP_SAMPLES);
  const int n = int(idx / (int64_t(M) * PE_MLP_SAMPLES));
  const DevTerm tm = terms[m];
  double acc = 0.0;
  for (int j = 0; j < PE_MLP_SAMPLES; ++j) {
    const double t = (t0 + double(n) * dT) + (double(j) / 7.0) * dT;
    acc += B.q[j * PE_MLP_SAMPLES + i] * term_time(tm, t);
  }
  Cp[idx] = acc;
}

size_t learned_coef_bytes(pe_grid g, int N) {
  return Arena::need(sizeof(double) * size_t(N) * PE_MLP_SAMPLES * std::max(g->n_terms, 1));
}

pe_status learned_coefs(pe_grid g, int N, double t0, double dT, double *Cp, hipStream_t st) {
  const int64_t tot = int64_t(N) * PE_MLP_SAMPLES * g->n_terms;
  if (tot == 0) return PE_OK;
  k_learned_coefs<<<unsigned((tot + 255) / 256), 256, 0, st>>>(N, t0, dT, g->d_terms, g->n_terms,
                                                               sample_basis(), Cp);
  PE_HIP(hipGetLastError());
  return PE_OK;
}

// ------------------------------------------------------------ training rows
struct RowsArgs {
  int d, n0, n1, n2, M;
  const double *lam0, *lam1, *lam2;
  const double *sp0, *sp1, *sp2;   // per-axis term spectra [M][n_a]
  const double *Cp;                // [N][8][M]
  double D, dT;
  const void *R, *r;
  int fp64;
  int64_t dof, total;
};

// Polynomial coefficients c[8] of the forcing samples of row (n, k).
__device__ inline void row_coeffs(const RowsArgs &a, int64_t row, double *c) {
  const int64_t n = row / a.dof, k = row - n * a.dof;
  int k0 = 0, k1 = 0, k2 = 0;
  if (a.d == 1) {
    k0 = int(k);
  } else if (a.d == 2) {
    k0 = int(k / a.n1);
    k1 = int(k % a.n1);
  } else {
    k2 = int(k % a.n2);
    const int64_t r = k / a.n2;
    k0 = int(r / a.n1);
    k1 = int(r % a.n1);
  }
  for (int i = 0; i < PE_MLP_SAMPLES; ++i) c[i] = 0.0;
  const double *cp = a.Cp + n * PE_MLP_SAMPLES * a.M;
  for (int m = 0; m < a.M; ++m) {
    double G = a.sp0[int64_t(m) * a.n0 + k0];
    if (a.d > 1) G *= a.sp1[int64_t(m) * a.n1 + k1];
    if (a.d > 2) G *= a.sp2[int64_t(m) * a.n2 + k2];
    for (int i = 0; i < PE_MLP_SAMPLES; ++i) c[i] += cp[i * a.M + m] * G;
  }
}

__device__ inline double row_scale(const RowsArgs &a, int64_t row, double *c) {
  row_coeffs(a, row, c);
  double hn = 0.0;
  for (int i = 4; i < PE_MLP_SAMPLES; ++i) hn += c[i] * c[i];
  return sqrt(hn);
}

__global__ void k_rows_max(RowsArgs a, double *part) {
  __shared__ double sm[256];
  double mx = 0.0;
  for (int64_t row = int64_t(blockIdx.x) * 256 + threadIdx.x; row < a.total;
       row += int64_t(gridDim.x) * 256) {
    double c[PE_MLP_SAMPLES];
    mx = fmax(mx, row_scale(a, row, c));
  }
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ void k_rows_max_final(const double *part, int nb, double *out) {
  double mx = 0.0;
  for (int i = 0; i < nb; ++i) mx = fmax(mx, part[i]);
  *out = mx;
}

// counts[b] = qualifying rows of block b (one row per thread)
__global__ void k_rows_count(RowsArgs a, const double *smax, double rel, int *counts) {
  __shared__ int sc[4];
  const int64_t row = int64_t(blockIdx.x) * 256 + threadIdx.x;
  bool q = false;
  if (row < a.total) {
    double c[PE_MLP_SAMPLES];
    const double sg = row_scale(a, row, c);
    q = sg > rel * (*smax) && sg > 0.0;
  }
  const unsigned long long bal = __ballot(q);
  if ((threadIdx.x & 63) == 0) sc[threadIdx.x >> 6] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = sc[0] + sc[1] + sc[2] + sc[3];
}

// exclusive scan of the block counts (one block, in order); total -> *total
__global__ void k_rows_scan(const int *counts, int nb, int64_t *offsets, int64_t *total) {
  if (threadIdx.x != 0) return;
  int64_t acc = 0;
  for (int i = 0; i < nb; ++i) {
    offsets[i] = acc;
    acc += counts[i];
  }
  *total = acc;
}

__global__ void k_rows_write(RowsArgs a, const double *smax, double rel, const int64_t *offsets,
                             int64_t max_rows, float *x, float *tg, float *scale_out) {
  __shared__ int sc[4];
  const int64_t row = int64_t(blockIdx.x) * 256 + threadIdx.x;
  bool q = false;
  double c[PE_MLP_SAMPLES];
  double sg = 0.0;
  if (row < a.total) {
    sg = row_scale(a, row, c);
    q = sg > rel * (*smax) && sg > 0.0;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long bal = __ballot(q);
  if (lane == 0) sc[wave] = __popcll(bal);
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wave; ++w) before += sc[w];
  const int local = before + __popcll(bal & ((1ull << lane) - 1ull));
  const int64_t pos = offsets[blockIdx.x] + local;
  if (!q || pos >= max_rows) return;
  const int64_t k = row % a.dof;
  const double lam = mode_lambda(a.d, a.n1, a.n2, a.lam0, a.lam1, a.lam2, k);
  float f[PE_MLP_INPUTS];
  z_features(a.D * lam * a.dT, f);
  coeff_features(c, f, sg);
  for (int i = 0; i < PE_MLP_INPUTS; ++i) x[pos * PE_MLP_INPUTS + i] = f[i];
  const double Rv = a.fp64 ? static_cast<const double *>(a.R)[row]
                           : double(static_cast<const float *>(a.R)[row]);
  const double rv = a.fp64 ? static_cast<const double *>(a.r)[row]
                           : double(static_cast<const float *>(a.r)[row]);
  tg[pos] = float((Rv - rv) / (sg * a.dT));
  if (scale_out) scale_out[pos] = float(sg);
}

static RowsArgs rows_args(pe_grid g, int N, double dT, const double *Cp, const void *R,
                          const void *r) {
  RowsArgs a{};
  a.d = g->dim;
  a.M = g->n_terms;
  a.n0 = g->ax[0].n;
  a.n1 = g->dim > 1 ? g->ax[1].n : 1;
  a.n2 = g->dim > 2 ? g->ax[2].n : 1;
  a.lam0 = g->ax[0].d_lam;
  a.lam1 = g->ax[1].d_lam;
  a.lam2 = g->ax[2].d_lam;
  a.sp0 = g->d_spec[0];
  a.sp1 = g->d_spec[1];
  a.sp2 = g->d_spec[2];
  a.Cp = Cp;
  a.D = g->D;
  a.dT = dT;
  a.R = R;
  a.r = r;
  a.fp64 = g->precision == PE_FP64;
  a.dof = g->dof;
  a.total = int64_t(N) * g->dof;
  return a;
}

}  // namespace pe

using namespace pe;

extern "C" {

size_t pe_learned_samples_workspace_bytes(pe_grid g, int32_t n_slices) {
  if (!g || n_slices < 1) return 0;
  return 4 * 256 + size_t(n_slices) * PE_MLP_SAMPLES * sample_field_bytes(g);
}

pe_status pe_learned_samples(pe_grid g, int32_t n_slices, double t0, double dT, void *d_samples,
                             void *d_work, size_t work_bytes, void *stream) {
  clear_error();
  if (!g || !d_samples) return set_error(PE_E_ARG, "null argument");
  if (n_slices < 1 || !(dT > 0)) return set_error(PE_E_ARG, "bad n_slices / dT");
  if (g->n_hats > 0) return set_error(PE_E_ARG, "the learned inputs do not cover moving sources");
  if (has_periodic(g)) return set_error(PE_E_ARG, "the learned inputs are built for Dirichlet axes");
  hipStream_t st = as_stream(stream);
  const size_t sb = g->precision == PE_FP64 ? sizeof(double) : sizeof(float);
  if (g->n_terms == 0) {
    PE_HIP(hipMemsetAsync(d_samples, 0, sb * size_t(n_slices) * PE_MLP_SAMPLES * g->dof, st));
    return PE_OK;
  }
  if (!d_work) return set_error(PE_E_ARG, "null workspace");
  const size_t per_slice = PE_MLP_SAMPLES * sample_field_bytes(g);
  if (work_bytes < 4 * 256 + per_slice)
    return set_error(PE_E_WORKSPACE, "workspace %zu B below %zu B", work_bytes, 4 * 256 + per_slice);
  const int nb = int(std::min<size_t>(n_slices, (work_bytes - 4 * 256) / per_slice));
  Arena ar(d_work, work_bytes);
  double *coef = ar.take<double>(size_t(nb) * PE_MLP_SAMPLES * std::max(g->n_terms, 1));
  char *w0 = ar.take<char>(size_t(nb) * PE_MLP_SAMPLES * field_bytes(g));
  char *w1 = ar.take<char>(size_t(nb) * PE_MLP_SAMPLES * field_bytes(g));
  if (!coef || !w0 || !w1) return set_error(PE_E_WORKSPACE, "internal: workspace split failed");
  for (int n0 = 0; n0 < n_slices; n0 += nb) {
    FieldBatch b{};
    b.n0 = n0;
    b.nslices = std::min(nb, n_slices - n0);
    b.j0 = 0;
    b.jc = 1;
    b.s = PE_MLP_SAMPLES;
    b.t0 = t0;
    b.dT = dT;
    b.dt = dT;
    for (int q = 0; q < PE_MLP_SAMPLES; ++q) b.c[q] = double(q) / 7.0;
    void *res = nullptr;
    PE_TRY(load_and_transform(g, b, w0, w1, coef, &res, st));
    const int64_t count = b.count();
    char *dst = static_cast<char *>(d_samples) + size_t(n0) * PE_MLP_SAMPLES * g->dof * sb;
    const Axis *A = g->ax;
    if (g->precision == PE_FP64)
      k_compact_fields<double><<<nblk(count * g->dof), 256, 0, st>>>(
          g->dim, A[0].n, A[1].n, A[2].n, A[0].np, A[1].np, A[2].np, A[0].Kh, A[1].Kh, A[2].Kh,
          A[0].d_sig, A[1].d_sig, A[2].d_sig, static_cast<const double *>(res),
          reinterpret_cast<double *>(dst), count, g->dof, g->dofp);
    else
      k_compact_fields<float><<<nblk(count * g->dof), 256, 0, st>>>(
          g->dim, A[0].n, A[1].n, A[2].n, A[0].np, A[1].np, A[2].np, A[0].Kh, A[1].Kh, A[2].Kh,
          A[0].d_sig, A[1].d_sig, A[2].d_sig, static_cast<const float *>(res),
          reinterpret_cast<float *>(dst), count, g->dof, g->dofp);
    PE_HIP(hipGetLastError());
  }
  return PE_OK;
}

size_t pe_learned_rows_workspace_bytes(pe_grid g, int32_t n_slices) {
  if (!g || n_slices < 1) return 0;
  const int64_t blocks = (int64_t(n_slices) * g->dof + 255) / 256;
  return 8 * 256 + size_t(blocks) * (sizeof(int) + sizeof(int64_t)) + sizeof(double) * 65538 +
         sizeof(int64_t) + learned_coef_bytes(g, n_slices);
}

pe_status pe_learned_rows(pe_grid g, int32_t n_slices, double t0, double dT, const void *d_R,
                          const void *d_r, double rel_thresh, float *d_x, float *d_t, float *d_s,
                          int64_t max_rows, int64_t *h_count, void *d_work, size_t work_bytes,
                          void *stream) {
  clear_error();
  if (!g || !d_R || !d_r || !d_x || !d_t || !h_count || !d_work)
    return set_error(PE_E_ARG, "null argument");
  if (n_slices < 1 || !(dT > 0) || max_rows < 0 || !(rel_thresh >= 0) || !std::isfinite(t0))
    return set_error(PE_E_ARG, "bad arguments");
  if (g->n_hats > 0) return set_error(PE_E_ARG, "the learned inputs do not cover moving sources");
  if (has_periodic(g)) return set_error(PE_E_ARG, "the learned inputs are built for Dirichlet axes");
  if (work_bytes < pe_learned_rows_workspace_bytes(g, n_slices))
    return set_error(PE_E_WORKSPACE, "workspace too small");
  hipStream_t st = as_stream(stream);
  if (g->n_terms == 0) {
    *h_count = 0;
    return PE_OK;
  }
  Arena ar(d_work, work_bytes);
  double *Cp = ar.take<double>(size_t(n_slices) * PE_MLP_SAMPLES * g->n_terms);
  RowsArgs a = rows_args(g, n_slices, dT, Cp, d_R, d_r);
  const int64_t blocks = (a.total + 255) / 256;
  if (blocks > (int64_t(1) << 24)) return set_error(PE_E_ARG, "too many rows");
  int *counts = ar.take<int>(blocks);
  int64_t *offsets = ar.take<int64_t>(blocks);
  const unsigned mb = nblk(a.total);
  double *part = ar.take<double>(mb);
  double *smax = ar.take<double>(1);
  int64_t *total = ar.take<int64_t>(1);
  if (!Cp || !counts || !offsets || !part || !smax || !total)
    return set_error(PE_E_WORKSPACE, "internal: workspace split failed");
  PE_TRY(learned_coefs(g, n_slices, t0, dT, Cp, st));
  k_rows_max<<<mb, 256, 0, st>>>(a, part);
  k_rows_max_final<<<1, 1, 0, st>>>(part, int(mb), smax);
  k_rows_count<<<unsigned(blocks), 256, 0, st>>>(a, smax, rel_thresh, counts);
  k_rows_scan<<<1, 64, 0, st>>>(counts, int(blocks), offsets, total);
  k_rows_write<<<unsigned(blocks), 256, 0, st>>>(a, smax, rel_thresh, offsets, max_rows, d_x, d_t,
                                                 d_s);
  PE_HIP(hipGetLastError());
  PE_HIP(hipMemcpyAsync(h_count, total, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  PE_HIP(hipStreamSynchronize(st));
  return PE_OK;
}

}  // extern "C"
