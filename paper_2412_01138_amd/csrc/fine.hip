// Fine propagator F on all Parareal slices at once, and the projection P_h.
//
// Paper eq. (2.6): one EIFE-linear step
//     W <- exp(-h D lambda) W + h sum_i b_i(h D lambda) ghat(t + c_i h),
// ghat(t) = Q^T F(t) the spectral coefficients of P_h f(t), F(t) the Q1 load
// vector.  Section 2.3: F^J is J such steps of size dt = dT/J with q nodes,
// applied to every slice n in parallel (Algorithm 1, the parallel line).
//
// Because the forcing does not depend on the state (linear problem), the
// load vectors of all (slice, step, stage) fields of a batch are evaluated
// and transformed together (large launches), and the diagonal update then
// walks the steps of the batch in order, keeping each coefficient's state in
// a register.
#include <algorithm>
#include <vector>

#include "pe_internal.h"

namespace pe {

// coef[f][m] = amp_m tau_m(t_f) for every field f of the batch
__global__ void k_time_coefs(FieldBatch b, const DevTerm *terms, int n_terms, double *coef,
                             int64_t count) {
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < count * n_terms;
       idx += int64_t(gridDim.x) * blockDim.x) {
  int64_t f = idx / n_terms;
  int m = int(idx - f * n_terms);
  int64_t per_slice = int64_t(b.jc) * b.s;
  int n = b.n0 + int(f / per_slice);
  int rem = int(f - (f / per_slice) * per_slice);
  int j = b.j0 + rem / b.s;
  int i = rem - (rem / b.s) * b.s;
  double t = ((b.t0 + double(n) * b.dT) + double(j) * b.dt) + b.c[i] * b.dt;
  coef[idx] = term_time(terms[m], t);
  }
}

struct Dims {
  int d;
  int n[PE_MAX_DIM];
  int np[PE_MAX_DIM];
  int Kh[PE_MAX_DIM];
  int per[PE_MAX_DIM];   // periodic axis: the transform writes modes in their own order
};

static Dims dims_of(pe_grid g) {
  Dims D{};
  D.d = g->dim;
  for (int a = 0; a < PE_MAX_DIM; ++a) {
    D.n[a] = a < g->dim ? g->ax[a].n : 1;
    D.np[a] = a < g->dim ? g->ax[a].np : 1;
    D.Kh[a] = a < g->dim ? g->ax[a].Kh : 1;
    D.per[a] = a < g->dim && g->ax[a].periodic ? 1 : 0;
  }
  return D;
}

// position of mode k of axis a in a transformed field
__device__ inline int mode_pos(const Dims &D, int a, int k) {
  return D.per[a] ? k : fold_pos(k, D.Kh[a]);
}

// Load vectors of `count` fields on the padded grid (pads = 0):
//   F_f[j] = sum_m coef[f][m] prod_a C_a[m][j_a]
// (the tensor Gauss rule applied to a separable term factorises into 1D
// rules, so C_a are the per-axis element-quadrature loads).  Block = one row
// (all axes but the last fixed) at a time: the row's factors
// coef[f][m] prod_{a<d-1} C_a[m][j_a] are formed once in LDS, then each
// thread sums them against the last-axis table for its nodes (the product
// order of a per-node evaluation, so the values are the same).
template <typename TG>
__global__ __launch_bounds__(256) void k_load_fields(Dims D, const double *__restrict__ C0,
                                                     const double *__restrict__ C1,
                                                     const double *__restrict__ C2, int n_terms,
                                                     const double *__restrict__ coef,
                                                     TG *__restrict__ out, int64_t rows_total,
                                                     int64_t rows_per_field) {
  __shared__ double pre[PE_MAX_TERMS];
  const int last = D.d - 1;
  const int npl = D.np[last], nl = D.n[last];
  const double *Cl = last == 0 ? C0 : (last == 1 ? C1 : C2);
  for (int64_t row = blockIdx.x; row < rows_total; row += gridDim.x) {
    const int64_t f = row / rows_per_field;
    int64_t r = row - f * rows_per_field;
    int j[2] = {0, 0};
    bool inside = true;
    for (int a = last - 1; a >= 0; --a) {
      j[a] = int(r % D.np[a]);
      r /= D.np[a];
      inside = inside && j[a] < D.n[a];
    }
    __syncthreads();   // the previous row's factors are read
    for (int m = threadIdx.x; m < n_terms; m += blockDim.x) {
      double v = coef[f * n_terms + m];
      if (last >= 1) v *= C0[int64_t(m) * D.np[0] + j[0]];
      if (last >= 2) v *= C1[int64_t(m) * D.np[1] + j[1]];
      pre[m] = inside ? v : 0.0;
    }
    __syncthreads();
    TG *o = out + row * npl;
    for (int jl = threadIdx.x; jl < npl; jl += blockDim.x) {
      double x = 0.0;
      if (jl < nl)
        for (int m = 0; m < n_terms; ++m) x += pre[m] * Cl[int64_t(m) * npl + jl];
      o[jl] = TG(x);
    }
  }
}

// Moving hat sources (Example 5.4) added to the load fields of a batch: for
// field f at time t_f and node j,
//   sum_s amp_s tau_s(t_f) H_s(t_f)[j_axis] prod_{b != axis} Chat_b[s][j_b],
// H_s(t)[j] the q-point Gauss rule of max(1 - |x - c_s(t)| / w_s, 0) phi_j(x)
// on the two elements of node j (as the 1D loads of the separable terms).
struct HatGeom {
  double lo[PE_MAX_DIM], h[PE_MAX_DIM];
};

__device__ inline double hat_load(const DevHat &hs, double t, int j, double lo, double h,
                                  const GaussRule &rule) {
  const double c = hs.c0 + hs.c1 * sin(hs.omega * t + hs.phase);
  double acc = 0.0;
  for (int gq = 0; gq < rule.q; ++gq) {
    const double xi = rule.x[gq];
    const double xl = lo + h * (double(j) + xi);
    const double xr = lo + h * (double(j + 1) + xi);
    const double Xl = fmax(1.0 - fabs(xl - c) / hs.width, 0.0);
    const double Xr = fmax(1.0 - fabs(xr - c) / hs.width, 0.0);
    acc += rule.w[gq] * (Xl * xi + Xr * (1.0 - xi));
  }
  return acc * h;
}

template <typename TG>
__global__ void k_add_hats(Dims D, FieldBatch b, HatGeom geo, GaussRule rule,
                           const DevHat *__restrict__ hats, int nh, const double *__restrict__ C0,
                           const double *__restrict__ C1, const double *__restrict__ C2,
                           TG *__restrict__ out, int64_t dofp, int64_t total) {
  const double *C[3] = {C0, C1, C2};
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * blockDim.x) {
    const int64_t f = idx / dofp;
    int64_t r = idx - f * dofp;
    int j[3] = {0, 0, 0};
    for (int a = D.d - 1; a >= 0; --a) {
      j[a] = int(r % D.np[a]);
      r /= D.np[a];
    }
    bool inside = true;
    for (int a = 0; a < D.d; ++a) inside = inside && (j[a] < D.n[a]);
    if (!inside) continue;
    const int64_t per_slice = int64_t(b.jc) * b.s;
    const int n = b.n0 + int(f / per_slice);
    const int rem = int(f - (f / per_slice) * per_slice);
    const int js = b.j0 + rem / b.s;
    const int i = rem - (rem / b.s) * b.s;
    const double t = ((b.t0 + double(n) * b.dT) + double(js) * b.dt) + b.c[i] * b.dt;
    double v = 0.0;
    for (int s = 0; s < nh; ++s) {
      const DevHat &hs = hats[s];
      double prod = term_time(hs.time, t);
      for (int a = 0; a < D.d; ++a)
        prod *= a == hs.axis ? hat_load(hs, t, j[a], geo.lo[a], geo.h[a], rule)
                             : C[a][int64_t(s) * D.np[a] + j[a]];
      v += prod;
    }
    out[idx] = TG(double(out[idx]) + v);
  }
}

// The fused diagonal update of eq. (2.6) over the jc steps of a batch, for
// every slice and every (unpadded) coefficient k:
//     V <- E_k V + sum_i B_ik sigma_k G[f(n, j, i)][p(k)]
// sigma_k = prod_a 1/sqrt(mu_a(k_a)) turns DST coefficients into
// M-orthonormal ones.  Uin == nullptr means a zero initial state.
template <typename TS, typename TG>
__global__ void k_update(Dims D, const double *__restrict__ sig0, const double *__restrict__ sig1,
                         const double *__restrict__ sig2, const double *__restrict__ E,
                         const double *__restrict__ B, int s, const TS *Uin, TS *Uout,
                         const TG *__restrict__ G, int nslices, int chunk, int jc, int64_t dof,
                         int64_t dofp) {
  // thread = (slice chunk, coefficient): the tables of coefficient k are read
  // once and applied to `chunk` consecutive slices
  const int nchunks = (nslices + chunk - 1) / chunk;
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < int64_t(nchunks) * dof;
       idx += int64_t(gridDim.x) * blockDim.x) {
    const int64_t c = idx / dof;
    const int64_t k = idx - c * dof;
    int kk[3] = {0, 0, 0};
    int64_t r = k;
    for (int a = D.d - 1; a >= 0; --a) {
      kk[a] = int(r % D.n[a]);
      r /= D.n[a];
    }
    int64_t p = 0;   // position of mode k in the folded mode order of every axis
    for (int a = 0; a < D.d; ++a) p = p * D.np[a] + mode_pos(D, a, kk[a]);
    double sig = sig0[kk[0]];
    if (D.d > 1) sig *= sig1[kk[1]];
    if (D.d > 2) sig *= sig2[kk[2]];
    const double e = E[k];
    double bs[PE_MAX_STAGES];
    for (int i = 0; i < s; ++i) bs[i] = B[int64_t(i) * dof + k] * sig;
    const int n1 = int(c * chunk) + chunk < nslices ? int(c * chunk) + chunk : nslices;
    for (int n = int(c * chunk); n < n1; ++n) {
      const int64_t o = int64_t(n) * dof + k;
      double V = Uin ? double(Uin[o]) : 0.0;
      const TG *Gn = G + (int64_t(n) * jc) * int64_t(s) * dofp + p;
      for (int j = 0; j < jc; ++j) {
        double v = e * V;
        for (int i = 0; i < s; ++i) v += bs[i] * double(Gn[(int64_t(j) * s + i) * dofp]);
        V = v;
      }
      Uout[o] = TS(V);
    }
  }
}

// Slices per update thread: enough threads to fill the chip (about 2^21),
// the rest of the batch's slices walked by each thread.
static int update_chunk(int nslices, int64_t dof) {
  const int64_t want = int64_t(1) << 21;
  int64_t c = (int64_t(nslices) * dof + want - 1) / want;
  return int(std::max<int64_t>(1, std::min<int64_t>(c, nslices)));
}

template <typename TS>
__global__ void k_decay(const double *__restrict__ E, const TS *Uin, TS *Uout, int nslices, int jc,
                        int64_t dof) {
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < int64_t(nslices) * dof;
       idx += int64_t(gridDim.x) * blockDim.x) {
    int64_t k = idx % dof;
    double e = E[k];
    double V = Uin ? double(Uin[idx]) : 0.0;
    for (int j = 0; j < jc; ++j) V = e * V;
    Uout[idx] = TS(V);
  }
}

// W[k] = sigma_k G[p(k)]  (projection output, one field; p(k) = folded position)
template <typename TS, typename TG>
__global__ void k_scale_compact(Dims D, const double *sig0, const double *sig1, const double *sig2,
                                const TG *G, TS *W, int64_t dof) {
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < dof;
       k += int64_t(gridDim.x) * blockDim.x) {
    int kk[3] = {0, 0, 0};
    int64_t r = k;
    for (int a = D.d - 1; a >= 0; --a) {
      kk[a] = int(r % D.n[a]);
      r /= D.n[a];
    }
    int64_t p = 0;
    for (int a = 0; a < D.d; ++a) p = p * D.np[a] + mode_pos(D, a, kk[a]);
    double sig = sig0[kk[0]];
    if (D.d > 1) sig *= sig1[kk[1]];
    if (D.d > 2) sig *= sig2[kk[2]];
    W[k] = TS(sig * double(G[p]));
  }
}

// Flat launches use grid-stride loops over at most 2^16 blocks (HIP limits a
// grid dimension to 2^32 work-items).
static inline unsigned blocks_for(int64_t n, int bs = 256) {
  int64_t b = (n + bs - 1) / bs;
  return unsigned(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

static pe_status launch_load(pe_grid g, double *const *C, int n_terms, const double *coef,
                             void *out, int64_t count, hipStream_t st) {
  Dims D = dims_of(g);
  const double sb = g->precision == PE_FP64 ? 8.0 : 4.0;
  TimedScope ts(g, PE_K_LOAD, 0.0, double(count) * double(g->dof) * sb, st);
  const int64_t per_field = g->dofp / g->ax[g->dim - 1].np;
  const int64_t rows = count * per_field;
  const unsigned blocks = unsigned(std::min<int64_t>(std::max<int64_t>(rows, 1), 65536));
  if (g->precision == PE_FP64)
    k_load_fields<double><<<blocks, 256, 0, st>>>(D, C[0], C[1], C[2], n_terms, coef,
                                                   static_cast<double *>(out), rows, per_field);
  else
    k_load_fields<float><<<blocks, 256, 0, st>>>(D, C[0], C[1], C[2], n_terms, coef,
                                                  static_cast<float *>(out), rows, per_field);
  PE_HIP(hipGetLastError());
  return PE_OK;
}

static pe_status transform(pe_grid g, int64_t count, const GenSrc *gen, void *work0, void *work1,
                           void **result, hipStream_t st, int stop_axis = 0,
                           bool *axis0_outer = nullptr) {
  if (axis0_outer) *axis0_outer = false;
  if (g->transform == PE_TRANSFORM_FFT) {
    double *r = nullptr;
    PE_TRY(dst_fields_fft(g, count, gen, static_cast<double *>(work0), static_cast<double *>(work1),
                          &r, st, stop_axis));
    *result = r;
  } else if (g->precision == PE_FP64) {
    double *r = nullptr;
    PE_TRY(dst_fields_f64(g, count, gen, static_cast<double *>(work0), static_cast<double *>(work1),
                          &r, st, stop_axis));
    *result = r;
  } else {
    float *r = nullptr;
    GenSrcF gf;
    if (gen) {
      gf.C0 = gen->C0;
      gf.C1 = gen->C1;
      gf.coef = gen->coef;
      gf.Cf = gen->Cf;
      gf.Cft = gen->Cft;
      gf.M = gen->M;
    }
    PE_TRY(dst_fields_split(g, count, gen ? &gf : nullptr, static_cast<float *>(work0),
                            static_cast<float *>(work1), &r, st, stop_axis, axis0_outer));
    *result = r;
  }
  return PE_OK;
}

pe_status load_and_transform(pe_grid g, const FieldBatch &b, void *work0, void *work1,
                             double *coef, void **result, hipStream_t st, int stop_axis,
                             bool *axis0_outer) {
  if (axis0_outer) *axis0_outer = false;
  int64_t count = b.count();
  int64_t nc = count * g->n_terms;
  k_time_coefs<<<blocks_for(nc), 256, 0, st>>>(b, g->d_terms, g->n_terms, coef, count);
  PE_HIP(hipGetLastError());
  // moving sources are not separable in t and x: their loads go into
  // written fields, which the non-generating passes transform
  const bool hats = g->n_hats > 0;
  const bool fused = !hats && (g->precision == PE_FP64 ? gen_supported(g, g->n_terms)
                                                       : gen_supported_split(g, g->n_terms));
  if (fused) {
    // quadrature fused into the first transform pass
    GenSrc gs;
    gs.C0 = g->dim >= 2 ? g->d_C[0] : nullptr;
    gs.C1 = g->dim >= 3 ? g->d_C[1] : nullptr;
    gs.coef = coef;
    gs.Cf = g->d_Cf;
    gs.Cft = g->d_Cft;
    gs.Cl = g->d_C[g->dim - 1];
    gs.M = g->n_terms;
    return transform(g, count, &gs, work0, work1, result, st, stop_axis, axis0_outer);
  }
  PE_TRY(launch_load(g, g->d_C, g->n_terms, coef, work0, count, st));
  if (hats) {
    Dims D = dims_of(g);
    HatGeom geo{};
    for (int a = 0; a < g->dim; ++a) {
      geo.lo[a] = g->ax[a].lo;
      geo.h[a] = g->ax[a].h;
    }
    const GaussRule rule = gauss_rule(g->quad_q);
    const int64_t total = count * g->dofp;
    if (g->precision == PE_FP64)
      k_add_hats<double><<<blocks_for(total), 256, 0, st>>>(
          D, b, geo, rule, g->d_hats, g->n_hats, g->d_Chat[0], g->d_Chat[1], g->d_Chat[2],
          static_cast<double *>(work0), g->dofp, total);
    else
      k_add_hats<float><<<blocks_for(total), 256, 0, st>>>(
          D, b, geo, rule, g->d_hats, g->n_hats, g->d_Chat[0], g->d_Chat[1], g->d_Chat[2],
          static_cast<float *>(work0), g->dofp, total);
    PE_HIP(hipGetLastError());
  }
  return transform(g, count, nullptr, work0, work1, result, st, stop_axis);
}

static size_t per_field_bytes(pe_grid g) {
  return 2 * field_bytes(g) + sizeof(double) * size_t(std::max(g->n_terms, 1));
}

// Run the batches of one F pass (or of the coarse forcing, with a zero
// initial state): slices [0, N), J steps of size dt starting at t0 + n dT.
pe_status run_propagation(pe_grid g, int N, double t0, double dT, double dt, int J, int s,
                          const double *c, const double *d_E, const double *d_B, const void *d_Uin,
                          void *d_Uout, void *d_work, size_t work_bytes, hipStream_t st) {
  const int64_t dof = g->dof;
  const bool fp64 = g->precision == PE_FP64;
  const size_t sbytes = fp64 ? sizeof(double) : sizeof(float);
  Dims D = dims_of(g);
  if (g->n_terms == 0 && g->n_hats == 0) {
    // no forcing: pure decay, J steps at once
    int64_t tot = int64_t(N) * dof;
    if (fp64)
      k_decay<double><<<blocks_for(tot), 256, 0, st>>>(d_E, static_cast<const double *>(d_Uin),
                                                        static_cast<double *>(d_Uout), N, J, dof);
    else
      k_decay<float><<<blocks_for(tot), 256, 0, st>>>(d_E, static_cast<const float *>(d_Uin),
                                                       static_cast<float *>(d_Uout), N, J, dof);
    PE_HIP(hipGetLastError());
    return PE_OK;
  }
  // the axis-0 pass fused with the update needs its tables at folded
  // positions; without room for them the separate pass + update run
  const size_t tbytes = fused_update_table_bytes(g);
  size_t pf = per_field_bytes(g);
  size_t overhead = 3 * 256;
  const bool fused = tbytes > 0 && work_bytes >= overhead + tbytes + pf * size_t(s);
  if (fused) overhead += tbytes;
  if (work_bytes < overhead + pf * size_t(s))
    return set_error(PE_E_WORKSPACE, "workspace %zu B below the minimum %zu B", work_bytes,
                     overhead + pf * size_t(s));
  int64_t fit = int64_t((work_bytes - overhead) / pf);
  int64_t total = int64_t(N) * J * s;
  // batches of equal size (the last one never much smaller than the rest):
  // `count` items in ceil(count / most) batches
  auto even = [](int count, int64_t most) {
    const int64_t nb = (count + most - 1) / most;
    return int((count + nb - 1) / nb);
  };
  int Nb, Jc;
  if (fit >= total) {
    Nb = N;
    Jc = J;
  } else if (fused && fit >= int64_t(J) * s) {
    // the fused update walks a slice's fields in one block: whole slices
    // (all J steps) per batch, so each block amortises its operator load
    // over the slice's J s fields and the states never leave its registers
    Nb = even(N, fit / (int64_t(J) * s));
    Jc = J;
  } else if (fit >= int64_t(N) * s) {
    Nb = N;
    Jc = even(J, fit / (int64_t(N) * s));
  } else {
    Nb = even(N, fit / s);
    Jc = 1;
  }
  int64_t maxf = int64_t(Nb) * Jc * s;
  Arena ar(d_work, work_bytes);
  double *coef = ar.take<double>(size_t(maxf) * std::max(g->n_terms, 1));
  char *w0 = ar.take<char>(size_t(maxf) * field_bytes(g));
  char *w1 = ar.take<char>(size_t(maxf) * field_bytes(g));
  double *Tp = fused ? ar.take<double>(size_t(g->dofp) * (1 + s)) : nullptr;
  if (!coef || !w0 || !w1 || (fused && !Tp))
    return set_error(PE_E_WORKSPACE, "internal: workspace split failed");
  if (fused) PE_TRY(fused_update_tables(g, s, d_E, d_B, Tp, st));

  for (int n0 = 0; n0 < N; n0 += Nb) {
    int nb = std::min(Nb, N - n0);
    for (int j0 = 0; j0 < J; j0 += Jc) {
      int jc = std::min(Jc, J - j0);
      FieldBatch b{};
      b.n0 = n0;
      b.nslices = nb;
      b.j0 = j0;
      b.jc = jc;
      b.s = s;
      b.t0 = t0;
      b.dT = dT;
      b.dt = dt;
      for (int i = 0; i < s; ++i) b.c[i] = c[i];
      void *res = nullptr;
      bool outer = false;
      PE_TRY(load_and_transform(g, b, w0, w1, coef, &res, st, fused ? 1 : 0, &outer));
      const char *uin = (j0 == 0) ? static_cast<const char *>(d_Uin)
                                  : static_cast<const char *>(d_Uout);
      if (uin) uin += size_t(n0) * dof * sbytes;
      char *uout = static_cast<char *>(d_Uout) + size_t(n0) * dof * sbytes;
      if (fused) {
        PE_TRY(final_pass_update(g, b, res, Tp, uin, uout, st, outer));
        continue;
      }
      const int chunk = update_chunk(nb, dof);
      const int64_t tot = int64_t((nb + chunk - 1) / chunk) * dof;
      // state read + write, jc*s stage fields read, tables read once per chunk
      TimedScope ts(g, PE_K_UPDATE, 0.0,
                    double(nb) * dof * sbytes * (2.0 + double(jc) * s) +
                        double(1 + s) * dof * 8.0 * double((nb + chunk - 1) / chunk),
                    st);
      if (fp64)
        k_update<double, double><<<blocks_for(tot), 256, 0, st>>>(
            D, g->ax[0].d_sig, g->ax[1].d_sig, g->ax[2].d_sig, d_E, d_B, s,
            reinterpret_cast<const double *>(uin), reinterpret_cast<double *>(uout),
            static_cast<const double *>(res), nb, chunk, jc, dof, g->dofp);
      else
        k_update<float, float><<<blocks_for(tot), 256, 0, st>>>(
            D, g->ax[0].d_sig, g->ax[1].d_sig, g->ax[2].d_sig, d_E, d_B, s,
            reinterpret_cast<const float *>(uin), reinterpret_cast<float *>(uout),
            static_cast<const float *>(res), nb, chunk, jc, dof, g->dofp);
      PE_HIP(hipGetLastError());
    }
  }
  return PE_OK;
}

pe_status build_loads(pe_grid g, int n_terms, const pe_term *terms, double **dst, hipStream_t st);
DevTerm to_dev_term(const pe_term &t);

}  // namespace pe

using namespace pe;

extern "C" {

size_t pe_fine_workspace_bytes(pe_grid g, int64_t fields) {
  if (!g || fields < 1) return 0;
  return 3 * 256 + size_t(fields) * per_field_bytes(g) + 3 * 256 + fused_update_table_bytes(g);
}

pe_status pe_fine_propagate(pe_grid g, int32_t n_slices, double t0, double dT, int32_t J,
                            int32_t q, const double *cF, const double *d_EF, const double *d_BF,
                            const void *d_Uin, void *d_Uout, void *d_work, size_t work_bytes,
                            void *stream) {
  clear_error();
  if (!g || !cF || !d_EF || !d_BF || !d_Uin || !d_Uout) return set_error(PE_E_ARG, "null argument");
  if (n_slices < 1 || J < 1) return set_error(PE_E_ARG, "n_slices and J must be >= 1");
  if (q < 1 || q > PE_MAX_STAGES) return set_error(PE_E_ARG, "q must be 1..%d", PE_MAX_STAGES);
  if (!(dT > 0) || !std::isfinite(dT) || !std::isfinite(t0)) return set_error(PE_E_ARG, "bad dT/t0");
  if (d_Uin == d_Uout) return set_error(PE_E_ARG, "d_Uin and d_Uout must not overlap");
  if (g->n_terms > 0 && !d_work) return set_error(PE_E_ARG, "null workspace");
  return run_propagation(g, n_slices, t0, dT, dT / J, J, q, cF, d_EF, d_BF, d_Uin, d_Uout, d_work,
                         work_bytes, as_stream(stream));
}

size_t pe_project_workspace_bytes(pe_grid g) {
  if (!g) return 0;
  size_t b = 10 * 256 + 2 * field_bytes(g);
  for (int a = 0; a < g->dim; ++a) b += sizeof(double) * PE_MAX_TERMS * g->ax[a].np;
  b += sizeof(double) * PE_MAX_TERMS + sizeof(DevTerm) * PE_MAX_TERMS;
  b += sizeof(double) * 2 * PE_MAX_TERMS * g->ax[g->dim - 1].Kh;
  if (g->precision != PE_FP64) b += split_gen_table_bytes(g);
  return b;
}

// P_h of n_terms separable terms plus explicit-table terms `der` (their
// amplitudes already include any time factor): W = (kron Q_a)^T F.
static pe_status project_impl(pe_grid g, int32_t n_terms, const pe_term *terms,
                              const std::vector<DerivedTerm> &der, void *d_W, void *d_work,
                              size_t work_bytes, hipStream_t st) {
  size_t sbytes = g->precision == PE_FP64 ? sizeof(double) : sizeof(float);
  const int M = n_terms + int(der.size());
  if (M == 0) {
    PE_HIP(hipMemsetAsync(d_W, 0, size_t(g->dof) * sbytes, st));
    return PE_OK;
  }
  if (M > PE_MAX_TERMS)
    return set_error(PE_E_ARG, "%d terms + %d from the boundary data exceed %d", n_terms,
                     int(der.size()), PE_MAX_TERMS);
  if (!d_work) return set_error(PE_E_ARG, "null workspace");
  if (work_bytes < pe_project_workspace_bytes(g))
    return set_error(PE_E_WORKSPACE, "workspace %zu B below %zu B", work_bytes,
                     pe_project_workspace_bytes(g));
  Arena ar(d_work, work_bytes);
  double *C[PE_MAX_DIM] = {nullptr, nullptr, nullptr};
  for (int a = 0; a < g->dim; ++a) C[a] = ar.take<double>(size_t(M) * g->ax[a].np);
  double *coef = ar.take<double>(M);
  double *Cf = ar.take<double>(2 * size_t(M) * g->ax[g->dim - 1].Kh);
  uint16_t *Cft = g->precision != PE_FP64 ? ar.take<uint16_t>(split_gen_table_bytes(g) / 2) : nullptr;
  char *w0 = ar.take<char>(field_bytes(g));
  char *w1 = ar.take<char>(field_bytes(g));
  if (!coef || !Cf || !w0 || !w1 || (g->precision != PE_FP64 && !Cft))
    return set_error(PE_E_WORKSPACE, "internal: workspace split failed");
  if (n_terms > 0) PE_TRY(build_loads(g, n_terms, terms, C, st));
  PE_TRY(upload_derived(g, der, n_terms, C, st));
  std::vector<double> amps(M);
  for (int m = 0; m < n_terms; ++m) amps[m] = terms[m].amp;
  for (size_t m = 0; m < der.size(); ++m) amps[n_terms + m] = der[m].time.amp;
  PE_HIP(hipMemcpyAsync(coef, amps.data(), sizeof(double) * M, hipMemcpyHostToDevice, st));
  void *res = nullptr;
  const bool fused = g->precision == PE_FP64 ? gen_supported(g, M) : gen_supported_split(g, M);
  if (fused) {
    PE_TRY(fold_table(g, C[g->dim - 1], M, Cf, st));
    if (Cft) PE_TRY(split_gen_table(g, Cf, M, Cft, st));
    GenSrc gs;
    gs.C0 = g->dim >= 2 ? C[0] : nullptr;
    gs.C1 = g->dim >= 3 ? C[1] : nullptr;
    gs.coef = coef;
    gs.Cf = Cf;
    gs.Cft = Cft;
    gs.Cl = C[g->dim - 1];
    gs.M = M;
    PE_TRY(transform(g, 1, &gs, w0, w1, &res, st));
  } else {
    PE_TRY(launch_load(g, C, M, coef, w0, 1, st));
    PE_TRY(transform(g, 1, nullptr, w0, w1, &res, st));
  }
  Dims D = dims_of(g);
  if (g->precision == PE_FP64)
    k_scale_compact<double, double><<<blocks_for(g->dof), 256, 0, st>>>(
        D, g->ax[0].d_sig, g->ax[1].d_sig, g->ax[2].d_sig, static_cast<const double *>(res),
        static_cast<double *>(d_W), g->dof);
  else
    k_scale_compact<float, float><<<blocks_for(g->dof), 256, 0, st>>>(
        D, g->ax[0].d_sig, g->ax[1].d_sig, g->ax[2].d_sig, static_cast<const float *>(res),
        static_cast<float *>(d_W), g->dof);
  PE_HIP(hipGetLastError());
  PE_HIP(hipStreamSynchronize(st));   // amps is host memory read by the copy
  return PE_OK;
}

pe_status pe_project(pe_grid g, int32_t n_terms, const pe_term *terms, void *d_W, void *d_work,
                     size_t work_bytes, void *stream) {
  clear_error();
  if (!g || !d_W) return set_error(PE_E_ARG, "null argument");
  if (n_terms < 0 || n_terms > PE_MAX_TERMS) return set_error(PE_E_ARG, "n_terms out of range");
  if (n_terms > 0 && !terms) return set_error(PE_E_ARG, "null terms");
  return project_impl(g, n_terms, terms, {}, d_W, d_work, work_bytes, as_stream(stream));
}

pe_status pe_project_state(pe_grid g, int32_t n_terms, const pe_term *terms, double t, void *d_W,
                           void *d_work, size_t work_bytes, void *stream) {
  clear_error();
  if (!g || !d_W) return set_error(PE_E_ARG, "null argument");
  if (n_terms < 0 || n_terms > PE_MAX_TERMS) return set_error(PE_E_ARG, "n_terms out of range");
  if (n_terms > 0 && !terms) return set_error(PE_E_ARG, "null terms");
  if (!std::isfinite(t)) return set_error(PE_E_ARG, "bad t");
  std::vector<DerivedTerm> der;
  boundary_terms(g, true, t, der);
  return project_impl(g, n_terms, terms, der, d_W, d_work, work_bytes, as_stream(stream));
}

}  // extern "C"
