// Coarse propagator G, the Parareal correction sweep and the jump norms.
//
// Paper Section 2.3: G(v; T_n) = exp(-dT L_h) v + dT sum_i b_i(-dT L_h)
// P_h f(T_n + c_i dT) -- in spectral space G(v) = E_G v + r_n with the
// state-independent forcing response r_n.  Algorithm 1 runs G sequentially
// over the slices; eq. (2.8) is the correction
//     U^{n+1,(k+1)} = G(U^{n,(k+1)}) + Fbar^{n+1} - G(U^{n,(k)}).
// The sweep is a first-order linear recurrence per coefficient: one thread
// owns one coefficient and walks n = 0..N-1, reading each slice once
// (coalesced across threads).  The squared norms of the jump, of the new
// iterate and of the previous iterate's residual U^{n+1,(k)} - Fbar^{n+1}
// (Fbar = F^J(U^{n,(k)}), both already read for eq. (2.8)) are accumulated
// in FP64 with a fixed reduction order.
#include <algorithm>
#include <mutex>

#include "pe_internal.h"

namespace pe {

pe_status run_propagation(pe_grid g, int N, double t0, double dT, double dt, int J, int s,
                          const double *c, const double *d_E, const double *d_B, const void *d_Uin,
                          void *d_Uout, void *d_work, size_t work_bytes, hipStream_t st);

constexpr int SWEEP_BS = 256;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

constexpr int NORMS = 3;   // jump, new iterate, residual of the previous iterate

// Block-wide sums of NORMS values in a fixed order; results valid in thread 0.
__device__ inline void block_sum(double (&v)[NORMS]) {
  __shared__ double sh[NORMS][SWEEP_BS / 64];
  int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NORMS; ++i) {
    v[i] = wave_sum(v[i]);
    if (lane == 0) sh[i][wave] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NORMS; ++i) {
      double x = 0;
      for (int w = 0; w < SWEEP_BS / 64; ++w) x += sh[i][w];
      v[i] = x;
    }
  }
}

// CORR: a learned correction is added to r; CORRECT: the correction sweep
// (Uprev and Fout given).  The reads of a slice do not depend on the
// recurrence, so those of the next two slices are issued ahead.
template <typename TS, bool CORR, bool CORRECT>
__global__ __launch_bounds__(SWEEP_BS) void k_sweep(const double *__restrict__ E,
                                                    const TS *__restrict__ r,
                                                    const TS *__restrict__ corr,
                                                    const TS *__restrict__ Uprev,
                                                    const TS *__restrict__ Fout,
                                                    TS *__restrict__ U, int N, int64_t dof,
                                                    double *partials) {
  int64_t k = int64_t(blockIdx.x) * SWEEP_BS + threadIdx.x;
  double acc[NORMS] = {0.0, 0.0, 0.0};   // jump, norm, residual
  if (k < dof) {
    const double e = E[k];
    double u = double(U[k]);
    double up = CORRECT ? double(Uprev[k]) : 0.0;
    // slice n: base = r (+ corr), fo = Fout, un = Uprev[n+1]
    struct Slice {
      double base, fo, un;
    };
    auto fetch = [&](int n) {
      const int64_t o = int64_t(n) * dof + k;
      Slice v;
      v.base = double(r[o]);
      if (CORR) v.base += double(corr[o]);
      v.fo = CORRECT ? double(Fout[o]) : 0.0;
      v.un = CORRECT ? double(Uprev[o + dof]) : 0.0;
      return v;
    };
    auto step = [&](int n, const Slice &c) {
      const int64_t o = int64_t(n) * dof + k;
      const double gnew = e * u + c.base;             // G(U^{n,(k+1)})
      double next = gnew;
      if (CORRECT) {
        const double gold = e * up + c.base;          // G(U^{n,(k)})
        next = (gnew + c.fo) - gold;                  // eq. (2.8)
      }
      const TS stored = TS(next);
      U[o + dof] = stored;
      const double nv = double(stored);
      if (CORRECT) {
        const double dlt = nv - c.un;
        acc[0] += dlt * dlt;
        const double res = c.un - c.fo;               // U^{n+1,(k)} - F^J(U^{n,(k)})
        acc[2] += res * res;
        up = c.un;
      }
      acc[1] += nv * nv;
      u = nv;
    };
    // two slice sets, each refilled right after use, without branches in the
    // loop (fetches past the last slice re-read it), so the loads of the
    // next slices stay in flight across the steps
    const int last = N - 1;
    Slice A = fetch(0), B = fetch(last < 1 ? last : 1);
    int n = 0;
    for (; n + 1 < N; n += 2) {
      step(n, A);
      A = fetch(n + 2 < last ? n + 2 : last);
      step(n + 1, B);
      B = fetch(n + 3 < last ? n + 3 : last);
    }
    if (n < N) step(n, A);
  }
  if (partials) {
    block_sum(acc);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < NORMS; ++i) partials[NORMS * blockIdx.x + i] = acc[i];
    }
  }
}

template <typename TS>
static void launch_sweep(int nb, hipStream_t st, const double *E, const void *r, const void *corr,
                         const void *Uprev, const void *Fout, void *U, int N, int64_t dof,
                         double *partials) {
  const TS *rr = static_cast<const TS *>(r), *cc = static_cast<const TS *>(corr);
  const TS *up = static_cast<const TS *>(Uprev), *fo = static_cast<const TS *>(Fout);
  TS *uu = static_cast<TS *>(U);
  if (Uprev) {
    if (corr)
      k_sweep<TS, true, true><<<nb, SWEEP_BS, 0, st>>>(E, rr, cc, up, fo, uu, N, dof, partials);
    else
      k_sweep<TS, false, true><<<nb, SWEEP_BS, 0, st>>>(E, rr, cc, up, fo, uu, N, dof, partials);
  } else {
    if (corr)
      k_sweep<TS, true, false><<<nb, SWEEP_BS, 0, st>>>(E, rr, cc, up, fo, uu, N, dof, partials);
    else
      k_sweep<TS, false, false><<<nb, SWEEP_BS, 0, st>>>(E, rr, cc, up, fo, uu, N, dof, partials);
  }
}

// One block: out[0..NORMS-1] = sums of the block partials, in a fixed order.
__global__ __launch_bounds__(SWEEP_BS) void k_reduce_partials(const double *partials, int nblocks,
                                                              double *out) {
  double v[NORMS] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nblocks; i += SWEEP_BS) {
#pragma unroll
    for (int j = 0; j < NORMS; ++j) v[j] += partials[NORMS * i + j];
  }
  block_sum(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NORMS; ++j) out[j] = v[j];
  }
}

static size_t partial_bytes(pe_grid g) {
  int64_t nb = (g->dof + SWEEP_BS - 1) / SWEEP_BS;
  return Arena::need(sizeof(double) * NORMS * size_t(nb));
}

pe_status sweep(pe_grid g, int N, const double *d_EG, const void *d_r, const void *d_corr,
                const void *d_Uprev, const void *d_Fout, void *d_U, double *d_norms,
                double *partials, hipStream_t st, bool timed) {
  int nb = int((g->dof + SWEEP_BS - 1) / SWEEP_BS);
  const double sb = g->precision == PE_FP64 ? 8.0 : 4.0;
  int arrays = 2 + (d_corr ? 1 : 0) + (d_Uprev ? 2 : 0);   // r, U write, corr, Uprev, Fout
  TimedScope ts(timed ? g : nullptr, PE_K_SWEEP, 0.0,
                double(N) * double(g->dof) * sb * arrays + g->dof * 8.0, st);
  if (g->precision == PE_FP64)
    launch_sweep<double>(nb, st, d_EG, d_r, d_corr, d_Uprev, d_Fout, d_U, N, g->dof,
                         d_norms ? partials : nullptr);
  else
    launch_sweep<float>(nb, st, d_EG, d_r, d_corr, d_Uprev, d_Fout, d_U, N, g->dof,
                        d_norms ? partials : nullptr);
  PE_HIP(hipGetLastError());
  if (d_norms) {
    k_reduce_partials<<<1, SWEEP_BS, 0, st>>>(partials, nb, d_norms);
    PE_HIP(hipGetLastError());
  }
  return PE_OK;
}

size_t coarse_partials_bytes(pe_grid g) { return partial_bytes(g); }

// ---------------------------------------------------------------------------
// Norm partials for pe_coarse_sweep_noalloc: a static device array (one copy
// per GPU, held until the process ends) instead of caller workspace.  Host
// code must not pass the array's name to a kernel (on the host it is only a
// stand-in for the symbol): its device address is looked up once per device
// and kept in scratch_ptr.
constexpr int64_t NOALLOC_BLOCKS = (int64_t(PE_NOALLOC_MAX_DOF) + SWEEP_BS - 1) / SWEEP_BS;
static __device__ __align__(256) double scratch[NORMS * NOALLOC_BLOCKS];

constexpr int MAX_DEVICES = 64;
static std::mutex scratch_mu;
static double *scratch_ptr[MAX_DEVICES] = {};

// Look up (once per device) the address of `scratch` on the current device.
pe_status sweep_scratch_setup(double **out) {
  int dev = -1;
  PE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES)
    return set_error(PE_E_UNSUPPORTED, "device %d: the static sweep scratch covers devices 0..%d",
                     dev, MAX_DEVICES - 1);
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void *p = nullptr;
    PE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return set_error(PE_E_HIP, "hipGetSymbolAddress returned a null address");
    scratch_ptr[dev] = static_cast<double *>(p);
  }
  if (out) *out = scratch_ptr[dev];
  return PE_OK;
}

}  // namespace pe

using namespace pe;

extern "C" {

size_t pe_coarse_workspace_bytes(pe_grid g, int32_t n_slices, int32_t p) {
  if (!g || n_slices < 1 || p < 1) return 0;
  return partial_bytes(g) + 256 + pe_fine_workspace_bytes(g, int64_t(n_slices) * p);
}

pe_status pe_coarse_sweep(pe_grid g, int32_t n_slices, double t0, double dT, int32_t p,
                          const double *cG, const double *d_EG, const double *d_BG,
                          int32_t compute_r, void *d_r, const void *d_corr, const void *d_Uprev,
                          const void *d_Fout, void *d_U, double *d_norms, void *d_work,
                          size_t work_bytes, void *stream) {
  clear_error();
  if (!g || !d_EG || !d_r || !d_U) return set_error(PE_E_ARG, "null argument");
  if (n_slices < 1) return set_error(PE_E_ARG, "n_slices must be >= 1");
  if ((d_Uprev == nullptr) != (d_Fout == nullptr))
    return set_error(PE_E_ARG, "d_Uprev and d_Fout must be given together");
  if (d_Uprev == d_U || d_r == d_U || (d_Fout && d_Fout == d_U) || (d_corr && d_corr == d_U))
    return set_error(PE_E_ARG, "d_U must not overlap d_r, d_corr, d_Uprev or d_Fout");
  hipStream_t st = as_stream(stream);
  Arena ar(d_work, work_bytes);
  double *partials = nullptr;
  if (d_norms) {
    if (!d_work) return set_error(PE_E_ARG, "norms need a workspace");
    partials = ar.take<double>(partial_bytes(g) / sizeof(double));
    if (!partials) return set_error(PE_E_WORKSPACE, "workspace too small for the norm partials");
  }
  if (compute_r) {
    if (!cG || !d_BG) return set_error(PE_E_ARG, "null coarse nodes/tables");
    if (p < 1 || p > PE_MAX_STAGES) return set_error(PE_E_ARG, "p must be 1..%d", PE_MAX_STAGES);
    if (!(dT > 0) || !std::isfinite(dT)) return set_error(PE_E_ARG, "bad dT");
    size_t off = (ar.off + 255) & ~size_t(255);
    void *rest = d_work ? static_cast<char *>(d_work) + off : nullptr;
    size_t rest_bytes = work_bytes > off ? work_bytes - off : 0;
    TimingClassScope tc(g, PE_K_COARSE_FORCING);
    PE_TRY(run_propagation(g, n_slices, t0, dT, dT, 1, p, cG, d_EG, d_BG, nullptr, d_r, rest,
                           rest_bytes, st));
  }
  return sweep(g, n_slices, d_EG, d_r, d_corr, d_Uprev, d_Fout, d_U, d_norms, partials, st);
}

pe_status pe_coarse_sweep_noalloc(pe_grid g, int32_t n_slices, const double *d_EG,
                                  const void *d_r, const void *d_corr, const void *d_Uprev,
                                  const void *d_Fout, void *d_U, double *d_norms, void *stream) {
  clear_error();
  if (!g || !d_EG || !d_r || !d_U) return set_error(PE_E_ARG, "null argument");
  if (n_slices < 1) return set_error(PE_E_ARG, "n_slices must be >= 1");
  if (g->dof > PE_NOALLOC_MAX_DOF)
    return set_error(PE_E_ARG, "grid of %lld coefficients exceeds the no-allocation limit %d",
                     (long long)g->dof, PE_NOALLOC_MAX_DOF);
  if ((d_Uprev == nullptr) != (d_Fout == nullptr))
    return set_error(PE_E_ARG, "d_Uprev and d_Fout must be given together");
  if (d_Uprev == d_U || d_r == d_U || (d_Fout && d_Fout == d_U) || (d_corr && d_corr == d_U))
    return set_error(PE_E_ARG, "d_U must not overlap d_r, d_corr, d_Uprev or d_Fout");
  double *partials = nullptr;
  if (d_norms) PE_TRY(sweep_scratch_setup(&partials));
  return sweep(g, n_slices, d_EG, d_r, d_corr, d_Uprev, d_Fout, d_U, d_norms, partials,
               as_stream(stream), false);
}

}  // extern "C"
