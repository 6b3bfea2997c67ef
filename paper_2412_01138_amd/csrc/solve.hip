// Parareal driver (paper Algorithm 1) on one GPU.
//
//   U^(0): U_0 = P_h u0, then the sequential coarse sweep;
//   repeat: Fbar = F^J(U^(k)) on all slices (one batched fine pass, never
//           cached between iterations), correction sweep (eq. (2.8)) with the
//           jump and residual norms fused in, one 24-byte read-back, stop
//           test.
// The stopping rule (not fixed by the paper) is the relative jump
// ||U^(k) - U^(k-1)|| / ||U^(k)|| over all slice ends, compared with tol.
// The relative residual ||U^{n+1,(k)} - F^J(U^{n,(k)})|| / ||U^(k)|| of the
// iterate a fine pass starts from is reported beside it.
#include <algorithm>
#include <cmath>

#include "learned_feat.h"

namespace pe {

pe_status run_propagation(pe_grid g, int N, double t0, double dT, double dt, int J, int s,
                          const double *c, const double *d_E, const double *d_B, const void *d_Uin,
                          void *d_Uout, void *d_work, size_t work_bytes, hipStream_t st);

static size_t fixed_bytes(pe_grid g, const pe_solve_params *P) {
  size_t sb = g->precision == PE_FP64 ? sizeof(double) : sizeof(float);
  size_t dof = size_t(g->dof);
  size_t b = 0;
  b += Arena::need(sizeof(double) * dof * (1 + P->q));      // EF, BF
  b += Arena::need(sizeof(double) * dof * (1 + P->p));      // EG, BG
  b += Arena::need(sb * dof * (P->N + 1));                  // second iterate buffer
  b += Arena::need(sb * dof * P->N);                        // Fout
  b += Arena::need(sb * dof * P->N);                        // r
  b += Arena::need(sizeof(double) * 6);                     // norms (initial, correction)
  b += coarse_partials_bytes(g);
  if (P->mlp && !P->d_corr) {
    b += learned_coef_bytes(g, P->N);                       // sample-coefficient tables
    b += Arena::need(sb * dof * P->N);                      // learned correction
  }
  return b + 6 * 256;
}

static pe_status check_params(pe_grid g, const pe_solve_params *P) {
  if (!P) return set_error(PE_E_ARG, "null params");
  if (P->N < 1 || P->J < 1) return set_error(PE_E_ARG, "N and J must be >= 1");
  if (P->p < 1 || P->p > PE_MAX_STAGES || P->q < 1 || P->q > PE_MAX_STAGES)
    return set_error(PE_E_ARG, "p, q must be 1..%d", PE_MAX_STAGES);
  if (P->K_max < 1 || P->K_max > PE_MAX_ITERS)
    return set_error(PE_E_ARG, "K_max must be 1..%d", PE_MAX_ITERS);
  if (!(P->T > 0) || !std::isfinite(P->T) || !std::isfinite(P->t0))
    return set_error(PE_E_ARG, "bad T/t0");
  if (!(P->tol >= 0)) return set_error(PE_E_ARG, "tol must be >= 0");
  return PE_OK;
}

}  // namespace pe

using namespace pe;

extern "C" {

size_t pe_solve_workspace_bytes(pe_grid g, const pe_solve_params *P) {
  if (!g || check_params(g, P) != PE_OK) return 0;
  // batch space: all fields of one fine pass, capped at 32 GiB of stage
  // fields (two buffers) but never below one step of all slices (or one
  // stage field set)
  int64_t all = int64_t(P->N) * P->J * P->q;
  size_t pf = pe_fine_workspace_bytes(g, 2) - pe_fine_workspace_bytes(g, 1);
  size_t pf_fields = 2 * field_bytes(g);
  int64_t cap = int64_t((size_t(32) << 30) / std::max<size_t>(pf_fields, 1));
  int64_t want = std::min(all, std::max<int64_t>(cap, int64_t(P->N) * std::max(P->q, P->p)));
  want = std::max<int64_t>(want, std::max(P->q, P->p));
  return fixed_bytes(g, P) + pe_fine_workspace_bytes(g, want);
}

pe_status pe_parareal_solve(pe_grid g, const pe_solve_params *P, const void *d_U0, void *d_U,
                            void *d_work, size_t work_bytes, pe_solve_report *rep, void *stream) {
  clear_error();
  if (!g || !d_U || !d_work || !rep) return set_error(PE_E_ARG, "null argument");
  PE_TRY(check_params(g, P));
  hipStream_t st = as_stream(stream);
  const int N = P->N, J = P->J, p = P->p, q = P->q;
  const double dT = P->T / N, dt = dT / J;
  const size_t sb = g->precision == PE_FP64 ? sizeof(double) : sizeof(float);
  const size_t dof = size_t(g->dof);
  size_t fixed = fixed_bytes(g, P);
  if (work_bytes < fixed + pe_fine_workspace_bytes(g, std::max(p, q)))
    return set_error(PE_E_WORKSPACE, "workspace %zu B below the minimum %zu B", work_bytes,
                     fixed + pe_fine_workspace_bytes(g, std::max(p, q)));
  Arena ar(d_work, work_bytes);
  double *EF = ar.take<double>(dof * (1 + q));
  double *EG = ar.take<double>(dof * (1 + p));
  char *Ubuf = ar.take<char>(sb * dof * (N + 1));
  char *Fout = ar.take<char>(sb * dof * N);
  char *r = ar.take<char>(sb * dof * N);
  double *norms = ar.take<double>(6);   // [0..2] correction sweeps, [3..5] initial sweep
  double *partials = ar.take<double>(coarse_partials_bytes(g) / sizeof(double));
  const bool learn = P->mlp && !P->d_corr;
  const size_t coef_bytes = learn ? learned_coef_bytes(g, N) : 0;
  char *coefs = learn ? ar.take<char>(coef_bytes) : nullptr;
  char *lcorr = learn ? ar.take<char>(sb * dof * N) : nullptr;
  if (!EF || !EG || !Ubuf || !Fout || !r || !norms || !partials || (learn && (!coefs || !lcorr)))
    return set_error(PE_E_WORKSPACE, "internal: workspace split failed");
  const void *corr = P->d_corr;
  double *BF = EF + dof, *BG = EG + dof;
  size_t off = (ar.off + 255) & ~size_t(255);
  void *fwork = static_cast<char *>(d_work) + off;
  size_t fbytes = work_bytes - off;

  *rep = pe_solve_report{};
  hipEvent_t ev[5];
  for (auto &e : ev) PE_HIP(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t *e;
    ~EvGuard() {
      for (int i = 0; i < 5; ++i) event_free(e[i]);
    }
  } guard{ev};
  float ms = 0;
  double fine_ms = 0, sweep_ms = 0;

  PE_HIP(hipEventRecord(ev[0], st));
  PE_TRY(pe_phi_tables(g, dt, q, P->cF, EF, BF, stream));
  PE_TRY(pe_phi_tables(g, dT, p, P->cG, EG, BG, stream));
  PE_HIP(hipEventRecord(ev[1], st));

  // iterate buffers: U^(k) and U^(k+1) alternate between d_U and Ubuf
  char *cur = static_cast<char *>(d_U), *nxt = Ubuf;
  if (d_U0)
    PE_HIP(hipMemcpyAsync(cur, d_U0, sb * dof, hipMemcpyDeviceToDevice, st));
  else
    PE_HIP(hipMemsetAsync(cur, 0, sb * dof, st));
  // U^(0): r_n for all slices (and the learned correction), then the
  // sequential coarse sweep
  {
    TimingClassScope tc(g, PE_K_COARSE_FORCING);
    PE_TRY(run_propagation(g, N, P->t0, dT, dT, 1, p, P->cG, EG, BG, nullptr, r, fwork, fbytes,
                           st));
  }
  if (learn) {
    hipEvent_t l0, l1;
    PE_HIP(hipEventCreate(&l0));
    PE_HIP(hipEventCreate(&l1));
    PE_HIP(hipEventRecord(l0, st));
    int32_t fb = 0;
    pe_status s2 = pe_learned_correction(g, P->mlp, N, P->t0, dT, lcorr, &fb, coefs, coef_bytes,
                                         stream);
    float lms = 0;
    if (s2 == PE_OK && hipEventRecord(l1, st) == hipSuccess && hipEventSynchronize(l1) == hipSuccess)
      (void)hipEventElapsedTime(&lms, l0, l1);
    event_free(l0);
    event_free(l1);
    PE_TRY(s2);
    rep->ms_learned = lms;
    rep->fallback = fb;
    corr = lcorr;
  }
  PE_TRY(sweep(g, N, EG, r, corr, nullptr, nullptr, cur, norms + 3, partials, st));
  double h0[3] = {0, 0, 0};
  PE_HIP(hipMemcpyAsync(h0, norms + 3, sizeof(h0), hipMemcpyDeviceToHost, st));
  PE_HIP(hipEventRecord(ev[2], st));
  PE_HIP(hipEventSynchronize(ev[2]));
  double prev_norm2 = h0[1];   // ||U^(k)||^2 of the iterate the next fine pass starts from

  int k = 0;
  bool converged = false;
  while (k < P->K_max) {
    PE_HIP(hipEventRecord(ev[3], st));
    PE_TRY(run_propagation(g, N, P->t0, dT, dt, J, q, P->cF, EF, BF, cur, Fout, fwork, fbytes,
                           st));
    PE_HIP(hipEventRecord(ev[4], st));
    PE_HIP(hipMemcpyAsync(nxt, cur, sb * dof, hipMemcpyDeviceToDevice, st));   // U^{0,(k+1)} = U^0
    PE_TRY(sweep(g, N, EG, r, corr, cur, Fout, nxt, norms, partials, st));
    double hn[3] = {0, 0, 0};
    PE_HIP(hipMemcpyAsync(hn, norms, sizeof(hn), hipMemcpyDeviceToHost, st));
    PE_HIP(hipStreamSynchronize(st));
    PE_HIP(hipEventElapsedTime(&ms, ev[3], ev[4]));
    fine_ms += ms;
    ++k;
    std::swap(cur, nxt);
    if (!std::isfinite(hn[0]) || !std::isfinite(hn[1]) || !std::isfinite(hn[2]))
      return set_error(PE_E_NUMERIC, "non-finite jump or residual norm at iteration %d", k);
    double jump = hn[1] > 0 ? std::sqrt(hn[0]) / std::sqrt(hn[1]) : std::sqrt(hn[0]);
    rep->jumps[k - 1] = jump;
    rep->residuals[k - 1] =
        prev_norm2 > 0 ? std::sqrt(hn[2]) / std::sqrt(prev_norm2) : std::sqrt(hn[2]);
    prev_norm2 = hn[1];
    if (jump <= P->tol) {
      converged = true;
      break;
    }
  }
  if (cur != static_cast<char *>(d_U))
    PE_HIP(hipMemcpyAsync(d_U, cur, sb * dof * (N + 1), hipMemcpyDeviceToDevice, st));
  PE_HIP(hipEventRecord(ev[3], st));
  PE_HIP(hipEventSynchronize(ev[3]));
  rep->iterations = k;
  rep->converged = converged ? 1 : 0;
  PE_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
  rep->ms_tables = ms;
  PE_HIP(hipEventElapsedTime(&ms, ev[1], ev[2]));
  rep->ms_coarse = ms;
  PE_HIP(hipEventElapsedTime(&ms, ev[0], ev[3]));
  rep->ms_total = ms;
  rep->ms_fine = fine_ms;
  sweep_ms = rep->ms_total - rep->ms_tables - rep->ms_coarse - fine_ms;
  rep->ms_sweep = sweep_ms;
  return PE_OK;
}

}  // extern "C"
