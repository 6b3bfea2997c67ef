// Internal declarations of the PEIFE-linear library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "peifem.h"

namespace pe {

// Even/odd folding of the DST-I.  With L = n + 1 and S[k][j] =
// sqrt(2/L) sin(pi j k / L) (1-based), S[k][L - j] = (-1)^(k+1) S[k][j], so
//   odd modes  k = 2i+1 : y = S_odd  u,  u_p = x_p + x_{n-1-p} (p < H), u_H = x_H (n odd)
//   even modes k = 2i+2 : y = S_even v,  v_p = x_p - x_{n-1-p} (p < H)
// (0-based node p, H = n/2 pairs): each axis transform is two dense products
// of half size.  An axis of n nodes is stored with np = 2*Kh entries, Kh =
// ceil(n/2) rounded up to 32: in nodal order before its transform, in
// "folded mode order" after it (odd modes at [0, Kh), even modes at
// [Kh, 2Kh)); unused entries are zero.
constexpr int KHALF = 32;

inline int half_pad(int n) { return ((n + 1) / 2 + KHALF - 1) / KHALF * KHALF; }

// position of mode index k (0-based, mode k+1) in folded mode order
__host__ __device__ inline int fold_pos(int k, int Kh) { return (k & 1) ? Kh + (k >> 1) : (k >> 1); }

// mode index k at folded position p (inverse of fold_pos)
__host__ __device__ inline int unfold_pos(int p, int Kh) { return p < Kh ? 2 * p : 2 * (p - Kh) + 1; }

// Blocks are handed to the 8 XCDs round-robin by block index; remapping the
// index gives every XCD a contiguous range of logical tiles, so neighbouring
// tiles (the tiles of one field, the strips of one slice) share that XCD's L2.
__device__ inline int64_t xcd_remap(int64_t bid, int64_t nblocks) {
  if (nblocks % 8 != 0) return bid;
  return (bid % 8) * (nblocks / 8) + bid / 8;
}

struct Axis {
  int n = 0, np = 0, Kh = 0, H = 0;
  // periodic axis: n nodes per period (node j at lo + j h, h = (hi - lo)/n),
  // np = n, modes in cos/sin order (position 0: the constant, 2k - 1: cos k,
  // 2k: sin k, n - 1: the alternating mode k = n/2); no DST tables
  bool periodic = false;
  double lo = 0, hi = 0, h = 0;
  double *d_lam = nullptr;       // [n]   generalized eigenvalues lambda_a(k)
  double *d_sig = nullptr;       // [n]   1/sqrt(mu_a(k)), mu_a the mass eigenvalues
  double *d_Sh = nullptr;        // [2][Kh][Kh]  Sh[h][i][p]: odd (h=0) / even (h=1) half of S
  double *d_ShT = nullptr;       // [2][Kh][Kh]  transposed halves, ShT[h][p][i]
  uint16_t *d_Shi = nullptr;     // [2][Kh][Kh] bf16 high part of Sh
  uint16_t *d_Slo = nullptr;     // [2][Kh][Kh] bf16 low part of Sh (Sh - hi)
  // second even/odd level (n = 2 Kh - 1): Q = Kh / 2 and, for mode half h and
  // input parity g, Sq[h][g][i][jj] = S[2i+1+h][2jj+1+g] (1-based S indices)
  bool l2 = false;
  double *d_Sq = nullptr;        // [2][2][Q][Q]
  double *d_SqT = nullptr;       // [2][2][Q][Q], SqT[h][g][jj][i]
  // third level (generating last-axis pass, Q a multiple of 32): per half h,
  // the B operands [K][N] of its reduced products, 3 Q^2 / 2 doubles per h:
  //   h = 0: P00[jj][n] = Sq[0][0][i(n)][jj] (Q x Q; i(n) = n below Q/2, else
  //          3Q/2 - 1 - n), P01E[k][n] = Sq[0][1][n][2k], P01O[k][n] =
  //          Sq[0][1][n][2k+1] (Q/2 x Q/2 each)
  //   h = 1: P10S[k][n] = Sq[1][0][2n][k], P10D[k][n] = Sq[1][0][2n+1][k],
  //          P11S[k][n] = Sq[1][1][2n][k], P11D[k][n] = Sq[1][1][2n+1][k]
  bool l3 = false;
  double *d_L3 = nullptr;        // [2][3 Q^2 / 2]
  // FFT transform: w^k = exp(-2 pi i k / N), N = 2 (n + 1), as (re, im)
  double *d_tw = nullptr;        // [N][2]
};

// q-point Gauss-Legendre rule on [0, 1]
struct GaussRule {
  int q;
  double x[8], w[8];
};
GaussRule gauss_rule(int q);

struct PendingTiming {
  hipEvent_t start, stop;
  int cls;
  double flops, bytes;
};

struct DevTerm {                 // a forcing term as the kernels read it
  double amp;
  double alpha, omega, phase;
  double p[4];
  int deriv;                     // 1: the term carries tau'(t) instead of tau(t)
};

// amp tau(t) (or amp tau'(t)): the time factor of a forcing term with its
// amplitude; tau = e^{alpha t} cos(omega t + phase) P(t), P cubic.
__device__ inline double term_time(const DevTerm &tm, double t) {
  const double poly = tm.p[0] + t * (tm.p[1] + t * (tm.p[2] + t * tm.p[3]));
  if (!tm.deriv) return tm.amp * exp(tm.alpha * t) * cos(tm.omega * t + tm.phase) * poly;
  const double arg = tm.omega * t + tm.phase;
  const double dpoly = tm.p[1] + t * (2.0 * tm.p[2] + 3.0 * t * tm.p[3]);
  return tm.amp * exp(tm.alpha * t) *
         ((tm.alpha * cos(arg) - tm.omega * sin(arg)) * poly + cos(arg) * dpoly);
}

// a moving hat source as the kernels read it
struct DevHat {
  DevTerm time;                  // amp tau(t)
  double width, c0, c1, omega, phase;
  int axis;
};

// Non-homogeneous Dirichlet data g (Sections 3 and 4 note the extension):
// with g_h the Q1 interpolant of g on the boundary nodes, the interior load
// gains -(M_IB g_B' + D A_IB g_B).  For a separable data term
// amp tau(t) prod_a X_a, with xb_a the values of X_a at the n_a + 2 nodes of
// axis a and (interior rows i, boundary entries kept / dropped)
//   p_a = (Mbar xb_a)_I, q_a = M_II (xb_a)_I, r_a = (Abar xb_a)_I, s_a = A_II (xb_a)_I,
// that load is the sum of 2 + 2d separable terms with explicit 1D tables:
//   -amp tau' (x)p + amp tau' (x)q
//   - D amp tau sum_a (x)_{b!=a} p_b x r_a + D amp tau sum_a (x)_{b!=a} q_b x s_a.
struct DerivedTerm {
  DevTerm time;                          // amplitude and time factor (tau or tau')
  std::vector<double> table[PE_MAX_DIM]; // [n_a] 1D load per axis
};
constexpr int PE_BOUNDARY_EXPANSION_MAX = 2 + 2 * PE_MAX_DIM;   // terms per data term
// the derived terms of the grid's data: all of them (mass_only = false), or
// only the mass coupling at time t with the time factor folded into the
// amplitude (mass_only = true: the initial-value correction -M_IB g_B(t))
void boundary_terms(pe_grid g, bool mass_only, double t, std::vector<DerivedTerm> &out);
// their tables into rows row0.. of per-axis tables [rows][np_a] (device)
pe_status upload_derived(pe_grid g, const std::vector<DerivedTerm> &der, int row0, double **dst,
                         hipStream_t st);

}  // namespace pe

struct pe_grid_s {
  int dim = 0;
  int precision = PE_FP64;
  int quad_q = 3;
  int transform = PE_TRANSFORM_DENSE;
  // 3D split-bf16 grids: generating and middle-axis passes as one kernel
  bool fuse_gen_mid = true;
  double D = 0;
  int64_t dof = 0;               // prod n_a
  int64_t dofp = 0;              // prod np_a (padded field size)
  pe::Axis ax[PE_MAX_DIM];
  int n_terms = 0;
  pe::DevTerm h_terms[PE_MAX_TERMS];
  pe::DevTerm *d_terms = nullptr;        // [n_terms]
  // the descriptors as given: forcing terms and Dirichlet data terms (the
  // internal list is the forcing followed by the data's derived terms)
  std::vector<pe_term> src_forcing, src_boundary;
  // moving hat sources: descriptors, device copies, the other axes' factor
  // loads [n_hats][np_a]
  std::vector<pe_moving_hat> src_moving;
  int n_hats = 0;
  pe::DevHat *d_hats = nullptr;
  double *d_Chat[PE_MAX_DIM] = {nullptr, nullptr, nullptr};
  double *d_C[PE_MAX_DIM] = {nullptr, nullptr, nullptr};  // [n_terms][np_a] 1D loads
  double *d_Cf = nullptr;        // [2][n_terms][Kh_last] folded last-axis loads
  uint16_t *d_Cft = nullptr;     // split-bf16 grids: d_Cf as the generating pass reads it
  // spec_a[m][k] = sig_a(k) (S_a^T C_a[m])_k: spectral 1D loads of each term
  double *d_spec[PE_MAX_DIM] = {nullptr, nullptr, nullptr};  // [n_terms][n_a]
  // kernel timing (benchmark instrumentation); timing_class >= 0 books every
  // launch into that class (the coarse forcing's launches)
  bool timing = false;
  int timing_class = -1;
  std::vector<pe::PendingTiming> pending;
  pe_kernel_stat stats[PE_K_COUNT] = {};
};

namespace pe {

// ---------------------------------------------------------------- errors
pe_status set_error(pe_status st, const char *fmt, ...);
void clear_error();

#define PE_HIP(call)                                                              \
  do {                                                                            \
    hipError_t _e = (call);                                                       \
    if (_e != hipSuccess)                                                         \
      return ::pe::set_error(PE_E_HIP, "%s failed: %s (%s:%d)", #call,            \
                             hipGetErrorString(_e), __FILE__, __LINE__);          \
  } while (0)

#define PE_TRY(expr)                    \
  do {                                  \
    pe_status _s = (expr);              \
    if (_s != PE_OK) return _s;         \
  } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Release paths: a failure there has nothing left to report to.
inline void dev_free(void *p) {
  if (p) (void)hipFree(p);
}
inline void event_free(hipEvent_t e) { (void)hipEventDestroy(e); }

// ------------------------------------------------------------- workspace
// A bump allocator over the caller's workspace (256-byte aligned slices).
struct Arena {
  char *base;
  size_t size, off = 0;
  Arena(void *b, size_t s) : base(static_cast<char *>(b)), size(s) {}
  template <class T>
  T *take(size_t count) {
    size_t o = (off + 255) & ~size_t(255);
    size_t bytes = count * sizeof(T);
    if (o + bytes > size) return nullptr;
    off = o + bytes;
    return reinterpret_cast<T *>(base + o);
  }
  static size_t need(size_t bytes) { return (bytes + 255) & ~size_t(255); }
};

// ---------------------------------------------------------- field passes
// Per-field time stamps of a batch of stage fields: field f is slice
// n = n0 + f / (jc * s), step j = j0 + (f / s) % jc, stage i = f % s at time
// ((t0 + n*dT) + j*dt) + c_i*dt.
struct FieldBatch {
  int n0, nslices;      // slices in this batch
  int j0, jc;           // steps in this batch
  int s;                // stages
  double t0, dT, dt;
  double c[PE_MAX_STAGES];
  int64_t count() const { return int64_t(nslices) * jc * s; }
};

// Evaluate the load vectors of a batch of fields and transform them to DST
// coefficients (before the 1/sqrt(mu) scaling).  work0/work1 each hold
// batch.count() padded fields of the grid's stage type; coef holds
// count * n_terms doubles.  Returns the buffer holding the result.
// (axis0_outer, when given, receives the layout of a stop_axis = 1 result:
// false [count][R][np_0], true [count][np_0][R]; see dst_fields_split)
pe_status load_and_transform(pe_grid g, const FieldBatch &b, void *work0, void *work1,
                             double *coef, void **result, hipStream_t st, int stop_axis = 0,
                             bool *axis0_outer = nullptr);

// Axis-0 pass fused with the diagonal update (d >= 2): FP64 grids whose
// axis 0 has two fold levels and Q = Kh/2 a multiple of 16 up to 128;
// split-bf16 grids whose axis 0 has Kh = 64 or 128.  The update tables (E, and b_i sigma per stage, in the kernel's
// lane order) are built once per propagation into (1 + s) * DOF_padded
// doubles of the fused_update_table_bytes of workspace.
bool fused_update_supported(pe_grid g);
size_t fused_update_table_bytes(pe_grid g);
pe_status fused_update_tables(pe_grid g, int s, const double *E, const double *B, double *Tp,
                              hipStream_t st);
// X: the batch after the passes over axes d-1..1 (stage type of the grid;
// split grids: [count][R][np_0], or [count][np_0][R] with axis0_outer);
// Uin (nullable) / Uout: the batch's slice states (state type).
pe_status final_pass_update(pe_grid g, const FieldBatch &b, const void *X, const double *Tp,
                            const void *Uin, void *Uout, hipStream_t st, bool axis0_outer = false);

// Load-vector generation inside the first (last-axis) transform pass: the
// nodal load of field f at node (j_0, .., j_{d-1}) is
//   sum_m coef[f][m] prod_{a<d-1} C_a[m][j_a] * C_{d-1}[m][j_{d-1}],
// and the pass consumes its fold along the last axis, built from the folded
// last-axis table Cf[h][m][p].
struct GenSrc {
  const double *C0 = nullptr;     // [M][np_0]  (d >= 2)
  const double *C1 = nullptr;     // [M][np_1]  (d == 3)
  const double *coef = nullptr;   // [count][M]
  const double *Cf = nullptr;     // [2][M][Kh_last]
  const double *Cl = nullptr;     // [M][np_last] (the FFT transform's generation)
  const uint16_t *Cft = nullptr;  // split-bf16 grids: Cf^T as bf16 hi / lo (split_gen_table)
  int M = 0;
};

// Per-axis DST products of `count` padded fields (FP64).  With gen != null
// the first pass generates its input (buf0 is then not read); otherwise
// buf0 holds nodal fields.  Passes ping-pong between buf0 and buf1;
// *result receives the buffer holding the coefficients (folded mode order).
// With stop_axis = 1 the axis-0 pass is left out (done by the fused
// axis-0 pass + update instead).
pe_status dst_fields_f64(pe_grid g, int64_t count, const GenSrc *gen, double *buf0, double *buf1,
                         double **result, hipStream_t st, int stop_axis = 0);
// Split-bf16 variant (fp32 fields): each pass contracts the contiguous axis
// and writes it outermost, so after d passes the axes are back in order.
struct GenSrcF {
  const double *C0 = nullptr;     // [M][np_0]  (d >= 2)
  const double *C1 = nullptr;     // [M][np_1]  (d == 3)
  const double *coef = nullptr;   // [count][M]
  const double *Cf = nullptr;     // [2][M][Kh_last]
  const uint16_t *Cft = nullptr;  // [2 hi/lo][2 halves][Kh_last][32] bf16 bits of Cf^T
  int M = 0;
};
// Cft of a split-bf16 grid from Cf ([2][M][Kh_last], M <= 32); terms
// m >= M are zero.  split_gen_table_bytes is its size.
size_t split_gen_table_bytes(pe_grid g);
pe_status split_gen_table(pe_grid g, const double *Cf, int M, uint16_t *Cft, hipStream_t st);
// (stop_axis = 1 leaves out the last pass, the one that contracts axis 0:
// the batch is then [count][R][np_0] with the other axes transformed)
// With gen, stop_axis = 1 and axis0_outer set, 3D grids that qualify
// (split_gen_mid_supported) run the generating and middle-axis passes as one
// kernel whose result is [count][np_0][R] (axis 0 outermost, *axis0_outer =
// true); otherwise *axis0_outer = false.
pe_status dst_fields_split(pe_grid g, int64_t count, const GenSrcF *gen, float *buf0, float *buf1,
                           float **result, hipStream_t st, int stop_axis = 0,
                           bool *axis0_outer = nullptr);
bool gen_supported_split(pe_grid g, int n_terms);
bool split_gen_mid_supported(pe_grid g, int n_terms);
pe_status split_gen_mid(pe_grid g, int64_t count, const GenSrcF *gen, float *out, hipStream_t st);
// true when the fused generation path can take n_terms terms
bool gen_supported(pe_grid g, int n_terms);
// Cf[h][m][p] from C[m][j] of the last axis (device)
pe_status fold_table(pe_grid g, const double *C_last, int n_terms, double *Cf, hipStream_t st);
pe_status build_loads(pe_grid g, int n_terms, const pe_term *terms, double **dst, hipStream_t st);

// FFT transform (FP64): axes with n + 1 in {64, .., 512}; the twiddle
// tables are built by fft_prepare.  dst_fields_fft has the contract of
// dst_fields_f64 (gen->Cl the plain last-axis table); the fused axis-0 pass
// + update takes (1 + s) DOF_padded doubles of tables from fft_tables.
bool fft_axis_ok(int n);
bool fft_periodic_ok(int n);
bool fft_gen_supported(pe_grid g, int n_terms);
pe_status fft_prepare(pe_grid g);
pe_status dst_fields_fft(pe_grid g, int64_t count, const GenSrc *gen, double *buf0, double *buf1,
                         double **result, hipStream_t st, int stop_axis = 0);
bool fft_final_supported(pe_grid g);
pe_status fft_tables(pe_grid g, int s, const double *E, const double *B, double *Tf,
                     hipStream_t st);
pe_status fft_final_update(pe_grid g, const FieldBatch &b, const double *X, const double *Tf,
                           const double *Uin, double *Uout, hipStream_t st);

inline bool has_periodic(pe_grid g) {
  for (int a = 0; a < g->dim; ++a)
    if (g->ax[a].periodic) return true;
  return false;
}

// bytes of one padded stage field
size_t field_bytes(pe_grid g);

// Coarse / correction sweep over N slices (see pe_coarse_sweep) with the
// norm partials in `partials` (needed when d_norms is given); timed = false
// skips the kernel-timing events.
pe_status sweep(pe_grid g, int N, const double *d_EG, const void *d_r, const void *d_corr,
                const void *d_Uprev, const void *d_Fout, void *d_U, double *d_norms,
                double *partials, hipStream_t st, bool timed = true);
size_t coarse_partials_bytes(pe_grid g);

// Books the timed launches made during its lifetime into one class.
struct TimingClassScope {
  pe_grid g;
  int prev;
  TimingClassScope(pe_grid g_, int cls) : g(g_), prev(g_->timing_class) { g->timing_class = cls; }
  ~TimingClassScope() { g->timing_class = prev; }
};

// Device address, on the current device, of the static norm-partials array
// of pe_coarse_sweep_noalloc (looked up once per device; *out may be null).
pe_status sweep_scratch_setup(double **out);

// Brackets the launches made during its lifetime with HIP events when the
// grid's timing is enabled (no-op otherwise, and for a null grid).
struct TimedScope {
  pe_grid g;
  hipStream_t st;
  PendingTiming pt{};
  bool on;
  TimedScope(pe_grid g_, int cls, double flops, double bytes, hipStream_t s)
      : g(g_), st(s), on(g_ && g_->timing) {
    if (!on) return;
    pt.cls = g_->timing_class >= 0 ? g_->timing_class : cls;
    pt.flops = flops;
    pt.bytes = bytes;
    if (hipEventCreate(&pt.start) != hipSuccess || hipEventCreate(&pt.stop) != hipSuccess ||
        hipEventRecord(pt.start, st) != hipSuccess)
      on = false;
  }
  ~TimedScope() {
    if (!on) return;
    if (hipEventRecord(pt.stop, st) == hipSuccess) g->pending.push_back(pt);
  }
};

}  // namespace pe
