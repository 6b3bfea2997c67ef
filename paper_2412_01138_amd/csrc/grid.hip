// Grid set-up, forcing load tables and exponential Runge-Kutta tables.
//
// Paper, Section 2.1: tensor Q1 space on a uniform box mesh; Section 2.3
// (closing paragraph): the Q1 mass and stiffness matrices are diagonalised
// simultaneously by one orthogonal matrix.  In 1D both are polynomials in
// tridiag(1, 0, 1), whose orthonormal eigenvectors are the DST-I vectors
// s_k(j) = sqrt(2/(n+1)) sin(jk pi/(n+1)); the mass eigenvalue is
// mu(k) = (h/3)(2 + cos t_k) and the stiffness/mass ratio is
// lambda(k) = (6/h^2)(1 - cos t_k)/(2 + cos t_k), t_k = k pi/(n + 1).
// Eq. (2.7): b_i(z) = int_0^1 exp(-z(1 - theta)) l_i(theta) dtheta.
#include <cmath>
#include <cstring>
#include <vector>

#include "pe_internal.h"

namespace pe {

static thread_local std::string g_err;

pe_status set_error(pe_status st, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

void clear_error() { g_err.clear(); }

size_t field_bytes(pe_grid g) {
  return size_t(g->dofp) * (g->precision == PE_FP64 ? sizeof(double) : sizeof(float));
}

// ------------------------------------------------------------------ kernels

// bf16 round-to-nearest-even of a float, as raw bits
__device__ inline uint16_t f32_to_bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(r >> 16);
}
__device__ inline float bf16_bits_to_f32(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

__global__ void k_axis_eig(int n, double h, double *lam, double *sig) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double kk = double(k + 1);
  double s = sinpi(kk / (2.0 * (n + 1)));          // sin(t_k / 2)
  double c = cospi(kk / double(n + 1));            // cos(t_k)
  double mu = h / 3.0 * (2.0 + c);
  lam[k] = 12.0 / (h * h) * s * s / (2.0 + c);     // (6/h^2)(1 - cos)/(2 + cos)
  sig[k] = 1.0 / sqrt(mu);
}

// Periodic axis (n nodes per period): the circulant pair has the same
// eigenvalue formula at t_k = 2 pi k / n; position p holds mode k(p) of the
// cos/sin order (p = 0: k = 0; p = 2k - 1 and 2k: k; p = n - 1: k = n/2).
__global__ void k_axis_eig_periodic(int n, double h, double *lam, double *sig) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int k = p == 0 ? 0 : (p == n - 1 ? n / 2 : (p + 1) / 2);
  const double s = sinpi(double(k) / double(n));          // sin(t_k / 2)
  const double c = cospi(2.0 * double(k) / double(n));    // cos(t_k)
  const double mu = h / 3.0 * (2.0 + c);
  lam[p] = 12.0 / (h * h) * s * s / (2.0 + c);
  sig[p] = 1.0 / sqrt(mu);
}

// Odd (h = 0) and even (h = 1) halves of the orthonormal DST-I matrix:
// Sh[h][i][p] = S[2i+1+h][p+1] (1-based S), restricted to the folded inputs
// that exist (p < H, plus the middle node p = H for the odd half when n is
// odd); ShT is the transpose of each half.  Optional bf16 hi/lo split.
__global__ void k_dst_half(int n, int Kh, int H, double *Sh, double *ShT, uint16_t *Shi,
                           uint16_t *Slo) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  int i = blockIdx.y;
  int h = blockIdx.z;
  if (p >= Kh) return;
  int k = 2 * i + 1 + h;   // 1-based mode
  bool valid = k <= n && (p < H || (h == 0 && p == H && (n & 1)));
  double v = 0.0;
  if (valid) {
    long long m = (long long)k * (p + 1) % (2LL * (n + 1));   // exact angle reduction
    v = sqrt(2.0 / (n + 1)) * sinpi(double(m) / double(n + 1));
  }
  size_t o = (size_t(h) * Kh + i) * Kh + p;
  Sh[o] = v;
  ShT[(size_t(h) * Kh + p) * Kh + i] = v;
  if (Shi) {
    uint16_t hb = f32_to_bf16_bits(float(v));
    Shi[o] = hb;
    Slo[o] = f32_to_bf16_bits(float(v - double(bf16_bits_to_f32(hb))));
  }
}

// spec[m][k] = sig(k) sum_j S[k][j] C[m][j]: the spectral 1D load of each
// term on one axis (S the orthonormal sine basis, exact angle reduction).
__global__ void k_axis_spectra(const double *C, int np, int n, const double *sig, int n_terms,
                               double *spec) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (k >= n || m >= n_terms) return;
  const double *c = C + size_t(m) * np;
  const long long per = 2LL * (n + 1);
  double acc = 0.0;
  for (int j = 0; j < n; ++j) {
    const long long a = (long long)(k + 1) * (j + 1) % per;
    acc += sinpi(double(a) / double(n + 1)) * c[j];
  }
  spec[size_t(m) * n + k] = sig[k] * sqrt(2.0 / (n + 1)) * acc;
}

// Quarter blocks of the second even/odd level (n = 2 Kh - 1, Q = Kh / 2):
// Sq[h][g][i][jj] = S[k][j], k = 2i + 1 + h, j = 2jj + 1 + g (1-based),
// exact angle reduction as above; SqT is the transpose of each block.
__global__ void k_dst_quarter(int n, int Q, double *Sq, double *SqT) {
  const int jj = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  const int hg = blockIdx.z;   // 2 h + g
  if (jj >= Q) return;
  const int h = hg >> 1, g = hg & 1;
  const long long k = 2 * i + 1 + h, j = 2 * jj + 1 + g;
  const long long m = k * j % (2LL * (n + 1));
  const double v = sqrt(2.0 / (n + 1)) * sinpi(double(m) / double(n + 1));
  Sq[(size_t(hg) * Q + i) * Q + jj] = v;
  SqT[(size_t(hg) * Q + jj) * Q + i] = v;
}

// Third-level B operands from the quarter blocks (layout in pe_internal.h).
__global__ void k_dst_l3(int Q, const double *Sq, double *L3) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = 3 * Q * Q / 2, h = blockIdx.y, Q2 = Q / 2;
  if (e >= per) return;
  auto sq = [&](int hh, int g, int i, int jj) { return Sq[((size_t(2 * hh + g)) * Q + i) * Q + jj]; };
  double v = 0.0;
  if (h == 0) {
    if (e < Q * Q) {
      const int jj = e / Q, n = e % Q;
      v = sq(0, 0, n < Q2 ? n : 3 * Q2 - 1 - n, jj);
    } else {
      const int r = e - Q * Q, part = r / (Q2 * Q2), k = (r % (Q2 * Q2)) / Q2, n = r % Q2;
      v = sq(0, 1, n, 2 * k + part);
    }
  } else if (e < Q * Q) {
    const int part = e / (Q2 * Q2), k = (e % (Q2 * Q2)) / Q2, n = e % Q2;
    v = sq(1, part >> 1, 2 * n + (part & 1), k);
  }
  L3[size_t(h) * per + e] = v;
}

// Cf[h][m][p]: the even/odd fold of the last-axis 1D load table C[m][j].
__global__ void k_fold_table(const double *C, int np, int n, int H, int Kh, int n_terms,
                             double *Cf) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  int m = blockIdx.y;
  if (p >= Kh || m >= n_terms) return;
  const double *c = C + (size_t)m * np;
  double u = 0.0, v = 0.0;
  if (p < H) {
    u = c[p] + c[n - 1 - p];
    v = c[p] - c[n - 1 - p];
  } else if (p == H && (n & 1)) {
    u = c[p];
  }
  Cf[(size_t)m * Kh + p] = u;
  Cf[(size_t(n_terms) + m) * Kh + p] = v;
}

// C[m][j] = int X_m(x) phi_j(x) dx, j = 0..np-1 (zero for j >= n), by the
// q-point Gauss rule on the two elements around interior node j (global
// node j + 1): element [x_j, x_{j+1}] carries the hat as xi, element
// [x_{j+1}, x_{j+2}] as 1 - xi.
struct SpaceParams {
  double kappa, phase, q0, q1, q2;
};

// (periodic axis: node j at lo + j h collects element j - 1 (mod n, so node
// 0 takes the last element of the period) and element j)
__global__ void k_load_1d(int n, int np, double lo, double h, GaussRule rule,
                          const SpaceParams *sp, int n_terms, double *C, int periodic) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int m = blockIdx.y;
  if (j >= np || m >= n_terms) return;
  double acc = 0.0;
  if (j < n) {
    SpaceParams p = sp[m];
    const int el = periodic ? (j > 0 ? j - 1 : n - 1) : j;    // left element's first node
    const int er = periodic ? j : j + 1;                       // right element's first node
    for (int g = 0; g < rule.q; ++g) {
      double xi = rule.x[g];
      double xl = lo + h * (double(el) + xi);       // left element
      double xr = lo + h * (double(er) + xi);       // right element
      double Xl = (p.q0 + xl * (p.q1 + xl * p.q2)) * sin(p.kappa * xl + p.phase);
      double Xr = (p.q0 + xr * (p.q1 + xr * p.q2)) * sin(p.kappa * xr + p.phase);
      acc += rule.w[g] * (Xl * xi + Xr * (1.0 - xi));
    }
    acc *= h;
  }
  C[(size_t)m * np + j] = acc;
}

struct PhiArgs {
  int s;
  double h, D;
  double A[PE_MAX_STAGES][PE_MAX_STAGES];   // A[i][j] = a_ij (j)! : l_i = sum_j a_ij th^j
};

// phi_j(-z) for j = 1..s: Taylor series below the switch point z_s, the
// recurrence phi_j = (1/(j-1)! - phi_{j-1}) / z from phi_0 = e^{-z} above.
// Each recurrence step divides the previous rounding error by z while the
// subtraction loses ~ log10(j/z) digits, so the recurrence is accurate only
// once z is about s/2; the alternating Taylor series loses ~ z log10(e)
// digits.  z_s = 2 for s <= 4 and s/2 above keeps every phi_j within a few
// ulps up to s = 8 (checked against 80-digit values over 0 < z < 8).
__device__ inline void phi_all(double z, int s, double *phi) {
  const double zs = s <= 4 ? 2.0 : 0.5 * s;
  if (z < zs) {
    double x = -z;
    double fact = 1.0;   // j!
    for (int j = 1; j <= s; ++j) {
      fact *= j;
      double p = 1.0;
      for (int m = 32; m >= 1; --m) p = 1.0 + x * p / double(j + m);
      phi[j - 1] = p / fact;
    }
  } else {
    double prev = exp(-z);
    double inv_fact = 1.0;   // 1/(j-1)!
    for (int j = 1; j <= s; ++j) {
      double cur = (inv_fact - prev) / z;
      phi[j - 1] = cur;
      prev = cur;
      inv_fact /= j;
    }
  }
}

__global__ void k_phi_tables(int dim, int n0, int n1, int n2, const double *lam0,
                             const double *lam1, const double *lam2, PhiArgs a, double *E,
                             double *B, int64_t dof) {
  int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= dof) return;
  double lam;
  if (dim == 1) {
    lam = lam0[k];
  } else if (dim == 2) {
    lam = lam0[k / n1] + lam1[k % n1];
  } else {
    int64_t k2 = k % n2, r = k / n2;
    lam = lam0[r / n1] + lam1[r % n1] + lam2[k2];
  }
  double z = a.h * a.D * lam;
  double phi[PE_MAX_STAGES];
  phi_all(z, a.s, phi);
  E[k] = exp(-z);
  for (int i = 0; i < a.s; ++i) {
    double b = 0.0;
    for (int j = 0; j < a.s; ++j) b += a.A[i][j] * phi[j];
    B[(size_t)i * dof + k] = a.h * b;
  }
}

// ------------------------------------------------------------ host helpers

// Gauss-Legendre nodes/weights on [0, 1] by Newton's method on P_q.
GaussRule gauss_rule(int q) {
  GaussRule r{};
  r.q = q;
  for (int i = 0; i < q; ++i) {
    long double x = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (q + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = x;
      for (int k = 2; k <= q; ++k) {
        long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (q == 1) { p1 = x; p0 = 1; }
      dp = q * (x * p1 - p0) / (x * x - 1);
      long double dx = p1 / dp;
      x -= dx;
      if (fabsl(dx) < 1e-30L) break;
    }
    long double w = 2 / ((1 - x * x) * dp * dp);
    r.x[q - 1 - i] = double((x + 1) / 2);
    r.w[q - 1 - i] = double(w / 2);
  }
  return r;
}

// Lagrange coefficients a_ij (l_i(th) = sum_j a_ij th^j) times j!, in long
// double; fails for repeated nodes.
static pe_status lagrange_A(int s, const double *c, double A[PE_MAX_STAGES][PE_MAX_STAGES]) {
  for (int i = 0; i < s; ++i) {
    long double poly[PE_MAX_STAGES + 1] = {0};
    poly[0] = 1;
    int deg = 0;
    long double denom = 1;
    for (int m = 0; m < s; ++m) {
      if (m == i) continue;
      long double d = (long double)c[i] - c[m];
      if (d == 0) return set_error(PE_E_ARG, "stage nodes must be distinct (c[%d] == c[%d])", i, m);
      for (int p = deg + 1; p >= 1; --p) poly[p] = poly[p - 1] - c[m] * poly[p];
      poly[0] = -c[m] * poly[0];
      ++deg;
      denom *= d;
    }
    long double fact = 1;
    for (int j = 0; j < s; ++j) {
      if (j > 0) fact *= j;
      A[i][j] = double(poly[j] / denom * fact);
    }
  }
  return PE_OK;
}

static void free_grid_tables(pe_grid g) {
  for (int a = 0; a < PE_MAX_DIM; ++a) {
    dev_free(g->ax[a].d_lam);
    dev_free(g->ax[a].d_sig);
    dev_free(g->ax[a].d_Sh);
    dev_free(g->ax[a].d_ShT);
    dev_free(g->ax[a].d_Shi);
    dev_free(g->ax[a].d_Slo);
    dev_free(g->ax[a].d_Sq);
    dev_free(g->ax[a].d_SqT);
    dev_free(g->ax[a].d_L3);
    dev_free(g->ax[a].d_tw);
    dev_free(g->d_C[a]);
    dev_free(g->d_spec[a]);
    dev_free(g->d_Chat[a]);
  }
  dev_free(g->d_terms);
  dev_free(g->d_Cf);
  dev_free(g->d_Cft);
  dev_free(g->d_hats);
}

pe_status build_loads(pe_grid g, int n_terms, const pe_term *terms, double **dst, hipStream_t st) {
  GaussRule rule = gauss_rule(g->quad_q);
  std::vector<SpaceParams> sp(std::max(n_terms, 1));
  SpaceParams *d_sp = nullptr;
  PE_HIP(hipMalloc(&d_sp, sizeof(SpaceParams) * sp.size()));
  for (int a = 0; a < g->dim; ++a) {
    for (int m = 0; m < n_terms; ++m) {
      const pe_space_factor &f = terms[m].space[a];
      sp[m] = SpaceParams{f.kappa, f.phase, f.poly[0], f.poly[1], f.poly[2]};
    }
    hipError_t e = hipMemcpyAsync(d_sp, sp.data(), sizeof(SpaceParams) * n_terms,
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess) { dev_free(d_sp); PE_HIP(e); }
    const Axis &ax = g->ax[a];
    dim3 grid((ax.np + 127) / 128, n_terms);
    if (n_terms > 0)
      k_load_1d<<<grid, 128, 0, st>>>(ax.n, ax.np, ax.lo, ax.h, rule, d_sp, n_terms, dst[a],
                                      ax.periodic ? 1 : 0);
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) { dev_free(d_sp); PE_HIP(e); }
  }
  dev_free(d_sp);
  PE_HIP(hipGetLastError());
  return PE_OK;
}

pe_status fold_table(pe_grid g, const double *C_last, int n_terms, double *Cf, hipStream_t st) {
  const Axis &ax = g->ax[g->dim - 1];
  if (n_terms <= 0) return PE_OK;
  k_fold_table<<<dim3((ax.Kh + 127) / 128, n_terms), 128, 0, st>>>(C_last, ax.np, ax.n, ax.H, ax.Kh,
                                                                   n_terms, Cf);
  PE_HIP(hipGetLastError());
  return PE_OK;
}

DevTerm to_dev_term(const pe_term &t) {
  DevTerm d;
  d.amp = t.amp;
  d.alpha = t.time.alpha;
  d.omega = t.time.omega;
  d.phase = t.time.phase;
  for (int i = 0; i < 4; ++i) d.p[i] = t.time.poly[i];
  d.deriv = 0;
  return d;
}

static double space_value(const pe_space_factor &f, double x) {
  return (f.poly[0] + x * (f.poly[1] + x * f.poly[2])) * std::sin(f.kappa * x + f.phase);
}

static double time_value(const pe_time_factor &tf, double t) {
  const double poly = tf.poly[0] + t * (tf.poly[1] + t * (tf.poly[2] + t * tf.poly[3]));
  return std::exp(tf.alpha * t) * std::cos(tf.omega * t + tf.phase) * poly;
}

void boundary_terms(pe_grid g, bool mass_only, double t, std::vector<DerivedTerm> &out) {
  const int d = g->dim;
  for (const pe_term &bt : g->src_boundary) {
    // the 1D products of the data's nodal values on each axis
    std::vector<double> P[PE_MAX_DIM], Qv[PE_MAX_DIM], R[PE_MAX_DIM], S[PE_MAX_DIM];
    for (int a = 0; a < d; ++a) {
      const Axis &ax = g->ax[a];
      const int n = ax.n;
      const double h = ax.h;
      std::vector<double> xb(n + 2);
      for (int j = 0; j < n + 2; ++j) xb[j] = space_value(bt.space[a], ax.lo + h * j);
      P[a].resize(n);
      Qv[a].resize(n);
      R[a].resize(n);
      S[a].resize(n);
      for (int i = 0; i < n; ++i) {
        const double xl = xb[i], xc = xb[i + 1], xr = xb[i + 2];
        const double xli = i > 0 ? xl : 0.0, xri = i < n - 1 ? xr : 0.0;
        P[a][i] = (h / 6.0) * xl + (4.0 * h / 6.0) * xc + (h / 6.0) * xr;
        Qv[a][i] = (h / 6.0) * xli + (4.0 * h / 6.0) * xc + (h / 6.0) * xri;
        R[a][i] = (2.0 * xc - xl - xr) / h;
        S[a][i] = (2.0 * xc - xli - xri) / h;
      }
    }
    auto add = [&](double amp, bool deriv, const std::vector<double> *const *tabs) {
      DerivedTerm dt;
      dt.time = to_dev_term(bt);
      dt.time.amp = amp;
      dt.time.deriv = deriv ? 1 : 0;
      if (mass_only) {   // constant in time: the factor at t folded into amp
        dt.time.amp = amp * time_value(bt.time, t);
        dt.time.alpha = dt.time.omega = 0.0;
        dt.time.phase = 0.0;
        dt.time.p[0] = 1.0;
        dt.time.p[1] = dt.time.p[2] = dt.time.p[3] = 0.0;
      }
      for (int a = 0; a < d; ++a) dt.table[a] = *tabs[a];
      out.push_back(std::move(dt));
    };
    const std::vector<double> *tp[PE_MAX_DIM], *tq[PE_MAX_DIM];
    for (int a = 0; a < d; ++a) {
      tp[a] = &P[a];
      tq[a] = &Qv[a];
    }
    // -M_IB g_B' (or -M_IB g_B(t) for the initial value)
    add(-bt.amp, !mass_only, tp);
    add(bt.amp, !mass_only, tq);
    if (mass_only) continue;
    // -D A_IB g_B
    for (int a = 0; a < d; ++a) {
      const std::vector<double> *tr[PE_MAX_DIM], *ts[PE_MAX_DIM];
      for (int b = 0; b < d; ++b) {
        tr[b] = b == a ? &R[b] : &P[b];
        ts[b] = b == a ? &S[b] : &Qv[b];
      }
      add(-g->D * bt.amp, false, tr);
      add(g->D * bt.amp, false, ts);
    }
  }
}

// The 1D tables of explicit-vector terms into rows row0.. of the per-axis
// tables (stride np_a, zero beyond n_a).
pe_status upload_derived(pe_grid g, const std::vector<DerivedTerm> &der, int row0, double **dst,
                         hipStream_t st) {
  for (int a = 0; a < g->dim; ++a) {
    const Axis &ax = g->ax[a];
    std::vector<double> rows(size_t(ax.np) * der.size(), 0.0);
    for (size_t m = 0; m < der.size(); ++m)
      for (int i = 0; i < ax.n; ++i) rows[m * ax.np + i] = der[m].table[a][i];
    if (!rows.empty()) {
      PE_HIP(hipMemcpyAsync(dst[a] + size_t(row0) * ax.np, rows.data(), sizeof(double) * rows.size(),
                            hipMemcpyHostToDevice, st));
      PE_HIP(hipStreamSynchronize(st));   // rows is host memory read by the copy
    }
  }
  return PE_OK;
}

}  // namespace pe

using namespace pe;

extern "C" {

const char *pe_last_error(void) { return g_err.c_str(); }

int64_t pe_grid_dof(pe_grid g) { return g ? g->dof : -1; }

static void drop_pending(pe_grid g) {
  for (auto &p : g->pending) {
    event_free(p.start);
    event_free(p.stop);
  }
  g->pending.clear();
}

pe_status pe_set_timing(pe_grid g, int32_t enable) {
  clear_error();
  if (!g) return set_error(PE_E_ARG, "null grid");
  if (enable) {
    PE_HIP(hipDeviceSynchronize());
    drop_pending(g);
    for (auto &s : g->stats) s = pe_kernel_stat{};
  }
  g->timing = enable != 0;
  return PE_OK;
}

pe_status pe_get_timing(pe_grid g, pe_kernel_stat *out) {
  clear_error();
  if (!g || !out) return set_error(PE_E_ARG, "null argument");
  for (auto &p : g->pending) {
    PE_HIP(hipEventSynchronize(p.stop));
    float ms = 0;
    PE_HIP(hipEventElapsedTime(&ms, p.start, p.stop));
    pe_kernel_stat &s = g->stats[p.cls];
    s.launches += 1;
    s.ms += ms;
    s.flops += p.flops;
    s.bytes += p.bytes;
  }
  drop_pending(g);
  for (int i = 0; i < PE_K_COUNT; ++i) out[i] = g->stats[i];
  return PE_OK;
}
int32_t pe_grid_precision(pe_grid g) { return g ? g->precision : -1; }

static pe_status init_grid(pe_grid *out, int32_t dim, const int32_t *n, const double *lo,
                           const double *hi, double D, int32_t precision, int32_t quad_q,
                           const int32_t *periodic, void *stream) {
  if (!out || !n || !lo || !hi) return set_error(PE_E_ARG, "null argument");
  *out = nullptr;
  if (dim < 1 || dim > PE_MAX_DIM) return set_error(PE_E_ARG, "dim must be 1..3 (got %d)", dim);
  if (!(D > 0) || !std::isfinite(D)) return set_error(PE_E_ARG, "D must be > 0");
  if (precision != PE_FP64 && precision != PE_SPLIT_BF16)
    return set_error(PE_E_ARG, "unknown precision %d", precision);
  if (quad_q < 1 || quad_q > 8) return set_error(PE_E_ARG, "quad_q must be 1..8");
  bool any_periodic = false;
  for (int a = 0; a < dim; ++a) {
    if (n[a] < 1 || n[a] > 8191) return set_error(PE_E_ARG, "n[%d] must be 1..8191", a);
    if (!(hi[a] > lo[a])) return set_error(PE_E_ARG, "hi[%d] must exceed lo[%d]", a, a);
    if (periodic && periodic[a]) {
      any_periodic = true;
      if (!fft_periodic_ok(n[a]))
        return set_error(PE_E_ARG, "periodic axis %d: n must be 64, 128, 256, 512 or 1024", a);
    }
  }
  if (any_periodic) {
    // periodic axes run on the FFT transform: FP64, and every other axis
    // must suit it too
    if (precision != PE_FP64) return set_error(PE_E_ARG, "periodic axes need an FP64 grid");
    for (int a = 0; a < dim; ++a)
      if (!periodic[a] && !fft_axis_ok(n[a]))
        return set_error(PE_E_ARG, "axis %d: with periodic axes n + 1 must be 64..512 (a power of 2)", a);
  }
  hipStream_t st = as_stream(stream);
  pe_grid g = new pe_grid_s();
  g->dim = dim;
  g->precision = precision;
  g->quad_q = quad_q;
  g->D = D;
  g->dof = 1;
  g->dofp = 1;
  auto fail = [&](pe_status s) {
    free_grid_tables(g);
    delete g;
    return s;
  };
  for (int a = 0; a < dim; ++a) {
    Axis &ax = g->ax[a];
    ax.n = n[a];
    ax.lo = lo[a];
    ax.hi = hi[a];
    if (periodic && periodic[a]) {
      ax.periodic = true;
      ax.Kh = ax.H = n[a] / 2;
      ax.np = n[a];
      ax.h = (hi[a] - lo[a]) / n[a];
      g->dof *= ax.n;
      g->dofp *= ax.np;
      hipError_t e = hipMalloc(&ax.d_lam, sizeof(double) * ax.n);
      if (e == hipSuccess) e = hipMalloc(&ax.d_sig, sizeof(double) * ax.n);
      if (e != hipSuccess)
        return fail(set_error(PE_E_HIP, "grid table allocation failed: %s", hipGetErrorString(e)));
      k_axis_eig_periodic<<<(ax.n + 127) / 128, 128, 0, st>>>(ax.n, ax.h, ax.d_lam, ax.d_sig);
      continue;
    }
    ax.Kh = half_pad(n[a]);
    ax.H = n[a] / 2;
    ax.np = 2 * ax.Kh;
    ax.h = (hi[a] - lo[a]) / (n[a] + 1);
    g->dof *= ax.n;
    g->dofp *= ax.np;
    size_t s2 = size_t(2) * ax.Kh * ax.Kh;
    hipError_t e = hipMalloc(&ax.d_lam, sizeof(double) * ax.n);
    if (e == hipSuccess) e = hipMalloc(&ax.d_sig, sizeof(double) * ax.n);
    if (e == hipSuccess) e = hipMalloc(&ax.d_Sh, sizeof(double) * s2);
    if (e == hipSuccess) e = hipMalloc(&ax.d_ShT, sizeof(double) * s2);
    if (e == hipSuccess && precision == PE_SPLIT_BF16) {
      e = hipMalloc(&ax.d_Shi, sizeof(uint16_t) * s2);
      if (e == hipSuccess) e = hipMalloc(&ax.d_Slo, sizeof(uint16_t) * s2);
    }
    // second fold level: FP64 grids whose axis has n = 2 Kh - 1
    ax.l2 = precision == PE_FP64 && ax.n == 2 * ax.Kh - 1;
    if (e == hipSuccess && ax.l2) {
      const size_t q2 = size_t(ax.Kh / 2) * (ax.Kh / 2) * 4;
      e = hipMalloc(&ax.d_Sq, sizeof(double) * q2);
      if (e == hipSuccess) e = hipMalloc(&ax.d_SqT, sizeof(double) * q2);
    }
    // third level for the generating pass of the last axis
    ax.l3 = ax.l2 && a == dim - 1 && (ax.Kh == 64 || ax.Kh == 128);
    if (e == hipSuccess && ax.l3)
      e = hipMalloc(&ax.d_L3, sizeof(double) * 3 * size_t(ax.Kh / 2) * (ax.Kh / 2));
    if (e != hipSuccess)
      return fail(set_error(PE_E_HIP, "grid table allocation failed: %s", hipGetErrorString(e)));
    k_axis_eig<<<(ax.n + 127) / 128, 128, 0, st>>>(ax.n, ax.h, ax.d_lam, ax.d_sig);
    k_dst_half<<<dim3((ax.Kh + 127) / 128, ax.Kh, 2), 128, 0, st>>>(ax.n, ax.Kh, ax.H, ax.d_Sh,
                                                                     ax.d_ShT, ax.d_Shi, ax.d_Slo);
    if (ax.l2)
      k_dst_quarter<<<dim3((ax.Kh / 2 + 127) / 128, ax.Kh / 2, 4), 128, 0, st>>>(
          ax.n, ax.Kh / 2, ax.d_Sq, ax.d_SqT);
    if (ax.l3) {
      const int Q = ax.Kh / 2;
      k_dst_l3<<<dim3((3 * Q * Q / 2 + 255) / 256, 2), 256, 0, st>>>(Q, ax.d_Sq, ax.d_L3);
    }
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess)
    return fail(set_error(PE_E_HIP, "grid set-up kernels failed: %s", hipGetErrorString(e)));
  if (any_periodic) {
    pe_status ps = fft_prepare(g);
    if (ps != PE_OK) return fail(ps);
    g->transform = PE_TRANSFORM_FFT;
  }
  // the device address of pe_coarse_sweep_noalloc's static scratch
  pe_status ps = sweep_scratch_setup(nullptr);
  if (ps != PE_OK) return fail(ps);
  *out = g;
  return PE_OK;
}

pe_status pe_init_grid(pe_grid *out, int32_t dim, const int32_t *n, const double *lo,
                       const double *hi, double D, int32_t precision, int32_t quad_q,
                       void *stream) {
  clear_error();
  return init_grid(out, dim, n, lo, hi, D, precision, quad_q, nullptr, stream);
}

pe_status pe_init_grid_periodic(pe_grid *out, int32_t dim, const int32_t *n, const double *lo,
                                const double *hi, double D, int32_t precision, int32_t quad_q,
                                const int32_t *periodic, void *stream) {
  clear_error();
  if (!periodic) return set_error(PE_E_ARG, "null periodic flags");
  return init_grid(out, dim, n, lo, hi, D, precision, quad_q, periodic, stream);
}

void pe_free_grid(pe_grid g) {
  if (!g) return;
  drop_pending(g);
  free_grid_tables(g);
  delete g;
}

pe_status pe_set_transform(pe_grid g, int32_t kind) {
  clear_error();
  if (!g) return set_error(PE_E_ARG, "null grid");
  bool any_periodic = false;
  for (int a = 0; a < g->dim; ++a) any_periodic = any_periodic || g->ax[a].periodic;
  if (kind == PE_TRANSFORM_DENSE) {
    if (any_periodic) return set_error(PE_E_ARG, "periodic axes need the FFT transform");
    g->transform = kind;
    return PE_OK;
  }
  if (kind == PE_TRANSFORM_FFT && any_periodic) return PE_OK;
  if (kind != PE_TRANSFORM_FFT) return set_error(PE_E_ARG, "unknown transform %d", kind);
  if (g->precision != PE_FP64) return set_error(PE_E_ARG, "the FFT transform needs an FP64 grid");
  for (int a = 0; a < g->dim; ++a)
    if (!fft_axis_ok(g->ax[a].n))
      return set_error(PE_E_ARG, "the FFT transform needs n + 1 in {64, 128, 256, 512} (axis %d: n = %d)",
                       a, g->ax[a].n);
  PE_TRY(fft_prepare(g));
  g->transform = kind;
  return PE_OK;
}

pe_status pe_set_fusion(pe_grid g, int32_t enable) {
  clear_error();
  if (!g) return set_error(PE_E_ARG, "null grid");
  g->fuse_gen_mid = enable != 0;
  return PE_OK;
}

// The internal term list: the forcing (loads by the grid's Gauss rule)
// followed by the derived terms of the Dirichlet data (explicit tables).
static pe_status rebuild_terms(pe_grid g, hipStream_t st) {
  for (int a = 0; a < PE_MAX_DIM; ++a) {
    dev_free(g->d_C[a]);
    g->d_C[a] = nullptr;
    dev_free(g->d_spec[a]);
    g->d_spec[a] = nullptr;
  }
  dev_free(g->d_terms);
  g->d_terms = nullptr;
  dev_free(g->d_Cf);
  g->d_Cf = nullptr;
  dev_free(g->d_Cft);
  g->d_Cft = nullptr;
  std::vector<DerivedTerm> der;
  boundary_terms(g, false, 0.0, der);
  const int mf = int(g->src_forcing.size());
  const int n_terms = mf + int(der.size());
  g->n_terms = 0;
  if (n_terms > PE_MAX_TERMS)
    return set_error(PE_E_ARG, "%d forcing terms + %d from the boundary data exceed %d", mf,
                     int(der.size()), PE_MAX_TERMS);
  if (n_terms == 0) return PE_OK;
  for (int m = 0; m < mf; ++m) g->h_terms[m] = to_dev_term(g->src_forcing[m]);
  for (size_t m = 0; m < der.size(); ++m) g->h_terms[mf + m] = der[m].time;
  PE_HIP(hipMalloc(&g->d_terms, sizeof(DevTerm) * n_terms));
  PE_HIP(hipMemcpyAsync(g->d_terms, g->h_terms, sizeof(DevTerm) * n_terms, hipMemcpyHostToDevice,
                        st));
  for (int a = 0; a < g->dim; ++a)
    PE_HIP(hipMalloc(&g->d_C[a], sizeof(double) * size_t(n_terms) * g->ax[a].np));
  if (mf > 0) PE_TRY(build_loads(g, mf, g->src_forcing.data(), g->d_C, st));
  PE_TRY(upload_derived(g, der, mf, g->d_C, st));
  const Axis &last = g->ax[g->dim - 1];
  PE_HIP(hipMalloc(&g->d_Cf, sizeof(double) * 2 * size_t(n_terms) * last.Kh));
  PE_TRY(fold_table(g, g->d_C[g->dim - 1], n_terms, g->d_Cf, st));
  if (g->precision != PE_FP64 && gen_supported_split(g, n_terms)) {
    PE_HIP(hipMalloc(&g->d_Cft, split_gen_table_bytes(g)));
    PE_TRY(split_gen_table(g, g->d_Cf, n_terms, g->d_Cft, st));
  }
  for (int a = 0; a < g->dim; ++a) {
    const Axis &ax = g->ax[a];
    PE_HIP(hipMalloc(&g->d_spec[a], sizeof(double) * size_t(n_terms) * ax.n));
    k_axis_spectra<<<dim3((ax.n + 127) / 128, n_terms), 128, 0, st>>>(g->d_C[a], ax.np, ax.n,
                                                                      ax.d_sig, n_terms,
                                                                      g->d_spec[a]);
    PE_HIP(hipGetLastError());
  }
  PE_HIP(hipStreamSynchronize(st));
  g->n_terms = n_terms;
  return PE_OK;
}

pe_status pe_set_forcing(pe_grid g, int32_t n_terms, const pe_term *terms, void *stream) {
  clear_error();
  if (!g) return set_error(PE_E_ARG, "null grid");
  if (n_terms < 0 || n_terms > PE_MAX_TERMS)
    return set_error(PE_E_ARG, "n_terms must be 0..%d", PE_MAX_TERMS);
  if (n_terms > 0 && !terms) return set_error(PE_E_ARG, "null terms");
  if (n_terms + (2 + 2 * g->dim) * int(g->src_boundary.size()) > PE_MAX_TERMS)
    return set_error(PE_E_ARG, "%d forcing terms + the boundary data's terms exceed %d", n_terms,
                     PE_MAX_TERMS);
  g->src_forcing.assign(terms, terms + n_terms);
  return rebuild_terms(g, as_stream(stream));
}

pe_status pe_set_moving_sources(pe_grid g, int32_t n, const pe_moving_hat *src, void *stream) {
  clear_error();
  if (!g) return set_error(PE_E_ARG, "null grid");
  if (n < 0 || n > PE_MAX_MOVING) return set_error(PE_E_ARG, "n must be 0..%d", PE_MAX_MOVING);
  if (n > 0 && !src) return set_error(PE_E_ARG, "null sources");
  for (int i = 0; i < n; ++i) {
    const pe_moving_hat &h = src[i];
    if (h.axis < 0 || h.axis >= g->dim) return set_error(PE_E_ARG, "source %d: bad axis", i);
    if (g->ax[h.axis].periodic) return set_error(PE_E_ARG, "source %d: periodic axis", i);
    if (!(h.width > 0) || !std::isfinite(h.width) || !std::isfinite(h.amp) ||
        !std::isfinite(h.c0) || !std::isfinite(h.c1) || !std::isfinite(h.omega) ||
        !std::isfinite(h.phase))
      return set_error(PE_E_ARG, "source %d: bad parameters", i);
  }
  hipStream_t st = as_stream(stream);
  for (int a = 0; a < PE_MAX_DIM; ++a) {
    dev_free(g->d_Chat[a]);
    g->d_Chat[a] = nullptr;
  }
  dev_free(g->d_hats);
  g->d_hats = nullptr;
  g->n_hats = 0;
  g->src_moving.assign(src, src + n);
  if (n == 0) return PE_OK;
  std::vector<DevHat> dh(n);
  std::vector<pe_term> factors(n);
  for (int i = 0; i < n; ++i) {
    const pe_moving_hat &h = src[i];
    pe_term tm{};
    tm.amp = h.amp;
    tm.time = h.time;
    for (int a = 0; a < PE_MAX_DIM; ++a) tm.space[a] = h.space[a];
    factors[i] = tm;
    dh[i].time = to_dev_term(tm);
    dh[i].width = h.width;
    dh[i].c0 = h.c0;
    dh[i].c1 = h.c1;
    dh[i].omega = h.omega;
    dh[i].phase = h.phase;
    dh[i].axis = h.axis;
  }
  PE_HIP(hipMalloc(&g->d_hats, sizeof(DevHat) * n));
  PE_HIP(hipMemcpyAsync(g->d_hats, dh.data(), sizeof(DevHat) * n, hipMemcpyHostToDevice, st));
  for (int a = 0; a < g->dim; ++a)
    PE_HIP(hipMalloc(&g->d_Chat[a], sizeof(double) * size_t(n) * g->ax[a].np));
  PE_TRY(build_loads(g, n, factors.data(), g->d_Chat, st));   // synchronises
  g->n_hats = n;
  return PE_OK;
}

pe_status pe_set_boundary(pe_grid g, int32_t n_terms, const pe_term *terms, void *stream) {
  clear_error();
  if (!g) return set_error(PE_E_ARG, "null grid");
  for (int a = 0; a < g->dim; ++a)
    if (g->ax[a].periodic && n_terms > 0)
      return set_error(PE_E_ARG, "Dirichlet data on a grid with periodic axes");
  if (n_terms < 0 || n_terms > PE_MAX_TERMS)
    return set_error(PE_E_ARG, "n_terms must be 0..%d", PE_MAX_TERMS);
  if (n_terms > 0 && !terms) return set_error(PE_E_ARG, "null terms");
  const int per = 2 + 2 * g->dim;
  if (int(g->src_forcing.size()) + per * n_terms > PE_MAX_TERMS)
    return set_error(PE_E_ARG, "%d forcing terms + %d x %d from the boundary data exceed %d",
                     int(g->src_forcing.size()), n_terms, per, PE_MAX_TERMS);
  g->src_boundary.assign(terms, terms + n_terms);
  return rebuild_terms(g, as_stream(stream));
}

pe_status pe_phi_tables(pe_grid g, double h, int32_t s, const double *c, double *d_E, double *d_B,
                        void *stream) {
  clear_error();
  if (!g || !c || !d_E || !d_B) return set_error(PE_E_ARG, "null argument");
  if (!(h > 0) || !std::isfinite(h)) return set_error(PE_E_ARG, "h must be > 0");
  if (s < 1 || s > PE_MAX_STAGES) return set_error(PE_E_ARG, "s must be 1..%d", PE_MAX_STAGES);
  for (int i = 0; i < s; ++i)
    if (!(c[i] >= 0.0 && c[i] <= 1.0)) return set_error(PE_E_ARG, "node c[%d] outside [0,1]", i);
  PhiArgs a{};
  a.s = s;
  a.h = h;
  a.D = g->D;
  PE_TRY(lagrange_A(s, c, a.A));
  hipStream_t st = as_stream(stream);
  int64_t blocks = (g->dof + 255) / 256;
  k_phi_tables<<<dim3(unsigned(blocks)), 256, 0, st>>>(
      g->dim, g->ax[0].n, g->ax[1].n, g->ax[2].n, g->ax[0].d_lam, g->ax[1].d_lam,
      g->ax[2].d_lam, a, d_E, d_B, g->dof);
  PE_HIP(hipGetLastError());
  return PE_OK;
}

}  // extern "C"
