// Per-axis DST-I by FFT (FP64), the alternative to the dense matrix-core
// products of the fine propagator.
//
// Section 2.3 applies the diagonalising sine matrix with a fast transform.
// With L = n + 1 (a power of two) and S[k][j] = sqrt(2/L) sin(pi j k / L), a
// line x_1..x_n is extended to the odd sequence z of length 2L
//     z_0 = z_L = 0,   z_j = x_j,   z_{2L-j} = -x_j   (1 <= j < L),
// whose DFT is Z_k = -2i sum_j x_j sin(pi j k / L).  Two real lines x, x' go
// into one complex sequence z + i z', so one complex DFT of length N = 2L
// gives both transforms:
//     (S x)_k = -Im Z_k / sqrt(2L),   (S x')_k = Re Z_k / sqrt(2L).
// The DFT is a Stockham autosort FFT in LDS: radix-8 stages, then one radix-4
// or radix-2 stage, 512 threads per block holding 4096 complex points (4096/N
// line pairs), N/8 threads per FFT.  Results are written in the folded mode
// order of the dense path, so both paths feed the same update.
//
// Kernels: k_fft_pass (one axis of a batch of fields; on the last axis it can
// generate its input from the separable load tables) and k_fft_final (axis 0
// fused with the diagonal update of eq. (2.6): a block owns one slice and a
// strip of columns and walks the slice's stage fields with the states in
// registers).
#include <algorithm>
#include <cmath>

#include "pe_internal.h"

namespace pe {

namespace {

using c2 = double2;

constexpr int FFT_THREADS = 512;
constexpr int FFT_POINTS = 4096;       // complex points per block
constexpr int FFT_GEN_MAX_TERMS = 32;  // separable terms generated in registers

template <int N>
struct Shape {
  static constexpr int L = N / 2;           // n + 1
  static constexpr int P = FFT_POINTS / N;  // FFTs (line pairs) per block
  static constexpr int LINES = 2 * P;
  static constexpr int TF = N / 8;          // threads per FFT
  // LDS stride of one FFT in complex entries: one pad entry per 8 (the
  // stride-R writes of a stage spread over the banks), plus one so that the
  // FFTs of a block start on different banks
  static constexpr int FS = N + N / 8 + 1;
  static_assert(P * TF == FFT_THREADS, "one radix-8 butterfly per thread and stage");
};

__device__ __forceinline__ int pidx(int i) { return i + (i >> 3); }

__device__ __forceinline__ c2 cadd(c2 a, c2 b) { return c2{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ c2 csub(c2 a, c2 b) { return c2{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ c2 cmul(c2 a, c2 b) {
  return c2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// -i z
__device__ __forceinline__ c2 mul_mi(c2 a) { return c2{a.y, -a.x}; }

// In-register DFTs, natural order in and out: v_r <- sum_q v_q e^{-2 pi i q r / R}.
__device__ __forceinline__ void dft2(c2 *v) {
  const c2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
__device__ __forceinline__ void dft4(c2 &x0, c2 &x1, c2 &x2, c2 &x3) {
  const c2 s0 = cadd(x0, x2), d0 = csub(x0, x2), s1 = cadd(x1, x3), d1 = mul_mi(csub(x1, x3));
  x0 = cadd(s0, s1);
  x2 = csub(s0, s1);
  x1 = cadd(d0, d1);
  x3 = csub(d0, d1);
}
__device__ __forceinline__ void dft8(c2 *v) {
  constexpr double R2 = 0.70710678118654752440;   // sqrt(1/2)
  c2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  c2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  // o_r times w^r, w = e^{-2 pi i / 8} = sqrt(1/2) (1 - i)
  o1 = c2{R2 * (o1.x + o1.y), R2 * (o1.y - o1.x)};
  o2 = mul_mi(o2);
  o3 = c2{R2 * (o3.y - o3.x), -R2 * (o3.x + o3.y)};
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

// Radix of the last Stockham stage (radix-8 stages, then the remainder).
constexpr int last_radix(int N) {
  int ns = 1, r = 8;
  while (ns < N) {
    r = N / ns >= 8 ? 8 : N / ns;
    ns *= r;
  }
  return r;
}

// The FFTs of up to 512 points run inside one wave (N/8 <= 64 threads), so
// their stages need only the wave's own ordering of its LDS accesses; longer
// ones span two waves and take the block barrier.
template <int N>
__device__ __forceinline__ void fft_sync() {
  if constexpr (N / 8 <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// One Stockham stage of radix R on the sub-transforms of size NS: butterfly
// j takes the R inputs j + r N/R, twists input r by w_N^{r k N/(NS R)}
// (k = j mod NS), transforms them and stores output r at
// (j / NS) NS R + k + r NS.  A thread does 8/R butterflies; all reads come
// before any write (the stage is in place).  Without STORE the outputs stay
// in v.
template <int N, int R, int NS, bool STORE>
__device__ __forceinline__ void fft_stage(c2 *Z, const c2 *__restrict__ tw, int u, c2 (&v)[8]) {
  constexpr int B = 8 / R;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = u + b * (N / 8);
#pragma unroll
    for (int r = 0; r < R; ++r) v[b * R + r] = Z[pidx(j + r * (N / R))];
  }
  fft_sync<N>();
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = u + b * (N / 8);
    const int k = j % NS;
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[b * R + r] = cmul(v[b * R + r], tw[r * k * (N / (NS * R))]);
    }
    if constexpr (R == 8) dft8(&v[b * R]);
    if constexpr (R == 4) dft4(v[b * R], v[b * R + 1], v[b * R + 2], v[b * R + 3]);
    if constexpr (R == 2) dft2(&v[b * R]);
    if constexpr (STORE) {
      const int dst = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) Z[pidx(dst + r * NS)] = v[b * R + r];
    }
  }
  if constexpr (STORE) fft_sync<N>();
}

// All stages of the FFT in Z (thread u of its N/8).  With KEEP_LAST the last
// stage's outputs stay in v: there NS = N/R, so butterfly j = u + b N/8 holds
// the outputs j + r N/R, and those below L = N/2 (the sine sums) are the
// four slots s = b (R/2) + r, r < R/2 (last_slot).
template <int N, int NS, bool KEEP_LAST>
__device__ __forceinline__ void fft_run(c2 *Z, const c2 *__restrict__ tw, int u, c2 (&v)[8]) {
  if constexpr (NS < N) {
    constexpr int R = N / NS >= 8 ? 8 : N / NS;
    fft_stage<N, R, NS, !(KEEP_LAST && NS * R == N)>(Z, tw, u, v);
    fft_run<N, NS * R, KEEP_LAST>(Z, tw, u, v);
  }
}

// slot s (0..3) of a kept last stage: register vi and DFT index fi < L
template <int N>
__device__ __forceinline__ void last_slot(int u, int s, int &vi, int &fi) {
  constexpr int R = last_radix(N), H = R / 2;
  const int b = s / H, r = s % H;
  vi = b * R + r;
  fi = u + b * (N / 8) + r * (N / R);
}

// Writes node j (0-based, value x) of tile line l into the odd extension:
// line l is the real (l < P) or imaginary part of FFT l mod P.  The thread of
// the position j = L - 1 (beyond the last node) writes the two zeros.
template <int N>
__device__ __forceinline__ void put_node(double *Zd, int l, int j, double x) {
  using Sh = Shape<N>;
  const int p = l % Sh::P, part = l / Sh::P;
  double *z = Zd + 2 * p * Sh::FS + part;
  if (j < Sh::L - 1) {
    z[2 * pidx(j + 1)] = x;
    z[2 * pidx(N - 1 - j)] = -x;
  } else {
    z[2 * pidx(0)] = 0.0;
    z[2 * pidx(Sh::L)] = 0.0;
  }
}

// Raw sine sum of mode m (0-based) of tile line l, times sqrt(2L).
template <int N>
__device__ __forceinline__ double get_mode(const c2 *Zs, int l, int m) {
  using Sh = Shape<N>;
  const int p = l % Sh::P, part = l / Sh::P;
  const c2 F = Zs[p * Sh::FS + pidx(m + 1)];
  return part ? F.x : -F.y;
}

}  // namespace

struct FftPassArgs {
  const double *in;          // nodal lines (unused when generating)
  double *out;               // DST coefficients, folded mode order
  int64_t nlines;            // lines of the pass
  int64_t inner;             // stride between the nodes of a line
  const c2 *tw;              // [N] e^{-2 pi i k / N}
  // load generation (last axis): node (f, r, j) has the load
  // sum_m coef[f][m] pre_r[m] Cl[m][j], pre_r the product of the other axes'
  // tables at the line's nodes
  const double *coef;        // [fields][M]
  const double *C0, *C1;     // [M][np_0], [M][np_1] (d >= 2, d == 3)
  const double *Cl;          // [M][L] last-axis loads
  int M, d, np0, np1;
  int64_t rows;              // lines per field (product of the other axes' np)
};

// One axis of a batch of fields, lines read from `in`.  Block = LINES
// lines; contiguous lines (the last axis) are read and written by the wave
// that transforms them, strided lines (adjacent columns) across the block.
template <int N, bool CONTIG>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_pass(FftPassArgs a) {
  using Sh = Shape<N>;
  constexpr int L = Sh::L, LINES = Sh::LINES;
  __shared__ c2 Zs[Sh::P * Sh::FS];
  double *Zd = reinterpret_cast<double *>(Zs);
  const int t = threadIdx.x;
  const int64_t l0 = int64_t(blockIdx.x) * LINES;
  auto line_base = [&](int64_t ln) -> int64_t {
    if (CONTIG) return ln * L;
    const int64_t o = ln / a.inner;
    return o * L * a.inner + (ln - o * a.inner);
  };
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int e = t + k * FFT_THREADS;
    // contiguous lines: consecutive threads walk a line; strided lines:
    // consecutive threads take consecutive lines (adjacent columns)
    const int l = CONTIG ? e / L : e % LINES;
    const int j = CONTIG ? e % L : e / LINES;
    const int64_t ln = l0 + l;
    const double x = (ln < a.nlines && j < L - 1) ? a.in[line_base(ln) + int64_t(j) * a.inner] : 0.0;
    put_node<N>(Zd, l, j, x);
  }
  __syncthreads();
  const int p = t / Sh::TF, u = t % Sh::TF;
  c2 v[8];
  fft_run<N, 1, CONTIG>(Zs + p * Sh::FS, a.tw, u, v);

  const double scale = 1.0 / sqrt(double(N));
  if constexpr (CONTIG) {
    // straight from the registers: the FFT's two lines, mode m = fi - 1 at
    // folded position fold_pos(m); the slot of fi = 0 writes the pad L - 1
    const int64_t ln0 = l0 + p, ln1 = l0 + p + Sh::P;
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      int vi, fi;
      last_slot<N>(u, sl, vi, fi);
      const int q = fi > 0 ? fold_pos(fi - 1, L / 2) : L - 1;
      if (ln0 < a.nlines) a.out[ln0 * L + q] = fi > 0 ? -v[vi].y * scale : 0.0;
      if (ln1 < a.nlines) a.out[ln1 * L + q] = fi > 0 ? v[vi].x * scale : 0.0;
    }
  } else {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = t + k * FFT_THREADS;
      const int l = e % LINES, q = e / LINES;
      const int64_t ln = l0 + l;
      if (ln >= a.nlines) continue;
      const int m = unfold_pos(q, L / 2);
      const double y = m < L - 1 ? get_mode<N>(Zs, l, m) * scale : 0.0;
      a.out[line_base(ln) + int64_t(q) * a.inner] = y;
    }
  }
}

// The last-axis pass generating its lines from the separable load tables:
// block = LINES lines, the thread's node position j = t mod L.  MT: the
// terms rounded up (8, 16 or 32; sizes the factor buffer and the table
// registers).  (A persistent form that keeps the table column in registers
// across tiles holds too many registers for two blocks per CU and is slower.)
template <int N, int MT>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_gen(FftPassArgs a) {
  using Sh = Shape<N>;
  constexpr int L = Sh::L, LINES = Sh::LINES;
  __shared__ c2 Zs[Sh::P * Sh::FS];
  __shared__ double pre[LINES * MT];
  double *Zd = reinterpret_cast<double *>(Zs);
  const int t = threadIdx.x;
  const int64_t l0 = int64_t(blockIdx.x) * LINES;
  // factor (l, m): coef[f][m] times the other axes' tables at the line's
  // nodes (zero beyond the lines)
  for (int e = t; e < LINES * a.M; e += FFT_THREADS) {
    const int l = e / a.M, m = e - l * a.M;
    const int64_t ln = l0 + l;
    double v = 0.0;
    if (ln < a.nlines) {
      const int64_t f = ln / a.rows;
      const int64_t r = ln - f * a.rows;
      v = a.coef[f * a.M + m];
      if (a.d == 2) v *= a.C0[int64_t(m) * a.np0 + r];
      if (a.d == 3) {
        v *= a.C0[int64_t(m) * a.np0 + r / a.np1];
        v *= a.C1[int64_t(m) * a.np1 + r % a.np1];
      }
    }
    pre[l * MT + m] = v;
  }
  const int j = t % L;
  double cl[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) cl[m] = (m < a.M && j < L - 1) ? a.Cl[int64_t(m) * L + j] : 0.0;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int l = t / L + k * (FFT_THREADS / L);
    const double *pl = pre + l * MT;
    double x = 0.0;
#pragma unroll
    for (int m = 0; m < MT; ++m)
      if (m < a.M) x += pl[m] * cl[m];
    put_node<N>(Zd, l, j, x);
  }
  __syncthreads();
  const int p = t / Sh::TF, u = t % Sh::TF;
  c2 v[8];
  fft_run<N, 1, true>(Zs + p * Sh::FS, a.tw, u, v);
  const double scale = 1.0 / sqrt(double(N));
  const int64_t ln0 = l0 + p, ln1 = ln0 + Sh::P;
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    int vi, fi;
    last_slot<N>(u, sl, vi, fi);
    const int q = fi > 0 ? fold_pos(fi - 1, L / 2) : L - 1;
    if (ln0 < a.nlines) a.out[ln0 * L + q] = fi > 0 ? -v[vi].y * scale : 0.0;
    if (ln1 < a.nlines) a.out[ln1 * L + q] = fi > 0 ? v[vi].x * scale : 0.0;
  }
}

// Axis-0 pass fused with the update.  Block = (slice nl, strip of LINES
// columns).  The strip is loaded across the block (adjacent columns per
// thread), transformed per line pair inside a wave, and the thread updates
// the modes of its own last FFT stage: slot s (0..3) and part h (0: the real
// line p, 1: the imaginary line p + P), state k = 2 s + h.
struct FftFinalArgs {
  const double *X;        // [fields][L][inner] after the other axes' passes
  const double *Tf;       // update tables in the thread order (fft_tables)
  const double *Uin;      // nullable
  double *Uout;
  const c2 *tw;
  int64_t inner, dof;
  int nslices, strips, jc, s;
  int n1, Kh1, n2, Kh2, np2, d;
  int per1, per2;         // inner axes periodic (position = mode, no fold)
};

// state index of (mode m, padded column c) or -1 at pads (DOF < 2^31 here)
__device__ __forceinline__ int fft_state_index(const FftFinalArgs &a, int L, int m, int64_t c) {
  if (m < 0 || m >= L - 1) return -1;
  int k1, k2 = 0;
  if (a.d == 3) {
    const int p1 = int(c / a.np2), p2 = int(c % a.np2);
    k1 = a.per1 ? p1 : unfold_pos(p1, a.Kh1);
    k2 = a.per2 ? p2 : unfold_pos(p2, a.Kh2);
    if (k2 >= a.n2) return -1;
  } else {
    k1 = a.per1 ? int(c) : unfold_pos(int(c), a.Kh1);
  }
  if (k1 >= a.n1) return -1;
  return (m * a.n1 + k1) * (a.d == 3 ? a.n2 : 1) + k2;
}

// (mode, column) of state k of thread t in strip `strip`
template <int N>
__device__ __forceinline__ void final_state(int t, int k, int64_t strip, int &m, int64_t &col) {
  using Sh = Shape<N>;
  const int p = t / Sh::TF, u = t % Sh::TF;
  int vi, fi;
  last_slot<N>(u, k / 2, vi, fi);
  m = fi - 1;
  col = strip * Sh::LINES + p + (k & 1) * Sh::P;
}

template <int N>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_final(FftFinalArgs a) {
  using Sh = Shape<N>;
  constexpr int L = Sh::L, LINES = Sh::LINES;
  __shared__ c2 Zs[Sh::P * Sh::FS];
  double *Zd = reinterpret_cast<double *>(Zs);
  const int t = threadIdx.x;
  const int nl = int(blockIdx.x % a.nslices);
  const int strip = int(blockIdx.x / a.nslices);
  const int p = t / Sh::TF, u = t % Sh::TF;
  const int nf = a.jc * a.s;

  int kidx[8];
  double W[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int m;
    int64_t c;
    final_state<N>(t, k, strip, m, c);
    kidx[k] = fft_state_index(a, L, m, c);
    W[k] = (a.Uin && kidx[k] >= 0) ? a.Uin[int64_t(nl) * a.dof + kidx[k]] : 0.0;
  }
  // loader: thread = column l (adjacent across threads), rows j = t / LINES + k 512/LINES
  const int l = t % LINES;
  const double *Xs = a.X + int64_t(nl) * nf * L * a.inner + int64_t(strip) * LINES + l;
  const double *Tl = a.Tf + int64_t(strip) * (1 + a.s) * 8 * FFT_THREADS + t;
  double S[8];
  auto load = [&](int e) {
    const double *Xf = Xs + int64_t(e) * L * a.inner;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int j = t / LINES + k * (FFT_THREADS / LINES);
      S[k] = j < L - 1 ? Xf[int64_t(j) * a.inner] : 0.0;
    }
  };
  load(0);
  for (int e = 0; e < nf; ++e) {
#pragma unroll
    for (int k = 0; k < 8; ++k) put_node<N>(Zd, l, t / LINES + k * (FFT_THREADS / LINES), S[k]);
    __syncthreads();
    // the field's tables, issued before the next strip's loads (loads
    // complete in issue order: the update then waits for its tables only)
    const int i = e % a.s;
    const double *Ti = Tl + (1 + i) * 8 * FFT_THREADS;
    double tb[8], te[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      tb[k] = Ti[k * FFT_THREADS];
      te[k] = i == 0 ? Tl[k * FFT_THREADS] : 1.0;
    }
    if (e + 1 < nf) load(e + 1);   // in flight during the transform
    c2 v[8];
    fft_run<N, 1, true>(Zs + p * Sh::FS, a.tw, u, v);
    // eq. (2.6): W = E W at a step's first stage, then W += (b_i sigma) y;
    // the tables carry sigma and the 1/sqrt(2L)
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      int vi, fi;
      last_slot<N>(u, sl, vi, fi);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = 2 * sl + h;
        const double y = h ? v[vi].x : -v[vi].y;
        double w = W[k];
        if (i == 0) w = te[k] * w;
        W[k] = w + tb[k] * y;
      }
    }
    __syncthreads();   // every wave is done with LDS before the next strip lands
  }
  double *Uo = a.Uout + int64_t(nl) * a.dof;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (kidx[k] >= 0) Uo[kidx[k]] = W[k];
}

// Tables of k_fft_final: Tf[strip][tbl][k][t], tbl 0 = E, tbl 1 + i =
// b_i sigma / sqrt(2L) (zero at pads).
__global__ void k_fft_tables(FftFinalArgs a, int L, const double *__restrict__ sig0,
                             const double *__restrict__ sig1, const double *__restrict__ sig2,
                             const double *__restrict__ E, const double *__restrict__ B,
                             double *Tf) {
  const int64_t total = int64_t(a.strips) * (1 + a.s) * 8 * FFT_THREADS;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int t = int(e % FFT_THREADS);
    const int k = int((e / FFT_THREADS) % 8);
    const int tbl = int((e / (8 * FFT_THREADS)) % (1 + a.s));
    const int64_t strip = e / (int64_t(8) * FFT_THREADS * (1 + a.s));
    int m;
    int64_t col;
    if (L == 64) final_state<128>(t, k, strip, m, col);
    else if (L == 128) final_state<256>(t, k, strip, m, col);
    else if (L == 256) final_state<512>(t, k, strip, m, col);
    else final_state<1024>(t, k, strip, m, col);
    const int64_t ki = fft_state_index(a, L, m, col);
    double v = 0.0;
    if (ki >= 0) {
      if (tbl == 0) {
        v = E[ki];
      } else {
        const int64_t rest = ki % (a.dof / (L - 1));
        double sig = sig0[m];
        if (a.d == 3) {
          sig *= sig1[rest / a.n2];
          sig *= sig2[rest % a.n2];
        } else {
          sig *= sig1[rest];
        }
        v = B[int64_t(tbl - 1) * a.dof + ki] * sig * (1.0 / sqrt(2.0 * L));
      }
    }
    Tf[e] = v;
  }
}

// One periodic axis (N = n nodes per period) of a batch of fields.  Two real
// lines x, x' ride in one complex FFT of z = x + i x' (no extension); with
// Z = DFT(z), X_k = (Z_k + conj Z_{N-k}) / 2 and X'_k = (Z_k - conj Z_{N-k}) / 2i,
// and the orthonormal cos/sin coefficients of a line are Re X_0 / sqrt(N)
// (position 0), sqrt(2/N) Re X_k (cos k, position 2k - 1), -sqrt(2/N) Im X_k
// (sin k, position 2k) and Re X_{N/2} / sqrt(N) (position N - 1).
template <int N, bool CONTIG>
__device__ __forceinline__ int64_t periodic_line_base(const FftPassArgs &a, int64_t ln) {
  if (CONTIG) return ln * N;
  const int64_t o = ln / a.inner;
  return o * N * a.inner + (ln - o * a.inner);
}

// The block's lines in Zs (line l: FFT l % P, real part for l < P): FFT
// and the cos/sin coefficients out.
template <int N, bool CONTIG>
__device__ __forceinline__ void periodic_fft_out(c2 *Zs, const FftPassArgs &a, int64_t l0, int t) {
  using Sh = Shape<N>;
  constexpr int LINES = Sh::LINES;
  constexpr int PER_THREAD = LINES * N / FFT_THREADS;
  c2 v[8];
  fft_run<N, 1, false>(Zs + (t / Sh::TF) * Sh::FS, a.tw, t % Sh::TF, v);
  __syncthreads();
  const double s0 = 1.0 / sqrt(double(N)), s1 = sqrt(2.0 / double(N));
#pragma unroll
  for (int k = 0; k < PER_THREAD; ++k) {
    const int e = t + k * FFT_THREADS;
    const int l = CONTIG ? e / N : e % LINES;
    const int q = CONTIG ? e % N : e / LINES;
    const int64_t ln = l0 + l;
    if (ln >= a.nlines) continue;
    const int p = l % Sh::P, part = l / Sh::P;
    const int kk = q == 0 ? 0 : (q == N - 1 ? N / 2 : (q + 1) / 2);
    const c2 Zk = Zs[p * Sh::FS + pidx(kk)];
    const c2 Zm = Zs[p * Sh::FS + pidx((N - kk) % N)];
    const double re = part ? 0.5 * (Zk.y + Zm.y) : 0.5 * (Zk.x + Zm.x);
    const double im = part ? -0.5 * (Zk.x - Zm.x) : 0.5 * (Zk.y - Zm.y);
    const double y = (q == 0 || q == N - 1) ? re * s0 : ((q & 1) ? re * s1 : -im * s1);
    a.out[periodic_line_base<N, CONTIG>(a, ln) + int64_t(q) * a.inner] = y;
  }
}

template <int N, bool CONTIG>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_pass_periodic(FftPassArgs a) {
  using Sh = Shape<N>;
  constexpr int LINES = Sh::LINES;
  constexpr int PER_THREAD = LINES * N / FFT_THREADS;
  __shared__ c2 Zs[Sh::P * Sh::FS];
  double *Zd = reinterpret_cast<double *>(Zs);
  const int t = threadIdx.x;
  const int64_t l0 = int64_t(blockIdx.x) * LINES;
#pragma unroll
  for (int k = 0; k < PER_THREAD; ++k) {
    const int e = t + k * FFT_THREADS;
    const int l = CONTIG ? e / N : e % LINES;
    const int j = CONTIG ? e % N : e / LINES;
    const int64_t ln = l0 + l;
    const double x =
        ln < a.nlines ? a.in[periodic_line_base<N, CONTIG>(a, ln) + int64_t(j) * a.inner] : 0.0;
    Zd[2 * ((l % Sh::P) * Sh::FS + pidx(j)) + l / Sh::P] = x;
  }
  __syncthreads();
  periodic_fft_out<N, CONTIG>(Zs, a, l0, t);
}

// Generating pass on a periodic last axis (contiguous lines): the load value
// of node j of line (f, r) is sum_m coef[f][m] pre_r[m] Cl[m][j], as in
// k_fft_gen, formed in registers and then transformed as in
// k_fft_pass_periodic (Cl rows have N entries: a periodic axis has np = n).
// The factor table pre[l][m] borrows the FFT buffer (it is dead once the
// values are formed).  MT: the terms rounded up.
template <int N, int MT>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_gen_periodic(FftPassArgs a) {
  using Sh = Shape<N>;
  constexpr int LINES = Sh::LINES;
  constexpr int PER_THREAD = LINES * N / FFT_THREADS;
  // node positions of a thread: t mod N when N divides the block, else
  // t + FFT_THREADS jd (element k has jd = k mod JD, line k / JD)
  constexpr int JD = N > FFT_THREADS ? N / FFT_THREADS : 1;
  static_assert(N % FFT_THREADS == 0 || FFT_THREADS % N == 0, "node mapping");
  static_assert(LINES * MT <= 2 * Sh::P * Sh::FS, "the factors fit the FFT buffer");
  __shared__ c2 Zs[Sh::P * Sh::FS];
  double *Zd = reinterpret_cast<double *>(Zs);
  double *pre = Zd;
  const int t = threadIdx.x;
  const int64_t l0 = int64_t(blockIdx.x) * LINES;
  for (int e = t; e < LINES * a.M; e += FFT_THREADS) {
    const int l = e / a.M, m = e - l * a.M;
    const int64_t ln = l0 + l;
    double v = 0.0;
    if (ln < a.nlines) {
      const int64_t f = ln / a.rows;
      const int64_t r = ln - f * a.rows;
      v = a.coef[f * a.M + m];
      if (a.d == 2) v *= a.C0[int64_t(m) * a.np0 + r];
      if (a.d == 3) {
        v *= a.C0[int64_t(m) * a.np0 + r / a.np1];
        v *= a.C1[int64_t(m) * a.np1 + r % a.np1];
      }
    }
    pre[l * MT + m] = v;
  }
  __syncthreads();
  double x[PER_THREAD];
#pragma unroll
  for (int jd = 0; jd < JD; ++jd) {
    const int j = JD > 1 ? t + jd * FFT_THREADS : t % N;
    double cl[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) cl[m] = m < a.M ? a.Cl[int64_t(m) * N + j] : 0.0;
#pragma unroll
    for (int k = jd; k < PER_THREAD; k += JD) {
      const int l = (t + k * FFT_THREADS) / N;
      const double *pl = pre + l * MT;
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < MT; ++m)
        if (m < a.M) s += pl[m] * cl[m];
      x[k] = s;
    }
  }
  __syncthreads();   // the factors are dead: the buffer takes the lines
#pragma unroll
  for (int k = 0; k < PER_THREAD; ++k) {
    const int e = t + k * FFT_THREADS;
    const int l = e / N, j = e % N;
    Zd[2 * ((l % Sh::P) * Sh::FS + pidx(j)) + l / Sh::P] = x[k];
  }
  __syncthreads();
  periodic_fft_out<N, true>(Zs, a, l0, t);
}

// Axis-0 periodic pass fused with the update.  Block = (slice nl, strip of
// LINES columns); thread t owns column l = t mod LINES and the PT = 16
// consecutive positions q0 + k, q0 = 16 (t / LINES), of it on axis 0 (so its
// loads, LDS offsets and tables are fixed offsets from one base each), loads
// those nodes of every field (adjacent columns across threads), and after
// the block's FFTs reads its coefficients as k_fft_pass_periodic does and
// updates its states (eq. 2.6; the tables carry sigma and the cos/sin
// scale).
constexpr int FFTP_PT = 16;

template <int N>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_final_periodic(FftFinalArgs a) {
  using Sh = Shape<N>;
  constexpr int LINES = Sh::LINES;
  constexpr int PT = FFTP_PT;
  static_assert(LINES * N == PT * FFT_THREADS, "16 positions per thread");
  __shared__ c2 Zs[Sh::P * Sh::FS];
  double *Zd = reinterpret_cast<double *>(Zs);
  const int t = threadIdx.x;
  const int nl = int(blockIdx.x % a.nslices);
  const int strip = int(blockIdx.x / a.nslices);
  const int nf = a.jc * a.s;
  const int l = t % LINES, lp = l % Sh::P, part = l / Sh::P;
  const int q0 = PT * (t / LINES);
  const int64_t col = int64_t(strip) * LINES + l;
  const int inner = int(a.inner);

  double W[PT];
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    const int ki = fft_state_index(a, N + 1, q0 + k, col);
    W[k] = (a.Uin && ki >= 0) ? a.Uin[int64_t(nl) * a.dof + ki] : 0.0;
  }
  const double *Xs = a.X + int64_t(nl) * nf * N * a.inner + int64_t(q0) * inner + col;
  const double *Tl = a.Tf + (int64_t(strip) * (1 + a.s) * FFT_THREADS + t) * PT;
  c2 *Zl = Zs + lp * Sh::FS;
  double S[PT];
  auto load = [&](int e) {
    const double *Xf = Xs + int64_t(e) * N * inner;
#pragma unroll
    for (int k = 0; k < PT; ++k) S[k] = Xf[k * inner];
  };
  load(0);
  for (int e = 0; e < nf; ++e) {
#pragma unroll
    for (int k = 0; k < PT; ++k) reinterpret_cast<double *>(Zl + pidx(q0 + k))[part] = S[k];
    __syncthreads();
    if (e + 1 < nf) load(e + 1);   // in flight during the transform
    c2 v[8];
    fft_run<N, 1, false>(Zs + (t / Sh::TF) * Sh::FS, a.tw, t % Sh::TF, v);
    __syncthreads();
    const int i = e % a.s;
    const double *Te = Tl, *Ti = Tl + int64_t(1 + i) * FFT_THREADS * PT;
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      const int q = q0 + k;
      const int kk = q == 0 ? 0 : (q == N - 1 ? N / 2 : (q + 1) / 2);
      const c2 Zk = Zl[pidx(kk)];
      const c2 Zm = Zl[pidx((N - kk) % N)];
      const double re = part ? Zk.y + Zm.y : Zk.x + Zm.x;
      const double im = part ? Zm.x - Zk.x : Zk.y - Zm.y;
      const double y = (q == 0 || q == N - 1 || (q & 1)) ? re : -im;
      double w = W[k];
      if (i == 0) w = Te[k] * w;
      W[k] = w + Ti[k] * y;
    }
    __syncthreads();   // every wave is done with LDS before the next strip lands
  }
  double *Uo = a.Uout + int64_t(nl) * a.dof;
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    const int ki = fft_state_index(a, N + 1, q0 + k, col);
    if (ki >= 0) Uo[ki] = W[k];
  }
}

// Tables of k_fft_final_periodic: Tf[strip][tbl][t][k], tbl 0 = E, tbl 1 + i
// = b_i sigma times the coefficient scale of position q (1/(2 sqrt N) for
// the constant and alternating modes, 1/sqrt(2N) for cos/sin: the kernel
// forms twice Re X_k or -Im X_k), zero at pads.
__global__ void k_fft_tables_periodic(FftFinalArgs a, int N, int lines, const double *__restrict__ sig0,
                                      const double *__restrict__ sig1,
                                      const double *__restrict__ sig2,
                                      const double *__restrict__ E, const double *__restrict__ B,
                                      double *Tf) {
  const int64_t total = int64_t(a.strips) * (1 + a.s) * FFT_THREADS * FFTP_PT;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int k = int(e % FFTP_PT);
    const int t = int((e / FFTP_PT) % FFT_THREADS);
    const int tbl = int((e / (int64_t(FFTP_PT) * FFT_THREADS)) % (1 + a.s));
    const int64_t strip = e / (int64_t(FFTP_PT) * FFT_THREADS * (1 + a.s));
    const int q = FFTP_PT * (t / lines) + k;
    const int64_t col = strip * lines + t % lines;
    const int64_t ki = fft_state_index(a, N + 1, q, col);
    double v = 0.0;
    if (ki >= 0) {
      if (tbl == 0) {
        v = E[ki];
      } else {
        const int64_t rest = ki % (a.dof / N);
        double sig = sig0[q];
        if (a.d == 3) {
          sig *= sig1[rest / a.n2];
          sig *= sig2[rest % a.n2];
        } else {
          sig *= sig1[rest];
        }
        const double sc = (q == 0 || q == N - 1) ? 0.5 / sqrt(double(N)) : 1.0 / sqrt(2.0 * N);
        v = B[int64_t(tbl - 1) * a.dof + ki] * sig * sc;
      }
    }
    Tf[e] = v;
  }
}

// ------------------------------------------------------------------ host

bool fft_axis_ok(int n) {
  const int L = n + 1;
  return L == 64 || L == 128 || L == 256 || L == 512;
}

bool fft_periodic_ok(int n) { return n == 64 || n == 128 || n == 256 || n == 512 || n == 1024; }

bool fft_gen_supported(pe_grid g, int n_terms) {
  (void)g;
  return n_terms >= 1 && n_terms <= FFT_GEN_MAX_TERMS;
}

__global__ void k_fft_twiddles(int N, c2 *tw) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  double s, c;
  sincospi(2.0 * double(k) / double(N), &s, &c);
  tw[k] = c2{c, -s};
}

pe_status fft_prepare(pe_grid g) {
  for (int a = 0; a < g->dim; ++a) {
    Axis &ax = g->ax[a];
    if (ax.d_tw) continue;
    const int N = ax.periodic ? ax.n : 2 * (ax.n + 1);
    PE_HIP(hipMalloc(&ax.d_tw, sizeof(c2) * size_t(N)));
    k_fft_twiddles<<<(N + 255) / 256, 256>>>(N, reinterpret_cast<c2 *>(ax.d_tw));
    PE_HIP(hipGetLastError());
  }
  PE_HIP(hipDeviceSynchronize());
  return PE_OK;
}

template <int N>
static void launch_pass(const FftPassArgs &a, bool gen, bool contig, hipStream_t st) {
  const int64_t tiles = (a.nlines + Shape<N>::LINES - 1) / Shape<N>::LINES;
  if (gen) {
    if (a.M <= 8)
      k_fft_gen<N, 8><<<unsigned(tiles), FFT_THREADS, 0, st>>>(a);
    else if (a.M <= 16)
      k_fft_gen<N, 16><<<unsigned(tiles), FFT_THREADS, 0, st>>>(a);
    else
      k_fft_gen<N, FFT_GEN_MAX_TERMS><<<unsigned(tiles), FFT_THREADS, 0, st>>>(a);
  } else if (contig) {
    k_fft_pass<N, true><<<unsigned(tiles), FFT_THREADS, 0, st>>>(a);
  } else {
    k_fft_pass<N, false><<<unsigned(tiles), FFT_THREADS, 0, st>>>(a);
  }
}

template <int N>
static void launch_pass_periodic(const FftPassArgs &a, bool gen, bool contig, hipStream_t st) {
  const unsigned blocks = unsigned((a.nlines + Shape<N>::LINES - 1) / Shape<N>::LINES);
  if (gen) {
    // (the generating pass runs on the last axis, whose lines are contiguous)
    if (a.M <= 8)
      k_fft_gen_periodic<N, 8><<<blocks, FFT_THREADS, 0, st>>>(a);
    else if (a.M <= 16)
      k_fft_gen_periodic<N, 16><<<blocks, FFT_THREADS, 0, st>>>(a);
    else
      k_fft_gen_periodic<N, FFT_GEN_MAX_TERMS><<<blocks, FFT_THREADS, 0, st>>>(a);
  } else if (contig)
    k_fft_pass_periodic<N, true><<<blocks, FFT_THREADS, 0, st>>>(a);
  else
    k_fft_pass_periodic<N, false><<<blocks, FFT_THREADS, 0, st>>>(a);
}

pe_status dst_fields_fft(pe_grid g, int64_t count, const GenSrc *gen, double *buf0, double *buf1,
                         double **result, hipStream_t st, int stop_axis) {
  double *in = buf0, *out = buf1;
  const int d = g->dim;
  for (int ax_i = d - 1; ax_i >= stop_axis; --ax_i) {
    const Axis &ax = g->ax[ax_i];
    const int N = ax.periodic ? ax.n : 2 * (ax.n + 1);
    FftPassArgs a{};
    int64_t inner = 1;
    for (int b = ax_i + 1; b < d; ++b) inner *= g->ax[b].np;
    a.in = in;
    a.out = out;
    a.inner = inner;
    a.nlines = count * (g->dofp / ax.np);
    a.tw = reinterpret_cast<const c2 *>(ax.d_tw);
    const bool gen_pass = gen && ax_i == d - 1;
    if (gen_pass) {
      a.coef = gen->coef;
      a.C0 = gen->C0;
      a.C1 = gen->C1;
      a.Cl = gen->Cl;
      a.M = gen->M;
      a.d = d;
      a.np0 = g->ax[0].np;
      a.np1 = d == 3 ? g->ax[1].np : 1;
      a.rows = g->dofp / ax.np;
    }
    if (a.nlines / Shape<128>::LINES >= (int64_t(1) << 31))
      return set_error(PE_E_ARG, "internal: FFT pass grid too large");
    // flops of a complex FFT of N points, 5 N log2 N, per line pair
    const double lines = double(count) * double(g->dof / ax.n);
    const double flops = lines * 2.5 * N * std::log2(double(N));
    const double fb = double(count) * double(g->dof) * 8.0;
    TimedScope ts(g, ax_i == d - 1 ? PE_K_DST_LAST : PE_K_DST_MID, flops,
                  gen_pass ? fb : 2.0 * fb, st);
    const bool contig = inner == 1;
    if (ax.periodic) {
      if (gen_pass && !contig) return set_error(PE_E_ARG, "internal: generating pass on strided lines");
      switch (N) {
        case 64: launch_pass_periodic<64>(a, gen_pass, contig, st); break;
        case 128: launch_pass_periodic<128>(a, gen_pass, contig, st); break;
        case 256: launch_pass_periodic<256>(a, gen_pass, contig, st); break;
        case 512: launch_pass_periodic<512>(a, gen_pass, contig, st); break;
        case 1024: launch_pass_periodic<1024>(a, gen_pass, contig, st); break;
        default: return set_error(PE_E_ARG, "internal: periodic FFT length %d", N);
      }
      PE_HIP(hipGetLastError());
      std::swap(in, out);
      continue;
    }
    switch (N) {
      case 128: launch_pass<128>(a, gen_pass, contig, st); break;
      case 256: launch_pass<256>(a, gen_pass, contig, st); break;
      case 512: launch_pass<512>(a, gen_pass, contig, st); break;
      case 1024: launch_pass<1024>(a, gen_pass, contig, st); break;
      default: return set_error(PE_E_ARG, "internal: FFT length %d", N);
    }
    PE_HIP(hipGetLastError());
    std::swap(in, out);
  }
  *result = in;
  return PE_OK;
}

static FftFinalArgs final_args(pe_grid g, int s) {
  FftFinalArgs a{};
  const Axis &x0 = g->ax[0];
  a.inner = g->dofp / x0.np;
  a.dof = g->dof;
  a.d = g->dim;
  a.n1 = g->ax[1].n;
  a.Kh1 = g->ax[1].Kh;
  if (g->dim == 3) {
    a.n2 = g->ax[2].n;
    a.Kh2 = g->ax[2].Kh;
    a.np2 = g->ax[2].np;
  } else {
    a.n2 = a.Kh2 = a.np2 = 1;
  }
  a.per1 = g->ax[1].periodic ? 1 : 0;
  a.per2 = g->dim == 3 && g->ax[2].periodic ? 1 : 0;
  a.s = s;
  const int N = x0.periodic ? x0.n : 2 * (x0.n + 1);
  a.strips = int(a.inner / (2 * (FFT_POINTS / N)));
  a.tw = reinterpret_cast<const c2 *>(x0.d_tw);
  return a;
}

bool fft_final_supported(pe_grid g) {
  if (g->dim < 2 || g->dofp >= (int64_t(1) << 31) || g->dof >= (int64_t(1) << 31)) return false;
  const Axis &x0 = g->ax[0];
  const int N = x0.periodic ? x0.n : 2 * (x0.n + 1);
  // a block takes 2 FFT_POINTS / N whole columns
  return (g->dofp / x0.np) % (2 * (FFT_POINTS / N)) == 0;
}

pe_status fft_tables(pe_grid g, int s, const double *E, const double *B, double *Tf,
                     hipStream_t st) {
  FftFinalArgs a = final_args(g, s);
  const double *sig2 = g->dim > 2 ? g->ax[2].d_sig : nullptr;
  if (g->ax[0].periodic) {
    const int N = g->ax[0].n, lines = 2 * (FFT_POINTS / N);
    const int64_t n = int64_t(a.strips) * (1 + s) * FFT_THREADS * FFTP_PT;
    const unsigned blocks = unsigned(std::min<int64_t>((n + 255) / 256, 65536));
    k_fft_tables_periodic<<<blocks, 256, 0, st>>>(a, N, lines, g->ax[0].d_sig, g->ax[1].d_sig,
                                                   sig2, E, B, Tf);
    PE_HIP(hipGetLastError());
    return PE_OK;
  }
  const int L = g->ax[0].n + 1;
  const int64_t n = int64_t(a.strips) * (1 + s) * 8 * FFT_THREADS;
  const unsigned blocks = unsigned(std::min<int64_t>((n + 255) / 256, 65536));
  k_fft_tables<<<blocks, 256, 0, st>>>(a, L, g->ax[0].d_sig, g->ax[1].d_sig, sig2, E, B, Tf);
  PE_HIP(hipGetLastError());
  return PE_OK;
}

pe_status fft_final_update(pe_grid g, const FieldBatch &b, const double *X, const double *Tf,
                           const double *Uin, double *Uout, hipStream_t st) {
  FftFinalArgs a = final_args(g, b.s);
  a.X = X;
  a.Tf = Tf;
  a.Uin = Uin;
  a.Uout = Uout;
  a.jc = b.jc;
  a.nslices = b.nslices;
  const Axis &x0 = g->ax[0];
  const int N = x0.periodic ? x0.n : 2 * (x0.n + 1);
  const int64_t blocks = int64_t(b.nslices) * a.strips;
  if (blocks >= (int64_t(1) << 31)) return set_error(PE_E_ARG, "internal: FFT grid too large");
  const double fields = double(b.count());
  const double flops = fields * double(g->dof / x0.n) * 2.5 * N * std::log2(double(N));
  const double bytes = fields * double(g->dof) * 8.0 + 2.0 * b.nslices * double(g->dof) * 8.0 +
                       double(1 + b.s) * double(g->dof) * 8.0;
  TimedScope ts(g, PE_K_MID_UPDATE, flops, bytes, st);
  const dim3 grid = dim3(unsigned(blocks));
  if (x0.periodic) {
    switch (N) {
      case 64: k_fft_final_periodic<64><<<grid, FFT_THREADS, 0, st>>>(a); break;
      case 128: k_fft_final_periodic<128><<<grid, FFT_THREADS, 0, st>>>(a); break;
      case 256: k_fft_final_periodic<256><<<grid, FFT_THREADS, 0, st>>>(a); break;
      case 512: k_fft_final_periodic<512><<<grid, FFT_THREADS, 0, st>>>(a); break;
      case 1024: k_fft_final_periodic<1024><<<grid, FFT_THREADS, 0, st>>>(a); break;
      default: return set_error(PE_E_ARG, "internal: periodic FFT length %d", N);
    }
    PE_HIP(hipGetLastError());
    return PE_OK;
  }
  switch (N) {
    case 128: k_fft_final<128><<<dim3(unsigned(blocks)), FFT_THREADS, 0, st>>>(a); break;
    case 256: k_fft_final<256><<<dim3(unsigned(blocks)), FFT_THREADS, 0, st>>>(a); break;
    case 512: k_fft_final<512><<<dim3(unsigned(blocks)), FFT_THREADS, 0, st>>>(a); break;
    case 1024: k_fft_final<1024><<<dim3(unsigned(blocks)), FFT_THREADS, 0, st>>>(a); break;
    default: return set_error(PE_E_ARG, "internal: FFT length %d", N);
  }
  PE_HIP(hipGetLastError());
  return PE_OK;
}

}  // namespace pe
