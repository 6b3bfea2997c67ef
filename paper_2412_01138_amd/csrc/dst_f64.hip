// Per-axis DST-I passes in FP64 on the matrix cores (v_mfma_f64_16x16x4f64).
//
// The transform (kron_a S_a) F of a d-D field is d mode products, one per
// axis (paper Section 2.3, closing paragraph: mass and stiffness matrices are
// diagonalised by one orthogonal matrix applied with tensor products).  Each
// mode product is done on the even/odd fold of its axis (see pe_internal.h):
// two dense half-size products per axis, i.e. half the multiply-adds of the
// plain dense product, all of it on MFMA.
//
//   last axis  ("LAST"): X viewed as [R][np]
//       Y[r][h*Kh + i] = sum_p fold_h(X[r][.])[p] * Sh[h][i][p]      (A = folded X, B = ShT[h])
//   other axis ("MID"):  X viewed as [O][np][I]
//       Y[o][h*Kh + i][t] = sum_p Sh[h][i][p] * fold_h(X[o][.][t])[p] (A = Sh[h], B = folded X)
//
// The first pass of a batch may generate its input instead of reading it:
// the stage load vectors are evaluated tile by tile from the per-axis
// quadrature tables inside the A-operand loader, so the nodal load fields
// never travel through HBM.
//
// Block: 256 threads = 4 waves in 2 x 2, block tile BM x BN, wave tile
// (BM/2) x (BN/2), k-step KB = 16, LDS double-buffered with register
// prefetch (one barrier per k-step).  MFMA f64 16x16x4 lane layout: lane l
// supplies A[l%16][l/16] and B[l/16][l%16] and receives C[l/16 + 4r][l%16].
#include <algorithm>

#include "pe_internal.h"

namespace pe {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int KB = 16;
constexpr int NT = 256;
constexpr int GEN_MAX_TERMS = 32;

template <int BM, int BN>
struct Cfg {
  static constexpr int TM = BM / 32;           // MFMA tiles per wave along M
  static constexpr int TN = BN / 32;           // ... along N
  static constexpr int B_PER = KB * BN / NT;   // B elements per thread per k-step
  static constexpr int TPR = NT / BM;          // threads per A row
  static constexpr int CPT = KB / TPR;         // A columns per thread
};

template <int BM, int BN>
struct Smem {
  double A[2][KB][BM + 1];   // k-major A tiles
  double B[2][KB][BN + 1];   // k-major B tiles
};

template <int BM, int BN>
__device__ inline void mma_stage(const double (&As)[KB][BM + 1], const double (&Bs)[KB][BN + 1],
                                 d4 (&acc)[BM / 32][BN / 32], int wm, int wn, int lr, int lk) {
  constexpr int TM = BM / 32, TN = BN / 32;
#pragma unroll
  for (int kk = 0; kk < KB; kk += 4) {
    double a[TM], b[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) a[i] = As[kk + lk][wm * (BM / 2) + i * 16 + lr];
#pragma unroll
    for (int j = 0; j < TN; ++j) b[j] = Bs[kk + lk][wn * (BN / 2) + j * 16 + lr];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
  }
}

// Tile layout of the two-level last pass for NTH threads: 2 x NW/2 waves,
// each (BM/2) x (BN/(NW/2)) outputs of both parities.
template <int BM, int BN, int NTH>
struct Cfg2 {
  static constexpr int NW = NTH / 64;
  static constexpr int WN = NW / 2;
  static constexpr int TM = BM / 2 / 16;       // MFMA tiles per wave along M
  static constexpr int TN = BN / WN / 16;      // ... along N
  static constexpr int B_PER = KB * BN / NTH;  // B elements per thread per k-step
  static constexpr int TPR = NTH / BM;         // threads per A row
  static constexpr int CPT = KB / TPR;         // A columns per thread
};

template <int TM, int TN, int LDA, int LDB>
__device__ inline void mma_tile(const double (&As)[KB][LDA], const double (&Bs)[KB][LDB],
                                d4 (&acc)[TM][TN], int mb, int nb, int lr, int lk) {
#pragma unroll
  for (int kk = 0; kk < KB; kk += 4) {
    double av[TM], bv[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) av[i] = As[kk + lk][mb + i * 16 + lr];
#pragma unroll
    for (int j = 0; j < TN; ++j) bv[j] = Bs[kk + lk][nb + j * 16 + lr];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
  }
}

// Even/odd fold of a nodal line at folded index p, split into the two raw
// loads (issued early, in-bounds clamped indices, no dependent arithmetic)
// and the combination (done later, when the k-step is written to LDS).
struct FoldIdx {
  int pa, pb;        // clamped node indices of x_p and its mirror x_{n-1-p}
  bool has_a, has_b;
};

__device__ inline FoldIdx fold_idx(int n, int H, int h, int p) {
  FoldIdx f;
  f.pa = p < n ? p : n - 1;
  f.pb = n - 1 - p > 0 ? n - 1 - p : 0;
  f.has_a = p < H || (h == 0 && p == H && (n & 1));
  f.has_b = p < H;
  return f;
}

__device__ inline double fold_val(double a, double b, int h, bool has_a, bool has_b) {
  const double av = has_a ? a : 0.0;
  const double bv = has_b ? (h == 0 ? b : -b) : 0.0;
  return av + bv;
}

struct LastArgs {
  const double *X;     // [R][np] nodal input (unused when generating)
  double *Y;           // [R][np] output
  int64_t R;
  int np, n, H, Kh;
  const double *ShT;   // [2][Kh][Kh]
  const double *L3;    // third-level B operands (generating pass), or null
  int tiles_m, tiles_n;
  // generation (GEN kernels)
  int d;               // dimension
  int64_t rows_per_field;
  int np0, np1;
  GenSrc gen;
};

// ---------------------------------------------------------------- LAST pass
// GM = 0: read nodal input; GM > 0: generate it from at most GM forcing terms
// (factors of the unused terms are zero).
template <int BM, int BN, int GM>
__global__ __launch_bounds__(NT) void k_pass_last(LastArgs a) {
  constexpr bool GEN = GM > 0;
  using C = Cfg<BM, BN>;
  __shared__ Smem<BM, BN> sm;

  int64_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const int tn = int(bid % a.tiles_n);
  bid /= a.tiles_n;
  const int h = int(bid % 2);
  const int64_t tm = bid / 2;
  const int64_t m0 = tm * BM;
  const int n0 = tn * BN;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1, lr = lane & 15, lk = lane >> 4;

  // thread -> A row ra, columns ca0 .. ca0 + CPT - 1 of each k-step
  const int ra = t / C::TPR;
  const int ca0 = (t % C::TPR) * C::CPT;
  const int64_t grow = m0 + ra;
  const bool row_ok = grow < a.R;

  // GEN: the load tile of a k-step is the product rf[BM x GM] * cf[GM x KB]
  // of the row factors rf[r][m] = coef[f][m] * prod_{a<d-1} C_a[m][j_a] and
  // the folded last-axis table cf (kept in LDS), computed with 16x16x4
  // MFMAs.  Each lane holds its MFMA A-operands rf[row][term] in registers.
  constexpr int RW = BM / 4;                 // rows generated per wave
  constexpr int RT = RW / 16 > 0 ? RW / 16 : 1;
  constexpr int GK = GM > 0 ? GM / 4 : 1;    // MFMA k-steps over the terms
  double rfa[RT][GK];
  if constexpr (GEN) {
    const int M = a.gen.M;
    const double *C0 = a.d >= 2 ? a.gen.C0 : nullptr;
    const double *C1 = a.d == 3 ? a.gen.C1 : nullptr;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int64_t gr0 = m0 + wave * RW + rt * 16 + lr;
      const bool ok = gr0 < a.R;
      const int64_t gr = ok ? gr0 : a.R - 1;
      const int64_t f = gr / a.rows_per_field;
      const int64_t rem = gr - f * a.rows_per_field;
      int j0 = 0, j1 = 0;
      if (a.d == 2) j0 = int(rem);
      if (a.d == 3) {
        j0 = int(rem / a.np1);
        j1 = int(rem - int64_t(j0) * a.np1);
      }
#pragma unroll
      for (int kk = 0; kk < GK; ++kk) {
        const int m = lk + 4 * kk;
        const int mm = m < M ? m : M - 1;
        double v = a.gen.coef[f * M + mm];
        if (C0) v *= C0[int64_t(mm) * a.np0 + j0];
        if (C1) v *= C1[int64_t(mm) * a.np1 + j1];
        rfa[rt][kk] = (m < M && ok) ? v : 0.0;
      }
    }
  }
  // GEN: the folded last-axis table of this half, [M][Kh], read through the
  // cache (a copy in LDS would cost the second block per CU)
  const double *cf_half = GEN ? a.gen.Cf + int64_t(h) * a.gen.M * a.Kh : nullptr;

  // prefetch registers: raw loads only; the arithmetic happens in store()
  double ra_a[GEN ? 1 : C::CPT], ra_b[GEN ? 1 : C::CPT], rb[C::B_PER];
  const double *xrow = GEN ? nullptr : a.X + (row_ok ? grow : a.R - 1) * a.np;
  auto load = [&](int k0) {
    if constexpr (!GEN) {
#pragma unroll
      for (int c = 0; c < C::CPT; ++c) {
        FoldIdx fi = fold_idx(a.n, a.H, h, k0 + ca0 + c);
        ra_a[c] = xrow[fi.pa];
        ra_b[c] = xrow[fi.pb];
      }
    }
#pragma unroll
    for (int q = 0; q < C::B_PER; ++q) {
      int e = t + q * NT;
      int k = e / BN, nl = e % BN;
      int col = n0 + nl;
      rb[q] = a.ShT[(int64_t(h) * a.Kh + k0 + k) * a.Kh + (col < a.Kh ? col : a.Kh - 1)];
    }
  };
  auto store = [&](int buf, int k0) {
    if constexpr (GEN) {
      const int Mm1 = a.gen.M - 1;
      double cfb[GK];
#pragma unroll
      for (int kk = 0; kk < GK; ++kk) {
        const int term = lk + 4 * kk;
        cfb[kk] = cf_half[(term < Mm1 ? term : Mm1) * a.Kh + k0 + lr];
      }
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        d4 gacc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < GK; ++kk)
          gacc = __builtin_amdgcn_mfma_f64_16x16x4f64(rfa[rt][kk], cfb[kk], gacc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) sm.A[buf][lr][wave * RW + rt * 16 + lk + 4 * r] = gacc[r];
      }
    } else {
#pragma unroll
      for (int c = 0; c < C::CPT; ++c) {
        FoldIdx fi = fold_idx(a.n, a.H, h, k0 + ca0 + c);
        sm.A[buf][ca0 + c][ra] = row_ok ? fold_val(ra_a[c], ra_b[c], h, fi.has_a, fi.has_b) : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < C::B_PER; ++q) {
      int e = t + q * NT;
      int col = n0 + e % BN;
      sm.B[buf][e / BN][e % BN] = col < a.Kh ? rb[q] : 0.0;
    }
  };

  d4 acc[C::TM][C::TN];
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int nk = a.Kh / KB;
  load(0);
  store(0, 0);
  __syncthreads();
  int buf = 0;
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load((kt + 1) * KB);
    mma_stage<BM, BN>(sm.A[buf], sm.B[buf], acc, wm, wn, lr, lk);
    if (kt + 1 < nk) store(buf ^ 1, (kt + 1) * KB);
    __syncthreads();
    buf ^= 1;
  }

#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      int col = n0 + wn * (BN / 2) + j * 16 + lr;
      if (col >= a.Kh) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int64_t row = m0 + wm * (BM / 2) + i * 16 + lk + 4 * r;
        if (row < a.R) a.Y[row * a.np + h * a.Kh + col] = acc[i][j][r];
      }
    }
}

// ----------------------------------------------------------------- MID pass
struct MidArgs {
  const double *X;     // [O][np][I]
  double *Y;           // [O][np][I]
  int64_t O, I;
  int np, n, H, Kh;
  const double *Sh;    // [2][Kh][Kh]
  int tiles_m, tiles_n;
};

template <int BM, int BN>
__global__ __launch_bounds__(NT) void k_pass_mid(MidArgs a) {
  using C = Cfg<BM, BN>;
  __shared__ Smem<BM, BN> sm;

  int64_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const int tn = int(bid % a.tiles_n);
  bid /= a.tiles_n;
  const int tm = int(bid % a.tiles_m);
  bid /= a.tiles_m;
  const int h = int(bid % 2);
  const int64_t o = bid / 2;
  const int m0 = tm * BM;
  const int64_t n0 = int64_t(tn) * BN;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1, lr = lane & 15, lk = lane >> 4;
  const double *X = a.X + o * a.np * a.I;
  const double *S = a.Sh + int64_t(h) * a.Kh * a.Kh;

  const int ra = t / C::TPR;
  const int ca0 = (t % C::TPR) * C::CPT;

  const bool arow_ok = m0 + ra < a.Kh;
  const double *Srow = S + int64_t(arow_ok ? m0 + ra : a.Kh - 1) * a.Kh;

  // prefetch registers: raw loads only; the fold happens in store()
  double pa[C::CPT], rxa[C::B_PER], rxb[C::B_PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int c = 0; c < C::CPT; ++c) pa[c] = Srow[k0 + ca0 + c];
#pragma unroll
    for (int q = 0; q < C::B_PER; ++q) {
      int e = t + q * NT;
      int k = e / BN, nl = e % BN;
      int64_t col = n0 + nl;
      const double *x = X + (col < a.I ? col : a.I - 1);
      FoldIdx fi = fold_idx(a.n, a.H, h, k0 + k);
      rxa[q] = x[int64_t(fi.pa) * a.I];
      rxb[q] = x[int64_t(fi.pb) * a.I];
    }
  };
  auto store = [&](int buf, int k0) {
#pragma unroll
    for (int c = 0; c < C::CPT; ++c) sm.A[buf][ca0 + c][ra] = arow_ok ? pa[c] : 0.0;
#pragma unroll
    for (int q = 0; q < C::B_PER; ++q) {
      int e = t + q * NT;
      int k = e / BN, nl = e % BN;
      FoldIdx fi = fold_idx(a.n, a.H, h, k0 + k);
      double v = fold_val(rxa[q], rxb[q], h, fi.has_a, fi.has_b);
      sm.B[buf][k][nl] = (n0 + nl < a.I) ? v : 0.0;
    }
  };

  d4 acc[C::TM][C::TN];
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int nk = a.Kh / KB;
  load(0);
  store(0, 0);
  __syncthreads();
  int buf = 0;
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load((kt + 1) * KB);
    mma_stage<BM, BN>(sm.A[buf], sm.B[buf], acc, wm, wn, lr, lk);
    if (kt + 1 < nk) store(buf ^ 1, (kt + 1) * KB);
    __syncthreads();
    buf ^= 1;
  }

  double *Y = a.Y + o * a.np * a.I;
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      int64_t col = n0 + wn * (BN / 2) + j * 16 + lr;
      if (col >= a.I) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = m0 + wm * (BM / 2) + i * 16 + lk + 4 * r;
        if (row < a.Kh) Y[int64_t(h * a.Kh + row) * a.I + col] = acc[i][j][r];
      }
    }
}

// ------------------------------------------------- MID pass, second level
// For n = 2 Kh - 1 (M = Kh, Q = M / 2) each half of the fold splits again:
// with u = fold_h(x), the output pair (i, i') of half h relates by
//     S[k(i')][j] = (-1)^{j+1} S[k(i)][j],   i' = M-1-i (h = 0), M-2-i (h = 1),
// so A_i = sum_{j odd} S[k(i)][j] u_j and B_i = sum_{j even} S[k(i)][j] u_j
// give y_i = A_i + B_i and y_i' = A_i - B_i: two Q x Q products per half
// instead of one M x M, half the multiply-adds.  Row i = Q-1 of half 1 is
// its own partner (its B vanishes); position M-1 of half 1 is a pad (zero).
struct Mid2Args {
  const double *X;     // [O][np][I]
  double *Y;           // [O][np][I]
  int64_t O, I;
  int np, n, H, Kh, Q;
  const double *Sq;    // [2][2][Q][Q]
  int tiles_m, tiles_n;
};

template <int BM, int BN>
struct Smem2 {
  double A[2][2][KB][BM + 1];   // [buffer][parity g][k][row]
  double B[2][2][KB][BN + 1];
};

template <int BM, int BN>
__global__ __launch_bounds__(NT) void k_pass_mid2(Mid2Args a) {
  using C = Cfg<BM, BN>;
  __shared__ Smem2<BM, BN> sm;

  int64_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const int tn = int(bid % a.tiles_n);
  bid /= a.tiles_n;
  const int tm = int(bid % a.tiles_m);
  bid /= a.tiles_m;
  const int h = int(bid % 2);
  const int64_t o = bid / 2;
  const int m0 = tm * BM;
  const int64_t n0 = int64_t(tn) * BN;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1, lr = lane & 15, lk = lane >> 4;
  const double *X = a.X + o * a.np * a.I;

  const int ra = t / C::TPR;
  const int ca0 = (t % C::TPR) * C::CPT;
  const bool arow_ok = m0 + ra < a.Q;
  const int arow = arow_ok ? m0 + ra : a.Q - 1;
  const double *S0 = a.Sq + (int64_t(2 * h) * a.Q + arow) * a.Q;
  const double *S1 = a.Sq + (int64_t(2 * h + 1) * a.Q + arow) * a.Q;

  // raw prefetch (input rows p = 2 jj + g and their mirrors n-1-p; p <= H)
  double pa0[C::CPT], pa1[C::CPT], xa[2][C::B_PER], xb[2][C::B_PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int c = 0; c < C::CPT; ++c) {
      pa0[c] = S0[k0 + ca0 + c];
      pa1[c] = S1[k0 + ca0 + c];
    }
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int q = 0; q < C::B_PER; ++q) {
        const int e = t + q * NT;
        const int k = e / BN, nl = e % BN;
        const int64_t col = n0 + nl;
        const double *x = X + (col < a.I ? col : a.I - 1);
        const int p = 2 * (k0 + k) + g;
        xa[g][q] = x[int64_t(p) * a.I];
        xb[g][q] = x[int64_t(a.n - 1 - p) * a.I];
      }
  };
  auto store = [&](int buf, int k0) {
#pragma unroll
    for (int c = 0; c < C::CPT; ++c) {
      sm.A[buf][0][ca0 + c][ra] = arow_ok ? pa0[c] : 0.0;
      sm.A[buf][1][ca0 + c][ra] = arow_ok ? pa1[c] : 0.0;
    }
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int q = 0; q < C::B_PER; ++q) {
        const int e = t + q * NT;
        const int k = e / BN, nl = e % BN;
        const int p = 2 * (k0 + k) + g;
        double v;
        if (p < a.H)
          v = h == 0 ? xa[g][q] + xb[g][q] : xa[g][q] - xb[g][q];
        else   // p == H: the middle node counts once in half 0, not at all in half 1
          v = h == 0 ? xa[g][q] : 0.0;
        sm.B[buf][g][k][nl] = (n0 + nl < a.I) ? v : 0.0;
      }
  };

  d4 acc0[C::TM][C::TN], acc1[C::TM][C::TN];
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) acc0[i][j] = acc1[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int nk = a.Q / KB;
  load(0);
  store(0, 0);
  __syncthreads();
  int buf = 0;
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load((kt + 1) * KB);
    mma_stage<BM, BN>(sm.A[buf][0], sm.B[buf][0], acc0, wm, wn, lr, lk);
    mma_stage<BM, BN>(sm.A[buf][1], sm.B[buf][1], acc1, wm, wn, lr, lk);
    if (kt + 1 < nk) store(buf ^ 1, (kt + 1) * KB);
    __syncthreads();
    buf ^= 1;
  }

  double *Y = a.Y + o * a.np * a.I;
  const int M = a.Kh;
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      const int64_t col = n0 + wn * (BN / 2) + j * 16 + lr;
      if (col >= a.I) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * (BM / 2) + i * 16 + lk + 4 * r;
        if (row >= a.Q) continue;
        const double A = acc0[i][j][r], B = acc1[i][j][r];
        // streaming stores: the next pass reads every field once
        __builtin_nontemporal_store(A + B, &Y[int64_t(h * a.Kh + row) * a.I + col]);
        int pos2;
        double v2;
        if (h == 0) {
          pos2 = M - 1 - row;
          v2 = A - B;
        } else if (row < a.Q - 1) {
          pos2 = M - 2 - row;
          v2 = A - B;
        } else {
          pos2 = M - 1;   // pad position of half 1
          v2 = 0.0;
        }
        __builtin_nontemporal_store(v2, &Y[int64_t(h * a.Kh + pos2) * a.I + col]);
      }
    }
}

// ------------------------------------------------ LAST pass, second level
// Same split as the MID pass above, on the contiguous axis: for half h and
// parity g the folded input row is sampled at p = 2 jj + g (A operand,
// rows r x jj, or generated from the quadrature tables at those p), the B
// operand is SqT[h][g] (jj x i); the row of outputs gets y_i = C_0 + C_1
// and y_i' = C_0 - C_1.
// NTH = 512 (the generating pass): 8 waves of (BM/2) x (BN/4) outputs, two
// blocks per CU (the LDS of two), so four waves share each SIMD; a wave
// generates one 16-row tile of one parity.  NTH = 256: 4 waves of
// (BM/2) x (BN/2), a wave generates one row tile of both parities.
// RTB > 1 (generating pass): a block walks RTB consecutive 64-row tiles,
// loading the next tile's row factors while the current one finishes, so
// the set-up latency of a short block (row factors, first k-tile) is paid
// once per RTB tiles.
template <int BM, int BN, int GM, int NTH, int RTB>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(NTH == 512 ? 4 : 1)))
void k_pass_last2(LastArgs a) {
  constexpr bool GEN = GM > 0;
  using C = Cfg2<BM, BN, NTH>;
  static_assert(BM == 64 && (NTH == 256 || NTH == 512), "tile layout");
  static_assert(RTB == 1 || GEN, "several row tiles per block only when generating");
  __shared__ Smem2<BM, BN> sm;

  const int Q = a.Kh / 2;
  int64_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const int tn = int(bid % a.tiles_n);
  bid /= a.tiles_n;
  const int h = int(bid % 2);
  const int64_t tmb = bid / 2;   // group of RTB row tiles
  const int n0 = tn * BN;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave / C::WN, wn = wave % C::WN, lr = lane & 15, lk = lane >> 4;

  const int ra = t / C::TPR;
  const int ca0 = (t % C::TPR) * C::CPT;

  // generation: the wave's 16-row tile and its parities [g0, g0 + GPW)
  constexpr int RTILES = BM / 16;
  constexpr int GPW = 2 * RTILES / C::NW;
  const int grt = wave % RTILES, g0 = GPW == 2 ? 0 : wave / RTILES;
  constexpr int GK = GM > 0 ? GM / 4 : 1;    // MFMA k-steps over the terms
  // row factors of the wave's generated rows of the tile starting at row m0
  auto row_factors = [&](int64_t m0, double (&rf)[GK]) {
    const int M = a.gen.M;
    const double *C0 = a.d >= 2 ? a.gen.C0 : nullptr;
    const double *C1 = a.d == 3 ? a.gen.C1 : nullptr;
    const int64_t gr0 = m0 + grt * 16 + lr;
    const bool ok = gr0 < a.R;
    const int64_t gr = ok ? gr0 : a.R - 1;
    const int64_t f = gr / a.rows_per_field;
    const int64_t rem = gr - f * a.rows_per_field;
    int j0 = 0, j1 = 0;
    if (a.d == 2) j0 = int(rem);
    if (a.d == 3) {
      j0 = int(rem / a.np1);
      j1 = int(rem - int64_t(j0) * a.np1);
    }
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      const int m = lk + 4 * kk;
      const int mm = m < M ? m : M - 1;
      double v = a.gen.coef[f * M + mm];
      if (C0) v *= C0[int64_t(mm) * a.np0 + j0];
      if (C1) v *= C1[int64_t(mm) * a.np1 + j1];
      rf[kk] = (m < M && ok) ? v : 0.0;
    }
  };
  // GEN: the folded last-axis table of this half, [M][Kh], read through the
  // cache (a copy in LDS would leave room for one block per CU only)
  const double *cf_half = GEN ? a.gen.Cf + int64_t(h) * a.gen.M * a.Kh : nullptr;
  const double *SqT = a.ShT;   // [2][2][Q][Q] when set up for this pass
  const int nk = Q / KB;
  const int mb = wm * (BM / 2), nb = wn * (BN / C::WN);
  const int M = a.Kh;

  double rfa[GK], rfn[GK];
  if constexpr (GEN) row_factors(tmb * RTB * BM, rfa);
  for (int rtb = 0; rtb < RTB; ++rtb) {
    const int64_t tm = tmb * RTB + rtb;
    if (tm >= a.tiles_m) break;
    const int64_t m0 = tm * BM;
    const int64_t grow = m0 + ra;
    const bool row_ok = grow < a.R;
    if (rtb > 0) {
#pragma unroll
      for (int kk = 0; kk < GK; ++kk) rfa[kk] = rfn[kk];
      __syncthreads();   // the last products of the previous tile read the LDS tiles
    }

    // raw prefetch: input rows at p = 2 jj + g and their mirrors (p <= H)
    double ra_a[GEN ? 1 : 2][GEN ? 1 : C::CPT], ra_b[GEN ? 1 : 2][GEN ? 1 : C::CPT];
    double rb[2][C::B_PER];
    const double *xrow = GEN ? nullptr : a.X + (row_ok ? grow : a.R - 1) * a.np;
    auto load = [&](int k0) {
      if constexpr (!GEN) {
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
          for (int c = 0; c < C::CPT; ++c) {
            const int p = 2 * (k0 + ca0 + c) + g;
            ra_a[g][c] = xrow[p];
            ra_b[g][c] = xrow[a.n - 1 - p];
          }
      }
#pragma unroll
      for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int q = 0; q < C::B_PER; ++q) {
          const int e = t + q * NTH;
          const int k = e / BN, nl = e % BN;
          const int col = n0 + nl;
          rb[g][q] = SqT[(int64_t(2 * h + g) * Q + k0 + k) * Q + (col < Q ? col : Q - 1)];
        }
    };
    auto store = [&](int buf, int k0) {
      if constexpr (GEN) {
        const int Mm1 = a.gen.M - 1;
#pragma unroll
        for (int gg = 0; gg < GPW; ++gg) {
          const int g = g0 + gg;
          double cfb[GK];
#pragma unroll
          for (int kk = 0; kk < GK; ++kk) {
            const int term = lk + 4 * kk;
            cfb[kk] = cf_half[(term < Mm1 ? term : Mm1) * a.Kh + 2 * (k0 + lr) + g];
          }
          d4 gacc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int kk = 0; kk < GK; ++kk)
            gacc = __builtin_amdgcn_mfma_f64_16x16x4f64(rfa[kk], cfb[kk], gacc, 0, 0, 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) sm.A[buf][g][lr][grt * 16 + lk + 4 * r] = gacc[r];
        }
      } else {
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
          for (int c = 0; c < C::CPT; ++c) {
            const int p = 2 * (k0 + ca0 + c) + g;
            double v;
            if (p < a.H)
              v = h == 0 ? ra_a[g][c] + ra_b[g][c] : ra_a[g][c] - ra_b[g][c];
            else
              v = h == 0 ? ra_a[g][c] : 0.0;
            sm.A[buf][g][ca0 + c][ra] = row_ok ? v : 0.0;
          }
      }
#pragma unroll
      for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int q = 0; q < C::B_PER; ++q) {
          const int e = t + q * NTH;
          const int col = n0 + e % BN;
          sm.B[buf][g][e / BN][e % BN] = col < Q ? rb[g][q] : 0.0;
        }
    };

    d4 acc0[C::TM][C::TN], acc1[C::TM][C::TN];
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int j = 0; j < C::TN; ++j) acc0[i][j] = acc1[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    // the last k-tile is peeled off the loop: a loop body without branches
    // keeps the accumulators in the matrix-core registers across iterations
    // (with the prefetch made conditional the compiler copied them out to
    // plain registers and back around every k-tile, which also made each
    // k-tile wait for all of its products)
    load(0);
    store(0, 0);
    __syncthreads();
    int buf = 0;
    for (int kt = 0; kt + 1 < nk; ++kt) {
      load((kt + 1) * KB);
      mma_tile<C::TM, C::TN, BM + 1, BN + 1>(sm.A[buf][0], sm.B[buf][0], acc0, mb, nb, lr, lk);
      mma_tile<C::TM, C::TN, BM + 1, BN + 1>(sm.A[buf][1], sm.B[buf][1], acc1, mb, nb, lr, lk);
      store(buf ^ 1, (kt + 1) * KB);
      __syncthreads();
      buf ^= 1;
    }
    // the next tile's row factors (their loads land during the last
    // products and the stores)
    if constexpr (GEN)
      if (rtb + 1 < RTB && tm + 1 < a.tiles_m) row_factors(m0 + BM, rfn);
    mma_tile<C::TM, C::TN, BM + 1, BN + 1>(sm.A[buf][0], sm.B[buf][0], acc0, mb, nb, lr, lk);
    mma_tile<C::TM, C::TN, BM + 1, BN + 1>(sm.A[buf][1], sm.B[buf][1], acc1, mb, nb, lr, lk);

#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        const int col = n0 + nb + j * 16 + lr;
        if (col >= Q) continue;
        int pos2;
        bool diff;
        if (h == 0) {
          pos2 = M - 1 - col;
          diff = true;
        } else if (col < Q - 1) {
          pos2 = M - 2 - col;
          diff = true;
        } else {
          pos2 = M - 1;   // pad position of half 1
          diff = false;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = m0 + mb + i * 16 + lk + 4 * r;
          if (row >= a.R) continue;
          const double A = acc0[i][j][r], B = acc1[i][j][r];
          __builtin_nontemporal_store(A + B, &a.Y[row * a.np + h * a.Kh + col]);
          __builtin_nontemporal_store(diff ? A - B : 0.0, &a.Y[row * a.np + h * a.Kh + pos2]);
        }
      }
  }
}

// ------------------------------ generating LAST pass, three fold levels
// For two-level axes with Q = Kh/2 in {32, 64} the generating pass splits
// three of its four Q x Q quarter products once more (the fourth, a DST-IV,
// has no sign symmetry):
//   h = 0, g = 1 (a DST-III): rows i and Q-1-i differ by the sign (-1)^jj,
//     so E_i (even jj) and O_i (odd jj) give B_i = E_i + O_i and
//     B_{Q-1-i} = E_i - O_i for i < Q/2;
//   h = 1, g = 0 (a DST-II): inputs jj and Q-1-jj enter row i with the sign
//     (-1)^i, so even rows take their sums and odd rows their differences;
//   h = 1, g = 1 (a DST-I of size Q-1): inputs jj and Q-2-jj likewise (the
//     middle input jj = Q/2-1 counts once in the sums; the last input is
//     multiplied by zeros throughout).
// The matrix-core work drops from 4 Q^2 to 5 Q^2 / 2 multiply-adds per row.
// Every input-side combination is linear in the quadrature table, so it is
// applied to the table (the K-column table cfl, built per block) rather than
// to data; the generated inputs come out of the transposed quadrature MFMA,
// C[k][r] = sum_m cfl[m][k] rf[r][m], already in the A-fragment layout of the
// transform MFMAs (lane l: k = l/16 + 4 r', r = l%16).  A wave owns a 16-row
// tile and every output of its half and walks the block's row tiles; the
// block keeps its half's reduced B operands (3 Q^2 / 2 doubles) in LDS, each
// [K][N] matrix with N >= 32 stored with its two 16-lane row groups in
// opposite bank halves (column n of row k at n ^ 16 (k & 1)).
// 16-row tiles per block: up to LG_TILES_MAX (the block's LDS staging is
// amortised over its tiles), fewer for small launches so that about 1024
// blocks fill the chip
constexpr int LG_TILES_MAX = 128;
// 8 waves per block: two blocks (the LDS of two) per compute unit then keep
// four waves on each SIMD to hide the latency of the chained products
constexpr int L3_NT = 512;
constexpr int L3_NW = L3_NT / 64;
static int64_t lg_tiles(int64_t tiles) {
  return std::max<int64_t>(4, std::min<int64_t>(LG_TILES_MAX, tiles / 512));
}

// x of lane (i - 1) mod 16 within each 16-lane row (DPP row_ror:1, on the
// two 32-bit halves)
__device__ inline double row_rotate1(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const int lo = __builtin_amdgcn_update_dpp(0, int(uint32_t(u)), 0x121, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(uint32_t(u >> 32)), 0x121, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
}

// One reduced product over a row tile: KCN chunks of 16 generated inputs
// (K columns from chunk KC0 of cfl) times the [K][N] operand at sb + Boff,
// accumulated into tiles [ACC0, ACC0 + N/16).
template <int Q, int GK, int KC0, int KCN, int N, int ACC0, int NACC>
__device__ inline void l3_product(const double *sb, int Boff, const double (*cfl)[2 * Q],
                                  const double (&rf)[GK], d4 (&acc)[NACC], int lr, int lk) {
  constexpr int NTL = N / 16;
  constexpr int SW = N >= 32 ? 16 : 0;
#pragma unroll 1
  for (int cc = 0; cc < KCN; ++cc) {
    d4 gen = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < GK; ++kk)
      gen = __builtin_amdgcn_mfma_f64_16x16x4f64(cfl[4 * kk + lk][16 * (KC0 + cc) + lr], rf[kk],
                                                 gen, 0, 0, 0);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int k = 16 * cc + 4 * rr + lk;
      const int sw = (k & 1) * SW;
#pragma unroll
      for (int j = 0; j < NTL; ++j) {
        const double b = sb[Boff + k * N + ((16 * j + lr) ^ sw)];
        acc[ACC0 + j] = __builtin_amdgcn_mfma_f64_16x16x4f64(gen[rr], b, acc[ACC0 + j], 0, 0, 0);
      }
    }
  }
}

template <int Q, int GK>
__global__ __launch_bounds__(L3_NT) __attribute__((amdgpu_waves_per_eu(GK <= 4 ? 4 : 2)))
void k_last3_gen(LastArgs a, int64_t tiles, int64_t per_block) {
  constexpr int Q2 = Q / 2;
  constexpr int NACC = Q / 8;          // accumulator tiles of a row tile
  constexpr int PER = 3 * Q * Q / 2;   // B operands per half
  __shared__ __attribute__((aligned(16))) double sb[PER];
  __shared__ double cfl[4 * GK][2 * Q];

  const int h = int(blockIdx.x & 1);
  const int64_t tile0 = int64_t(blockIdx.x >> 1) * per_block;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int M = a.gen.M;

  // this half's reduced B operands -> LDS
  {
    const double *src = a.L3 + int64_t(h) * PER;
    const int nb = h == 0 ? PER : Q * Q;
    for (int e = 2 * t; e < nb; e += 2 * L3_NT) {
      int base, N, r;
      if (h == 0 && e < Q * Q) {
        base = 0;
        N = Q;
        r = e;
      } else {
        const int e2 = h == 0 ? e - Q * Q : e;
        base = (h == 0 ? Q * Q : 0) + (e2 / (Q2 * Q2)) * Q2 * Q2;
        N = Q2;
        r = e2 % (Q2 * Q2);
      }
      const int k = r / N, n = r - k * N;   // n even: the pair (n, n+1) moves together
      const int sw = N >= 32 ? (k & 1) * 16 : 0;
      *reinterpret_cast<double2 *>(&sb[base + k * N + (n ^ sw)]) =
          *reinterpret_cast<const double2 *>(src + e);
    }
  }
  // K-column table of this half (input-side folds applied to the table)
  {
    const double *cf = a.gen.Cf + int64_t(h) * M * a.Kh;
    for (int e = t; e < 4 * GK * 2 * Q; e += L3_NT) {
      const int m = e / (2 * Q), kc = e - m * 2 * Q;
      double v = 0.0;
      if (m < M) {
        const double *c = cf + int64_t(m) * a.Kh;
        if (h == 0) {
          if (kc < Q)
            v = c[2 * kc];
          else if (kc < 3 * Q2)
            v = c[2 * (2 * (kc - Q)) + 1];
          else
            v = c[2 * (2 * (kc - 3 * Q2) + 1) + 1];
        } else if (kc < Q) {
          const int jj = kc < Q2 ? kc : kc - Q2;
          v = kc < Q2 ? c[2 * jj] + c[2 * (Q - 1 - jj)] : c[2 * jj] - c[2 * (Q - 1 - jj)];
        } else {
          const int jj = kc < 3 * Q2 ? kc - Q : kc - 3 * Q2;
          if (jj < Q2 - 1)
            v = kc < 3 * Q2 ? c[2 * jj + 1] + c[2 * (Q - 2 - jj) + 1]
                            : c[2 * jj + 1] - c[2 * (Q - 2 - jj) + 1];
          else
            v = kc < 3 * Q2 ? c[2 * jj + 1] : 0.0;
        }
      }
      cfl[m][kc] = v;
    }
  }
  __syncthreads();

  const double *C0 = a.d >= 2 ? a.gen.C0 : nullptr;
  const double *C1 = a.d == 3 ? a.gen.C1 : nullptr;
  // row factors rf[r][m] of row r = l%16 of a tile, m = 4 kk + l/16
  auto row_factors = [&](int64_t tile, double (&rf)[GK]) {
    const int64_t gr = tile * 16 + lr;
    const int64_t f = gr / a.rows_per_field;
    const int64_t rem = gr - f * a.rows_per_field;
    int j0 = 0, j1 = 0;
    if (a.d == 2) j0 = int(rem);
    if (a.d == 3) {
      j0 = int(rem / a.np1);
      j1 = int(rem - int64_t(j0) * a.np1);
    }
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      const int m = 4 * kk + lk;
      const int mm = m < M ? m : M - 1;
      double v = a.gen.coef[f * M + mm];
      if (C0) v *= C0[int64_t(mm) * a.np0 + j0];
      if (C1) v *= C1[int64_t(mm) * a.np1 + j1];
      rf[kk] = m < M ? v : 0.0;
    }
  };

  const int Mh = a.Kh;
  const int64_t tend = std::min<int64_t>(tile0 + per_block, tiles);
  int64_t tile = tile0 + wave;
  double rf[GK], rfn[GK];
  if (tile < tend) row_factors(tile, rf);
  // the next tile's row factors are loaded after this tile's products:
  // their use waits for every older memory operation, and by then the
  // previous tile's output stores have drained (loaded before the products,
  // each tile waited for the stores just issued)
  for (; tile < tend; tile += L3_NW) {
    d4 acc[NACC];
#pragma unroll
    for (int j = 0; j < NACC; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
    if (h == 0) {
      l3_product<Q, GK, 0, Q / 16, Q, 0, NACC>(sb, 0, cfl, rf, acc, lr, lk);
      l3_product<Q, GK, Q / 16, Q / 32, Q2, Q / 16, NACC>(sb, Q * Q, cfl, rf, acc, lr, lk);
      l3_product<Q, GK, 3 * Q / 32, Q / 32, Q2, 3 * Q / 32, NACC>(sb, Q * Q + Q2 * Q2, cfl, rf,
                                                                   acc, lr, lk);
      if (tile + L3_NW < tend) row_factors(tile + L3_NW, rfn);
      // outputs: A from P00 (upper slots reversed), B from E +- O
#pragma unroll
      for (int tt = 0; tt < Q / 32; ++tt) {
        const int ilo = 16 * tt + lr, ihi = Q - 1 - ilo;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = tile * 16 + lk + 4 * r;
          double *y = a.Y + row * a.np;
          const double Alo = acc[tt][r], Ahi = acc[Q / 32 + tt][r];
          const double E = acc[Q / 16 + tt][r], O = acc[3 * Q / 32 + tt][r];
          const double Blo = E + O, Bhi = E - O;
          __builtin_nontemporal_store(Alo + Blo, &y[ilo]);
          __builtin_nontemporal_store(Alo - Blo, &y[Mh - 1 - ilo]);
          __builtin_nontemporal_store(Ahi + Bhi, &y[ihi]);
          __builtin_nontemporal_store(Ahi - Bhi, &y[Mh - 1 - ihi]);
        }
      }
    } else {
      l3_product<Q, GK, 0, Q / 32, Q2, 0, NACC>(sb, 0, cfl, rf, acc, lr, lk);
      l3_product<Q, GK, Q / 32, Q / 32, Q2, Q / 32, NACC>(sb, Q2 * Q2, cfl, rf, acc, lr, lk);
      l3_product<Q, GK, Q / 16, Q / 32, Q2, Q / 16, NACC>(sb, 2 * Q2 * Q2, cfl, rf, acc, lr, lk);
      l3_product<Q, GK, 3 * Q / 32, Q / 32, Q2, 3 * Q / 32, NACC>(sb, 3 * Q2 * Q2, cfl, rf, acc,
                                                                   lr, lk);
      if (tile + L3_NW < tend) row_factors(tile + L3_NW, rfn);
      // outputs: even rows from the sums, odd rows from the differences.
      // Lane k (= 16 tt + l%16) writes the pair (2k, 2k+1) and the partner
      // pair (M-2-2k, M-1-2k); the second partner is lane k-1's odd one
      // (M-2-(2k-1)), brought over by a rotation within the 16-lane row,
      // with lane 15 of the previous tile (or the pad, 0) for k's first lane.
      double carry[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int tt = 0; tt < Q / 32; ++tt) {
        const int ie = 2 * (16 * tt + lr);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = tile * 16 + lk + 4 * r;
          double *y = a.Y + row * a.np + Mh;
          const double Ae = acc[tt][r], Ao = acc[Q / 32 + tt][r];
          const double Be = acc[Q / 16 + tt][r], Bo = acc[3 * Q / 32 + tt][r];
          const d2 yy = {Ae + Be, Ao + Bo};
          __builtin_nontemporal_store(yy, reinterpret_cast<d2 *>(&y[ie]));
          const double rot = row_rotate1(Ao - Bo);   // lane i gets lane (i - 1) mod 16
          const d2 pp = {Ae - Be, lr == 0 ? carry[r] : rot};
          carry[r] = rot;   // its lane 0 holds this tile's lane 15
          __builtin_nontemporal_store(pp, reinterpret_cast<d2 *>(&y[Mh - 2 - ie]));
        }
      }
    }
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) rf[kk] = rfn[kk];
  }
}

template <int Q, int GM>
static pe_status launch_last3_gen(const LastArgs &a, hipStream_t st) {
  constexpr int GK = (GM + 3) / 4;
  const int64_t tiles = a.R / 16;
  const int64_t per = lg_tiles(tiles);
  const int64_t blocks = 2 * ((tiles + per - 1) / per);
  if (blocks >= (int64_t(1) << 31)) return set_error(PE_E_ARG, "internal: LAST3 grid too large");
  k_last3_gen<Q, GK><<<dim3(unsigned(blocks)), L3_NT, 0, st>>>(a, tiles, per);
  PE_HIP(hipGetLastError());
  return PE_OK;
}

// ------------------------------------------------------------------ dispatch
static int pick(int64_t extent) { return extent >= 128 ? 128 : (extent >= 64 ? 64 : 32); }

constexpr int64_t MAX_BLOCKS = (int64_t(1) << 24) - 1;   // 2^32 work-items per grid dimension

template <int BM, int BN, int GM>
static pe_status launch_last_t(LastArgs a, size_t dyn, hipStream_t st) {
  constexpr bool GEN = GM > 0;
  const int64_t per_row_tile = int64_t(a.tiles_n) * 2;
  // row chunks: whole fields when generating, at most MAX_BLOCKS blocks
  int64_t max_tm = MAX_BLOCKS / per_row_tile;
  if (GEN) {
    int64_t fields_per_chunk = std::max<int64_t>(1, max_tm * BM / a.rows_per_field);
    max_tm = fields_per_chunk * a.rows_per_field / BM;
    if (max_tm < 1 || (fields_per_chunk * a.rows_per_field) % BM != 0)
      max_tm = (a.R + BM - 1) / BM;   // single launch (small batches)
  }
  const int64_t total_tm = a.tiles_m;
  for (int64_t tm0 = 0; tm0 < total_tm; tm0 += max_tm) {
    int64_t ntm = std::min(max_tm, total_tm - tm0);
    if (ntm * per_row_tile > MAX_BLOCKS) return set_error(PE_E_ARG, "internal: LAST grid too large");
    LastArgs b = a;
    int64_t r0 = tm0 * BM;
    b.R = std::min<int64_t>(a.R - r0, ntm * BM);
    b.tiles_m = int(ntm);
    if (!GEN) b.X = a.X + r0 * a.np;
    b.Y = a.Y + r0 * a.np;
    if (GEN) b.gen.coef = a.gen.coef + (r0 / a.rows_per_field) * a.gen.M;
    k_pass_last<BM, BN, GM><<<dim3(unsigned(ntm * per_row_tile)), NT, dyn, st>>>(b);
    PE_HIP(hipGetLastError());
  }
  return PE_OK;
}

template <int GM>
static pe_status launch_last(LastArgs a, hipStream_t st) {
  int bm = a.R >= 128 ? 128 : 64;
  int bn = pick(a.Kh);
  a.tiles_m = int((a.R + bm - 1) / bm);
  a.tiles_n = (a.Kh + bn - 1) / bn;
  const size_t dyn = 0;
#define PE_LAST(BMv, BNv) \
  if (bm == BMv && bn == BNv) return launch_last_t<BMv, BNv, GM>(a, dyn, st);
  PE_LAST(128, 128) PE_LAST(128, 64) PE_LAST(128, 32)
  PE_LAST(64, 128) PE_LAST(64, 64) PE_LAST(64, 32)
#undef PE_LAST
  return set_error(PE_E_ARG, "internal: no LAST tile for %d x %d", bm, bn);
}

template <int BM, int BN>
static pe_status launch_mid_t(MidArgs a, hipStream_t st) {
  const int64_t per_o = int64_t(a.tiles_m) * a.tiles_n * 2;
  const int64_t max_o = std::max<int64_t>(1, MAX_BLOCKS / per_o);
  if (per_o > MAX_BLOCKS) return set_error(PE_E_ARG, "internal: MID grid too large");
  for (int64_t o0 = 0; o0 < a.O; o0 += max_o) {
    MidArgs b = a;
    b.O = std::min(max_o, a.O - o0);
    b.X = a.X + o0 * a.np * a.I;
    b.Y = a.Y + o0 * a.np * a.I;
    k_pass_mid<BM, BN><<<dim3(unsigned(b.O * per_o)), NT, 0, st>>>(b);
    PE_HIP(hipGetLastError());
  }
  return PE_OK;
}

static pe_status launch_mid(MidArgs a, hipStream_t st) {
  int bm = pick(a.Kh);
  int bn = pick(a.I);
  a.tiles_m = (a.Kh + bm - 1) / bm;
  a.tiles_n = int((a.I + bn - 1) / bn);
#define PE_MID(BMv, BNv) \
  if (bm == BMv && bn == BNv) return launch_mid_t<BMv, BNv>(a, st);
  PE_MID(128, 128) PE_MID(128, 64) PE_MID(128, 32)
  PE_MID(64, 128) PE_MID(64, 64) PE_MID(64, 32)
  PE_MID(32, 128) PE_MID(32, 64) PE_MID(32, 32)
#undef PE_MID
  return set_error(PE_E_ARG, "internal: no MID tile for %d x %d", bm, bn);
}

template <int BM, int BN, int GM, int NTH, int RTB>
static pe_status launch_last2_t(LastArgs a, size_t dyn, hipStream_t st) {
  constexpr bool GEN = GM > 0;
  const int64_t per_row_tile = int64_t(a.tiles_n) * 2;
  int64_t max_tm = MAX_BLOCKS / per_row_tile;
  if (GEN) {
    int64_t fields_per_chunk = std::max<int64_t>(1, max_tm * BM / a.rows_per_field);
    max_tm = fields_per_chunk * a.rows_per_field / BM;
    if (max_tm < 1 || (fields_per_chunk * a.rows_per_field) % BM != 0)
      max_tm = (a.R + BM - 1) / BM;   // single launch (small batches)
  }
  const int64_t total_tm = a.tiles_m;
  for (int64_t tm0 = 0; tm0 < total_tm; tm0 += max_tm) {
    int64_t ntm = std::min(max_tm, total_tm - tm0);
    if (ntm * per_row_tile > MAX_BLOCKS) return set_error(PE_E_ARG, "internal: LAST2 grid too large");
    LastArgs b = a;
    int64_t r0 = tm0 * BM;
    b.R = std::min<int64_t>(a.R - r0, ntm * BM);
    b.tiles_m = int(ntm);
    if (!GEN) b.X = a.X + r0 * a.np;
    b.Y = a.Y + r0 * a.np;
    if (GEN) b.gen.coef = a.gen.coef + (r0 / a.rows_per_field) * a.gen.M;
    const int64_t groups = (ntm + RTB - 1) / RTB;
    k_pass_last2<BM, BN, GM, NTH, RTB><<<dim3(unsigned(groups * per_row_tile)), NTH, dyn, st>>>(b);
    PE_HIP(hipGetLastError());
  }
  return PE_OK;
}

// row tiles per block of the generating two-level pass
constexpr int LAST2_RTB = 4;

// a.ShT must point at the axis' SqT blocks
template <int GM>
static pe_status launch_last2(LastArgs a, hipStream_t st) {
  constexpr int BM = 64, BN = 64;
  if constexpr (GM > 0) {
    if (a.L3 && a.R % 16 == 0 && a.Kh == 128) return launch_last3_gen<64, GM>(a, st);
    if (a.L3 && a.R % 16 == 0 && a.Kh == 64) return launch_last3_gen<32, GM>(a, st);
  }
  a.tiles_m = int((a.R + BM - 1) / BM);
  a.tiles_n = (a.Kh / 2 + BN - 1) / BN;
  if constexpr (GM > 0)
    return launch_last2_t<BM, BN, GM, 512, LAST2_RTB>(a, 0, st);
  else
    return launch_last2_t<BM, BN, GM, NT, 1>(a, 0, st);
}

static pe_status launch_mid2(Mid2Args a, hipStream_t st) {
  constexpr int BM = 64, BN = 64;
  a.tiles_m = (a.Q + BM - 1) / BM;
  a.tiles_n = int((a.I + BN - 1) / BN);
  const int64_t per_o = int64_t(a.tiles_m) * a.tiles_n * 2;
  if (per_o > MAX_BLOCKS) return set_error(PE_E_ARG, "internal: MID2 grid too large");
  const int64_t max_o = std::max<int64_t>(1, MAX_BLOCKS / per_o);
  for (int64_t o0 = 0; o0 < a.O; o0 += max_o) {
    Mid2Args b = a;
    b.O = std::min(max_o, a.O - o0);
    b.X = a.X + o0 * a.np * a.I;
    b.Y = a.Y + o0 * a.np * a.I;
    k_pass_mid2<BM, BN><<<dim3(unsigned(b.O * per_o)), NT, 0, st>>>(b);
    PE_HIP(hipGetLastError());
  }
  return PE_OK;
}

bool gen_supported(pe_grid g, int n_terms) {
  if (g->transform == PE_TRANSFORM_FFT) return fft_gen_supported(g, n_terms);
  return n_terms >= 1 && n_terms <= GEN_MAX_TERMS;
}

pe_status dst_fields_f64(pe_grid g, int64_t count, const GenSrc *gen, double *buf0, double *buf1,
                         double **result, hipStream_t st, int stop_axis) {
  double *in = buf0, *out = buf1;
  const int d = g->dim;
  for (int ax_i = d - 1; ax_i >= stop_axis; --ax_i) {
    const Axis &ax = g->ax[ax_i];
    int64_t inner = 1, outer = count;
    for (int b = ax_i + 1; b < d; ++b) inner *= g->ax[b].np;
    for (int b = 0; b < ax_i; ++b) outer *= g->ax[b].np;
    // algorithmic work per line of n nodes: one fold level,
    // ceil(n/2)^2 + floor(n/2)^2 multiply-adds; two levels, 4 (Kh/2)^2
    double lines = double(count) * double(g->dof) / ax.n;
    // (the generating pass on a three-level axis: 5/8 Kh^2; a batch whose
    // row count is not a multiple of 16 takes the two-level kernel)
    const bool l3_pass =
        gen && ax_i == d - 1 && ax.l3 && gen->M <= GEN_MAX_TERMS && outer % 16 == 0;
    double fl = l3_pass  ? 2.0 * lines * 0.625 * double(ax.Kh) * ax.Kh
                : ax.l2 ? 2.0 * lines * double(ax.Kh) * ax.Kh
                        : 2.0 * lines * (double((ax.n + 1) / 2) * ((ax.n + 1) / 2) + double(ax.H) * ax.H);
    // a generating pass writes its field and reads only the per-field
    // coefficients; the others read and write the field
    const bool gen_pass = gen && ax_i == d - 1;
    const double bytes = (gen_pass ? 1.0 : 2.0) * double(count) * double(g->dof) * sizeof(double) +
                         (gen_pass ? double(count) * gen->M * sizeof(double) : 0.0);
    TimedScope ts(g, ax_i == d - 1 ? PE_K_DST_LAST : PE_K_DST_MID, fl, bytes, st);
    if (ax_i == d - 1) {
      LastArgs a{};
      a.X = in;
      a.Y = out;
      a.R = outer;
      a.np = ax.np;
      a.n = ax.n;
      a.H = ax.H;
      a.Kh = ax.Kh;
      a.ShT = ax.d_ShT;
      a.d = d;
      a.rows_per_field = outer / count;
      a.np0 = g->ax[0].np;
      a.np1 = d >= 2 ? g->ax[1].np : 1;
      if (ax.l2) {
        a.ShT = ax.d_SqT;
        a.L3 = ax.l3 ? ax.d_L3 : nullptr;
        if (gen) {
          a.gen = *gen;
          if (gen->M <= 4)
            PE_TRY(launch_last2<4>(a, st));
          else if (gen->M <= 8)
            PE_TRY(launch_last2<8>(a, st));
          else if (gen->M <= 12)
            PE_TRY(launch_last2<12>(a, st));
          else if (gen->M <= 16)
            PE_TRY(launch_last2<16>(a, st));
          else
            PE_TRY(launch_last2<32>(a, st));
        } else {
          PE_TRY(launch_last2<0>(a, st));
        }
      } else if (gen) {
        a.gen = *gen;
        if (gen->M <= 4)
          PE_TRY(launch_last<4>(a, st));
        else if (gen->M <= 8)
          PE_TRY(launch_last<8>(a, st));
        else if (gen->M <= 12)
          PE_TRY(launch_last<12>(a, st));
        else if (gen->M <= 16)
          PE_TRY(launch_last<16>(a, st));
        else
          PE_TRY(launch_last<32>(a, st));
      } else {
        PE_TRY(launch_last<0>(a, st));
      }
    } else if (ax.l2) {
      Mid2Args a{};
      a.X = in;
      a.Y = out;
      a.O = outer;
      a.I = inner;
      a.np = ax.np;
      a.n = ax.n;
      a.H = ax.H;
      a.Kh = ax.Kh;
      a.Q = ax.Kh / 2;
      a.Sq = ax.d_Sq;
      PE_TRY(launch_mid2(a, st));
    } else {
      MidArgs a{};
      a.X = in;
      a.Y = out;
      a.O = outer;
      a.I = inner;
      a.np = ax.np;
      a.n = ax.n;
      a.H = ax.H;
      a.Kh = ax.Kh;
      a.Sh = ax.d_Sh;
      PE_TRY(launch_mid(a, st));
    }
    std::swap(in, out);
  }
  *result = in;
  return PE_OK;
}

}  // namespace pe
