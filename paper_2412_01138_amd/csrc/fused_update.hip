// Axis-0 transform pass fused with the diagonal update of eq. (2.6) (FP64,
// axes with two even/odd fold levels, d >= 2).
//
// After the passes over axes d-1..1 a batch holds, for every stage field f =
// (slice n, step j, stage i), the partial transform X_f[p][t]: p the nodes of
// axis 0, t the folded positions of the other axes.  The rest of one fine
// step is the axis-0 product and, per coefficient k of slice n,
//     W_k <- E_k W_k + sum_i (b_i sigma)_k ghat_{n,j,i}(k),   j in order
// (eq. 2.6 in the M-orthonormal basis; sigma_k turns DST coefficients into
// M-orthonormal ones).  The update of mode k needs the transformed value of
// mode k only, so a block owns one slice and a 16-wide strip of t and walks
// the slice's stage fields in order: each field's strip is folded into LDS
// (both halves), multiplied by the axis-0 quarter blocks Sq (kept in
// registers for the whole block), and the products go straight into the
// states, which stay in registers too.  The transformed stage fields never
// travel through HBM: one read of the partial transform per field replaces
// the write + read + read of the separate pass and update.
//
// Second fold level (axis 0, n = 2 Kh - 1, Q = Kh / 2): for half h and input
// parity g, C_g[i][t] = sum_jj Sq[h][g][i][jj] u_h[2 jj + g][t] with u_0 =
// x_p + x_{n-1-p}, u_1 = x_p - x_{n-1-p} (the middle node p = H counts once in
// half 0 only); folded position h Kh + i gets C_0 + C_1 and its partner i'
// (M-1-i for h = 0, M-2-i for h = 1; the last row of half 1 pairs with the pad
// position M-1) gets C_0 - C_1.
//
// Waves: HB halves per block x Q/16 row tiles.  Wave (h, rt) owns rows
// [16 rt, 16 rt + 16) of half h; with v_mfma_f64_16x16x4f64 (lane l supplies
// A[l%16][l/16], B[l/16][l%16], receives C[l/16 + 4r][l%16]) each lane holds
// the 4 rows l/16 + 4r of column l%16 for both parities, i.e. the states of
// 8 modes.  The rounding sequence of every state is the one of the separate
// update kernel (W = E W, then W += (b_i sigma) y per stage).
#include <algorithm>

#include "pe_internal.h"

namespace pe {

// fields per barrier of the FP64 kernel (two measured slower)
constexpr int FUSED_FPB = 1;
// strips in flight per block in the split-bf16 fused update (three or more
// cost the Kh = 64 kernel its second block per CU)
constexpr int SPLIT_DEPTH = 2;
// both halves of axis 0 in one block up to this Q (one half per block above)
constexpr int FUSED_HB2_MAX_Q = 64;

typedef double d4 __attribute__((ext_vector_type(4)));

struct FuArgs {
  const double *X;     // [count][np0][I]: partial transforms of the batch
  const double *Sq;    // [2][2][Q][Q] quarter blocks of axis 0
  // update tables in the kernel's lane order (zero at pads):
  // Tp[strip][ws][t][pair][lane][2], ws = h Q/16 + rt the wave slot, t = 0 the
  // decay e^{-z}, t = 1 + i the weight b_i(z) sigma, pair p holding the lane's
  // modes 2p (row l/16 + 4p of the tile) and 2p + 1 (its partner)
  const double *Tp;
  const double *Uin;   // [nslices][dof] states in, or null (zero)
  double *Uout;        // [nslices][dof] states out
  int64_t I;           // padded inner size prod_{a>0} np_a
  int64_t dofp;        // np0 * I
  int64_t dof;         // prod_a n_a
  int n0, Kh0;         // axis 0
  int n1, Kh1, n2, Kh2, np2;   // inner axes (2D: n2 = np2 = Kh2 = 1)
  int jc, s, strips, nslices;
  // split-bf16 grids: fp32 partial transforms and states, bf16 hi/lo halves
  // of axis 0's folded matrix
  const float *Xs;
  const float *Uins;
  float *Uouts;
  const uint16_t *Shi, *Slo;   // [2][Kh][Kh]
  int H0;
};

// compact index of the mode at folded position (P0, t), -1 at pads
__device__ inline int64_t mode_index(const FuArgs &a, int P0, int64_t t) {
  const int k0 = unfold_pos(P0, a.Kh0);
  const int p1 = int(t / a.np2), p2 = int(t - int64_t(p1) * a.np2);
  const int k1 = unfold_pos(p1, a.Kh1), k2 = unfold_pos(p2, a.Kh2);
  if (k0 >= a.n0 || k1 >= a.n1 || k2 >= a.n2) return -1;
  return (int64_t(k0) * a.n1 + k1) * a.n2 + k2;
}

template <int Q, int HB, int FPB>
__global__ __launch_bounds__(HB * Q * 4) void k_final_update(FuArgs a) {
  constexpr int RT = Q / 16;            // row tiles per half
  constexpr int NTH = HB * RT * 64;     // threads
  constexpr int KS = Q / 4;             // k-steps per parity
  constexpr int KH = 2 * Q;             // folded rows per half
  constexpr int ITEMS = KH * 8 / NTH;   // (row, column pair) loader items per thread
  static_assert(ITEMS * NTH == KH * 8, "loader items must tile the strip");
  // [stage][field of the group][half][parity][jj][column]
  __shared__ __attribute__((aligned(16))) double F[2][FPB][HB][2][Q][16];

  // strip-major block order: the blocks an XCD runs share a few strips (and
  // so the few update-table columns its L2 has to hold), each reading other
  // slices' fields
  int64_t bid = xcd_remap(blockIdx.x, gridDim.x);
  int hb = 0;
  if (HB == 1) {
    hb = int(bid % 2);
    bid /= 2;
  }
  const int nl = int(bid % a.nslices);
  const int strip = int(bid / a.nslices);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int hl = HB == 2 ? wave / RT : 0;
  const int h = HB == 2 ? hl : hb;
  const int rt = wave % RT;
  const int lr = lane & 15, lk = lane >> 4;
  const int M = a.Kh0;

  // quarter blocks of this wave's rows, both parities, as MFMA A fragments
  double s0[KS], s1[KS];
  {
    const double *S0 = a.Sq + (int64_t(2 * h) * Q + rt * 16 + lr) * Q + lk;
    const double *S1 = S0 + int64_t(Q) * Q;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      s0[ks] = S0[4 * ks];
      s1[ks] = S1[4 * ks];
    }
  }

  // folded positions of the lane's 8 modes (row pair r: first, partner)
  const int64_t col = int64_t(strip) * 16 + lr;
  int off[8];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = rt * 16 + lk + 4 * r;
    const int i2 = h == 0 ? M - 1 - i : (i < Q - 1 ? M - 2 - i : M - 1);
    off[2 * r] = int((h * M + i) * a.I + col);
    off[2 * r + 1] = int((h * M + i2) * a.I + col);
  }

  const int nf = a.jc * a.s;
  const double *Tl = a.Tp + (int64_t(strip) * (2 * RT) + h * RT + rt) * (1 + a.s) * 512 + 2 * lane;
  const double *Uin = a.Uin ? a.Uin + int64_t(nl) * a.dof : nullptr;
  double W[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int64_t k = mode_index(a, off[m] / int(a.I), col);
    W[m] = (Uin && k >= 0) ? Uin[k] : 0.0;
  }

  // strip loader: item = (folded row p, column pair), raw x_p and x_{n-1-p}
  const int64_t fstride = int64_t(2 * M) * a.I;
  const double *Xs = a.X + int64_t(nl) * nf * fstride + int64_t(strip) * 16;
  // one half per block (four loader items): the strip moves in two parts, the
  // second loaded while the first half of the products runs, so only two
  // items are ever live
  constexpr int PARTS = HB == 1 ? 2 : 1;
  constexpr int PI = ITEMS / PARTS;   // items per part
  static_assert(PARTS == 1 || FPB == 1, "split loader only with one field per barrier");
  struct Raw {
    double2 xa[PI], xb[PI];
  };
  Raw S[FPB];
  auto load = [&](Raw &R, int e, int part) {
    const double *Xf = Xs + e * fstride;
#pragma unroll
    for (int q = 0; q < PI; ++q) {
      const int idx = t + (part * PI + q) * NTH, p = idx >> 3, c = (idx & 7) * 2;
      R.xa[q] = *reinterpret_cast<const double2 *>(Xf + int64_t(p) * a.I + c);
      R.xb[q] = *reinterpret_cast<const double2 *>(Xf + int64_t(a.n0 - 1 - p) * a.I + c);
    }
  };
  auto stash = [&](const Raw &R, int stage, int slot, int part) {
#pragma unroll
    for (int q = 0; q < PI; ++q) {
      const int idx = t + (part * PI + q) * NTH, p = idx >> 3, c = (idx & 7) * 2;
      const int g = p & 1, jj = p >> 1;
      const bool mid = p == KH - 1;   // p = H: the middle node
      double2 u, v;
      u.x = mid ? R.xa[q].x : R.xa[q].x + R.xb[q].x;
      u.y = mid ? R.xa[q].y : R.xa[q].y + R.xb[q].y;
      v.x = mid ? 0.0 : R.xa[q].x - R.xb[q].x;
      v.y = mid ? 0.0 : R.xa[q].y - R.xb[q].y;
      if (HB == 2) {
        *reinterpret_cast<double2 *>(&F[stage][slot][0][g][jj][c]) = u;
        *reinterpret_cast<double2 *>(&F[stage][slot][HB - 1][g][jj][c]) = v;
      } else {
        // a select per component (as a select of the two structs the
        // compiler went through scratch memory, whose reload then waited
        // behind the strip prefetch)
        double2 w;
        w.x = hb == 0 ? u.x : v.x;
        w.y = hb == 0 ? u.y : v.y;
        *reinterpret_cast<double2 *>(&F[stage][slot][0][g][jj][c]) = w;
      }
    }
  };
  auto load2 = [&](const double *src, double (&dst)[8]) {
#pragma unroll
    for (int pp = 0; pp < 4; ++pp) {
      const double2 v = *reinterpret_cast<const double2 *>(src + pp * 128);
      dst[2 * pp] = v.x;
      dst[2 * pp + 1] = v.y;
    }
  };

  // Fields go in groups of FPB: the group's products from LDS stage g & 1,
  // the next group's strips stashed into the other stage (its last readers
  // passed the barrier that ended the previous group), then the updates of
  // the lane's states in field order, one barrier per group.
  for (int f = 0; f < FPB && f < nf; ++f)
    for (int part = 0; part < PARTS; ++part) {
      load(S[f], f, part);
      stash(S[f], 0, f, part);
    }
  __syncthreads();
  for (int e0 = 0; e0 < nf; e0 += FPB) {
    const int stage = (e0 / FPB) & 1;
    const int nxt = e0 + FPB;
    // tables of the group (16-byte loads, contiguous across the wave): the
    // decay once per group (it does not depend on the stage), a weight set
    // per field; ahead of the products (also with one half per block, where
    // it costs a few spilled registers but no longer exposes the tables'
    // latency after the products), and
    // issued before the next strip's loads: memory loads complete in issue
    // order, so the update's wait for its tables then leaves the strip in
    // flight
    int ist[FPB];
    bool need_e = false;
#pragma unroll
    for (int f = 0; f < FPB; ++f) {
      ist[f] = (e0 + f) % a.s;
      need_e = need_e || (ist[f] == 0 && e0 + f < nf);
    }
    double bw[FPB][8], ew[8];
    auto tables = [&]() {
#pragma unroll
      for (int f = 0; f < FPB; ++f) load2(Tl + (1 + ist[f]) * 512, bw[f]);
      if (need_e) load2(Tl, ew);
    };
    tables();
#pragma unroll
    for (int f = 0; f < FPB; ++f)
      if (nxt + f < nf) load(S[f], nxt + f, 0);
    d4 c0[FPB], c1[FPB];
#pragma unroll
    for (int f = 0; f < FPB; ++f) c0[f] = c1[f] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      if (PARTS == 2 && ks == KS / 2 && nxt < nf) {
        stash(S[0], stage ^ 1, 0, 0);
        load(S[0], nxt, 1);
      }
#pragma unroll
      for (int f = 0; f < FPB; ++f) {
        const double b0 = F[stage][f][hl][0][4 * ks + lk][lr];
        const double b1 = F[stage][f][hl][1][4 * ks + lk][lr];
        c0[f] = __builtin_amdgcn_mfma_f64_16x16x4f64(s0[ks], b0, c0[f], 0, 0, 0);
        c1[f] = __builtin_amdgcn_mfma_f64_16x16x4f64(s1[ks], b1, c1[f], 0, 0, 0);
      }
    }
#pragma unroll
    for (int f = 0; f < FPB; ++f)
      if (nxt + f < nf) stash(S[f], stage ^ 1, f, PARTS - 1);
#pragma unroll
    for (int f = 0; f < FPB; ++f) {
      if (e0 + f >= nf) break;   // a short last group (its LDS slot holds no field)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double y1 = c0[f][r] + c1[f][r], y2 = c0[f][r] - c1[f][r];
        double w1 = W[2 * r], w2 = W[2 * r + 1];
        if (ist[f] == 0) {
          w1 = ew[2 * r] * w1;
          w2 = ew[2 * r + 1] * w2;
        }
        W[2 * r] = w1 + bw[f][2 * r] * y1;
        W[2 * r + 1] = w2 + bw[f][2 * r + 1] * y2;
      }
    }
    __syncthreads();
  }

  double *Uout = a.Uout + int64_t(nl) * a.dof;
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int64_t k = mode_index(a, off[m] / int(a.I), col);
    if (k >= 0) Uout[k] = W[m];
  }
}

// The update tables in the fused kernel's lane order (layout at FuArgs::Tp):
// entry (strip, ws, t, pair, lane, c) is the table t of the lane's mode 2
// pair + c, i.e. E[k] or B[t-1][k] sigma_k for the mode k at its folded
// position (zero at pads); sigma_k = prod_a sig_a(k_a), in the product order
// of the separate update kernel.
__global__ void k_update_tables(FuArgs a, int RT, const double *__restrict__ sig0,
                                const double *__restrict__ sig1, const double *__restrict__ sig2,
                                const double *__restrict__ E, const double *__restrict__ B,
                                double *Tp, int d) {
  const int nt = 1 + a.s;
  const int64_t total = int64_t(a.strips) * 2 * RT * nt * 512;
  const int M = a.Kh0, Q = M / 2;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int c = int(e & 1), lane = int((e >> 1) & 63), pp = int((e >> 7) & 3);
    const int64_t rest = e >> 9;
    const int tt = int(rest % nt);
    const int64_t ws_all = rest / nt;
    const int ws = int(ws_all % (2 * RT)), strip = int(ws_all / (2 * RT));
    const int h = ws / RT, rt = ws % RT, lr = lane & 15, lk = lane >> 4;
    const int i = rt * 16 + lk + 4 * pp;
    const int i2 = h == 0 ? M - 1 - i : (i < Q - 1 ? M - 2 - i : M - 1);
    const int P0 = h * M + (c == 0 ? i : i2);
    const int64_t col = int64_t(strip) * 16 + lr;
    const int64_t k = mode_index(a, P0, col);
    double v = 0.0;
    if (k >= 0) {
      if (tt == 0) {
        v = E[k];
      } else {
        const int k0 = unfold_pos(P0, a.Kh0);
        const int p1 = int(col / a.np2), p2 = int(col - int64_t(p1) * a.np2);
        const int k1 = unfold_pos(p1, a.Kh1), k2 = unfold_pos(p2, a.Kh2);
        double sig = sig0[k0];
        if (d > 1) sig *= sig1[k1];
        if (d > 2) sig *= sig2[k2];
        v = B[int64_t(tt - 1) * a.dof + k] * sig;
      }
    }
    Tp[e] = v;
  }
}

// ------------------------------------------------------ split-bf16 grids
// In the split path every pass contracts the contiguous axis and writes it
// outermost, so the last pass contracts axis 0 and its input is
// X[f][r][p] (r the folded positions of the other axes, p the nodes of axis
// 0).  Fused with the update: a block owns one slice and 16 rows r and walks
// the slice's stage fields; each field's 16 rows are read once (float4 runs,
// the mirrored half as one ascending run), folded for both halves, split into
// bf16 hi + lo in LDS, and multiplied on v_mfma_f32_16x16x32_bf16 by the
// bf16 halves of Sh held in registers: three products per k-step (hi hi, hi
// lo, lo hi) with fp32 accumulation, in the order of the separate split pass.
// Waves: half h = wave / 4 and TM = Kh/64 mode tiles each; lane l holds
// C[4 (l/16) + r][l%16], i.e. 4 TM modes of row l%16, whose states stay in
// FP64 registers for the whole slice (as the separate update computes them).
// AXIS0_OUTER: the input is X[f][p][r] (the fused generating and
// middle-axis pass writes axis 0 outermost); a block then owns 32 rows, two
// row tiles, so that it reads whole 128-byte lines.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef float f4u_t __attribute__((ext_vector_type(4), aligned(4)));
typedef uint16_t u16x8_t __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4_t __attribute__((ext_vector_type(4)));
// the fourth word of a raw (unswizzled, stride 0) buffer resource on gfx950:
// 32-bit data format, no index swizzle; loads past num_records return zero
constexpr int BUFFER_RSRC_WORD3 = 0x00020000;

template <int KH, int DEPTH, bool AXIS0_OUTER>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(KH == 64 ? 4 : 1)))
void k_split_final_update(FuArgs a) {
  constexpr int NTH = 512;
  constexpr int TM = KH / 64;     // mode tiles per wave
  constexpr int KT = KH / 32;     // k-steps
  constexpr int LDB = KH + 8;     // bf16 per LDS row (16-byte pad)
  constexpr int CPR = KH / 4;     // 4-wide p chunks per row
  // AXIS0_OUTER: two adjacent 16-row tiles per block, so that every p of a
  // field is read as whole 128-byte lines (32 rows)
  constexpr int NR = AXIS0_OUTER ? 2 : 1;
  constexpr int ROWS = 16 * NR;
  constexpr int ITEMS = ROWS * CPR;                // loader items
  constexpr int IPT = (ITEMS + NTH - 1) / NTH;     // ... per thread
  static_assert(TM >= 1 && ITEMS <= IPT * NTH && (IPT == 1 || ITEMS % NTH == 0), "Kh of 64 or 128");
  constexpr bool ALL_ACTIVE = ITEMS == IPT * NTH;  // every thread loads every item
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][2][2][ROWS][LDB];   // [buf][h][hi/lo][row][p]
  // Kh = 128 with two row tiles: the lo halves of the Sh fragments live in
  // LDS (each wave its own, lane-contiguous 16-byte entries), which leaves
  // the registers to the prefetched tables of both tiles
  constexpr bool AL_LDS = KH == 128 && AXIS0_OUTER;
  __shared__ __attribute__((aligned(16))) u16x8_t AlS[AL_LDS ? 8 * TM * KT * 64 : 1];

  const int64_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const int nl = int(bid % a.nslices);
  const int rt0 = int(bid / a.nslices) * NR;   // first 16-row tile (strip-major: shared tables per XCD)
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int h = wave >> 2, wt = wave & 3;
  const int lr = lane & 15, lk = lane >> 4;

  // bf16 hi / lo of the wave's rows of Sh[h] as MFMA A fragments
  bf16x8_t ah[TM][KT], al[AL_LDS ? 1 : TM][AL_LDS ? 1 : KT];
  auto al_slot = [&](int tm, int kt) -> u16x8_t & { return AlS[((wave * TM + tm) * KT + kt) * 64 + lane]; };
#pragma unroll
  for (int tm = 0; tm < TM; ++tm)
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      const int64_t o = (int64_t(h) * KH + 16 * (wt * TM + tm) + lr) * KH + 32 * kt + 8 * lk;
      ah[tm][kt] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u16x8_t *>(a.Shi + o));
      const u16x8_t lo = *reinterpret_cast<const u16x8_t *>(a.Slo + o);
      if constexpr (AL_LDS)
        al_slot(tm, kt) = lo;   // read back by this lane only
      else
        al[tm][kt] = __builtin_bit_cast(bf16x8_t, lo);
    }

  // the lane's modes in tile n: m = 4 tm + q -> folded position (h Kh + i, row)
  const int nf = a.jc * a.s;
  const float *Uin = a.Uins ? a.Uins + int64_t(nl) * a.dof : nullptr;
  double W[NR][4 * TM];
#pragma unroll
  for (int n = 0; n < NR; ++n)
#pragma unroll
    for (int m = 0; m < 4 * TM; ++m) {
      const int i = 16 * (wt * TM + m / 4) + 4 * lk + (m % 4);
      const int64_t k = mode_index(a, h * KH + i, int64_t(rt0 + n) * 16 + lr);
      W[n][m] = (Uin && k >= 0) ? double(Uin[k]) : 0.0;
    }
  // the wave's tables of tile n as a buffer (base and size uniform); the lane
  // reads its 16 bytes of each 1 KiB row
  const double *Tw = a.Tp + (int64_t(rt0) * 8 + wave) * (1 + a.s) * (2 * TM * 128);
  const int64_t tstride = int64_t(8) * (1 + a.s) * (2 * TM * 128);   // next tile's tables
  const int trows = (1 + a.s) * 2 * TM;
  __amdgpu_buffer_rsrc_t Tr[NR];
#pragma unroll
  for (int n = 0; n < NR; ++n)
    Tr[n] = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(Tw + n * tstride), 0, trows * 1024,
                                              BUFFER_RSRC_WORD3);
  const int tlane = lane * 16;

  // loader items: row lrow of the block's rows, p = 4 c .. 4 c + 3.
  // The kernel is bound by HBM: DEPTH register sets keep the strips of the
  // next DEPTH fields in flight (field e + 1 + DEPTH is loaded right after
  // field e + 1 is stashed), so each load has DEPTH fields of time to land.
  // The strips are read once: streaming (nontemporal) loads leave L2 to the
  // update tables, which every step of the slice reads again.  AXIS0_OUTER:
  // the input is X[f][p][r] instead (the fused generating and middle-axis
  // pass writes axis 0 outermost); an item then reads its four p of one row
  // as single values, 32 consecutive rows (one 128-byte line) per p.
  const int64_t fstride = int64_t(a.I) * (2 * KH);
  int lrow[IPT], p0[IPT];
  bool active[IPT];
  const float *Xr[IPT];
  // AXIS0_OUTER: each field is read as a buffer from (p = 0, first row of
  // the block): byte offsets of (p0, row) and of the mirror (n0-4-p0, row)
  // per lane, and the e2-th value of an item 4 e2 I bytes further (the
  // mirror: 4 (3 - e2) I), a uniform offset.  No 64-bit address stays live.
  int oa[IPT], ob[IPT];
  const float *Xb = a.Xs + int64_t(nl) * nf * fstride + int64_t(rt0) * 16;
  const int xbytes = int((fstride - int64_t(rt0) * 16) * 4);   // to the field's end
#pragma unroll
  for (int q = 0; q < IPT; ++q) {
    const int it = t + q * NTH;
    lrow[q] = AXIS0_OUTER ? it % ROWS : it / CPR;
    p0[q] = 4 * (AXIS0_OUTER ? it / ROWS : it % CPR);
    active[q] = ALL_ACTIVE || it < ITEMS;
    Xr[q] = a.Xs + int64_t(nl) * nf * fstride +
            (int64_t(rt0) * 16 + (active[q] ? lrow[q] : 0)) * (AXIS0_OUTER ? 1 : 2 * KH);
    oa[q] = int((int64_t(p0[q]) * a.I + lrow[q]) * 4);
    ob[q] = int((int64_t(a.n0 - 4 - p0[q]) * a.I + lrow[q]) * 4);
  }
  struct Raw {
    f4_t xa[IPT], xb[IPT];
  };
  Raw S[DEPTH];
  // (past the last field the last one is loaded again, unused: no branch
  // around the loads, whose waits would otherwise be merged conservatively
  // with the path that skips them)
  auto load = [&](Raw &R, int e) {
    e = e < nf ? e : nf - 1;
    if constexpr (AXIS0_OUTER) {
      // (the mirror index n0-1-p0-e2 >= n0-Kh >= 0 for axes with Kh = 64 or
      // 128: the host checks it)
      const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float *>(Xb + int64_t(e) * fstride), 0, xbytes, BUFFER_RSRC_WORD3);
#pragma unroll
      for (int q = 0; q < IPT; ++q) {
        if (!ALL_ACTIVE && !active[q]) continue;
#pragma unroll
        for (int e2 = 0; e2 < 4; ++e2) {
          R.xa[q][e2] = __builtin_bit_cast(
              float, __builtin_amdgcn_raw_buffer_load_b32(xr, oa[q], int(e2 * a.I * 4), 0));
          R.xb[q][e2] = __builtin_bit_cast(
              float, __builtin_amdgcn_raw_buffer_load_b32(xr, ob[q], int((3 - e2) * a.I * 4), 0));
        }
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
      if (!ALL_ACTIVE && !active[q]) continue;
      const float *x = Xr[q] + e * fstride;
      R.xa[q] = __builtin_nontemporal_load(reinterpret_cast<const f4_t *>(x + p0[q]));
      const int mb = a.n0 - 4 - p0[q];   // x[n-1-p0-e], e = 0..3: one ascending run
      if (mb >= 0) {
        const f4u_t v = __builtin_nontemporal_load(reinterpret_cast<const f4u_t *>(x + mb));
        R.xb[q] = f4_t{v.w, v.z, v.y, v.x};
      } else {
#pragma unroll
        for (int e2 = 0; e2 < 4; ++e2) {
          const int i = a.n0 - 1 - p0[q] - e2;
          R.xb[q][e2] = x[i > 0 ? i : 0];
        }
      }
    }
  };
  auto stash = [&](const Raw &R, int buf) {
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
      if (!ALL_ACTIVE && !active[q]) continue;
      f4_t u, v;
      // AXIS0_OUTER: a wave's items cover two p0 (known from the wave index);
      // below the middle node both fold terms exist for every lane
      const bool interior = AXIS0_OUTER && 4 * ((wave * 64 + q * NTH + 63) / ROWS) + 3 < a.H0;
      if (interior) {
        u = R.xa[q] + R.xb[q];
        v = R.xa[q] - R.xb[q];
      } else {
#pragma unroll
        for (int e2 = 0; e2 < 4; ++e2) {
          const int p = p0[q] + e2;
          const bool has_b = p < a.H0;
          const bool has_a0 = has_b || (p == a.H0 && (a.n0 & 1));
          u[e2] = (has_a0 ? R.xa[q][e2] : 0.0f) + (has_b ? R.xb[q][e2] : 0.0f);
          v[e2] = (has_b ? R.xa[q][e2] : 0.0f) + (has_b ? -R.xb[q][e2] : 0.0f);
        }
      }
      const bf16x4_t uh = __builtin_convertvector(u, bf16x4_t);
      const bf16x4_t ul = __builtin_convertvector(u - __builtin_convertvector(uh, f4_t), bf16x4_t);
      const bf16x4_t vh = __builtin_convertvector(v, bf16x4_t);
      const bf16x4_t vl = __builtin_convertvector(v - __builtin_convertvector(vh, f4_t), bf16x4_t);
      *reinterpret_cast<u16x4_t *>(&Bs[buf][0][0][lrow[q]][p0[q]]) = __builtin_bit_cast(u16x4_t, uh);
      *reinterpret_cast<u16x4_t *>(&Bs[buf][0][1][lrow[q]][p0[q]]) = __builtin_bit_cast(u16x4_t, ul);
      *reinterpret_cast<u16x4_t *>(&Bs[buf][1][0][lrow[q]][p0[q]]) = __builtin_bit_cast(u16x4_t, vh);
      *reinterpret_cast<u16x4_t *>(&Bs[buf][1][1][lrow[q]][p0[q]]) = __builtin_bit_cast(u16x4_t, vl);
    }
  };

  // the update tables of tile n: the decay (the same every step, loaded
  // once) and the weights of field e's stage e % s, loaded one field ahead,
  // right after the previous field's update of the tile, so that the loads
  // have a whole field's products to land in instead of stalling the update
  double bw[NR][4 * TM], ew[NR][4 * TM];
  auto row = [&](int n, int r) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(Tr[n], tlane, r * 1024, 0));
  };
  auto load_tables = [&](int n, int e) {
    e = e < nf ? e : nf - 1;   // (unconditional, as the field loads)
    const int i_st = e % a.s;
#pragma unroll
    for (int pp = 0; pp < 2 * TM; ++pp) {
      const double2 w2 = row(n, (1 + i_st) * 2 * TM + pp);
      bw[n][2 * pp] = w2.x;
      bw[n][2 * pp + 1] = w2.y;
    }
  };
#pragma unroll
  for (int n = 0; n < NR; ++n)
#pragma unroll
    for (int pp = 0; pp < 2 * TM; ++pp) {
      const double2 w2 = row(n, pp);
      ew[n][2 * pp] = w2.x;
      ew[n][2 * pp + 1] = w2.y;
    }

  // one field: the products of both row tiles from LDS buffer e & 1, the
  // next field stashed from its register set (then refilled DEPTH fields
  // ahead), the update of each tile and its next tables
  auto field = [&](int e, Raw &nextset) {
    const int buf = e & 1;
    const int i_st = e % a.s;
    // the products of both row tiles in one k-loop (the A fragments serve both)
    f4_t acc[NR][TM];
#pragma unroll
    for (int n = 0; n < NR; ++n)
#pragma unroll
      for (int tm = 0; tm < TM; ++tm) acc[n][tm] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      bf16x8_t bh[NR], bl[NR];
#pragma unroll
      for (int n = 0; n < NR; ++n) {
        bh[n] = __builtin_bit_cast(
            bf16x8_t, *reinterpret_cast<const u16x8_t *>(&Bs[buf][h][0][16 * n + lr][32 * kt + 8 * lk]));
        bl[n] = __builtin_bit_cast(
            bf16x8_t, *reinterpret_cast<const u16x8_t *>(&Bs[buf][h][1][16 * n + lr][32 * kt + 8 * lk]));
      }
#pragma unroll
      for (int tm = 0; tm < TM; ++tm) {
        bf16x8_t alo;
        if constexpr (AL_LDS)
          alo = __builtin_bit_cast(bf16x8_t, al_slot(tm, kt));
        else
          alo = al[tm][kt];
#pragma unroll
        for (int n = 0; n < NR; ++n) {
          acc[n][tm] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[tm][kt], bh[n], acc[n][tm], 0, 0, 0);
          acc[n][tm] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[tm][kt], bl[n], acc[n][tm], 0, 0, 0);
          acc[n][tm] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bh[n], acc[n][tm], 0, 0, 0);
        }
      }
    }
    // (after the last field the stash writes a buffer nobody reads)
    stash(nextset, buf ^ 1);
    load(nextset, e + 1 + DEPTH);
    // the decay once per step (a uniform branch, not a select per mode)
    if (i_st == 0) {
#pragma unroll
      for (int n = 0; n < NR; ++n)
#pragma unroll
        for (int m = 0; m < 4 * TM; ++m) W[n][m] = ew[n][m] * W[n][m];
    }
#pragma unroll
    for (int n = 0; n < NR; ++n) {
#pragma unroll
      for (int m = 0; m < 4 * TM; ++m) W[n][m] = W[n][m] + bw[n][m] * double(acc[n][m / 4][m % 4]);
      load_tables(n, e + 1);
    }
    __syncthreads();
  };

  // set d holds field d (d < DEPTH); field 0 goes to LDS and its set is
  // refilled with field DEPTH; then field 0's tables.  (The loads leave in
  // the order of every field's: field loads, then tables, so that the waits
  // the compiler counts at the loop head hold for the first pass too and
  // do not fall back to waiting for everything.)
#pragma unroll
  for (int d = 0; d < DEPTH; ++d) load(S[d], d);
  stash(S[0], 0);
  load(S[0], DEPTH);
#pragma unroll
  for (int n = 0; n < NR; ++n) load_tables(n, 0);
  __syncthreads();
  for (int e0 = 0; e0 < nf; e0 += DEPTH) {
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) {
      if (e0 + d >= nf) break;
      field(e0 + d, S[(d + 1) % DEPTH]);
    }
  }

  float *Uout = a.Uouts + int64_t(nl) * a.dof;
#pragma unroll
  for (int n = 0; n < NR; ++n)
#pragma unroll
    for (int m = 0; m < 4 * TM; ++m) {
      const int i = 16 * (wt * TM + m / 4) + 4 * lk + (m % 4);
      const int64_t k = mode_index(a, h * KH + i, int64_t(rt0 + n) * 16 + lr);
      if (k >= 0) Uout[k] = float(W[n][m]);
    }
}

// Update tables in the split kernel's lane order: entry (rt, wave, t, pair,
// lane, c) is table t of the lane's mode 2 pair + c (rows of tile rt).
__global__ void k_split_tables(FuArgs a, int TM, const double *__restrict__ sig0,
                               const double *__restrict__ sig1, const double *__restrict__ sig2,
                               const double *__restrict__ E, const double *__restrict__ B,
                               double *Tp, int d) {
  const int nt = 1 + a.s, NP = 2 * TM;
  const int64_t total = (a.I / 16) * 8 * nt * NP * 128;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int c = int(e & 1), lane = int((e >> 1) & 63);
    int64_t rest = e >> 7;
    const int pp = int(rest % NP);
    rest /= NP;
    const int tt = int(rest % nt);
    rest /= nt;
    const int wave = int(rest % 8);
    const int64_t rt = rest / 8;
    const int h = wave >> 2, wt = wave & 3, lr = lane & 15, lk = lane >> 4;
    const int m = 2 * pp + c;
    const int i = 16 * (wt * TM + m / 4) + 4 * lk + (m % 4);
    const int P0 = h * a.Kh0 + i;
    const int64_t row = rt * 16 + lr;
    const int64_t k = mode_index(a, P0, row);
    double v = 0.0;
    if (k >= 0) {
      if (tt == 0) {
        v = E[k];
      } else {
        const int k0 = unfold_pos(P0, a.Kh0);
        const int p1 = int(row / a.np2), p2 = int(row - int64_t(p1) * a.np2);
        const int k1 = unfold_pos(p1, a.Kh1), k2 = unfold_pos(p2, a.Kh2);
        double sig = sig0[k0];
        if (d > 1) sig *= sig1[k1];
        if (d > 2) sig *= sig2[k2];
        v = B[int64_t(tt - 1) * a.dof + k] * sig;
      }
    }
    Tp[e] = v;
  }
}

static FuArgs base_args(pe_grid g, int s) {
  FuArgs a{};
  const Axis &x0 = g->ax[0];
  a.I = g->dofp / x0.np;
  a.dofp = g->dofp;
  a.dof = g->dof;
  a.n0 = x0.n;
  a.Kh0 = x0.Kh;
  a.n1 = g->ax[1].n;
  a.Kh1 = g->ax[1].Kh;
  if (g->dim == 3) {
    a.n2 = g->ax[2].n;
    a.Kh2 = g->ax[2].Kh;
    a.np2 = g->ax[2].np;
  } else {
    a.n2 = a.Kh2 = a.np2 = 1;
  }
  a.s = s;
  a.strips = int(a.I / 16);
  return a;
}

// Largest Q whose quarter blocks, loader and states fit the 256 registers of
// a lane at two waves per SIMD without spilling.
constexpr int FUSED_MAX_Q = 128;

bool fused_update_supported(pe_grid g) {
  if (g->transform == PE_TRANSFORM_FFT) return fft_final_supported(g);
  if (g->dim < 2) return false;
  const Axis &x0 = g->ax[0];
  if (g->precision == PE_SPLIT_BF16)
    return (x0.Kh == 64 || x0.Kh == 128) && x0.d_Shi && (g->dofp / x0.np) % 16 == 0 &&
           g->dofp < (int64_t(1) << 31);
  if (g->precision != PE_FP64) return false;
  const int Q = x0.Kh / 2;
  return x0.l2 && x0.n == 2 * x0.Kh - 1 && Q % 16 == 0 && Q >= 16 && Q <= FUSED_MAX_Q &&
         (g->dofp / x0.np) % 16 == 0 && g->dofp < (int64_t(1) << 31);
}

// (the packed tables hold strips * Q/8 wave slots * (1 + s) * 512 = (1 + s)
// DOF_padded doubles)
size_t fused_update_table_bytes(pe_grid g) {
  if (!fused_update_supported(g)) return 0;
  return Arena::need(sizeof(double) * size_t(g->dofp) * (1 + PE_MAX_STAGES)) + 256;
}

pe_status fused_update_tables(pe_grid g, int s, const double *E, const double *B, double *Tp,
                              hipStream_t st) {
  if (g->transform == PE_TRANSFORM_FFT) return fft_tables(g, s, E, B, Tp, st);
  FuArgs a = base_args(g, s);
  if (g->precision == PE_SPLIT_BF16) {
    const int TM = g->ax[0].Kh / 64;
    const int64_t n = (a.I / 16) * 8 * (1 + s) * 2 * TM * 128;
    const unsigned blocks = unsigned(std::min<int64_t>((n + 255) / 256, 65536));
    k_split_tables<<<blocks, 256, 0, st>>>(a, TM, g->ax[0].d_sig, g->ax[1].d_sig,
                                            g->dim > 2 ? g->ax[2].d_sig : nullptr, E, B, Tp,
                                            g->dim);
    PE_HIP(hipGetLastError());
    return PE_OK;
  }
  const int RT = g->ax[0].Kh / 32;
  const int64_t n = int64_t(a.strips) * 2 * RT * (1 + s) * 512;
  const unsigned blocks = unsigned(std::min<int64_t>((n + 255) / 256, 65536));
  k_update_tables<<<blocks, 256, 0, st>>>(a, RT, g->ax[0].d_sig, g->ax[1].d_sig,
                                           g->dim > 2 ? g->ax[2].d_sig : nullptr, E, B, Tp,
                                           g->dim);
  PE_HIP(hipGetLastError());
  return PE_OK;
}

template <int Q>
static void launch_q(const FuArgs &a, int64_t nslices, hipStream_t st) {
  constexpr int HB = Q <= FUSED_HB2_MAX_Q ? 2 : 1;
  constexpr int FPB = HB == 2 ? FUSED_FPB : 1;   // two strips fit the registers at Q <= 64
  const int64_t blocks = nslices * a.strips * (2 / HB);
  k_final_update<Q, HB, FPB><<<dim3(unsigned(blocks)), HB * Q * 4, 0, st>>>(a);
}

template <int KH>
static void launch_split_final(const FuArgs &a, int64_t blocks, bool axis0_outer, hipStream_t st) {
  // (32 rows per block: one strip in flight holds as many bytes as two of 16)
  if (axis0_outer)
    k_split_final_update<KH, SPLIT_DEPTH / 2, true><<<dim3(unsigned(blocks)), 512, 0, st>>>(a);
  else
    k_split_final_update<KH, SPLIT_DEPTH, false><<<dim3(unsigned(blocks)), 512, 0, st>>>(a);
}

static pe_status split_final_update(pe_grid g, const FieldBatch &b, FuArgs a, bool axis0_outer,
                                    hipStream_t st) {
  const Axis &x0 = g->ax[0];
  a.Shi = x0.d_Shi;
  a.Slo = x0.d_Slo;
  a.H0 = x0.H;
  if (axis0_outer && (a.I / 16) % 2 != 0)
    return set_error(PE_E_ARG, "internal: odd tile count for the axis-0-outer fused update");
  // (the axis-0-outer loader reads the mirror node n0-1-p for p < Kh without
  // a clamp, and addresses a field with 32-bit byte offsets)
  if (axis0_outer && x0.n < x0.Kh)
    return set_error(PE_E_ARG, "internal: axis 0 shorter than its half width");
  if (axis0_outer && g->dofp * int64_t(sizeof(float)) >= (int64_t(1) << 31))
    return set_error(PE_E_ARG, "internal: field too large for the axis-0-outer fused update");
  const int64_t blocks = int64_t(b.nslices) * (a.I / 16) / (axis0_outer ? 2 : 1);
  if (blocks >= (int64_t(1) << 31)) return set_error(PE_E_ARG, "internal: fused grid too large");
  // axis-0 products (three bf16 products of the folded pass) plus the update
  const double fields = double(b.count());
  const double lines = double(g->dof / x0.n);
  const double flops =
      fields * 3.0 * 2.0 * lines *
      (double((x0.n + 1) / 2) * ((x0.n + 1) / 2) + double(x0.H) * x0.H);
  const double bytes = fields * double(g->dof) * 4.0 + 2.0 * b.nslices * double(g->dof) * 4.0 +
                       double(1 + b.s) * double(g->dof) * 8.0;
  TimedScope ts(g, PE_K_MID_UPDATE, flops, bytes, st);
  if (x0.Kh == 128)
    launch_split_final<128>(a, blocks, axis0_outer, st);
  else
    launch_split_final<64>(a, blocks, axis0_outer, st);
  PE_HIP(hipGetLastError());
  return PE_OK;
}

pe_status final_pass_update(pe_grid g, const FieldBatch &b, const void *X, const double *Tp,
                            const void *Uin, void *Uout, hipStream_t st, bool axis0_outer) {
  if (!fused_update_supported(g)) return set_error(PE_E_ARG, "internal: no fused update here");
  if (g->transform == PE_TRANSFORM_FFT)
    return fft_final_update(g, b, static_cast<const double *>(X), Tp,
                            static_cast<const double *>(Uin), static_cast<double *>(Uout), st);
  FuArgs a = base_args(g, b.s);
  const Axis &x0 = g->ax[0];
  a.Tp = Tp;
  a.jc = b.jc;
  a.nslices = b.nslices;
  if (g->precision == PE_SPLIT_BF16) {
    a.Xs = static_cast<const float *>(X);
    a.Uins = static_cast<const float *>(Uin);
    a.Uouts = static_cast<float *>(Uout);
    return split_final_update(g, b, a, axis0_outer, st);
  }
  a.X = static_cast<const double *>(X);
  a.Sq = x0.d_Sq;
  a.Uin = static_cast<const double *>(Uin);
  a.Uout = static_cast<double *>(Uout);
  const int Q = x0.Kh / 2;
  const int64_t blocks = int64_t(b.nslices) * a.strips * (Q <= FUSED_HB2_MAX_Q ? 1 : 2);
  if (blocks >= (int64_t(1) << 31)) return set_error(PE_E_ARG, "internal: fused grid too large");
  // axis-0 products (two fold levels) plus the update's reads and writes
  const double fields = double(b.count());
  const double flops = fields * 2.0 * double(g->dof / x0.n) * double(x0.Kh) * x0.Kh;
  const double bytes = fields * double(g->dof) * 8.0 + 2.0 * b.nslices * double(g->dof) * 8.0 +
                       double(1 + b.s) * double(g->dof) * 8.0;
  TimedScope ts(g, PE_K_MID_UPDATE, flops, bytes, st);
  switch (Q) {
    case 16: launch_q<16>(a, b.nslices, st); break;
    case 32: launch_q<32>(a, b.nslices, st); break;
    case 48: launch_q<48>(a, b.nslices, st); break;
    case 64: launch_q<64>(a, b.nslices, st); break;
    case 80: launch_q<80>(a, b.nslices, st); break;
    case 96: launch_q<96>(a, b.nslices, st); break;
    case 112: launch_q<112>(a, b.nslices, st); break;
    case 128: launch_q<128>(a, b.nslices, st); break;
    default: return set_error(PE_E_ARG, "internal: fused update Q %d", Q);
  }
  PE_HIP(hipGetLastError());
  return PE_OK;
}

}  // namespace pe
