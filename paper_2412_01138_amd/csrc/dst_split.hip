// Per-axis DST-I passes in split-bf16 with fp32 accumulation, for fp32
// fields (v_mfma_f32_16x16x32_bf16).
//
// Every pass contracts the contiguous axis of its input and writes that axis
// outermost ("rotating" passes):  X[f][r][p] -> Y[f][k][r],
//     Y[f][h*Kh + i][r] = sum_p Sh[h][i][p] * fold_h(X[f][r][.])[p]
// with the even/odd fold of the DST-I (see pe_internal.h).  After d passes
// the axes are back in their natural order, each in folded mode order.  Both
// MFMA operands then run along p in memory, so no transposes are needed:
// A = Sh[h] (precomputed bf16 hi/lo split), B = the folded fp32 data, split
// on the fly into hi + lo bf16.  Three products per tile,
//     C += A_hi B_hi + A_hi B_lo + A_lo B_hi,
// accumulate in fp32 (the dropped A_lo B_lo term is below fp32 rounding of
// the inputs' second halves).
//
// The first pass can generate its input from the quadrature tables, as in the
// FP64 path: the folded load row of field f, row r is
//     sum_m rf[r][m] Cf[h][m][p],  rf = coef[f][m] prod_{a<d-1} C_a[m][j_a],
// a product with k = the (at most 32) forcing terms, done on the same bf16
// MFMA as the transform with hi/lo splits of both factors (three products,
// fp32 accumulation): A = Cf^T of this half (bf16 hi/lo, [p][m], built once
// per table by k_split_gen_table and read through the cache, so the block's
// LDS holds only its tiles), B = the wave's row factors (registers), C = the
// tile transposed, so a lane holds four consecutive p of one row.
//
// Block: 256 threads = 4 waves (2 x 2), tile BM (modes) x 128 (rows r) of
// one half (a generating block computes both halves of its tile in turn,
// forming the row factors once), k-step 32, single LDS buffer with register
// prefetch.
// MFMA f32 16x16x32 bf16 lane layout: lane l supplies A[l%16][8(l/16) + e]
// and B[8(l/16) + e][l%16] (e = 0..7) and receives C[4(l/16) + r][l%16].
#include <algorithm>

#include "pe_internal.h"

namespace pe {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int SKB = 32;          // k-step
constexpr int SBN = 128;         // block tile along r
constexpr int SLD = SKB + 8;     // LDS row length in bf16 (16-byte pad: conflict-free b128 reads)
constexpr int SNT = 256;
constexpr int SGEN_MAX_TERMS = 32;   // one 32-deep MFMA k-step over the terms

typedef float f8 __attribute__((ext_vector_type(8)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));   // dword-aligned loads
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// LDS ordering between lanes of one wave (no cross-wave exchange)
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// hi = bf16(v) (round to nearest even), lo = bf16(v - hi), 8 at a time
__device__ inline void split8(const f8 &v, bf16x8 &hi, bf16x8 &lo) {
  hi = __builtin_convertvector(v, bf16x8);
  const f8 hv = __builtin_convertvector(hi, f8);
  lo = __builtin_convertvector(v - hv, bf16x8);
}

struct SplitArgs {
  const float *X;          // [F][R][np]  (contracted axis contiguous)
  float *Y;                // [F][np][R]
  int64_t R;
  int np, n, H, Kh;
  const uint16_t *Shi, *Slo;   // [2][Kh][Kh]
  int tiles_m, tiles_n;
  // generation (first pass only; natural axis order)
  int d;
  int np0, np1;
  GenSrcF gen;
};

template <int BM>
struct alignas(16) SSmem {
  uint16_t Ahi[BM][SLD], Alo[BM][SLD];
  uint16_t Bhi[SBN][SLD], Blo[SBN][SLD];
};

template <int BM, bool GEN>
// (GEN: at most 168 registers, three waves per SIMD)
__global__ __launch_bounds__(SNT) __attribute__((amdgpu_waves_per_eu(GEN ? 3 : 1))) void k_split_pass(SplitArgs a) {
  constexpr int TM = BM / 32;                 // MFMA tiles per wave along the modes
  constexpr int TN = 4;                       // ... along r (64 per wave)
  constexpr int ACH = BM * (SKB / 8) / SNT;   // 16-byte A chunks per thread per array (2, 1, ..)
  constexpr int EB = 16;                      // p values of one B row per thread
  static_assert(ACH >= 1 || BM == 32, "A chunk mapping");
  __shared__ SSmem<BM> sm;

  int64_t bid = blockIdx.x;
  {
    const int64_t nb = gridDim.x;
    if (nb % 8 == 0) bid = (bid % 8) * (nb / 8) + bid / 8;   // one field's tiles on one XCD
  }
  // the two halves of a tile read the same rows: run them back to back (a
  // generating block runs both, sharing its row factors)
  int h = 0;
  if (!GEN) {
    h = int(bid % 2);
    bid /= 2;
  }
  const int tn = int(bid % a.tiles_n);
  bid /= a.tiles_n;
  const int tm = int(bid % a.tiles_m);
  const int64_t f = bid / a.tiles_m;
  const int m0 = tm * BM;
  const int64_t n0 = int64_t(tn) * SBN;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1, lr = lane & 15, lk = lane >> 4;

  // A-tile role: 16-byte chunks c = t + SNT u of the BM x 32 tile
  // (row c / 4, bf16 columns 8 (c % 4) ..); BM = 32 uses half the threads
  constexpr int AU = ACH > 0 ? ACH : 1;
  const bool a_active = ACH > 0 || t < BM * (SKB / 8);
  // B-tile role: row rb (an r index), p values pb0 .. pb0 + 16
  const int rb = t / 2, pb0 = (t % 2) * EB;
  const int64_t grow = n0 + rb;
  const bool brow_ok = grow < a.R;
  const int64_t grc = brow_ok ? grow : a.R - 1;

  // GEN: the wave's 32 rows of row factors as MFMA B fragments (two 16-row
  // tiles): lane supplies rf[row = 32 wave + 16 rt + lr][m = 8 lk + e]
  bf16x8 rfh[GEN ? 2 : 1], rfl[GEN ? 2 : 1];
  if constexpr (GEN) {
    const int M = a.gen.M;
    const double *C0 = a.d >= 2 ? a.gen.C0 : nullptr;
    const double *C1 = a.d == 3 ? a.gen.C1 : nullptr;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int64_t gr0 = n0 + 32 * wave + 16 * rt + lr;
      const bool ok = gr0 < a.R;
      const int64_t gr = ok ? gr0 : a.R - 1;
      int j0 = 0, j1 = 0;
      if (a.d == 2) j0 = int(gr);
      if (a.d == 3) {
        j0 = int(gr / a.np1);
        j1 = int(gr - int64_t(j0) * a.np1);
      }
      f8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int m = 8 * lk + e;
        const int mm = m < M ? m : M - 1;
        double x = a.gen.coef[f * M + mm];
        if (C0) x *= C0[int64_t(mm) * a.np0 + j0];
        if (C1) x *= C1[int64_t(mm) * a.np1 + j1];
        v[e] = (m < M && ok) ? float(x) : 0.0f;
      }
      split8(v, rfh[rt], rfl[rt]);
    }
  }
  // GEN: Cf^T as 16-byte pieces, [hi / lo][h][p][m / 8]
  const bf16x8 *cft = GEN ? reinterpret_cast<const bf16x8 *>(a.gen.Cft) : nullptr;
  const int64_t cft_lo = int64_t(2) * a.Kh * (SGEN_MAX_TERMS / 8);

  const float *xrow = GEN ? nullptr : a.X + (f * a.R + grc) * a.np;
  u16x8 pah[AU], pal[AU];
  float pxa[GEN ? 1 : EB], pxb[GEN ? 1 : EB];
  auto load = [&](int k0) {
    if (a_active) {
#pragma unroll
      for (int u = 0; u < AU; ++u) {
        const int c = t + SNT * u;
        const int row = m0 + c / 4;
        const int64_t arow = int64_t(h) * a.Kh + (row < a.Kh ? row : a.Kh - 1);
        const int64_t o = arow * a.Kh + k0 + 8 * (c % 4);
        pah[u] = *reinterpret_cast<const u16x8 *>(a.Shi + o);
        pal[u] = *reinterpret_cast<const u16x8 *>(a.Slo + o);
      }
    }
    if constexpr (!GEN) {
      const int p = k0 + pb0;
      // forward x[p .. p+15]: p + 15 < Kh <= np, inside the row
#pragma unroll
      for (int q = 0; q < EB / 4; ++q) {
        const f4u v = *reinterpret_cast<const f4u *>(xrow + p + 4 * q);
        pxa[4 * q] = v.x;
        pxa[4 * q + 1] = v.y;
        pxa[4 * q + 2] = v.z;
        pxa[4 * q + 3] = v.w;
      }
      // mirror x[n-1-p-e], e = 0..15: one ascending run from n-16-p
      const int mb = a.n - EB - p;
      if (mb >= 0) {
#pragma unroll
        for (int q = 0; q < EB / 4; ++q) {
          const f4u v = *reinterpret_cast<const f4u *>(xrow + mb + 4 * q);
          pxb[EB - 1 - 4 * q] = v.x;
          pxb[EB - 2 - 4 * q] = v.y;
          pxb[EB - 3 - 4 * q] = v.z;
          pxb[EB - 4 - 4 * q] = v.w;
        }
      } else {
#pragma unroll
        for (int e = 0; e < EB; ++e) {
          const int i = a.n - 1 - p - e;
          pxb[e] = xrow[i > 0 ? i : 0];
        }
      }
    }
  };
  auto store = [&](int k0) {
    if (a_active) {
#pragma unroll
      for (int u = 0; u < AU; ++u) {
        const int c = t + SNT * u;
        const bool ok = m0 + c / 4 < a.Kh;
        const u16x8 z = {0, 0, 0, 0, 0, 0, 0, 0};
        *reinterpret_cast<u16x8 *>(&sm.Ahi[c / 4][8 * (c % 4)]) = ok ? pah[u] : z;
        *reinterpret_cast<u16x8 *>(&sm.Alo[c / 4][8 * (c % 4)]) = ok ? pal[u] : z;
      }
    }
    if constexpr (GEN) {
      // B tile rows 32 wave .. + 32, p = k0 .. k0 + 32: C^T = Cf^T rf^T
      // (the A fragments are read here, not prefetched with the next step's
      // tiles: sixteen more live registers would cost a wave per SIMD)
      bf16x8 gth[2], gtl[2];
#pragma unroll
      for (int pt = 0; pt < 2; ++pt) {
        // this half's rows p = k0 + 16 pt + lr, terms m = 8 lk .. 8 lk + 7
        const int64_t o = (int64_t(h) * a.Kh + k0 + 16 * pt + lr) * (SGEN_MAX_TERMS / 8) + lk;
        gth[pt] = cft[o];
        gtl[pt] = cft[cft_lo + o];
      }
#pragma unroll
      for (int pt = 0; pt < 2; ++pt) {
        const bf16x8 ah = gth[pt], al = gtl[pt];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
          f4 c = f4{0.f, 0.f, 0.f, 0.f};
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, rfh[rt], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, rfl[rt], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, rfh[rt], c, 0, 0, 0);
          // lane holds p = 16 pt + 4 lk + r (r = 0..3) of row 32 wave + 16 rt + lr
          uint16_t hb[4], lb[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const __bf16 hv = static_cast<__bf16>(c[r]);
            hb[r] = __builtin_bit_cast(uint16_t, hv);
            lb[r] = __builtin_bit_cast(uint16_t, static_cast<__bf16>(c[r] - static_cast<float>(hv)));
          }
          const int row = 32 * wave + 16 * rt + lr, col = 16 * pt + 4 * lk;
          *reinterpret_cast<uint2 *>(&sm.Bhi[row][col]) =
              uint2{uint32_t(hb[0]) | (uint32_t(hb[1]) << 16), uint32_t(hb[2]) | (uint32_t(hb[3]) << 16)};
          *reinterpret_cast<uint2 *>(&sm.Blo[row][col]) =
              uint2{uint32_t(lb[0]) | (uint32_t(lb[1]) << 16), uint32_t(lb[2]) | (uint32_t(lb[3]) << 16)};
        }
      }
    } else {
#pragma unroll
      for (int g8 = 0; g8 < EB / 8; ++g8) {
        f8 v;
#pragma unroll
        for (int e8 = 0; e8 < 8; ++e8) {
          const int e = 8 * g8 + e8;
          const int p = k0 + pb0 + e;
          const bool has_b = p < a.H;
          const bool has_a = has_b || (h == 0 && p == a.H && (a.n & 1));
          float x = (has_a ? pxa[e] : 0.0f) + (has_b ? (h == 0 ? pxb[e] : -pxb[e]) : 0.0f);
          v[e8] = brow_ok ? x : 0.0f;
        }
        bf16x8 hi, lo;
        split8(v, hi, lo);
        *reinterpret_cast<bf16x8 *>(&sm.Bhi[rb][pb0 + 8 * g8]) = hi;
        *reinterpret_cast<bf16x8 *>(&sm.Blo[rb][pb0 + 8 * g8]) = lo;
      }
    }
  };

  for (int hh = 0; hh < (GEN ? 2 : 1); ++hh) {
    if (GEN) h = hh;
    f4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    const int nk = a.Kh / SKB;
    load(0);
    for (int kt = 0; kt < nk; ++kt) {
      store(kt * SKB);
      __syncthreads();
      if (kt + 1 < nk) load((kt + 1) * SKB);
      bf16x8 ah[TM], al[TM];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int row = wm * (BM / 2) + i * 16 + lr;
        ah[i] = *reinterpret_cast<const bf16x8 *>(&sm.Ahi[row][lk * 8]);
        al[i] = *reinterpret_cast<const bf16x8 *>(&sm.Alo[row][lk * 8]);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int col = wn * 64 + j * 16 + lr;
        const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(&sm.Bhi[col][lk * 8]);
        const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(&sm.Blo[col][lk * 8]);
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc[i][j], 0, 0, 0);
        }
      }
      __syncthreads();
    }

    // Output through a per-wave LDS scratch (the tile buffers are free after
    // the last barrier): each 16-row group of the wave's 64 columns is written
    // in MFMA layout, read back as rows and stored as float4 runs (256 B of
    // one output row per 16 lanes instead of 64 B pieces of four rows).
    float *Y = a.Y + f * int64_t(a.np) * a.R;
    constexpr int SCR = 68;   // scratch row stride (floats)
    static_assert(sizeof(SSmem<BM>) >= 4 * 16 * SCR * sizeof(float), "scratch fits");
    float *scr = reinterpret_cast<float *>(&sm) + wave * (16 * SCR);
    const bool vec_ok = (a.R & 3) == 0;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) scr[(4 * lk + r) * SCR + j * 16 + lr] = acc[i][j][r];
      wave_sync();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = (lane >> 4) + 4 * q, c4 = (lane & 15) * 4;
        const int row = m0 + wm * (BM / 2) + i * 16 + rr;
        const int64_t col = n0 + wn * 64 + c4;
        if (row >= a.Kh || col >= a.R) continue;
        const f4 v = *reinterpret_cast<const f4 *>(&scr[rr * SCR + c4]);
        float *dst = Y + int64_t(h * a.Kh + row) * a.R + col;
        if (vec_ok) {
          // R % 4 == 0: col + 3 < R; streaming store (read once by the next pass)
          __builtin_nontemporal_store(v, reinterpret_cast<f4 *>(dst));
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (col + e < a.R) dst[e] = v[e];
        }
      }
      wave_sync();
    }
    if (GEN && hh == 0) __syncthreads();   // the scratch is the next half's tile buffer
  }
}

// ------------------------------- generating + middle-axis pass, fused (3D)
// On 3D grids whose axis-0 pass is fused with the update, the first two
// passes run as one: for a stage field f and an axis-0 node i0 (a "plane")
// a block generates the load, transforms it along axis 2 and then along
// axis 1, and writes the plane once,
//     X1[i1][P2] = sum_p Sh2[h2][j][p] Lf_h2[i1][p]            (P2 = h2 Kh2 + j)
//     Z[P1][P2]  = sum_p Sh1[h1][i][p] fold_h1(X1[.][P2])[p]   (P1 = h1 Kh1 + i)
//     Y[f][i0][P1][P2] = Z[P1][P2],
// so the axis-2 results never travel through HBM.  The output keeps the
// natural axis order (axis 0 outermost); the fused axis-0 pass reads it that
// way.  A block owns one 64-wide chunk of P2 (its Sh2 rows, permuted as below,
// and this half's quadrature table stay in LDS) and walks planes.
//   Axis-2 step: a wave takes the 16 rows i1 = 16 t + x and their mirrors
//   n1 - 1 - (16 t + x) (x = 0..15): the quadrature MFMA leaves lane (x, q) the
//   loads of p = 4 q + r and 16 + 4 q + r (r = 0..3) of each 32-wide k-step,
//   and those eight values are the lane's A operand as they are (k slot
//   8 q + e holds p = 4 q + e for e < 4, 16 + 4 q + e - 4 above), the Sh2
//   rows being staged with the same order of p.  Lane (x, q) then holds
//   X1[p][P2] and X1[n1 - 1 - p][P2] for p = 16 t + 4 q + r, folds them for
//   both halves of axis 1 (as the separate middle pass does) and stores the
//   bf16 hi / lo parts to LDS.
//   Axis-1 step: A = Sh1 (the wave's mode rows, in registers for the whole
//   kernel), B = the folded plane from LDS, three products per k-step in the
//   order of the separate pass.
template <int KH1, int KH2>
struct alignas(16) GmSmem {
  uint16_t S2[2][64][KH2 + 8];         // [hi/lo][P2 of the chunk][p, permuted]
  uint16_t Cg[2][KH2][SGEN_MAX_TERMS + 8];   // [hi/lo][p][m] of this half's table
  uint16_t U[2][2][64][KH1 + 8];       // [h1][hi/lo][P2 of the chunk][p]
  float C1[SGEN_MAX_TERMS][2 * KH1];   // axis-1 factors of the terms, [m][i1] (fp32)
  double Pf[8][2][SGEN_MAX_TERMS];     // [wave][plane parity][m]: coef x axis-0 factor
};

struct GmArgs {
  float *Y;                 // [F][np0][np1][np2]
  int64_t planes;           // F * n0
  int n0, np0;
  int n1, H1, np1;          // axis 1 (Kh1 = np1 / 2)
  int np2;                  // axis 2 (Kh2 = np2 / 2)
  const uint16_t *S1hi, *S1lo, *S2hi, *S2lo;   // [2][Kh][Kh] of axes 1 and 2
  GenSrcF gen;
};

constexpr int GM_NT = 512;

template <int KH1, int KH2>
__global__ __launch_bounds__(GM_NT) void k_split_gen_mid(GmArgs a) {
  constexpr int NCH = KH2 / 32;        // 64-wide chunks of P2 (both halves)
  constexpr int KT1 = KH1 / 32, KT2 = KH2 / 32;
  constexpr int NPAIR = KH1 / 16;      // row tiles (with their mirrors)
  constexpr int WPP = 8 / NPAIR;       // waves per row tile (2 at Kh1 = 64)
  constexpr int JA = 4 / WPP;          // P2 tiles per wave, axis-2 step
  constexpr int IB = KH1 / 64;         // mode tiles per wave, axis-1 step
  static_assert(NPAIR * WPP == 8 && KH2 % 64 == 0, "shape");
  __shared__ GmSmem<KH1, KH2> sm;

  const int chunk = int(blockIdx.x % NCH);
  const int h2 = chunk / (KH2 / 64);
  const int c0 = (chunk % (KH2 / 64)) * 64;        // first j of the chunk in half h2
  const int P2b = h2 * KH2 + c0;
  const int64_t pstride = gridDim.x / NCH;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int M = a.gen.M;

  // Sh2 rows of the chunk, p permuted within each 32-wide k-step
  for (int e = t; e < 2 * 64 * KT2 * 8; e += GM_NT) {
    const int part = e & 1, g8 = (e >> 1) & 3, kp = (e >> 3) % KT2;
    const int n = (e >> 3) / KT2 % 64, hl = (e >> 3) / KT2 / 64;
    const int p = 32 * kp + 16 * part + 4 * g8;      // four p of this piece
    const uint16_t *src = (hl ? a.S2lo : a.S2hi) + (int64_t(h2) * KH2 + c0 + n) * KH2 + p;
    *reinterpret_cast<uint2 *>(&sm.S2[hl][n][32 * kp + 8 * g8 + 4 * part]) =
        *reinterpret_cast<const uint2 *>(src);
  }
  // this half's quadrature table Cf^T (bf16 hi / lo, [p][m])
  const uint16_t *cft = a.gen.Cft;
  for (int e = t; e < 2 * KH2 * 4; e += GM_NT) {
    const int q = e & 3, p = (e >> 2) % KH2, hl = (e >> 2) / KH2;
    const int64_t o = (int64_t(hl) * 2 * KH2 + int64_t(h2) * KH2 + p) * SGEN_MAX_TERMS + 8 * q;
    *reinterpret_cast<uint4 *>(&sm.Cg[hl][p][8 * q]) = *reinterpret_cast<const uint4 *>(cft + o);
  }
  // the wave's rows of Sh1 (axis-1 step A operands), kept for all planes
  const int h1 = wave >> 2;
  bf16x8 ah1[IB][KT1], al1[IB][KT1];
#pragma unroll
  for (int ii = 0; ii < IB; ++ii)
#pragma unroll
    for (int kp = 0; kp < KT1; ++kp) {
      const int64_t o = (int64_t(h1) * KH1 + 16 * ((wave & 3) * IB + ii) + lr) * KH1 + 32 * kp + 8 * lk;
      ah1[ii][kp] = *reinterpret_cast<const bf16x8 *>(a.S1hi + o);
      al1[ii][kp] = *reinterpret_cast<const bf16x8 *>(a.S1lo + o);
    }
  __syncthreads();

  const int rt = wave / WPP;               // row tile of the axis-2 step
  const int ja0 = (wave % WPP) * JA;       // its first P2 tile
  const double *C0 = a.gen.C0, *C1 = a.gen.C1;
  // Row factors of a plane's rows: coef_f[m] C0[m][i0] C1[m][i1].  The axis-1
  // factors (the same for every plane) sit in LDS in fp32 (the products are
  // rounded to fp32 anyway, and split into bf16 hi / lo); each wave keeps the
  // plane's coef x C0 products in an LDS slot of its own, loaded a plane
  // ahead (lane m, before the plane's axis-1 step) and written before its
  // stores: no global load waits at the start of a plane, where it would
  // also wait for the previous plane's stores (memory operations complete
  // in issue order).
  for (int e = t; e < SGEN_MAX_TERMS * 2 * KH1; e += GM_NT) {
    const int m = e / (2 * KH1), i1 = e - m * (2 * KH1);
    sm.C1[m][i1] = (m < M && i1 < a.n1) ? float(C1[int64_t(m) * a.np1 + i1]) : 0.0f;
  }
  const int mlane = lane < M ? lane : M - 1;   // lane m < 32 loads term m
  auto plane_factor = [&](int64_t pl) {       // coef x C0 of term mlane, plane pl
    pl = pl < a.planes ? pl : a.planes - 1;   // (past the last plane: loaded, unused)
    const int64_t fp = pl / a.n0;
    const int ip = int(pl - fp * a.n0);
    return a.gen.coef[fp * M + mlane] * C0[int64_t(mlane) * a.np0 + ip];
  };
  {
    const double pf0 = plane_factor(blockIdx.x / NCH);
    if (lane < SGEN_MAX_TERMS) sm.Pf[wave][0][lane] = pf0;
  }
  __syncthreads();
  int par = 0;
  for (int64_t pl = blockIdx.x / NCH; pl < a.planes; pl += pstride, par ^= 1) {
    const int64_t f = pl / a.n0;
    const int i0 = int(pl - f * a.n0);
    // row factors of the tile's rows and of their mirrors (MFMA B operands)
    bf16x8 rfh[2], rfl[2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
      const int i1 = mi == 0 ? 16 * rt + lr : a.n1 - 1 - (16 * rt + lr);
      f8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int m = 8 * lk + e;
        const double x = sm.Pf[wave][par][m] * double(sm.C1[m][i1]);
        v[e] = m < M ? float(x) : 0.0f;
      }
      split8(v, rfh[mi], rfl[mi]);
    }
    // axis 2: generated loads times the chunk's Sh2 rows
    f4 acc[2][JA];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int j = 0; j < JA; ++j) acc[mi][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kp = 0; kp < KT2; ++kp) {
      bf16x8 gh[2], gl[2];
#pragma unroll
      for (int pt = 0; pt < 2; ++pt) {
        gh[pt] = *reinterpret_cast<const bf16x8 *>(&sm.Cg[0][32 * kp + 16 * pt + lr][8 * lk]);
        gl[pt] = *reinterpret_cast<const bf16x8 *>(&sm.Cg[1][32 * kp + 16 * pt + lr][8 * lk]);
      }
      bf16x8 lh[2], ll[2];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) {
        f8 v;
#pragma unroll
        for (int pt = 0; pt < 2; ++pt) {
          f4 c = f4{0.f, 0.f, 0.f, 0.f};
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gh[pt], rfh[mi], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gh[pt], rfl[mi], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gl[pt], rfh[mi], c, 0, 0, 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) v[4 * pt + r] = c[r];
        }
        split8(v, lh[mi], ll[mi]);
      }
#pragma unroll
      for (int j = 0; j < JA; ++j) {
        const int n = 16 * (ja0 + j) + lr;
        const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(&sm.S2[0][n][32 * kp + 8 * lk]);
        const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(&sm.S2[1][n][32 * kp + 8 * lk]);
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) {
          acc[mi][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lh[mi], bh, acc[mi][j], 0, 0, 0);
          acc[mi][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ll[mi], bh, acc[mi][j], 0, 0, 0);
          acc[mi][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lh[mi], bl, acc[mi][j], 0, 0, 0);
        }
      }
    }
    // fold along axis 1 (p = 16 rt + 4 lk + r: x_p from the tile, x_{n1-1-p}
    // from the mirror tile), split, into the LDS plane
#pragma unroll
    for (int j = 0; j < JA; ++j) {
      f4 u, w;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = 16 * rt + 4 * lk + r;
        const bool has_b = p < a.H1;
        const bool has_a0 = has_b || (p == a.H1 && (a.n1 & 1));
        const float xa = acc[0][j][r], xb = acc[1][j][r];
        u[r] = (has_a0 ? xa : 0.0f) + (has_b ? xb : 0.0f);
        w[r] = (has_b ? xa : 0.0f) + (has_b ? -xb : 0.0f);
      }
      typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
      const bf16x4 uh = __builtin_convertvector(u, bf16x4);
      const bf16x4 ul = __builtin_convertvector(u - __builtin_convertvector(uh, f4), bf16x4);
      const bf16x4 wh = __builtin_convertvector(w, bf16x4);
      const bf16x4 wl = __builtin_convertvector(w - __builtin_convertvector(wh, f4), bf16x4);
      const int n = 16 * (ja0 + j) + lr, p0 = 16 * rt + 4 * lk;
      *reinterpret_cast<bf16x4 *>(&sm.U[0][0][n][p0]) = uh;
      *reinterpret_cast<bf16x4 *>(&sm.U[0][1][n][p0]) = ul;
      *reinterpret_cast<bf16x4 *>(&sm.U[1][0][n][p0]) = wh;
      *reinterpret_cast<bf16x4 *>(&sm.U[1][1][n][p0]) = wl;
    }
    __syncthreads();
    const double pf_next = plane_factor(pl + pstride);

    // axis 1: the wave's mode rows of half h1 times the folded plane
    f4 z[IB][4];
#pragma unroll
    for (int ii = 0; ii < IB; ++ii)
#pragma unroll
      for (int j = 0; j < 4; ++j) z[ii][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kp = 0; kp < KT1; ++kp) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(&sm.U[h1][0][16 * j + lr][32 * kp + 8 * lk]);
        const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(&sm.U[h1][1][16 * j + lr][32 * kp + 8 * lk]);
#pragma unroll
        for (int ii = 0; ii < IB; ++ii) {
          z[ii][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah1[ii][kp], bh, z[ii][j], 0, 0, 0);
          z[ii][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah1[ii][kp], bl, z[ii][j], 0, 0, 0);
          z[ii][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al1[ii][kp], bh, z[ii][j], 0, 0, 0);
        }
      }
    }
    // (read by this wave only, at its next plane)
    if (lane < SGEN_MAX_TERMS) sm.Pf[wave][par ^ 1][lane] = pf_next;
    // lane (x, q) holds modes 4 q + r of the tile at column x of each P2 tile
    float *Yp = a.Y + (f * a.np0 + i0) * int64_t(a.np1) * a.np2 + P2b + lr;
#pragma unroll
    for (int ii = 0; ii < IB; ++ii)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int P1 = h1 * KH1 + 16 * ((wave & 3) * IB + ii) + 4 * lk + r;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          __builtin_nontemporal_store(z[ii][j][r], Yp + int64_t(P1) * a.np2 + 16 * j);
      }
    __syncthreads();   // the plane buffer is the next plane's
  }
}

bool split_gen_mid_supported(pe_grid g, int n_terms) {
  if (g->dim != 3 || g->precision != PE_SPLIT_BF16 || !g->fuse_gen_mid) return false;
  if (!gen_supported_split(g, n_terms) || !fused_update_supported(g)) return false;
  const int k1 = g->ax[1].Kh, k2 = g->ax[2].Kh;
  // (the fused axis-0 pass addresses a field of this layout with 32-bit
  // byte offsets)
  return (k1 == 64 || k1 == 128) && (k2 == 64 || k2 == 128) &&
         g->dofp * int64_t(sizeof(float)) < (int64_t(1) << 31);
}

template <int KH1, int KH2>
static pe_status launch_gen_mid(const GmArgs &a, hipStream_t st) {
  constexpr int NCH = KH2 / 32;
  int dev = 0, cus = 0, per_cu = 0;
  PE_HIP(hipGetDevice(&dev));
  PE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  PE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_split_gen_mid<KH1, KH2>, GM_NT, 0));
  // persistent blocks, as many as fit at once (the LDS of one or two per
  // compute unit), each chunk served by the same number of them
  const int64_t per_chunk =
      std::max<int64_t>(1, std::min<int64_t>(int64_t(cus) * std::max(per_cu, 1) / NCH, a.planes));
  k_split_gen_mid<KH1, KH2><<<dim3(unsigned(per_chunk * NCH)), GM_NT, 0, st>>>(a);
  PE_HIP(hipGetLastError());
  return PE_OK;
}

pe_status split_gen_mid(pe_grid g, int64_t count, const GenSrcF *gen, float *out, hipStream_t st) {
  const Axis &x0 = g->ax[0], &x1 = g->ax[1], &x2 = g->ax[2];
  GmArgs a{};
  a.Y = out;
  a.planes = count * x0.n;
  a.n0 = x0.n;
  a.np0 = x0.np;
  a.n1 = x1.n;
  a.H1 = x1.H;
  a.np1 = x1.np;
  a.np2 = x2.np;
  a.S1hi = x1.d_Shi;
  a.S1lo = x1.d_Slo;
  a.S2hi = x2.d_Shi;
  a.S2lo = x2.d_Slo;
  a.gen = *gen;
  // work: both transforms (three bf16 products each, folded); bytes: one
  // write of the axis-0 nodes' planes plus the per-field coefficients
  const double lines2 = double(count) * x0.n * x1.n, lines1 = double(count) * x0.n * x2.n;
  const double fl = 3.0 * 2.0 *
                    (lines2 * (double((x2.n + 1) / 2) * ((x2.n + 1) / 2) + double(x2.H) * x2.H) +
                     lines1 * (double((x1.n + 1) / 2) * ((x1.n + 1) / 2) + double(x1.H) * x1.H));
  const double bytes = double(count) * x0.n * double(x1.np) * x2.np * sizeof(float) +
                       double(count) * gen->M * sizeof(double);
  TimedScope ts(g, PE_K_DST_LAST, fl, bytes, st);
  if (x1.Kh == 128 && x2.Kh == 128) return launch_gen_mid<128, 128>(a, st);
  if (x1.Kh == 128 && x2.Kh == 64) return launch_gen_mid<128, 64>(a, st);
  if (x1.Kh == 64 && x2.Kh == 128) return launch_gen_mid<64, 128>(a, st);
  if (x1.Kh == 64 && x2.Kh == 64) return launch_gen_mid<64, 64>(a, st);
  return set_error(PE_E_ARG, "internal: no fused generating pass for Kh %d / %d", x1.Kh, x2.Kh);
}

// ------------------------------------------------------------------ dispatch
constexpr int64_t SMAX_BLOCKS = (int64_t(1) << 24) - 1;

template <int BM, bool GEN>
static pe_status launch_split_t(SplitArgs a, int64_t count, hipStream_t st) {
  const int64_t per_f = int64_t(a.tiles_m) * a.tiles_n * (GEN ? 1 : 2);
  if (per_f > SMAX_BLOCKS) return set_error(PE_E_ARG, "internal: split grid too large");
  const int64_t max_f = std::max<int64_t>(1, SMAX_BLOCKS / per_f);
  for (int64_t f0 = 0; f0 < count; f0 += max_f) {
    const int64_t nf = std::min(max_f, count - f0);
    SplitArgs b = a;
    if (!GEN) b.X = a.X + f0 * a.R * a.np;
    b.Y = a.Y + f0 * a.R * a.np;
    if (GEN) b.gen.coef = a.gen.coef + f0 * a.gen.M;
    k_split_pass<BM, GEN><<<dim3(unsigned(nf * per_f)), SNT, 0, st>>>(b);
    PE_HIP(hipGetLastError());
  }
  return PE_OK;
}

template <bool GEN>
static pe_status launch_split(SplitArgs a, int64_t count, hipStream_t st) {
  const int bm = a.Kh >= 128 ? 128 : (a.Kh >= 64 ? 64 : 32);
  a.tiles_m = (a.Kh + bm - 1) / bm;
  a.tiles_n = int((a.R + SBN - 1) / SBN);
  if (bm == 128) return launch_split_t<128, GEN>(a, count, st);
  if (bm == 64) return launch_split_t<64, GEN>(a, count, st);
  return launch_split_t<32, GEN>(a, count, st);
}

bool gen_supported_split(pe_grid g, int n_terms) {
  return n_terms >= 1 && n_terms <= SGEN_MAX_TERMS;
}

// Cft[s][h][p][m] (s = 0: bf16 hi, 1: lo) of Cf[h][m][p], zero for m >= M
__global__ void k_split_gen_table(const double *Cf, int M, int Kh, uint16_t *Cft) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * Kh * SGEN_MAX_TERMS) return;
  const int m = i % SGEN_MAX_TERMS, p = (i / SGEN_MAX_TERMS) % Kh, h = i / (SGEN_MAX_TERMS * Kh);
  const float v = m < M ? float(Cf[(int64_t(h) * M + m) * Kh + p]) : 0.0f;
  const __bf16 hv = static_cast<__bf16>(v);
  const __bf16 lv = static_cast<__bf16>(v - static_cast<float>(hv));
  Cft[i] = __builtin_bit_cast(uint16_t, hv);
  Cft[2 * Kh * SGEN_MAX_TERMS + i] = __builtin_bit_cast(uint16_t, lv);
}

size_t split_gen_table_bytes(pe_grid g) {
  return 2 * 2 * size_t(g->ax[g->dim - 1].Kh) * SGEN_MAX_TERMS * sizeof(uint16_t);
}

pe_status split_gen_table(pe_grid g, const double *Cf, int M, uint16_t *Cft, hipStream_t st) {
  if (M < 1 || M > SGEN_MAX_TERMS)
    return set_error(PE_E_ARG, "internal: %d terms for the split generating table", M);
  const int Kh = g->ax[g->dim - 1].Kh;
  const int total = 2 * Kh * SGEN_MAX_TERMS;
  k_split_gen_table<<<(total + 255) / 256, 256, 0, st>>>(Cf, M, Kh, Cft);
  PE_HIP(hipGetLastError());
  return PE_OK;
}

pe_status dst_fields_split(pe_grid g, int64_t count, const GenSrcF *gen, float *buf0, float *buf1,
                           float **result, hipStream_t st, int stop_axis, bool *axis0_outer) {
  if (!g->ax[0].d_Shi) return set_error(PE_E_UNSUPPORTED, "grid has no split-bf16 tables");
  if (axis0_outer) *axis0_outer = false;
  if (gen && stop_axis == 1 && axis0_outer && split_gen_mid_supported(g, gen->M)) {
    if (!gen->Cft) return set_error(PE_E_ARG, "internal: split generating pass without its table");
    PE_TRY(split_gen_mid(g, count, gen, buf0, st));
    *result = buf0;
    *axis0_outer = true;
    return PE_OK;
  }
  float *in = buf0, *out = buf1;
  const int d = g->dim;
  // axis contracted by pass q: d-1, d-2, ..., 0 (rotating layout)
  for (int q = 0; q < d - stop_axis; ++q) {
    const int ax_i = d - 1 - q;
    const Axis &ax = g->ax[ax_i];
    const int64_t R = g->dofp / ax.np;
    double lines = double(count) * double(g->dof) / ax.n;
    // three bf16 products of the folded pass
    double fl = 3.0 * 2.0 * lines * (double((ax.n + 1) / 2) * ((ax.n + 1) / 2) + double(ax.H) * ax.H);
    const bool gen_pass = gen && q == 0;   // writes only (plus per-field coefficients)
    const double bytes = (gen_pass ? 1.0 : 2.0) * double(count) * double(g->dof) * sizeof(float) +
                         (gen_pass ? double(count) * gen->M * sizeof(double) : 0.0);
    TimedScope ts(g, q == 0 ? PE_K_DST_LAST : PE_K_DST_MID, fl, bytes, st);
    SplitArgs a{};
    a.X = in;
    a.Y = out;
    a.R = R;
    a.np = ax.np;
    a.n = ax.n;
    a.H = ax.H;
    a.Kh = ax.Kh;
    a.Shi = ax.d_Shi;
    a.Slo = ax.d_Slo;
    a.d = d;
    a.np0 = g->ax[0].np;
    a.np1 = d >= 2 ? g->ax[1].np : 1;
    if (q == 0 && gen) {
      if (!gen->Cft) return set_error(PE_E_ARG, "internal: split generating pass without its table");
      a.gen = *gen;
      PE_TRY(launch_split<true>(a, count, st));
    } else {
      PE_TRY(launch_split<false>(a, count, st));
    }
    std::swap(in, out);
  }
  *result = in;
  return PE_OK;
}

}  // namespace pe
