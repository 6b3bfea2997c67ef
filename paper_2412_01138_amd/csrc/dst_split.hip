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
                           float **result, hipStream_t st, int stop_axis) {
  if (!g->ax[0].d_Shi) return set_error(PE_E_UNSUPPORTED, "grid has no split-bf16 tables");
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
