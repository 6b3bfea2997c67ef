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
// evaluated in fp32 from the FP64 tables.
//
// Block: 256 threads = 4 waves (2 x 2), tile BM (modes) x 128 (rows r),
// k-step 32, single LDS buffer with register prefetch.
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
constexpr int SGEN_MAX_TERMS = 32;
constexpr int SGEN_MAX_CF = 8192;   // floats of one folded half table kept in LDS

typedef float f8 __attribute__((ext_vector_type(8)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));   // dword-aligned loads
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

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

template <int BM, int GM>
__global__ __launch_bounds__(SNT) void k_split_pass(SplitArgs a) {
  constexpr bool GEN = GM > 0;
  constexpr int TM = BM / 32;                 // MFMA tiles per wave along the modes
  constexpr int TN = 4;                       // ... along r (64 per wave)
  constexpr int ACH = BM * (SKB / 8) / SNT;   // 16-byte A chunks per thread per array (2, 1, ..)
  constexpr int EB = 16;                      // p values of one B row per thread
  static_assert(ACH >= 1 || BM == 32, "A chunk mapping");
  __shared__ SSmem<BM> sm;
  extern __shared__ float cf_lds[];           // GEN: [M][Kh] folded table of this half

  int64_t bid = blockIdx.x;
  {
    const int64_t nb = gridDim.x;
    if (nb % 8 == 0) bid = (bid % 8) * (nb / 8) + bid / 8;   // one field's tiles on one XCD
  }
  // the two halves of a tile read the same rows: run them back to back
  const int h = int(bid % 2);
  bid /= 2;
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

  float rf[GEN ? GM : 1];
  if constexpr (GEN) {
    const int M = a.gen.M;
    const int ncf = M * a.Kh;
    const double *cf_src = a.gen.Cf + int64_t(h) * ncf;
    for (int e = t; e < ncf; e += SNT) cf_lds[e] = float(cf_src[e]);
    int j0 = 0, j1 = 0;
    if (a.d == 2) j0 = int(grc);
    if (a.d == 3) {
      j0 = int(grc / a.np1);
      j1 = int(grc - int64_t(j0) * a.np1);
    }
    const double *C0 = a.d >= 2 ? a.gen.C0 : nullptr;
    const double *C1 = a.d == 3 ? a.gen.C1 : nullptr;
#pragma unroll
    for (int m = 0; m < GM; ++m) {
      const int mm = m < M ? m : M - 1;
      double v = a.gen.coef[f * M + mm];
      if (C0) v *= C0[int64_t(mm) * a.np0 + j0];
      if (C1) v *= C1[int64_t(mm) * a.np1 + j1];
      rf[m] = (m < M && brow_ok) ? float(v) : 0.0f;
    }
    __syncthreads();
  }

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
#pragma unroll
    for (int g8 = 0; g8 < EB / 8; ++g8) {
      f8 v;
#pragma unroll
      for (int e8 = 0; e8 < 8; ++e8) {
        const int e = 8 * g8 + e8;
        const int p = k0 + pb0 + e;
        float x;
        if constexpr (GEN) {
          const int Mm1 = a.gen.M - 1;
          x = 0.0f;
#pragma unroll
          for (int m = 0; m < GM; ++m) x += rf[m] * cf_lds[(m < Mm1 ? m : Mm1) * a.Kh + p];
        } else {
          const bool has_b = p < a.H;
          const bool has_a = has_b || (h == 0 && p == a.H && (a.n & 1));
          x = (has_a ? pxa[e] : 0.0f) + (has_b ? (h == 0 ? pxb[e] : -pxb[e]) : 0.0f);
          x = brow_ok ? x : 0.0f;
        }
        v[e8] = x;
      }
      bf16x8 hi, lo;
      split8(v, hi, lo);
      *reinterpret_cast<bf16x8 *>(&sm.Bhi[rb][pb0 + 8 * g8]) = hi;
      *reinterpret_cast<bf16x8 *>(&sm.Blo[rb][pb0 + 8 * g8]) = lo;
    }
  };

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

  float *Y = a.Y + f * int64_t(a.np) * a.R;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t col = n0 + wn * 64 + j * 16 + lr;
      if (col >= a.R) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * (BM / 2) + i * 16 + 4 * lk + r;
        if (row < a.Kh) Y[int64_t(h * a.Kh + row) * a.R + col] = acc[i][j][r];
      }
    }
}

// ------------------------------------------------------------------ dispatch
constexpr int64_t SMAX_BLOCKS = (int64_t(1) << 24) - 1;

template <int BM, int GM>
static pe_status launch_split_t(SplitArgs a, int64_t count, hipStream_t st) {
  const int64_t per_f = int64_t(a.tiles_m) * a.tiles_n * 2;
  if (per_f > SMAX_BLOCKS) return set_error(PE_E_ARG, "internal: split grid too large");
  const int64_t max_f = std::max<int64_t>(1, SMAX_BLOCKS / per_f);
  size_t dyn = GM > 0 ? sizeof(float) * size_t(a.gen.M) * a.Kh : 0;
  for (int64_t f0 = 0; f0 < count; f0 += max_f) {
    const int64_t nf = std::min(max_f, count - f0);
    SplitArgs b = a;
    if (GM == 0) b.X = a.X + f0 * a.R * a.np;
    b.Y = a.Y + f0 * a.R * a.np;
    if (GM > 0) b.gen.coef = a.gen.coef + f0 * a.gen.M;
    k_split_pass<BM, GM><<<dim3(unsigned(nf * per_f)), SNT, dyn, st>>>(b);
    PE_HIP(hipGetLastError());
  }
  return PE_OK;
}

template <int GM>
static pe_status launch_split(SplitArgs a, int64_t count, hipStream_t st) {
  const int bm = a.Kh >= 128 ? 128 : (a.Kh >= 64 ? 64 : 32);
  a.tiles_m = (a.Kh + bm - 1) / bm;
  a.tiles_n = int((a.R + SBN - 1) / SBN);
  if (bm == 128) return launch_split_t<128, GM>(a, count, st);
  if (bm == 64) return launch_split_t<64, GM>(a, count, st);
  return launch_split_t<32, GM>(a, count, st);
}

bool gen_supported_split(pe_grid g, int n_terms) {
  const Axis &last = g->ax[g->dim - 1];
  return n_terms >= 1 && n_terms <= SGEN_MAX_TERMS && int64_t(n_terms) * last.Kh <= SGEN_MAX_CF;
}

pe_status dst_fields_split(pe_grid g, int64_t count, const GenSrcF *gen, float *buf0, float *buf1,
                           float **result, hipStream_t st) {
  if (!g->ax[0].d_Shi) return set_error(PE_E_UNSUPPORTED, "grid has no split-bf16 tables");
  float *in = buf0, *out = buf1;
  const int d = g->dim;
  // axis contracted by pass q: d-1, d-2, ..., 0 (rotating layout)
  for (int q = 0; q < d; ++q) {
    const int ax_i = d - 1 - q;
    const Axis &ax = g->ax[ax_i];
    const int64_t R = g->dofp / ax.np;
    double lines = double(count) * double(g->dof) / ax.n;
    // three bf16 products of the folded pass
    double fl = 3.0 * 2.0 * lines * (double((ax.n + 1) / 2) * ((ax.n + 1) / 2) + double(ax.H) * ax.H);
    TimedScope ts(g, q == 0 ? PE_K_DST_LAST : PE_K_DST_MID, fl,
                  2.0 * double(count) * double(g->dof) * sizeof(float), st);
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
      a.gen = *gen;
      if (gen->M <= 8)
        PE_TRY(launch_split<8>(a, count, st));
      else if (gen->M <= 16)
        PE_TRY(launch_split<16>(a, count, st));
      else if (gen->M <= 24)
        PE_TRY(launch_split<24>(a, count, st));
      else
        PE_TRY(launch_split<32>(a, count, st));
    } else {
      PE_TRY(launch_split<0>(a, count, st));
    }
    std::swap(in, out);
  }
  *result = in;
  return PE_OK;
}

}  // namespace pe
