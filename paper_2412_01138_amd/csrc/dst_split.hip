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

__device__ inline uint16_t bf16_rn(float x) {
  uint32_t u = __float_as_uint(x);
  return uint16_t((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_val(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

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
struct SSmem {
  uint16_t Ahi[BM][SLD], Alo[BM][SLD];
  uint16_t Bhi[SBN][SLD], Blo[SBN][SLD];
};

template <int BM, int GM>
__global__ __launch_bounds__(SNT) void k_split_pass(SplitArgs a) {
  constexpr bool GEN = GM > 0;
  constexpr int TM = BM / 32;                 // MFMA tiles per wave along the modes
  constexpr int TN = 4;                       // ... along r (64 per wave)
  constexpr int TPR_A = SNT / BM;             // threads per A row
  constexpr int EA = SKB / TPR_A;             // bf16 of one A row per thread (4, 8, 16)
  constexpr int EB = 16;                      // p values of one B row per thread
  __shared__ SSmem<BM> sm;
  extern __shared__ float cf_lds[];           // GEN: [M][Kh] folded table of this half

  int64_t bid = blockIdx.x;
  {
    const int64_t nb = gridDim.x;
    if (nb % 8 == 0) bid = (bid % 8) * (nb / 8) + bid / 8;   // one field's tiles on one XCD
  }
  const int tn = int(bid % a.tiles_n);
  bid /= a.tiles_n;
  const int tm = int(bid % a.tiles_m);
  bid /= a.tiles_m;
  const int h = int(bid % 2);
  const int64_t f = bid / 2;
  const int m0 = tm * BM;
  const int64_t n0 = int64_t(tn) * SBN;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1, lr = lane & 15, lk = lane >> 4;

  // A-tile role: row ia, bf16 columns ka0 .. ka0 + EA
  const int ia = t / TPR_A, ka0 = (t % TPR_A) * EA;
  const bool arow_ok = m0 + ia < a.Kh;
  const int64_t arow = int64_t(h) * a.Kh + (arow_ok ? m0 + ia : a.Kh - 1);
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
  uint16_t pah[EA], pal[EA];
  float pxa[GEN ? 1 : EB], pxb[GEN ? 1 : EB];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      pah[e] = a.Shi[arow * a.Kh + k0 + ka0 + e];
      pal[e] = a.Slo[arow * a.Kh + k0 + ka0 + e];
    }
    if constexpr (!GEN) {
#pragma unroll
      for (int e = 0; e < EB; ++e) {
        const int p = k0 + pb0 + e;
        const int pa = p < a.n ? p : a.n - 1;
        const int pm = a.n - 1 - p > 0 ? a.n - 1 - p : 0;
        pxa[e] = xrow[pa];
        pxb[e] = xrow[pm];
      }
    }
  };
  auto store = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      sm.Ahi[ia][ka0 + e] = arow_ok ? pah[e] : uint16_t(0);
      sm.Alo[ia][ka0 + e] = arow_ok ? pal[e] : uint16_t(0);
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int p = k0 + pb0 + e;
      float v;
      if constexpr (GEN) {
        const int Mm1 = a.gen.M - 1;
        v = 0.0f;
#pragma unroll
        for (int m = 0; m < GM; ++m) v += rf[m] * cf_lds[(m < Mm1 ? m : Mm1) * a.Kh + p];
      } else {
        const bool has_a = p < a.H || (h == 0 && p == a.H && (a.n & 1));
        const bool has_b = p < a.H;
        v = (has_a ? pxa[e] : 0.0f) + (has_b ? (h == 0 ? pxb[e] : -pxb[e]) : 0.0f);
        v = brow_ok ? v : 0.0f;
      }
      const uint16_t hi = bf16_rn(v);
      const uint16_t lo = bf16_rn(v - bf16_val(hi));
      sm.Bhi[rb][pb0 + e] = hi;
      sm.Blo[rb][pb0 + e] = lo;
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
