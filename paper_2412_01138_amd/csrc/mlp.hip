// Per-mode coarse-correction network: bf16 weights, fp32 accumulation, all
// layer products on the matrix cores (v_mfma_f32_16x16x32_bf16).
//
// NN: x[12] -> 64 -> 64 -> 64 (GELU: x Phi(x)) -> 1 (linear), parameters
// W1[12][64] b1 W2[64][64] b2 W3[64][64] b3 w4[64] b4 (W[in][out]).
//
// Layer l is C = A W on 16-row groups: the MFMA A operand is the activation
// tile (row-major, k contiguous), the B operand the transposed weights
// Wt[out][in] (k contiguous).  The inputs enter as bf16 hi + lo halves in the
// 32-wide first-layer tile (W1t repeats its 12 columns), so layer 1 sees the
// fp32 features.  Backward:
//   dA_{l-1} = dZ_l W_l^T  (B operand = W_l[in][out] row-major),
//   dW_l    += A_{l-1}^T dZ_l (A operand = A^T[in][row], B = dZ^T[out][row]),
// with the row sums of the weight gradients taken on the matrix cores; every
// block writes its partial gradient, a second kernel adds the partials in a
// fixed order (bitwise-repeatable gradients).
//
// The learned correction (k_mlp_correct) gives each block 64 consecutive
// modes and walks the slices, one slice per wave at a time: per-mode inputs
// (z-features, term spectra) are formed once per block, the per-slice ones
// from the slice's sample-coefficient table.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "learned_feat.h"

namespace pe {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NIN = PE_MLP_INPUTS;   // 12
constexpr int KIN = 32;              // padded input width (MFMA k-step)
constexpr int WD = PE_MLP_WIDTH;     // 64
constexpr int NP = PE_MLP_PARAMS;    // 9217
constexpr int OW1 = 0, OB1 = OW1 + NIN * WD, OW2 = OB1 + WD, OB2 = OW2 + WD * WD, OW3 = OB2 + WD,
              OB3 = OW3 + WD * WD, OW4 = OB3 + WD, OB4 = OW4 + WD;
static_assert(OB4 + 1 == NP, "parameter layout");
static_assert(2 * NIN <= KIN, "hi/lo inputs fit the first-layer tile");

// packed bf16 weights (global): W1t[64][32], W2t[64][64], W3t[64][64],
// W2n[64][64], W3n[64][64], w4[64]
constexpr int PW1T = 0, PW2T = PW1T + WD * KIN, PW3T = PW2T + WD * WD, PW2N = PW3T + WD * WD,
              PW3N = PW2N + WD * WD, PW4 = PW3N + WD * WD, PTOT = PW4 + WD;

constexpr int LD1 = KIN + 8;   // LDS row stride (bf16) of 32-wide tiles
constexpr int LD2 = WD + 8;    // ... of 64-wide tiles (16-byte pad: conflict-free b128 reads)
constexpr int ROWS = 64;       // rows per tile
constexpr int MNT = 256;
constexpr int MAX_TRAIN_BLOCKS = 256;

}  // namespace pe

struct pe_mlp_s {
  float *master = nullptr;     // [NP]
  float *m = nullptr, *v = nullptr;
  uint16_t *packed = nullptr;  // [PTOT] bf16
  float *partials = nullptr;   // [MAX_TRAIN_BLOCKS][NP]
  float *loss_part = nullptr;  // [MAX_TRAIN_BLOCKS]
  float *grad = nullptr;       // [NP]
  int *flag = nullptr;         // non-finite output seen by the last correction
  int64_t step = 0;
};

namespace pe {

// round to nearest even (hardware conversion)
__device__ inline uint16_t f2bf(float x) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(x)); }
__device__ inline float bf2f(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

// Phi(-|x|) = erfc(|x|/sqrt 2)/2 by the rational approximation of
// Abramowitz & Stegun 7.1.26 (absolute error of erf below 1.5e-7), and
// e = exp(-x^2/2), shared with the normal density.
__device__ inline float normal_tail(float x, float &e) {
  const float u = fabsf(x) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, u, 1.0f));
  const float poly =
      t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f +
                                                                         t * 1.061405429f))));
  e = __expf(-u * u);
  return 0.5f * poly * e;
}
__device__ inline float gelu(float x) {
  float e;
  const float tail = normal_tail(x, e);
  return x * (x >= 0.f ? 1.0f - tail : tail);
}
__device__ inline float gelu_d(float x) {
  float e;
  const float tail = normal_tail(x, e);
  return (x >= 0.f ? 1.0f - tail : tail) + x * 0.39894228040143268f * e;
}

// LDS ordering between lanes of one wave (no cross-wave exchange)
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave: C[16][64] += A[16][K] * Bt[64][K]^T.  Lane (lr, lk) receives
// rows 4*lk + r, columns 16*j + lr.
template <int K>
__device__ inline void mm16x64(const uint16_t *A, int lda, const uint16_t *Bt, int ldb,
                               f4 (&acc)[4], int lr, int lk) {
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 32) {
    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(A + lr * lda + k0 + lk * 8);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bf16x8 b = *reinterpret_cast<const bf16x8 *>(Bt + (j * 16 + lr) * ldb + k0 + lk * 8);
      acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
    }
  }
}

// forward weights in LDS
struct alignas(16) FwdWeights {
  uint16_t W1t[WD][LD1];
  uint16_t W2t[WD][LD2], W3t[WD][LD2];
  float w4[WD], b1[WD], b2[WD], b3[WD], b4;
};

// forward + the transposed products of the backward pass
struct alignas(16) WeightsLds {
  FwdWeights f;
  uint16_t W2n[WD][LD2], W3n[WD][LD2];
};

__device__ inline void load_fwd_weights(FwdWeights &w, const uint16_t *packed,
                                        const float *master) {
  for (int e = threadIdx.x; e < WD * KIN; e += MNT) w.W1t[e / KIN][e % KIN] = packed[PW1T + e];
  for (int e = threadIdx.x; e < WD * WD; e += MNT) {
    const int r = e / WD, c = e % WD;
    w.W2t[r][c] = packed[PW2T + e];
    w.W3t[r][c] = packed[PW3T + e];
  }
  for (int e = threadIdx.x; e < WD; e += MNT) {
    w.w4[e] = bf2f(packed[PW4 + e]);
    w.b1[e] = master[OB1 + e];
    w.b2[e] = master[OB2 + e];
    w.b3[e] = master[OB3 + e];
  }
  if (threadIdx.x == 0) w.b4 = master[OB4];
}

__device__ inline void load_weights(WeightsLds &w, const uint16_t *packed, const float *master) {
  load_fwd_weights(w.f, packed, master);
  for (int e = threadIdx.x; e < WD * WD; e += MNT) {
    const int r = e / WD, c = e % WD;
    w.W2n[r][c] = packed[PW2N + e];
    w.W3n[r][c] = packed[PW3N + e];
  }
}

// First-layer input row: x = hi + lo (both bf16) in columns [0, 12) and
// [12, 24), zeros after (x may be null when !ok: a zero row).
__device__ inline void put_input(uint16_t *X, const float *x, bool ok) {
  uint32_t v[KIN / 2];
  uint16_t hi[NIN], lo[NIN];
  for (int i = 0; i < NIN; ++i) {
    const float f = ok ? x[i] : 0.f;
    hi[i] = f2bf(f);
    lo[i] = f2bf(f - bf2f(hi[i]));
  }
  for (int i = 0; i < KIN / 2; ++i) {
    const int e0 = 2 * i, e1 = 2 * i + 1;
    const uint16_t a = e0 < NIN ? hi[e0] : e0 < 2 * NIN ? lo[e0 - NIN] : uint16_t(0);
    const uint16_t b = e1 < NIN ? hi[e1] : e1 < 2 * NIN ? lo[e1 - NIN] : uint16_t(0);
    v[i] = uint32_t(a) | (uint32_t(b) << 16);
  }
  uint4 *dst = reinterpret_cast<uint4 *>(X);
  for (int q = 0; q < KIN / 8; ++q) dst[q] = uint4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
}

// Rows X[0..15] through the network (one wave; H1, H2: 16-row scratch).
// On return every lane of row group lk holds y - b4 of rows 4*lk + r in ys[r].
__device__ inline void forward16(const FwdWeights &w, const uint16_t *X, uint16_t (*H1)[LD2],
                                 uint16_t (*H2)[LD2], int lr, int lk, float (&ys)[4]) {
  f4 acc[4];
  for (int j = 0; j < 4; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
  mm16x64<KIN>(X, LD1, &w.W1t[0][0], LD1, acc, lr, lk);
  for (int j = 0; j < 4; ++j)
    for (int r = 0; r < 4; ++r) H1[4 * lk + r][j * 16 + lr] = f2bf(gelu(acc[j][r] + w.b1[j * 16 + lr]));
  wave_sync();
  for (int j = 0; j < 4; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
  mm16x64<WD>(&H1[0][0], LD2, &w.W2t[0][0], LD2, acc, lr, lk);
  for (int j = 0; j < 4; ++j)
    for (int r = 0; r < 4; ++r) H2[4 * lk + r][j * 16 + lr] = f2bf(gelu(acc[j][r] + w.b2[j * 16 + lr]));
  wave_sync();
  for (int j = 0; j < 4; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
  mm16x64<WD>(&H2[0][0], LD2, &w.W3t[0][0], LD2, acc, lr, lk);
  for (int r = 0; r < 4; ++r) ys[r] = 0.f;
  for (int j = 0; j < 4; ++j)
    for (int r = 0; r < 4; ++r) ys[r] += gelu(acc[j][r] + w.b3[j * 16 + lr]) * w.w4[j * 16 + lr];
  for (int r = 0; r < 4; ++r)
    for (int off = 8; off >= 1; off >>= 1) ys[r] += __shfl_xor(ys[r], off, 16);
}

// ------------------------------------------------- inference on given rows
struct alignas(16) InferWave {
  uint16_t X[16][LD1];
  uint16_t H1[16][LD2], H2[16][LD2];
};

// y[r] = NN(x[r]); each wave takes 16-row groups in turn.
__global__ __launch_bounds__(MNT) void k_mlp_infer(const uint16_t *packed, const float *master,
                                                   const float *x, int64_t rows, float *y) {
  __shared__ FwdWeights w;
  __shared__ InferWave iw[MNT / 64];
  load_fwd_weights(w, packed, master);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lr = lane & 15, lk = lane >> 4;
  InferWave &W = iw[wave];
  const int64_t groups = (rows + 15) / 16;
  for (int64_t gi = int64_t(blockIdx.x) * (MNT / 64) + wave; gi < groups;
       gi += int64_t(gridDim.x) * (MNT / 64)) {
    if (lane < 16) {
      const int64_t row = gi * 16 + lane;
      const bool ok = row < rows;
      put_input(&W.X[lane][0], ok ? x + row * NIN : nullptr, ok);
    }
    wave_sync();
    float ys[4];
    forward16(w, &W.X[0][0], W.H1, W.H2, lr, lk, ys);
    if (lr == 0)
      for (int r = 0; r < 4; ++r) {
        const int64_t row = gi * 16 + 4 * lk + r;
        if (row < rows) y[row] = ys[r] + w.b4;
      }
    wave_sync();
  }
}

// --------------------------------------------------- learned correction
struct CorrArgs {
  int d, n0, n1, n2, M, N;
  const double *lam0, *lam1, *lam2;
  const double *sp0, *sp1, *sp2;   // per-axis term spectra [M][n_a]
  const double *Cp;                // [N][8][M] sample-coefficient tables
  double D, dT;
  int64_t dof;
  int ktiles, nsplit;              // grid = ktiles x nsplit blocks
  void *corr;                      // [N][DOF] state dtype
  int fp64;
  int *bad;                        // set to 1 on a non-finite output
};

struct alignas(16) CorrWave {
  uint16_t X[ROWS][LD1];
  uint16_t H1[16][LD2], H2[16][LD2];
  float y[ROWS];
};

constexpr size_t lds_align(size_t b) { return (b + 15) & ~size_t(15); }
constexpr size_t CORR_LDS_FIXED = lds_align(sizeof(FwdWeights)) + (MNT / 64) * sizeof(CorrWave);

// Block (kt, sg): modes kt*64 .. kt*64+63; wave w takes slices
// n = 4 sg + w, 4 sg + w + 4 nsplit, ...  (no block-wide barrier in the loop:
// waves may run different slice counts).
__global__ __launch_bounds__(MNT) void k_mlp_correct(const uint16_t *packed, const float *master,
                                                     CorrArgs a) {
  extern __shared__ __align__(16) char lds[];
  FwdWeights &w = *reinterpret_cast<FwdWeights *>(lds);
  CorrWave *cw = reinterpret_cast<CorrWave *>(lds + lds_align(sizeof(FwdWeights)));
  double *Gs = reinterpret_cast<double *>(lds + CORR_LDS_FIXED);   // [M][64]
  load_fwd_weights(w, packed, master);
  const int t = threadIdx.x, lane = t & 63, lr = lane & 15, lk = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int kt = int(blockIdx.x % unsigned(a.ktiles));
  const int sg = int(blockIdx.x / unsigned(a.ktiles));
  for (int e = t; e < a.M * 64; e += MNT) {
    const int m = e >> 6;
    const int64_t kk = int64_t(kt) * 64 + (e & 63);
    double G = 0.0;
    if (kk < a.dof) {
      int k0 = 0, k1 = 0, k2 = 0;
      if (a.d == 1) {
        k0 = int(kk);
      } else if (a.d == 2) {
        k0 = int(kk / a.n1);
        k1 = int(kk % a.n1);
      } else {
        k2 = int(kk % a.n2);
        const int64_t r = kk / a.n2;
        k0 = int(r / a.n1);
        k1 = int(r % a.n1);
      }
      G = a.sp0[int64_t(m) * a.n0 + k0];
      if (a.d > 1) G *= a.sp1[int64_t(m) * a.n1 + k1];
      if (a.d > 2) G *= a.sp2[int64_t(m) * a.n2 + k2];
    }
    Gs[e] = G;
  }
  const int64_t k = int64_t(kt) * 64 + lane;
  const bool kv = k < a.dof;
  float zf[4] = {0.f, 0.f, 0.f, 0.f};
  if (kv) z_features(a.D * mode_lambda(a.d, a.n1, a.n2, a.lam0, a.lam1, a.lam2, k) * a.dT, zf);
  __syncthreads();
  CorrWave &W = cw[wave];
  for (int n = 4 * sg + wave; n < a.N; n += 4 * a.nsplit) {
    const double *cp = a.Cp + int64_t(n) * PE_MLP_SAMPLES * a.M;
    double c[PE_MLP_SAMPLES];
    for (int i = 0; i < PE_MLP_SAMPLES; ++i) c[i] = 0.0;
    for (int m = 0; m < a.M; ++m) {
      const double G = Gs[m * 64 + lane];
      for (int i = 0; i < PE_MLP_SAMPLES; ++i) c[i] += cp[i * a.M + m] * G;
    }
    float x[NIN];
    for (int i = 0; i < 4; ++i) x[i] = zf[i];
    double s;
    coeff_features(c, x, s);
    put_input(&W.X[lane][0], x, kv);
    wave_sync();
    for (int g = 0; g < ROWS / 16; ++g) {
      float ys[4];
      forward16(w, &W.X[16 * g][0], W.H1, W.H2, lr, lk, ys);
      if (lr == 0)
        for (int r = 0; r < 4; ++r) W.y[16 * g + 4 * lk + r] = ys[r] + w.b4;
      wave_sync();
    }
    if (kv) {
      double dlt = s > 0.0 ? s * a.dT * double(W.y[lane]) : 0.0;
      if (!isfinite(dlt)) {
        *a.bad = 1;
        dlt = 0.0;
      }
      const int64_t o = int64_t(n) * a.dof + k;
      if (a.fp64)
        static_cast<double *>(a.corr)[o] = dlt;
      else
        static_cast<float *>(a.corr)[o] = float(dlt);
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------- training
struct alignas(16) TrainLds {
  WeightsLds w;
  uint16_t X[ROWS][LD1];
  uint16_t XT[KIN][LD2];
  uint16_t H1[ROWS][LD2], H2[ROWS][LD2];
  uint16_t H1T[WD][LD2], H2T[WD][LD2];
  uint16_t dZ3[ROWS][LD2], dZ2[ROWS][LD2];
  uint16_t dZ3T[WD][LD2], dZ2T[WD][LD2], dZ1T[WD][LD2];
  float tgt[ROWS];
  float red[4][4][WD];   // [wave][quantity][col] bias/w4 partials
  float lossw[4];
};

__global__ __launch_bounds__(MNT) void k_mlp_train(const uint16_t *packed, const float *master,
                                                   const float *x, const float *tg, int64_t rows,
                                                   int64_t rows_per_block, float *partials,
                                                   float *loss_part) {
  extern __shared__ __align__(16) char smem_raw[];
  TrainLds &s = *reinterpret_cast<TrainLds *>(smem_raw);
  load_weights(s.w, packed, master);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, lr = lane & 15, lk = lane >> 4;
  const int r0 = wave * 16;
  const int64_t beg = int64_t(blockIdx.x) * rows_per_block;
  const int64_t end = beg + rows_per_block < rows ? beg + rows_per_block : rows;
  const float inv_b = 2.0f / float(rows);

  f4 gW1[4], gW2[4], gW3[4];
  for (int j = 0; j < 4; ++j) gW1[j] = gW2[j] = gW3[j] = f4{0.f, 0.f, 0.f, 0.f};
  float gb1[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0}, gb3[4] = {0, 0, 0, 0}, gw4[4] = {0, 0, 0, 0};
  float gb4 = 0.f, lsum = 0.f;

  for (int64_t base = beg; base < end; base += ROWS) {
    __syncthreads();
    if (t < ROWS) {
      const int64_t row = base + t;
      const bool ok = row < end;
      put_input(&s.X[t][0], ok ? x + row * NIN : nullptr, ok);
      // the weight gradient of layer 1 uses the hi part of the inputs
      for (int i = 0; i < KIN; ++i) s.XT[i][t] = i < NIN ? s.X[t][i] : uint16_t(0);
      s.tgt[t] = ok ? tg[row] : 0.f;
    }
    __syncthreads();
    f4 z1[4], z2[4], z3[4];
    for (int j = 0; j < 4; ++j) z1[j] = z2[j] = z3[j] = f4{0.f, 0.f, 0.f, 0.f};
    mm16x64<KIN>(&s.X[r0][0], LD1, &s.w.f.W1t[0][0], LD1, z1, lr, lk);
    for (int j = 0; j < 4; ++j)
      for (int r = 0; r < 4; ++r) {
        z1[j][r] += s.w.f.b1[j * 16 + lr];
        const uint16_t h = f2bf(gelu(z1[j][r]));
        s.H1[r0 + 4 * lk + r][j * 16 + lr] = h;
        s.H1T[j * 16 + lr][r0 + 4 * lk + r] = h;
      }
    __syncthreads();
    mm16x64<WD>(&s.H1[r0][0], LD2, &s.w.f.W2t[0][0], LD2, z2, lr, lk);
    for (int j = 0; j < 4; ++j)
      for (int r = 0; r < 4; ++r) {
        z2[j][r] += s.w.f.b2[j * 16 + lr];
        const uint16_t h = f2bf(gelu(z2[j][r]));
        s.H2[r0 + 4 * lk + r][j * 16 + lr] = h;
        s.H2T[j * 16 + lr][r0 + 4 * lk + r] = h;
      }
    __syncthreads();
    mm16x64<WD>(&s.H2[r0][0], LD2, &s.w.f.W3t[0][0], LD2, z3, lr, lk);
    float h3[4][4];
    float ys[4] = {0.f, 0.f, 0.f, 0.f};
    for (int j = 0; j < 4; ++j)
      for (int r = 0; r < 4; ++r) {
        z3[j][r] += s.w.f.b3[j * 16 + lr];
        h3[j][r] = gelu(z3[j][r]);
        ys[r] += h3[j][r] * s.w.f.w4[j * 16 + lr];
      }
    for (int r = 0; r < 4; ++r)
      for (int off = 8; off >= 1; off >>= 1) ys[r] += __shfl_xor(ys[r], off, 16);
    // dL/dy per row (zero for padding rows)
    float dy[4];
    for (int r = 0; r < 4; ++r) {
      const int lrow = r0 + 4 * lk + r;
      const bool ok = base + lrow < end;
      const float res = ok ? (ys[r] + s.w.f.b4 - s.tgt[lrow]) : 0.f;
      dy[r] = res * inv_b;
      if (lr == 0) lsum += res * res;
    }
    // output layer and dZ3
    for (int j = 0; j < 4; ++j)
      for (int r = 0; r < 4; ++r) {
        gw4[j] += h3[j][r] * dy[r];
        const float d = dy[r] * s.w.f.w4[j * 16 + lr] * gelu_d(z3[j][r]);
        gb3[j] += d;
        const uint16_t b = f2bf(d);
        s.dZ3[r0 + 4 * lk + r][j * 16 + lr] = b;
        s.dZ3T[j * 16 + lr][r0 + 4 * lk + r] = b;
      }
    if (lr == 0)
      for (int r = 0; r < 4; ++r) gb4 += dy[r];
    __syncthreads();
    // dW3 += H2^T dZ3 (rows of dW3 = in features 16*wave..)
    mm16x64<ROWS>(&s.H2T[r0][0], LD2, &s.dZ3T[0][0], LD2, gW3, lr, lk);
    // dA2 = dZ3 W3^T, dZ2
    f4 da[4];
    for (int j = 0; j < 4; ++j) da[j] = f4{0.f, 0.f, 0.f, 0.f};
    mm16x64<WD>(&s.dZ3[r0][0], LD2, &s.w.W3n[0][0], LD2, da, lr, lk);
    for (int j = 0; j < 4; ++j)
      for (int r = 0; r < 4; ++r) {
        const float d = da[j][r] * gelu_d(z2[j][r]);
        gb2[j] += d;
        const uint16_t b = f2bf(d);
        s.dZ2[r0 + 4 * lk + r][j * 16 + lr] = b;
        s.dZ2T[j * 16 + lr][r0 + 4 * lk + r] = b;
      }
    __syncthreads();
    mm16x64<ROWS>(&s.H1T[r0][0], LD2, &s.dZ2T[0][0], LD2, gW2, lr, lk);
    for (int j = 0; j < 4; ++j) da[j] = f4{0.f, 0.f, 0.f, 0.f};
    mm16x64<WD>(&s.dZ2[r0][0], LD2, &s.w.W2n[0][0], LD2, da, lr, lk);
    for (int j = 0; j < 4; ++j)
      for (int r = 0; r < 4; ++r) {
        const float d = da[j][r] * gelu_d(z1[j][r]);
        gb1[j] += d;
        s.dZ1T[j * 16 + lr][r0 + 4 * lk + r] = f2bf(d);
      }
    __syncthreads();
    if (wave < KIN / 16) mm16x64<ROWS>(&s.XT[r0][0], LD2, &s.dZ1T[0][0], LD2, gW1, lr, lk);
  }

  // per-block partial gradient, flat parameter layout
  float *P = partials + int64_t(blockIdx.x) * NP;
  for (int j = 0; j < 4; ++j)
    for (int r = 0; r < 4; ++r) {
      const int in = r0 + 4 * lk + r, out = j * 16 + lr;
      P[OW3 + in * WD + out] = gW3[j][r];
      P[OW2 + in * WD + out] = gW2[j][r];
      if (wave < KIN / 16 && in < NIN) P[OW1 + in * WD + out] = gW1[j][r];
    }
  // column sums over the 4 row groups of a wave, then over the waves, in order
  float vals[4][4];
  for (int j = 0; j < 4; ++j) {
    vals[0][j] = gb1[j];
    vals[1][j] = gb2[j];
    vals[2][j] = gb3[j];
    vals[3][j] = gw4[j];
  }
  for (int q = 0; q < 4; ++q)
    for (int j = 0; j < 4; ++j) {
      float v = vals[q][j];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      vals[q][j] = v;
    }
  __syncthreads();
  if (lk == 0)
    for (int q = 0; q < 4; ++q)
      for (int j = 0; j < 4; ++j) s.red[wave][q][j * 16 + lr] = vals[q][j];
  // loss and b4 partials: lanes with lr == 0 hold them; sum in a fixed order
  float lb[2] = {lsum, gb4};
  for (int q = 0; q < 2; ++q) {
    lb[q] += __shfl_xor(lb[q], 16, 64);
    lb[q] += __shfl_xor(lb[q], 32, 64);
  }
  if (lane == 0) s.lossw[wave] = lb[0];
  __shared__ float b4w[4];
  if (lane == 0) b4w[wave] = lb[1];
  __syncthreads();
  if (t < WD) {
    for (int q = 0; q < 4; ++q) {
      const float v = ((s.red[0][q][t] + s.red[1][q][t]) + s.red[2][q][t]) + s.red[3][q][t];
      const int off = q == 0 ? OB1 : q == 1 ? OB2 : q == 2 ? OB3 : OW4;
      P[off + t] = v;
    }
  }
  if (t == 0) {
    P[OB4] = ((b4w[0] + b4w[1]) + b4w[2]) + b4w[3];
    loss_part[blockIdx.x] = ((s.lossw[0] + s.lossw[1]) + s.lossw[2]) + s.lossw[3];
  }
}

__global__ void k_mlp_reduce(const float *partials, const float *loss_part, int nb, int64_t rows,
                             float *grad, float *loss_out, float *grad_out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NP) {
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += partials[int64_t(b) * NP + p];
    grad[p] = s;
    if (grad_out) grad_out[p] = s;
  }
  if (p == 0 && loss_out) {
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += loss_part[b];
    *loss_out = s / float(rows);
  }
}

__global__ void k_mlp_adam(float *w, float *m, float *v, const float *g, float lr, float c1,
                           float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  const float gi = g[p];
  const float mi = 0.9f * m[p] + 0.1f * gi;
  const float vi = 0.999f * v[p] + 0.001f * gi * gi;
  m[p] = mi;
  v[p] = vi;
  w[p] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// bf16 copies of the weights in the kernels' layouts
__global__ void k_mlp_pack(const float *w, uint16_t *pk) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < WD * KIN) {
    const int o = e / KIN, i = e % KIN;
    const int ii = i < NIN ? i : i - NIN;   // columns [12, 24) repeat [0, 12)
    pk[PW1T + e] = i < 2 * NIN ? f2bf(w[OW1 + ii * WD + o]) : uint16_t(0);
  }
  if (e < WD * WD) {
    const int a = e / WD, b = e % WD;
    pk[PW2T + e] = f2bf(w[OW2 + b * WD + a]);   // W2t[out=a][in=b]
    pk[PW3T + e] = f2bf(w[OW3 + b * WD + a]);
    pk[PW2N + e] = f2bf(w[OW2 + e]);            // W2n[in][out]
    pk[PW3N + e] = f2bf(w[OW3 + e]);
  }
  if (e < WD) pk[PW4 + e] = f2bf(w[OW4 + e]);
}

static pe_status repack(pe_mlp m, hipStream_t st) {
  k_mlp_pack<<<(WD * WD + 255) / 256, 256, 0, st>>>(m->master, m->packed);
  PE_HIP(hipGetLastError());
  return PE_OK;
}

static unsigned infer_blocks(int64_t rows) {
  const int64_t groups = (rows + 15) / 16;
  const int64_t b = (groups + MNT / 64 - 1) / (MNT / 64);
  return unsigned(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace pe

using namespace pe;

extern "C" {

pe_status pe_mlp_create(pe_mlp *out, const float *h_params, void *stream) {
  clear_error();
  if (!out || !h_params) return set_error(PE_E_ARG, "null argument");
  *out = nullptr;
  hipStream_t st = as_stream(stream);
  pe_mlp m = new pe_mlp_s();
  hipError_t e = hipMalloc(&m->master, sizeof(float) * NP);
  if (e == hipSuccess) e = hipMalloc(&m->m, sizeof(float) * NP);
  if (e == hipSuccess) e = hipMalloc(&m->v, sizeof(float) * NP);
  if (e == hipSuccess) e = hipMalloc(&m->packed, sizeof(uint16_t) * PTOT);
  if (e == hipSuccess) e = hipMalloc(&m->partials, sizeof(float) * NP * MAX_TRAIN_BLOCKS);
  if (e == hipSuccess) e = hipMalloc(&m->loss_part, sizeof(float) * MAX_TRAIN_BLOCKS);
  if (e == hipSuccess) e = hipMalloc(&m->grad, sizeof(float) * NP);
  if (e == hipSuccess) e = hipMalloc(&m->flag, sizeof(int));
  if (e == hipSuccess) e = hipMemcpyAsync(m->master, h_params, sizeof(float) * NP,
                                          hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(m->m, 0, sizeof(float) * NP, st);
  if (e == hipSuccess) e = hipMemsetAsync(m->v, 0, sizeof(float) * NP, st);
  if (e == hipSuccess) {
    k_mlp_pack<<<(WD * WD + 255) / 256, 256, 0, st>>>(m->master, m->packed);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    pe_mlp_free(m);
    return set_error(PE_E_HIP, "network allocation failed: %s", hipGetErrorString(e));
  }
  *out = m;
  return PE_OK;
}

void pe_mlp_free(pe_mlp m) {
  if (!m) return;
  dev_free(m->master);
  dev_free(m->m);
  dev_free(m->v);
  dev_free(m->packed);
  dev_free(m->partials);
  dev_free(m->loss_part);
  dev_free(m->grad);
  dev_free(m->flag);
  delete m;
}

pe_status pe_mlp_get_params(pe_mlp m, float *h_params, void *stream) {
  clear_error();
  if (!m || !h_params) return set_error(PE_E_ARG, "null argument");
  hipStream_t st = as_stream(stream);
  PE_HIP(hipMemcpyAsync(h_params, m->master, sizeof(float) * NP, hipMemcpyDeviceToHost, st));
  PE_HIP(hipStreamSynchronize(st));
  return PE_OK;
}

pe_status pe_mlp_set_params(pe_mlp m, const float *h_params, void *stream) {
  clear_error();
  if (!m || !h_params) return set_error(PE_E_ARG, "null argument");
  hipStream_t st = as_stream(stream);
  PE_HIP(hipMemcpyAsync(m->master, h_params, sizeof(float) * NP, hipMemcpyHostToDevice, st));
  PE_TRY(repack(m, st));
  PE_HIP(hipStreamSynchronize(st));
  return PE_OK;
}

pe_status pe_mlp_forward(pe_mlp m, int64_t rows, const float *d_x, float *d_y, void *stream) {
  clear_error();
  if (!m || !d_x || !d_y) return set_error(PE_E_ARG, "null argument");
  if (rows < 1) return set_error(PE_E_ARG, "rows must be >= 1");
  hipStream_t st = as_stream(stream);
  k_mlp_infer<<<infer_blocks(rows), MNT, 0, st>>>(m->packed, m->master, d_x, rows, d_y);
  PE_HIP(hipGetLastError());
  return PE_OK;
}

pe_status pe_mlp_train_step(pe_mlp m, int64_t rows, const float *d_x, const float *d_t, float lr,
                            int32_t apply, float *d_loss, float *d_grad, void *stream) {
  clear_error();
  if (!m || !d_x || !d_t) return set_error(PE_E_ARG, "null argument");
  if (rows < 1 || rows > (int64_t(1) << 24)) return set_error(PE_E_ARG, "rows must be 1..2^24");
  hipStream_t st = as_stream(stream);
  int64_t tiles = (rows + ROWS - 1) / ROWS;
  int nb = int(tiles < MAX_TRAIN_BLOCKS ? tiles : MAX_TRAIN_BLOCKS);
  int64_t tiles_per_block = (tiles + nb - 1) / nb;
  nb = int((tiles + tiles_per_block - 1) / tiles_per_block);
  size_t lds = sizeof(TrainLds);
  static bool attr_set = false;
  if (!attr_set) {
    PE_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_mlp_train),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    attr_set = true;
  }
  k_mlp_train<<<nb, MNT, lds, st>>>(m->packed, m->master, d_x, d_t, rows,
                                   tiles_per_block * ROWS, m->partials, m->loss_part);
  PE_HIP(hipGetLastError());
  k_mlp_reduce<<<(NP + 255) / 256, 256, 0, st>>>(m->partials, m->loss_part, nb, rows, m->grad,
                                                 d_loss, d_grad);
  PE_HIP(hipGetLastError());
  if (apply) {
    m->step += 1;
    const float c1 = 1.0f - powf(0.9f, float(m->step));
    const float c2 = 1.0f - powf(0.999f, float(m->step));
    k_mlp_adam<<<(NP + 255) / 256, 256, 0, st>>>(m->master, m->m, m->v, m->grad, lr, c1, c2);
    PE_HIP(hipGetLastError());
    PE_TRY(repack(m, st));
  }
  return PE_OK;
}

size_t pe_learned_correction_workspace_bytes(pe_grid g, int32_t n_slices) {
  if (!g || n_slices < 1) return 0;
  return learned_coef_bytes(g, n_slices);
}

pe_status pe_learned_correction(pe_grid g, pe_mlp m, int32_t n_slices, double t0, double dT,
                                void *d_corr, int32_t *h_fallback, void *d_work,
                                size_t work_bytes, void *stream) {
  clear_error();
  if (!g || !m || !d_corr) return set_error(PE_E_ARG, "null argument");
  if (n_slices < 1 || !(dT > 0) || !std::isfinite(t0))
    return set_error(PE_E_ARG, "bad n_slices / t0 / dT");
  if (g->n_hats > 0) return set_error(PE_E_ARG, "the learned inputs do not cover moving sources");
  if (has_periodic(g)) return set_error(PE_E_ARG, "the learned inputs are built for Dirichlet axes");
  hipStream_t st = as_stream(stream);
  const bool fp64 = g->precision == PE_FP64;
  const size_t sb = fp64 ? sizeof(double) : sizeof(float);
  if (h_fallback) *h_fallback = 0;
  if (g->n_terms == 0) {
    PE_HIP(hipMemsetAsync(d_corr, 0, sb * size_t(n_slices) * g->dof, st));
    return PE_OK;
  }
  if (!d_work || work_bytes < pe_learned_correction_workspace_bytes(g, n_slices))
    return set_error(PE_E_WORKSPACE, "workspace %zu B below %zu B", work_bytes,
                     pe_learned_correction_workspace_bytes(g, n_slices));
  double *Cp = static_cast<double *>(d_work);
  PE_TRY(learned_coefs(g, n_slices, t0, dT, Cp, st));
  CorrArgs a{};
  a.d = g->dim;
  a.M = g->n_terms;
  a.N = n_slices;
  a.n0 = g->ax[0].n;
  a.n1 = g->dim > 1 ? g->ax[1].n : 1;
  a.n2 = g->dim > 2 ? g->ax[2].n : 1;
  a.lam0 = g->ax[0].d_lam;
  a.lam1 = g->ax[1].d_lam;
  a.lam2 = g->ax[2].d_lam;
  a.sp0 = g->d_spec[0];
  a.sp1 = g->d_spec[1];
  a.sp2 = g->d_spec[2];
  a.Cp = Cp;
  a.D = g->D;
  a.dT = dT;
  a.dof = g->dof;
  a.corr = d_corr;
  a.fp64 = fp64;
  a.bad = m->flag;
  const int64_t ktiles = (g->dof + 63) / 64;
  const int64_t slice_groups = (int64_t(n_slices) + 3) / 4;
  const int64_t want = (2048 + ktiles - 1) / ktiles;
  const int64_t nsplit = std::max<int64_t>(1, std::min(slice_groups, want));
  if (ktiles * nsplit > (int64_t(1) << 24)) return set_error(PE_E_ARG, "grid too large");
  a.ktiles = int(ktiles);
  a.nsplit = int(nsplit);
  const size_t lds = CORR_LDS_FIXED + sizeof(double) * 64 * size_t(a.M);
  static bool attr_set = false;
  if (!attr_set) {
    PE_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_mlp_correct),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(CORR_LDS_FIXED + sizeof(double) * 64 * PE_MAX_TERMS)));
    attr_set = true;
  }
  PE_HIP(hipMemsetAsync(m->flag, 0, sizeof(int), st));
  k_mlp_correct<<<unsigned(ktiles * nsplit), MNT, lds, st>>>(m->packed, m->master, a);
  PE_HIP(hipGetLastError());
  int bad = 0;
  PE_HIP(hipMemcpyAsync(&bad, m->flag, sizeof(int), hipMemcpyDeviceToHost, st));
  PE_HIP(hipStreamSynchronize(st));
  if (bad) {
    PE_HIP(hipMemsetAsync(d_corr, 0, sb * size_t(n_slices) * g->dof, st));
    PE_HIP(hipStreamSynchronize(st));
  }
  if (h_fallback) *h_fallback = bad ? 1 : 0;
  return PE_OK;
}

}  // extern "C"
