// Per-axis DST-I products of batches of padded fields in FP64 on the matrix
// cores (v_mfma_f64_16x16x4f64).
//
// The tensor-product transform (kron_a S_a) F of a d-D field is d mode
// products, one per axis (paper Section 2.3, closing paragraph: the mass and
// stiffness matrices are diagonalised by one orthogonal matrix and applied
// with tensor-product operations).  Every mode product is a row-major GEMM
// C = A * B with A contiguous along k and B contiguous along n:
//   last axis   : X viewed as [rows][np]   ->  C[r][k] = sum_j X[r][j] S[j][k]
//   other axes  : X viewed as [outer][np][inner]
//                 -> C_o[k][i] = sum_j S[k][j] X_o[j][i]   (batched over o)
// S is symmetric, so the same matrix serves as either operand.
#include "pe_internal.h"

namespace pe {

typedef double d4 __attribute__((ext_vector_type(4)));

// Block tile BM x BN, k-step KB, 4 waves in a WAVES_M x WAVES_N arrangement.
// LDS holds the A tile k-major (As[k][m]) and the B tile k-major (Bs[k][n])
// so that the 16 lanes of an MFMA operand read 16 consecutive doubles.
//
// MFMA f64 16x16x4 lane layout: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; it receives C[l/16 + 4*r][l%16], r = 0..3.
template <int BM, int BN, int KB, int WAVES_M, int WAVES_N>
__global__ __launch_bounds__(256) void k_gemm_f64(const double *__restrict__ A, int64_t lda,
                                                  int64_t sA, const double *__restrict__ B,
                                                  int64_t ldb, int64_t sB, double *__restrict__ C,
                                                  int64_t ldc, int64_t sC, int M, int N, int K,
                                                  int tiles_n, int64_t tiles_per_batch) {
  constexpr int WM = BM / WAVES_M;
  constexpr int WN = BN / WAVES_N;
  constexpr int TM = WM / 16;
  constexpr int TN = WN / 16;
  constexpr int APAD = 4, BPAD = 4;
  __shared__ double As[KB][BM + APAD];
  __shared__ double Bs[KB][BN + BPAD];

  const int64_t bid = blockIdx.x;
  const int64_t batch = bid / tiles_per_batch;
  const int64_t t = bid - batch * tiles_per_batch;
  const int tm = int(t / tiles_n), tn = int(t - int64_t(tm) * tiles_n);
  A += batch * sA;
  B += batch * sB;
  C += batch * sC;
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;
  const int lr = lane & 15, lk = lane >> 4;

  d4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  for (int k0 = 0; k0 < K; k0 += KB) {
    // A tile: BM rows x KB columns (contiguous in k) -> As[k][m]
#pragma unroll
    for (int e = tid; e < BM * KB; e += 256) {
      int m = e / KB, k = e - (e / KB) * KB;
      double v = 0.0;
      if (m0 + m < M) v = A[int64_t(m0 + m) * lda + k0 + k];
      As[k][m] = v;
    }
    // B tile: KB rows x BN columns (contiguous in n) -> Bs[k][n]
#pragma unroll
    for (int e = tid; e < KB * BN; e += 256) {
      int k = e / BN, n = e - (e / BN) * BN;
      double v = 0.0;
      if (n0 + n < N) v = B[int64_t(k0 + k) * ldb + n0 + n];
      Bs[k][n] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KB; kk += 4) {
      double a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[kk + lk][wm * WM + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = Bs[kk + lk][wn * WN + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      int col = n0 + wn * WN + j * 16 + lr;
      if (col >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = m0 + wm * WM + i * 16 + lk + 4 * r;
        if (row < M) C[int64_t(row) * ldc + col] = acc[i][j][r];
      }
    }
}

constexpr int G_BM = 64, G_BN = 64, G_KB = 16;

static pe_status gemm_f64(const double *A, int64_t lda, int64_t sA, const double *B, int64_t ldb,
                          int64_t sB, double *C, int64_t ldc, int64_t sC, int M, int N, int K,
                          int64_t batch, hipStream_t st) {
  if (K % G_KB != 0) return set_error(PE_E_ARG, "internal: K=%d not a multiple of %d", K, G_KB);
  int tiles_m = (M + G_BM - 1) / G_BM;
  int tiles_n = (N + G_BN - 1) / G_BN;
  int64_t per = int64_t(tiles_m) * tiles_n;
  if (per <= 0 || batch <= 0) return PE_OK;
  // a grid dimension holds at most 2^32 work-items: launch batch chunks
  const int64_t max_blocks = (int64_t(1) << 24) - 1;
  if (per > max_blocks) return set_error(PE_E_ARG, "internal: GEMM tile count too large");
  int64_t bchunk = max_blocks / per;
  for (int64_t b0 = 0; b0 < batch; b0 += bchunk) {
    int64_t nb = batch - b0 < bchunk ? batch - b0 : bchunk;
    k_gemm_f64<G_BM, G_BN, G_KB, 2, 2><<<dim3(unsigned(per * nb)), 256, 0, st>>>(
        A + b0 * sA, lda, sA, B + b0 * sB, ldb, sB, C + b0 * sC, ldc, sC, M, N, K, tiles_n, per);
    PE_HIP(hipGetLastError());
  }
  return PE_OK;
}

// d mode products of `count` padded fields; buffers ping-pong.
pe_status dst_fields_f64(pe_grid g, int64_t count, double *buf0, double *buf1, double **result,
                         hipStream_t st) {
  double *in = buf0, *out = buf1;
  const int d = g->dim;
  for (int a = d - 1; a >= 0; --a) {
    const Axis &ax = g->ax[a];
    int64_t inner = 1, outer = count;
    for (int b = a + 1; b < d; ++b) inner *= g->ax[b].np;
    for (int b = 0; b < a; ++b) outer *= g->ax[b].np;
    // algorithmic work of this pass: 2 n_a flops per coefficient, one read
    // and one write of every (unpadded) field
    TimedScope ts(g, PE_K_TRANSFORM, 2.0 * double(count) * double(g->dof) * ax.n,
                  2.0 * double(count) * double(g->dof) * sizeof(double), st);
    if (a == d - 1) {
      int64_t rows = outer;   // inner == 1
      // row chunks keep the grid below 2^24 blocks of 256 work-items
      const int64_t max_rows = int64_t(1) << 26;
      for (int64_t r0 = 0; r0 < rows; r0 += max_rows) {
        int64_t nr = rows - r0 < max_rows ? rows - r0 : max_rows;
        PE_TRY(gemm_f64(in + r0 * ax.np, ax.np, 0, ax.d_S, ax.np, 0, out + r0 * ax.np, ax.np, 0,
                        int(nr), ax.np, ax.np, 1, st));
      }
    } else {
      if (inner > 0x7fffffff) return set_error(PE_E_ARG, "internal: inner extent too large");
      PE_TRY(gemm_f64(ax.d_S, ax.np, 0, in, inner, ax.np * inner, out, inner, ax.np * inner, ax.np,
                      int(inner), ax.np, outer, st));
    }
    double *tmp = in;
    in = out;
    out = tmp;
  }
  *result = in;
  return PE_OK;
}

}  // namespace pe
