// Batched dense linear algebra on CDNA4 matrix cores (MFMA), FP64 and FP32.
//
// Used for the subdomain Dirichlet and constrained-Neumann factorisations and
// the coarse matrix: blocked right-looking Cholesky with 32-wide panels, a
// triangular inverse by block forward substitution, and the product
// Y^T Y that turns the inverse factor into the inverse.  Every kernel takes a
// batch of equally sized, row-major matrices (stride between matrices) and
// runs one workgroup per (tile, matrix), so the same code factors one large
// coarse matrix or thousands of subdomain matrices.
//
// GEMM tile: 64 x 64 outputs per 256-thread workgroup, four 64-wide waves in
// a 2 x 2 arrangement, each wave owning 2 x 2 MFMA 16x16 blocks; the K loop
// stages 64 x 16 / 16 x 64 operand tiles in LDS.
#include "dense.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace cutbddc {
namespace {

constexpr int TM = 64;    // output tile rows
constexpr int TN = 64;    // output tile cols
constexpr int KT = 16;    // K per LDS stage
constexpr int BLK = 32;   // Cholesky panel width
constexpr int SUPER = 128; // super-panel width (K of the trailing updates)

template <typename T> struct Acc;
// Operand layouts of the 16x16x4 MFMAs (both types): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  Output element v of lane l is
// D[row(l, v)][l % 16], where the row mapping differs between the FP64 and
// FP32 instructions (measured on gfx950).
template <> struct Acc<double> {
  typedef double __attribute__((ext_vector_type(4))) type;
  __device__ static type mfma(double a, double b, type c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <> struct Acc<float> {
  typedef float __attribute__((ext_vector_type(4))) type;
  __device__ static type mfma(float a, float b, type c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// C[M x N] = alpha * op(A)[M x K] * op(B)[K x N] + beta * C
//   TA = 0: A(i,k) = A[i*lda + k];  TA = 1: A(i,k) = A[k*lda + i]
//   TB = 0: B(k,j) = B[k*ldb + j];  TB = 1: B(k,j) = B[j*ldb + k]
template <typename T, int TA, int TB>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, T alpha, const T* __restrict__ A,
                                                   int64_t lda, int64_t sA, const T* __restrict__ B,
                                                   int64_t ldb, int64_t sB, T beta, T* C, int64_t ldc,
                                                   int64_t sC, int mode) {
  __shared__ T As[TM][KT + 1];
  __shared__ T Bs[KT][TN + 1];
  const int row0 = blockIdx.y * TM;
  const int col0 = blockIdx.x * TN;
  const int64_t bz = blockIdx.z;
  if ((mode & GEMM_LOWER) && col0 > row0 + TM - 1) return;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  int kbeg = 0, kend = K;
  if (mode & GEMM_KFROM_DIAG) kbeg = (max(row0, col0) / KT) * KT;
  if (mode & GEMM_KTO_DIAG) kend = min(K, row0 + TM);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;
  typename Acc<T>::type acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = (typename Acc<T>::type){0, 0, 0, 0};
  for (int k0 = kbeg; k0 < kend; k0 += KT) {
    // stage A tile (TM x KT)
    for (int e = tid; e < TM * KT; e += 256) {
      int i, k;
      if (TA == 0) { i = e / KT; k = e % KT; } else { k = e / TM; i = e % TM; }
      const int gi = row0 + i, gk = k0 + k;
      T v = 0;
      if (gi < M && gk < kend) v = TA == 0 ? A[(int64_t)gi * lda + gk] : A[(int64_t)gk * lda + gi];
      As[i][k] = v;
    }
    for (int e = tid; e < KT * TN; e += 256) {
      int k, j;
      if (TB == 0) { k = e / TN; j = e % TN; } else { j = e / KT; k = e % KT; }
      const int gj = col0 + j, gk = k0 + k;
      T v = 0;
      if (gj < N && gk < kend) v = TB == 0 ? B[(int64_t)gk * ldb + gj] : B[(int64_t)gj * ldb + gk];
      Bs[k][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KT; kk += 4) {
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) {
        const T a = As[wr * 32 + mi * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
          const T b = Bs[kk + (lane >> 4)][wc * 32 + ni * 16 + (lane & 15)];
          acc[mi][ni] = Acc<T>::mfma(a, b, acc[mi][ni]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = row0 + wr * 32 + mi * 16 + Acc<T>::row(lane, v);
        const int gj = col0 + wc * 32 + ni * 16 + (lane & 15);
        if (gi >= M || gj >= N) continue;
        if ((mode & GEMM_LOWER) && gj > gi) continue;
        T* c = C + (int64_t)gi * ldc + gj;
        const T r = alpha * acc[mi][ni][v];
        *c = (beta == T(0)) ? r : r + beta * (*c);
      }
}

// Broadcast of lane `l`'s value (l uniform, a compile-time constant after
// unrolling) to the whole wave.
__device__ inline double bcast(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline float bcast(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Cholesky of the BLK x BLK diagonal tile at (k0, k0) of each matrix, held
// in registers of one wave (lane i < BLK owns row i; lanes >= BLK idle).
// Writes L (lower, upper part of the tile zeroed) and L^{-1} into
// Linv[bz][tile][BLK*BLK].  A non-positive or non-finite pivot sets
// info[bz] (first failing global row + 1) and is replaced by 1 so that the
// factorisation continues without NaNs.
template <typename T>
__global__ __launch_bounds__(64) void potrf_tile_kernel(T* A, int64_t lda, int64_t sA, int k0,
                                                        T* Linv, int64_t sL, int* info) {
  const int64_t bz = blockIdx.x;
  T* a = A + bz * sA + (int64_t)k0 * lda + k0;
  const int lane = threadIdx.x;
  const bool own = lane < BLK;
  T row[BLK];
#pragma unroll
  for (int c = 0; c < BLK; ++c) row[c] = own ? a[(int64_t)lane * lda + c] : T(0);
  int bad = 0;
#pragma unroll
  for (int j = 0; j < BLK; ++j) {
    T d = bcast(row[j], j);
    if (!(d > T(0)) || !(d < T(3.0e38))) {
      if (!bad) bad = k0 + j + 1;
      d = T(1);
    }
    const T piv = sqrt(d);
    const T lij = (lane == j) ? piv : row[j] / piv;
    if (lane >= j) row[j] = lij;
#pragma unroll
    for (int l = j + 1; l < BLK; ++l) {
      const T llj = bcast(row[j], l);
      if (lane >= l) row[l] -= lij * llj;
    }
  }
  // X = L^{-1} by forward elimination; lane i owns row i of X
  T x[BLK];
#pragma unroll
  for (int c = 0; c < BLK; ++c) x[c] = (c == lane) ? T(1) : T(0);
#pragma unroll
  for (int j = 0; j < BLK; ++j) {
    const T ljj = bcast(row[j], j);
    if (lane == j) {
#pragma unroll
      for (int c = 0; c <= j; ++c) x[c] = x[c] / ljj;
    }
#pragma unroll
    for (int c = 0; c <= j; ++c) {
      const T xjc = bcast(x[c], j);
      if (lane > j) x[c] -= row[j] * xjc;
    }
  }
  if (bad && lane == 0 && info && info[bz] == 0) info[bz] = bad;
  if (!own) return;
  T* li = Linv + bz * sL + (int64_t)(k0 / BLK) * BLK * BLK;
#pragma unroll
  for (int c = 0; c < BLK; ++c) {
    a[(int64_t)lane * lda + c] = (c <= lane) ? row[c] : T(0);
    li[lane * BLK + c] = x[c];
  }
}

// Copies the diagonal Linv tile into Y's diagonal block (rows/cols i0..i0+BLK).
template <typename T>
__global__ __launch_bounds__(256) void set_diag_block_kernel(T* Y, int64_t ldy, int64_t sY, int i0,
                                                             const T* Linv, int64_t sL, int tile) {
  const int64_t bz = blockIdx.x;
  T* y = Y + bz * sY;
  const T* li = Linv + bz * sL + (int64_t)tile * BLK * BLK;
  for (int e = threadIdx.x; e < BLK * BLK; e += 256)
    y[(int64_t)(i0 + e / BLK) * ldy + i0 + e % BLK] = li[e];
}

// Copies an m x n block (row-major, ld) between buffers of a batch.
template <typename T>
__global__ __launch_bounds__(256) void copy_block_kernel(const T* src, int64_t lds, int64_t sS, T* dst,
                                                         int64_t ldd, int64_t sD, int n) {
  const int64_t bz = blockIdx.y;
  const int r = blockIdx.x;
  const T* a = src + bz * sS + (int64_t)r * lds;
  T* b = dst + bz * sD + (int64_t)r * ldd;
  for (int c = threadIdx.x; c < n; c += 256) b[c] = a[c];
}

template <typename T>
__global__ __launch_bounds__(256) void zero_kernel(T* Y, int64_t ldy, int64_t sY, int nb) {
  T* y = Y + (int64_t)blockIdx.y * sY + (int64_t)blockIdx.x * ldy;
  for (int c = threadIdx.x; c < nb; c += 256) y[c] = T(0);
}

// out (full symmetric, row-major nb x nb) = D * sym(lower(in)) * D
template <typename T, typename TO>
__global__ __launch_bounds__(256) void symmetrize_scale_kernel(const T* in, int64_t ldi, int64_t sI,
                                                               TO* out, int64_t ldo, int64_t sO,
                                                               const double* D, int64_t sD, int nb) {
  const int64_t bz = blockIdx.y;
  const int r = blockIdx.x;
  const T* x = in + bz * sI;
  TO* o = out + bz * sO;
  const double* d = D + bz * sD;
  for (int c = threadIdx.x; c < nb; c += 256) {
    const T v = (c <= r) ? x[(int64_t)r * ldi + c] : x[(int64_t)c * ldi + r];
    o[(int64_t)r * ldo + c] = (TO)((double)v * d[r] * d[c]);
  }
}

}  // namespace

template <typename T>
void gemm(hipStream_t st, int TA, int TB, int M, int N, int K, T alpha, const T* A, int64_t lda,
          int64_t sA, const T* B, int64_t ldb, int64_t sB, T beta, T* C, int64_t ldc, int64_t sC,
          int batch, int mode) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM, batch);
#define GEMM_CASE(a, b)                                                                          \
  if (TA == a && TB == b) {                                                                      \
    hipLaunchKernelGGL((gemm_kernel<T, a, b>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda,   \
                       sA, B, ldb, sB, beta, C, ldc, sC, mode);                                  \
    return;                                                                                      \
  }
  GEMM_CASE(0, 0) GEMM_CASE(0, 1) GEMM_CASE(1, 0) GEMM_CASE(1, 1)
#undef GEMM_CASE
}

template <typename T>
void cholesky(hipStream_t st, T* A, int64_t lda, int64_t sA, int n, int batch, T* Linv, int64_t sL,
              int* info) {
  // Two-level right-looking blocking: 32-wide panels are factored inside a
  // SB-wide super-panel (narrow updates), then the trailing matrix gets one
  // rank-SB update (K = SB) per super-panel.
  for (int K0 = 0; K0 < n; K0 += SUPER) {
    const int kend = std::min(K0 + SUPER, n);
    for (int k0 = K0; k0 < kend; k0 += BLK) {
      hipLaunchKernelGGL(potrf_tile_kernel<T>, dim3(batch), dim3(64), 0, st, A, lda, sA, k0, Linv,
                         sL, info);
      const int rest = n - k0 - BLK;
      if (rest <= 0) break;
      T* panel = A + (int64_t)(k0 + BLK) * lda + k0;
      const T* li = Linv + (int64_t)(k0 / BLK) * BLK * BLK;
      // panel solve in place: X = A_panel L_kk^{-T} (each output tile reads
      // only its own rows of the panel)
      gemm<T>(st, 0, 1, rest, BLK, BLK, T(1), panel, lda, sA, li, BLK, sL, T(0), panel, lda, sA, batch, 0);
      const int ncols = kend - (k0 + BLK);
      if (ncols > 0)
        gemm<T>(st, 0, 1, rest, ncols, BLK, T(-1), panel, lda, sA, panel, lda, sA, T(1),
                A + (int64_t)(k0 + BLK) * lda + (k0 + BLK), lda, sA, batch, GEMM_LOWER);
    }
    const int rest = n - kend;
    if (rest > 0) {
      T* P = A + (int64_t)kend * lda + K0;
      gemm<T>(st, 0, 1, rest, rest, kend - K0, T(-1), P, lda, sA, P, lda, sA, T(1),
              A + (int64_t)kend * lda + kend, lda, sA, batch, GEMM_LOWER);
    }
  }
}

template <typename T>
void tri_inverse(hipStream_t st, const T* L, int64_t ldl, int64_t sL, int off, int nb, int batch,
                 const T* Linv, int64_t sLi, T* Y, int64_t ldy, int64_t sY, T* tmp, int64_t sT) {
  // Y = L_block^{-1} for the diagonal block [off, off+nb) of L (lower) by
  // block forward substitution on L Y = I.  Y holds the running right-hand
  // side R; within a SUPER-wide block row the 32-wide steps form
  // inv(L_SS); the block row's left part becomes inv(L_SS) R_S (through
  // tmp, SUPER x nb per matrix); rows below get one rank-SUPER update.
  hipLaunchKernelGGL(zero_kernel<T>, dim3(nb, batch), dim3(256), 0, st, Y, ldy, sY, nb);
  for (int S0 = 0; S0 < nb; S0 += SUPER) {
    const int send = std::min(S0 + SUPER, nb);
    for (int i0 = S0; i0 < send; i0 += BLK) {
      const T* li = Linv + (int64_t)((off + i0) / BLK) * BLK * BLK;
      if (i0 > S0)
        gemm<T>(st, 0, 0, BLK, i0 - S0, BLK, T(1), li, BLK, sLi, Y + (int64_t)i0 * ldy + S0, ldy, sY, T(0),
                Y + (int64_t)i0 * ldy + S0, ldy, sY, batch, 0);
      hipLaunchKernelGGL(set_diag_block_kernel<T>, dim3(batch), dim3(256), 0, st, Y, ldy, sY, i0, Linv, sLi,
                         (off + i0) / BLK);
      const int rin = send - i0 - BLK;
      if (rin > 0) {
        const T* Lli = L + (int64_t)(off + i0 + BLK) * ldl + (off + i0);
        gemm<T>(st, 0, 0, rin, i0 + BLK - S0, BLK, T(-1), Lli, ldl, sL, Y + (int64_t)i0 * ldy + S0, ldy, sY, T(1),
                Y + (int64_t)(i0 + BLK) * ldy + S0, ldy, sY, batch, 0);
      }
    }
    const int h = send - S0;
    if (S0 > 0) {
      // Y[S, 0:S0] = inv(L_SS) R_S[:, 0:S0]
      gemm<T>(st, 0, 0, h, S0, h, T(1), Y + (int64_t)S0 * ldy + S0, ldy, sY, Y + (int64_t)S0 * ldy, ldy, sY, T(0),
              tmp, S0, sT, batch, GEMM_KTO_DIAG);
      hipLaunchKernelGGL(copy_block_kernel<T>, dim3(h, batch), dim3(256), 0, st, (const T*)tmp, (int64_t)S0, sT,
                         Y + (int64_t)S0 * ldy, ldy, sY, S0);
    }
    const int rest = nb - send;
    if (rest > 0) {
      const T* LlS = L + (int64_t)(off + send) * ldl + (off + S0);
      gemm<T>(st, 0, 0, rest, send, h, T(-1), LlS, ldl, sL, Y + (int64_t)S0 * ldy, ldy, sY, T(1),
              Y + (int64_t)send * ldy, ldy, sY, batch, 0);
    }
  }
}

template <typename T, typename TO>
void symmetrize_scale(hipStream_t st, const T* in, int64_t ldi, int64_t sI, TO* out, int64_t ldo,
                      int64_t sO, const double* D, int64_t sD, int nb, int batch) {
  hipLaunchKernelGGL((symmetrize_scale_kernel<T, TO>), dim3(nb, batch), dim3(256), 0, st, in, ldi,
                     sI, out, ldo, sO, D, sD, nb);
}

#define INST(T)                                                                                 \
  template void gemm<T>(hipStream_t, int, int, int, int, int, T, const T*, int64_t, int64_t,    \
                        const T*, int64_t, int64_t, T, T*, int64_t, int64_t, int, int);         \
  template void cholesky<T>(hipStream_t, T*, int64_t, int64_t, int, int, T*, int64_t, int*);    \
  template void tri_inverse<T>(hipStream_t, const T*, int64_t, int64_t, int, int, int, const T*, \
                               int64_t, T*, int64_t, int64_t, T*, int64_t);
INST(double)
INST(float)
#undef INST
template void symmetrize_scale<double, double>(hipStream_t, const double*, int64_t, int64_t,
                                               double*, int64_t, int64_t, const double*, int64_t,
                                               int, int);
template void symmetrize_scale<float, float>(hipStream_t, const float*, int64_t, int64_t, float*,
                                             int64_t, int64_t, const double*, int64_t, int, int);
template void symmetrize_scale<float, double>(hipStream_t, const float*, int64_t, int64_t, double*,
                                              int64_t, int64_t, const double*, int64_t, int, int);

}  // namespace cutbddc
