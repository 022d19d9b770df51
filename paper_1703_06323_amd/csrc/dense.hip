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
// GEMM tiles: 64 or 128 rows x 64 or 128 columns per 256-thread workgroup,
// four 64-wide waves in a 2 x 2 arrangement; the shape per call comes from a
// small autotuner table (see gemm_autotune).
#include "dense.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

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

// C[M x N] = alpha * op(A)[M x K] * op(B)[K x N] + beta * C, BM x BN output
// tile per 256-thread workgroup: four waves in a 2 x 2 arrangement, each
// owning (BM/32) x (BN/32) MFMA 16x16 blocks; the K loop stages BM x 16 and
// 16 x BN operand tiles in LDS.
//   TA = 0: A(i,k) = A[i*lda + k];  TA = 1: A(i,k) = A[k*lda + i]
//   TB = 0: B(k,j) = B[k*ldb + j];  TB = 1: B(k,j) = B[j*ldb + k]
// C is written only after the whole K loop, so a call may overwrite its own
// B operand when each output tile reads only its own columns of B (and the
// same for A and rows); the dispatcher keeps such calls on 64-wide tiles.
template <typename T, int TA, int TB, int BM, int BN>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, T alpha, const T* __restrict__ A,
                                                   int64_t lda, int64_t sA, const T* __restrict__ B,
                                                   int64_t ldb, int64_t sB, T beta, T* C, int64_t ldc,
                                                   int64_t sC, int mode) {
  constexpr int WM = BM / 2, WN = BN / 2;       // per-wave outputs
  constexpr int FM = WM / 16, FN = WN / 16;     // MFMA blocks per wave
  __shared__ T As[BM][KT + 1];
  __shared__ T Bs[KT][BN + 1];
  const int row0 = blockIdx.y * BM;
  const int col0 = blockIdx.x * BN;
  const int64_t bz = blockIdx.z;
  if ((mode & GEMM_LOWER) && col0 > row0 + BM - 1) return;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  int kbeg = 0, kend = K;
  if (mode & GEMM_KFROM_DIAG) kbeg = (max(row0, col0) / KT) * KT;
  if (mode & GEMM_KTO_DIAG) kend = min(K, row0 + BM);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;
  typename Acc<T>::type acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = (typename Acc<T>::type){0, 0, 0, 0};
  for (int k0 = kbeg; k0 < kend; k0 += KT) {
    for (int e = tid; e < BM * KT; e += 256) {
      int i, k;
      if (TA == 0) { i = e / KT; k = e % KT; } else { k = e / BM; i = e % BM; }
      const int gi = row0 + i, gk = k0 + k;
      T v = 0;
      if (gi < M && gk < kend) v = TA == 0 ? A[(int64_t)gi * lda + gk] : A[(int64_t)gk * lda + gi];
      As[i][k] = v;
    }
    for (int e = tid; e < KT * BN; e += 256) {
      int k, j;
      if (TB == 0) { k = e / BN; j = e % BN; } else { j = e / KT; k = e % KT; }
      const int gj = col0 + j, gk = k0 + k;
      T v = 0;
      if (gj < N && gk < kend) v = TB == 0 ? B[(int64_t)gk * ldb + gj] : B[(int64_t)gj * ldb + gk];
      Bs[k][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KT; kk += 4) {
      T bv[FN];
#pragma unroll
      for (int ni = 0; ni < FN; ++ni) bv[ni] = Bs[kk + (lane >> 4)][wc * WN + ni * 16 + (lane & 15)];
#pragma unroll
      for (int mi = 0; mi < FM; ++mi) {
        const T av = As[wr * WM + mi * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int ni = 0; ni < FN; ++ni) acc[mi][ni] = Acc<T>::mfma(av, bv[ni], acc[mi][ni]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int mi = 0; mi < FM; ++mi)
#pragma unroll
    for (int ni = 0; ni < FN; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = row0 + wr * WM + mi * 16 + Acc<T>::row(lane, v);
        const int gj = col0 + wc * WN + ni * 16 + (lane & 15);
        if (gi >= M || gj >= N) continue;
        if ((mode & GEMM_LOWER) && gj > gi) continue;
        T* c = C + (int64_t)gi * ldc + gj;
        const T r = alpha * acc[mi][ni][v];
        *c = (beta == T(0)) ? r : r + beta * (*c);
      }
}

// Cholesky of the BLK x BLK diagonal tile at (k0, k0) of each matrix by one
// wave.  Thread t owns half (t & 1) of row (t >> 1) in registers (16
// values; the step loop is unrolled so every register index is static).  At
// step j the pivot and then the new column j go through small LDS vectors,
// so each step costs two barriers and a burst of independent LDS reads.
// L^{-1} follows by forward elimination on [L | I] with the same layout.
// Writes L (lower, upper part of the tile zeroed) and L^{-1} into
// Linv[bz][tile][BLK*BLK].  A non-positive or non-finite pivot sets
// info[bz] (first failing global row + 1) and is replaced by 1 so that the
// factorisation continues without NaNs.
template <typename T>
__global__ __launch_bounds__(64) void potrf_tile_kernel(T* A, int64_t lda, int64_t sA, int k0,
                                                        T* Linv, int64_t sL, int* info) {
  constexpr int H = BLK / 2;
  __shared__ T pv[BLK];
  __shared__ T colj[BLK];
  __shared__ T Lt[BLK][BLK + 1];
  const int64_t bz = blockIdx.x;
  T* a = A + bz * sA + (int64_t)k0 * lda + k0;
  const int t = threadIdx.x;
  const int i = t >> 1, c0 = (t & 1) * H;
  T r[H];
#pragma unroll
  for (int q = 0; q < H; ++q) r[q] = a[(int64_t)i * lda + c0 + q];
  int bad = 0;
#pragma unroll
  for (int j = 0; j < BLK; ++j) {
    const bool mine = (j >= c0 && j < c0 + H);   // this thread's half holds column j
    if (i == j && mine) {
      T d = r[j - c0];
      if (!(d > T(0)) || !(d < T(3.0e38))) d = T(-1);
      pv[j] = d;
    }
    __syncthreads();
    T d = pv[j];
    if (d < T(0)) {
      if (!bad) bad = k0 + j + 1;
      d = T(1);
    }
    const T piv = sqrt(d);
    if (mine) {
      if (i == j) r[j - c0] = piv;
      if (i > j) r[j - c0] = r[j - c0] / piv;
      if (i >= j) colj[i] = r[j - c0];
    }
    __syncthreads();
    if (i > j) {
      const T lij = colj[i];
#pragma unroll
      for (int q = 0; q < H; ++q) {
        const int l = c0 + q;
        if (l > j && l <= i) r[q] -= lij * colj[l];
      }
    }
  }
  // L to LDS, then X = L^{-1} row segments in registers
#pragma unroll
  for (int q = 0; q < H; ++q) Lt[i][c0 + q] = r[q];
  __syncthreads();
  T x[H];
#pragma unroll
  for (int q = 0; q < H; ++q) x[q] = (c0 + q == i) ? T(1) : T(0);
#pragma unroll
  for (int j = 0; j < BLK; ++j) {
    if (i == j) {
      const T inv = T(1) / Lt[j][j];
#pragma unroll
      for (int q = 0; q < H; ++q) {
        x[q] = x[q] * inv;
        colj[c0 + q] = x[q];
      }
    }
    __syncthreads();
    if (i > j) {
      const T lij = Lt[i][j];
#pragma unroll
      for (int q = 0; q < H; ++q)
        if (c0 + q <= j) x[q] -= lij * colj[c0 + q];
    }
    __syncthreads();
  }
  if (bad && t == 0 && info && info[bz] == 0) info[bz] = bad;
  T* li = Linv + bz * sL + (int64_t)(k0 / BLK) * BLK * BLK;
#pragma unroll
  for (int q = 0; q < H; ++q) {
    a[(int64_t)i * lda + c0 + q] = (c0 + q <= i) ? r[q] : T(0);
    li[i * BLK + c0 + q] = x[q];
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

// ---- GEMM dispatch and tile-shape autotuner -----------------------------
// Tile shapes: 0 = 64x64, 1 = 128x64, 2 = 64x128, 3 = 128x128.  The choice
// for a call is looked up by (type, TA, TB, mode bits, shape bucket); buckets
// are powers of two of M, N, K and of the batch size.  Calls that overwrite
// their own operand (in place) always use 64x64 tiles.  The table is filled
// by gemm_autotune(), which times every shape on scratch matrices of the
// bucket's size and keeps the fastest; untuned buckets use 64x64.
namespace {
struct TuneKey {
  int dt, ta, tb, mode, bm, bn, bk, bb;
  bool operator<(const TuneKey& o) const {
    return std::tie(dt, ta, tb, mode, bm, bn, bk, bb) < std::tie(o.dt, o.ta, o.tb, o.mode, o.bm, o.bn, o.bk, o.bb);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
inline int log2b(int x) {
  int b = 0;
  while ((1 << (b + 1)) <= x) ++b;
  return b;
}
bool autotune_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("CUTBDDC_AUTOTUNE");
    return !(e && e[0] == '0');
  }();
  return on;
}
template <typename T>
TuneKey tune_key(int TA, int TB, int M, int N, int K, int batch, int mode) {
  return TuneKey{(int)sizeof(T), TA, TB, mode & 7, log2b(M), log2b(N), log2b(std::max(K, 1)), log2b(batch)};
}

template <typename T>
void gemm_launch(int shape, hipStream_t st, int TA, int TB, int M, int N, int K, T alpha, const T* A,
                 int64_t lda, int64_t sA, const T* B, int64_t ldb, int64_t sB, T beta, T* C, int64_t ldc,
                 int64_t sC, int batch, int mode) {
  const int BM = (shape == 1 || shape == 3) ? 128 : 64;
  const int BN = (shape == 2 || shape == 3) ? 128 : 64;
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, batch);
#define GEMM_CASE(a, b, bm, bn)                                                                        \
  if (TA == a && TB == b && BM == bm && BN == bn) {                                                    \
    hipLaunchKernelGGL((gemm_kernel<T, a, b, bm, bn>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, \
                       sA, B, ldb, sB, beta, C, ldc, sC, mode);                                        \
    return;                                                                                            \
  }
#define GEMM_SHAPES(a, b) \
  GEMM_CASE(a, b, 64, 64) GEMM_CASE(a, b, 128, 64) GEMM_CASE(a, b, 64, 128) GEMM_CASE(a, b, 128, 128)
  GEMM_SHAPES(0, 0) GEMM_SHAPES(0, 1) GEMM_SHAPES(1, 0) GEMM_SHAPES(1, 1)
#undef GEMM_SHAPES
#undef GEMM_CASE
}
}  // namespace

template <typename T>
void gemm(hipStream_t st, int TA, int TB, int M, int N, int K, T alpha, const T* A, int64_t lda,
          int64_t sA, const T* B, int64_t ldb, int64_t sB, T beta, T* C, int64_t ldc, int64_t sC,
          int batch, int mode) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  int shape = 0;
  const bool in_place = ((const T*)C == A) || ((const T*)C == B);
  if (!in_place) {
    bool known = false;
    {
      std::lock_guard<std::mutex> g(g_tune_mu);
      auto it = g_tune.find(tune_key<T>(TA, TB, M, N, K, batch, mode));
      if (it != g_tune.end()) {
        shape = it->second;
        known = true;
      }
    }
    if (!known && autotune_enabled()) shape = gemm_autotune<T>(TA, TB, M, N, K, batch, mode);
  }
  gemm_launch<T>(shape, st, TA, TB, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, mode);
}

template <typename T>
int gemm_autotune(int TA, int TB, int M, int N, int K, int batch, int mode) {
  if (M <= 0 || N <= 0 || batch <= 0) return 0;
  const TuneKey key = tune_key<T>(TA, TB, M, N, K, batch, mode);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second;
  }
  const int64_t la = TA == 0 ? K : M, lb = TB == 0 ? N : K;
  const int64_t sA = (int64_t)(TA == 0 ? M : K) * la, sB = (int64_t)(TB == 0 ? K : N) * lb, sC = (int64_t)M * N;
  // scratch capped at ~2 GB: time a smaller batch for very large calls
  const int64_t per = (sA + sB + sC) * (int64_t)sizeof(T);
  batch = (int)std::max<int64_t>(1, std::min<int64_t>(batch, ((int64_t)2 << 30) / std::max<int64_t>(per, 1)));
  T *A = nullptr, *B = nullptr, *C = nullptr;
  if (hipMalloc(&A, sA * batch * sizeof(T)) != hipSuccess || hipMalloc(&B, sB * batch * sizeof(T)) != hipSuccess ||
      hipMalloc(&C, sC * batch * sizeof(T)) != hipSuccess) {
    (void)hipFree(A);
    (void)hipFree(B);
    (void)hipFree(C);
    return 0;
  }
  (void)hipMemset(A, 0, sA * batch * sizeof(T));
  (void)hipMemset(B, 0, sB * batch * sizeof(T));
  (void)hipMemset(C, 0, sC * batch * sizeof(T));
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  int best = 0;
  float best_ms = 1e30f;
  for (int shape = 0; shape < 4; ++shape) {
    float tot = 0.f;
    for (int rep = 0; rep < 3; ++rep) {
      (void)hipEventRecord(e0, nullptr);
      gemm_launch<T>(shape, nullptr, TA, TB, M, N, K, T(1), A, la, sA, B, lb, sB, T(1), C, N, sC, batch, mode);
      (void)hipEventRecord(e1, nullptr);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) tot += ms;
    }
    if (tot < best_ms) {
      best_ms = tot;
      best = shape;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(A);
  (void)hipFree(B);
  (void)hipFree(C);
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[key] = best;
  return best;
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
  template int gemm_autotune<T>(int, int, int, int, int, int, int);                              \
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
