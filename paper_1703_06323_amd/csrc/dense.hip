// Batched dense linear algebra on CDNA4 matrix cores (MFMA), FP64 and FP32.
//
// Used for the subdomain Dirichlet and constrained-Neumann factorisations and
// the coarse matrix: blocked right-looking Cholesky over 128-wide diagonal
// blocks (each factored and inverted in LDS), a triangular inverse by block
// forward substitution, and the product Y^T Y that turns the inverse factor
// into the inverse.  Every kernel takes a
// batch of equally sized, row-major matrices (stride between matrices) and
// runs one workgroup per (tile, matrix), so the same code factors one large
// coarse matrix or thousands of subdomain matrices.
//
// GEMM tiles: 64 or 128 rows x 64 or 128 columns per workgroup, one 64-wide
// wave per 32 x 32 sub-tile (4 to 16 waves); the shape per call comes from a
// small autotuner table (see gemm_autotune).
#include "dense.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

namespace cutbddc {
namespace {


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

template <typename T> struct Vec16;   // 16-byte vector of T
template <> struct Vec16<float> {
  typedef float __attribute__((ext_vector_type(4))) type;
};
template <> struct Vec16<double> {
  typedef double __attribute__((ext_vector_type(2))) type;
};

// C[M x N] = alpha * op(A)[M x K] * op(B)[K x N] + beta * C, BM x BN output
// tile per workgroup of (BM/32) x (BN/32) waves, each owning a 32 x 32
// sub-tile (2 x 2 MFMA 16x16 blocks): larger tiles keep the per-wave
// registers (and so the waves per SIMD) of the smallest one while sharing
// the LDS operand tiles among more waves.
//   TA = 0: A(i,k) = A[i*lda + k];  TA = 1: A(i,k) = A[k*lda + i]
//   TB = 0: B(k,j) = B[k*ldb + j];  TB = 1: B(k,j) = B[j*ldb + k]
// The K loop runs in stages of KT (KB bytes of k per row: 128, or 256 / 512
// for short K loops, which are bound by the load latency of each stage, not
// by the multiplies); both operand
// tiles sit in LDS with k contiguous (As[i][k], Bs[j][k]), double buffered:
// the global loads of stage s+1 are in flight while stage s is multiplied,
// and one barrier separates the stages.  Within a 16-wide k block the four
// MFMAs take k = 4*(lane/16) + q (q = 0..3) instead of consecutive k, so a
// lane fetches its 4 values of A and of B with one 16-byte LDS read each.
// vec: the operands allow 16-byte global loads (leading dimensions, batch
// strides and base addresses are multiples of 16 bytes); edge vectors fall
// back to element loads either way.
// C is written only after the whole K loop, so a call may overwrite its own
// B operand when each output tile reads only its own columns of B (and the
// same for A and rows); the dispatcher keeps such calls on 64-wide tiles.
template <typename T, int TA, int TB, int BM, int BN, int DEPTH = 1, int KB = 128>
__global__ __launch_bounds__(64 * (BM / 32) * (BN / 32)) void gemm_kernel(int M, int N, int K, T alpha, const T* __restrict__ A,
                                                   int64_t lda, int64_t sA, const T* __restrict__ B,
                                                   int64_t ldb, int64_t sB, T beta, T* C, int64_t ldc,
                                                   int64_t sC, int mode, int vec, int swz, GemmRows rows) {
  typedef typename Vec16<T>::type V;
  constexpr int VW = 16 / sizeof(T);            // elements per 16-byte vector
  constexpr int KT = KB / (int)sizeof(T);       // k per stage
  constexpr int LDK = KT;                       // LDS row length
  constexpr int CPR = KT / VW;                  // 16-byte chunks per [row][k] row
  constexpr int SWM = CPR >= 16 ? 15 : 7;       // swizzle mask
  static_assert(CPR >= 8 && (CPR & (CPR - 1)) == 0, "stage width");
  constexpr int WGN = BN / 32;                  // waves along N
  constexpr int NT = 64 * (BM / 32) * WGN;      // threads
  constexpr int WM = 32, WN = 32;               // per-wave outputs
  constexpr int FM = WM / 16, FN = WN / 16;     // MFMA blocks per wave
  constexpr int AV = BM * KT / VW / NT;         // vectors per thread per stage
  constexpr int BV = BN * KT / VW / NT;
  static_assert(AV >= 1 && BV >= 1, "tile too small");
  // An operand whose global rows run along k (TA = 0, TB = 1) sits in LDS
  // as [row][k] and is read 16 bytes at a time; the other kind (TA = 1,
  // TB = 0) sits as [k][row], so that its 16-byte global vectors go to LDS
  // unchanged (a [row][k] store would scatter them over rows and collide
  // in the banks), and is read one element per MFMA operand.
  // [row][k] rows are unpadded and the 16-byte chunk c of row r is kept at
  // chunk c ^ g(r), g(r) = (r ^ (r >> 1)) & SWM (a Gray code): the 16 rows
  // read by a wave at one k, and the rows stored by consecutive lanes, then
  // spread over distinct bank groups both for 8 lanes per LDS cycle over 32
  // banks and for 16 lanes over 64 banks.  [k][row] rows are padded by 4
  // elements so that the k rows 4 apart read by lane groups in one LDS
  // cycle fall in different banks.
  constexpr int PK = 4;
  constexpr int AR = TA == 0 ? BM : KT, AC = TA == 0 ? LDK : BM + PK;
  constexpr int BR = TB == 1 ? BN : KT, BC = TB == 1 ? LDK : BN + PK;
  __shared__ __align__(16) T As[2][AR][AC];
  __shared__ __align__(16) T Bs[2][BR][BC];
  // Workgroups are handed to the 8 XCDs round-robin by linear id; with swz
  // the tiles are renumbered so that each XCD runs a contiguous range of
  // (tile, matrix) pairs, i.e. whole matrices, whose operand panels then
  // stay in that XCD's L2.  The map is a bijection for any grid size.
  int64_t tx = blockIdx.x, ty = blockIdx.y, tz = blockIdx.z;
  if (swz) {
    const int64_t gx = gridDim.x, gxy = gx * gridDim.y;
    const int64_t tot = gxy * gridDim.z, L = tx + gx * ty + gxy * tz;
    const int64_t q = tot / 8, r = tot % 8, x = L % 8, s = L / 8;
    const int64_t Lp = x < r ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
    tz = Lp / gxy;
    ty = (Lp - tz * gxy) / gx;
    tx = Lp - tz * gxy - ty * gx;
  }
  const int row0 = (int)ty * BM;
  const int col0 = (int)tx * BN;
  const int64_t bz = tz;
  if ((mode & GEMM_LOWER) && col0 > row0 + BM - 1) return;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  int kbeg = 0, kend = K;
  if (mode & GEMM_KFROM_DIAG) kbeg = (max(row0, col0) / KT) * KT;
  if (mode & GEMM_KTO_DIAG) kend = min(K, row0 + BM);
  // padded batch (GemmRows): the nonzero index set of matrix bz is
  // [0, na) u [sp, sp + nb)
  int na = 0, nb = 0;
  const int sp = rows.split;
  auto meets = [&](int lo, int hi) { return (lo < na && hi > 0) || (nb > 0 && lo < sp + nb && hi > sp); };
  if (rows.na) {
    na = rows.na[bz];
    nb = rows.nb ? rows.nb[bz] : 0;
    const int g0 = kbeg + rows.k_off, g1 = kend + rows.k_off;
    int lo = g1, hi = g0;   // hull of the set within [g0, g1)
    if (g0 < na && g1 > 0) {
      lo = max(g0, 0);
      hi = min(g1, na);
    }
    if (nb > 0 && g0 < sp + nb && g1 > sp) {
      lo = min(lo, max(g0, sp));
      hi = max(hi, min(g1, sp + nb));
    }
    const bool live = lo < hi && meets(rows.r_off + row0, rows.r_off + row0 + BM) &&
                      meets(rows.c_off + col0, rows.c_off + col0 + BN);
    if (!live) {
      if (beta == T(1)) return;
      kend = kbeg;   // no product: the epilogue writes beta C
    } else {
      kbeg = max(kbeg, ((lo - rows.k_off) / KT) * KT);
      kend = hi - rows.k_off;
    }
  }
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int wr = wv / WGN, wc = wv % WGN;

  V ra[AV], rb[BV], ra2[AV], rb2[BV];
  // element offset within a [row][k] LDS row of the chunk holding k (k a
  // multiple of VW)
  auto sw = [](int r, int k) { return ((k / VW) ^ ((r ^ (r >> 1)) & SWM)) * VW; };
  // tile coordinates (row or column index, k) of the first element of
  // vector q of this thread
  auto a_coord = [&](int q, int& i, int& k) {
    const int v = tid + NT * q;
    if (TA == 0) {
      i = v / (KT / VW);
      k = (v % (KT / VW)) * VW;
    } else {
      k = v / (BM / VW);
      i = (v % (BM / VW)) * VW;
    }
  };
  auto b_coord = [&](int q, int& j, int& k) {
    const int v = tid + NT * q;
    if (TB == 1) {
      j = v / (KT / VW);
      k = (v % (KT / VW)) * VW;
    } else {
      k = v / (BN / VW);
      j = (v % (BN / VW)) * VW;
    }
  };
  auto load = [&](int k0, V (&ra)[AV], V (&rb)[BV]) {
#pragma unroll
    for (int q = 0; q < AV; ++q) {
      int i, k;
      a_coord(q, i, k);
      const int gi = row0 + i, gk = k0 + k;
      V x;
      if (TA == 0) {
        if (vec && gi < M && gk + VW <= kend) {
          x = *reinterpret_cast<const V*>(A + (int64_t)gi * lda + gk);
        } else {
#pragma unroll
          for (int c = 0; c < VW; ++c) x[c] = (gi < M && gk + c < kend) ? A[(int64_t)gi * lda + gk + c] : T(0);
        }
      } else {
        if (vec && gk < kend && gi + VW <= M) {
          x = *reinterpret_cast<const V*>(A + (int64_t)gk * lda + gi);
        } else {
#pragma unroll
          for (int c = 0; c < VW; ++c) x[c] = (gi + c < M && gk < kend) ? A[(int64_t)gk * lda + gi + c] : T(0);
        }
      }
      ra[q] = x;
    }
#pragma unroll
    for (int q = 0; q < BV; ++q) {
      int j, k;
      b_coord(q, j, k);
      const int gj = col0 + j, gk = k0 + k;
      V x;
      if (TB == 1) {
        if (vec && gj < N && gk + VW <= kend) {
          x = *reinterpret_cast<const V*>(B + (int64_t)gj * ldb + gk);
        } else {
#pragma unroll
          for (int c = 0; c < VW; ++c) x[c] = (gj < N && gk + c < kend) ? B[(int64_t)gj * ldb + gk + c] : T(0);
        }
      } else {
        if (vec && gk < kend && gj + VW <= N) {
          x = *reinterpret_cast<const V*>(B + (int64_t)gk * ldb + gj);
        } else {
#pragma unroll
          for (int c = 0; c < VW; ++c) x[c] = (gj + c < N && gk < kend) ? B[(int64_t)gk * ldb + gj + c] : T(0);
        }
      }
      rb[q] = x;
    }
  };
  auto store = [&](int buf, const V (&ra)[AV], const V (&rb)[BV]) {
#pragma unroll
    for (int q = 0; q < AV; ++q) {
      int i, k;
      a_coord(q, i, k);
      if constexpr (TA == 0) *reinterpret_cast<V*>(&As[buf][i][sw(i, k)]) = ra[q];
      else *reinterpret_cast<V*>(&As[buf][k][i]) = ra[q];
    }
#pragma unroll
    for (int q = 0; q < BV; ++q) {
      int j, k;
      b_coord(q, j, k);
      if constexpr (TB == 1) *reinterpret_cast<V*>(&Bs[buf][j][sw(j, k)]) = rb[q];
      else *reinterpret_cast<V*>(&Bs[buf][k][j]) = rb[q];
    }
  };

  typename Acc<T>::type acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = (typename Acc<T>::type){0, 0, 0, 0};

  // Old C values: loaded just before the last K stage is multiplied (the
  // stage-staging registers are free by then), so that their latency hides
  // behind that stage.  Only this workgroup writes its C tile, and only
  // after the loop, so the values are those of the call's start even when C
  // aliases A or B.
  T cold[FM][FN][4];
  auto load_c = [&]() {
#pragma unroll
    for (int mi = 0; mi < FM; ++mi)
#pragma unroll
      for (int ni = 0; ni < FN; ++ni)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int gi = row0 + wr * WM + mi * 16 + Acc<T>::row(lane, v);
          const int gj = col0 + wc * WN + ni * 16 + (lane & 15);
          const bool ok = gi < M && gj < N && !((mode & GEMM_LOWER) && gj > gi);
          cold[mi][ni][v] = (ok && beta != T(0)) ? C[(int64_t)gi * ldc + gj] : T(0);
        }
  };

  const int ks = 4 * (lane >> 4);
  // a wave whose 32 x 32 outputs all lie above the diagonal of a
  // lower-triangle product has nothing to store: it only helps stage the
  // operands and keeps the barriers
  // (likewise a wave whose rows or columns are padding only: its products
  // are exact zeros, and its outputs become beta C)
  const bool idle = ((mode & GEMM_LOWER) && col0 + wc * WN > row0 + wr * WM + WM - 1) ||
                    (rows.na && !(meets(rows.r_off + row0 + wr * WM, rows.r_off + row0 + wr * WM + WM) &&
                                  meets(rows.c_off + col0 + wc * WN, rows.c_off + col0 + wc * WN + WN)));
  auto compute = [&](int buf) {
    if (idle) return;
#pragma unroll
    for (int kb = 0; kb < KT; kb += 16) {
      T av[FM][4], bv[FN][4];
#pragma unroll
      for (int mi = 0; mi < FM; ++mi) {
        const int i = wr * WM + mi * 16 + (lane & 15);
        if constexpr (TA == 0) {
#pragma unroll
          for (int h = 0; h < 4; h += VW) {
            const V x = *reinterpret_cast<const V*>(&As[buf][i][sw(i, kb + ks + h)]);
#pragma unroll
            for (int c = 0; c < VW; ++c) av[mi][h + c] = x[c];
          }
        } else {
#pragma unroll
          for (int h = 0; h < 4; ++h) av[mi][h] = As[buf][kb + ks + h][i];
        }
      }
#pragma unroll
      for (int ni = 0; ni < FN; ++ni) {
        const int j = wc * WN + ni * 16 + (lane & 15);
        if constexpr (TB == 1) {
#pragma unroll
          for (int h = 0; h < 4; h += VW) {
            const V x = *reinterpret_cast<const V*>(&Bs[buf][j][sw(j, kb + ks + h)]);
#pragma unroll
            for (int c = 0; c < VW; ++c) bv[ni][h + c] = x[c];
          }
        } else {
#pragma unroll
          for (int h = 0; h < 4; ++h) bv[ni][h] = Bs[buf][kb + ks + h][j];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int mi = 0; mi < FM; ++mi)
#pragma unroll
          for (int ni = 0; ni < FN; ++ni) acc[mi][ni] = Acc<T>::mfma(av[mi][q], bv[ni][q], acc[mi][ni]);
    }
  };
  if (DEPTH == 1) {
    int buf = 0;
    if (kbeg < kend) {
      load(kbeg, ra, rb);
      store(0, ra, rb);
    }
    __syncthreads();
    int k0 = kbeg;
    for (; k0 + KT < kend; k0 += KT) {
      load(k0 + KT, ra, rb);
      compute(buf);
      store(buf ^ 1, ra, rb);
      __syncthreads();
      buf ^= 1;
    }
    load_c();
    if (k0 < kend) compute(buf);   // last stage (no LDS writes follow)
  } else {
    // two stages in flight: the registers of stage s+2 are loaded while
    // stage s is multiplied and stage s+1 waits in the other register set
    if (kbeg < kend) {
      load(kbeg, ra, rb);
      store(0, ra, rb);
    }
    if (kbeg + KT < kend) load(kbeg + KT, ra2, rb2);
    __syncthreads();
    for (int k0 = kbeg; k0 < kend; k0 += 2 * KT) {
      if (k0 + 2 * KT < kend) load(k0 + 2 * KT, ra, rb);
      compute(0);
      if (k0 + KT < kend) store(1, ra2, rb2);
      __syncthreads();
      if (k0 + KT >= kend) break;
      if (k0 + 3 * KT < kend) load(k0 + 3 * KT, ra2, rb2);
      compute(1);
      if (k0 + 2 * KT < kend) store(0, ra, rb);
      __syncthreads();
    }
    load_c();
  }
  // Epilogue
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
        const T r = alpha * acc[mi][ni][v];
        C[(int64_t)gi * ldc + gj] = (beta == T(0)) ? r : r + beta * cold[mi][ni][v];
      }
}

// Factors the b x b diagonal block (b <= DB) at (k0, k0) of every matrix and
// inverts the factor, in one pass.  The block is split into 8 x 8 tiles; the
// 136 lower tiles of L live in the registers of waves 0-2 (one tile per
// thread) and the 136 lower tiles of X = L^{-1} in waves 3-5, so no wave
// holds both kinds.  Step j (right-looking Cholesky and forward elimination
// on L X = I, both driven by column j of L):
//   1. the owner of the diagonal tile takes the pivot L_jj;
//   2. the owners of tile column j/8 of L scale column j and publish it in
//      LDS; the owners of tile row j/8 of X scale row j of X by 1 / L_jj and
//      publish it;
//   3. every L tile gets the rank-1 update with column j, and every X tile
//      below row j subtracts L_ij X_j.
// The published vectors are zero outside the rows (columns) they cover, so
// the updates need no element tests.  The step loop is unrolled by 8 so that
// every register index is static.  Rows and columns beyond b are identity.
// Writes L back (upper part of the block zeroed) and L^{-1} (zero above the
// diagonal) to the DB x DB block `blk` of Linv[bz].  A non-positive or
// non-finite pivot sets info[bz] (first failing global row + 1) and is
// replaced by 1.
constexpr int DF_THREADS = 384;
template <typename T>
__global__ __launch_bounds__(DF_THREADS) void diag_factor_kernel(T* A, int64_t lda, int64_t sA, int k0, int b,
                                                                 T* Linv, int64_t sL, int blk, int* info) {
  constexpr int TS = 8, NT = DB / TS, NLT = NT * (NT + 1) / 2, XOFF = 192;
  __shared__ T vec[DB];    // column j of L below the diagonal, zero elsewhere
  __shared__ T vecx[DB];   // row j of X up to the diagonal, zero elsewhere
  __shared__ T pinv;
  __shared__ int bad;
  const int64_t bz = blockIdx.x;
  T* a = A + bz * sA + (int64_t)k0 * lda + k0;
  const int t = threadIdx.x;
  const bool isL = t < NLT;
  const bool isX = t >= XOFF && t < XOFF + NLT;
  // lower tile (I, C), I >= C, of this thread: index = I (I + 1) / 2 + C
  int I = -1, C = -1;
  if (isL || isX) {
    int q = isL ? t : t - XOFF, r = 0;
    while (q > r) {
      q -= r + 1;
      ++r;
    }
    I = r;
    C = q;
  }
  if (t == 0) bad = 0;
  T r[TS][TS];
  if (isL) {
#pragma unroll
    for (int rr = 0; rr < TS; ++rr)
#pragma unroll
      for (int cc = 0; cc < TS; ++cc) {
        const int row = TS * I + rr, col = TS * C + cc;
        r[rr][cc] = (row < b && col < b) ? a[(int64_t)row * lda + col] : (row == col ? T(1) : T(0));
      }
  } else if (isX) {
#pragma unroll
    for (int rr = 0; rr < TS; ++rr)
#pragma unroll
      for (int cc = 0; cc < TS; ++cc) r[rr][cc] = (TS * I + rr == TS * C + cc) ? T(1) : T(0);
  }
  __syncthreads();
  const int nJ = (b + TS - 1) / TS;
  for (int J = 0; J < nJ; ++J) {
#pragma unroll
    for (int jj = 0; jj < TS; ++jj) {
      const int j = TS * J + jj;
      if (j >= b) break;
      if (isL && I == J && C == J) {
        T d = r[jj][jj];
        if (!(d > T(0)) || !(d < T(3.0e38))) {
          if (bad == 0) bad = k0 + j + 1;
          d = T(1);
        }
        d = sqrt(d);
        r[jj][jj] = d;
        pinv = T(1) / d;
      }
      __syncthreads();
      const T inv = pinv;
      if (isL && C == J) {
#pragma unroll
        for (int rr = 0; rr < TS; ++rr) {
          const int row = TS * I + rr;
          if (row > j) r[rr][jj] *= inv;
          vec[row] = row > j ? r[rr][jj] : T(0);
        }
      } else if (isX && I == J) {
#pragma unroll
        for (int cc = 0; cc < TS; ++cc) {
          const int col = TS * C + cc;
          if (col <= j) r[jj][cc] *= inv;
          vecx[col] = col <= j ? r[jj][cc] : T(0);
        }
      }
      __syncthreads();
      if (isL && C >= J) {
        T li[TS], lc[TS];
#pragma unroll
        for (int q = 0; q < TS; ++q) {
          li[q] = vec[TS * I + q];
          lc[q] = vec[TS * C + q];
        }
#pragma unroll
        for (int rr = 0; rr < TS; ++rr)
#pragma unroll
          for (int cc = 0; cc < TS; ++cc) r[rr][cc] = fma(-li[rr], lc[cc], r[rr][cc]);
      } else if (isX && I >= J && C <= J) {
        T lr[TS], xc[TS];
#pragma unroll
        for (int q = 0; q < TS; ++q) {
          lr[q] = vec[TS * I + q];
          xc[q] = vecx[TS * C + q];
        }
#pragma unroll
        for (int rr = 0; rr < TS; ++rr)
#pragma unroll
          for (int cc = 0; cc < TS; ++cc) r[rr][cc] = fma(-lr[rr], xc[cc], r[rr][cc]);
      }
    }
  }
  __syncthreads();
  T* li = Linv + bz * sL + (int64_t)blk * DB * DB;
  if (isL) {
#pragma unroll
    for (int rr = 0; rr < TS; ++rr)
#pragma unroll
      for (int cc = 0; cc < TS; ++cc) {
        const int row = TS * I + rr, col = TS * C + cc;
        if (row < b && col < b) a[(int64_t)row * lda + col] = col <= row ? r[rr][cc] : T(0);
      }
  } else if (isX) {
#pragma unroll
    for (int rr = 0; rr < TS; ++rr)
#pragma unroll
      for (int cc = 0; cc < TS; ++cc) {
        const int row = TS * I + rr, col = TS * C + cc;
        li[row * DB + col] = (row < b && col < b && col <= row) ? r[rr][cc] : T(0);
      }
  }
  // upper tiles: zero in the block of A and in the inverse
  for (int e = t; e < DB * DB; e += DF_THREADS) {
    const int row = e / DB, col = e - row * DB;
    if (col / TS > row / TS) {
      li[e] = T(0);
      if (row < b && col < b) a[(int64_t)row * lda + col] = T(0);
    }
  }
  if (t == 0 && bad && info && info[bz] == 0) info[bz] = bad;
}

// Blocked variant of the diagonal step for blocks of order b, b a multiple
// of 16 (b <= DB): the same outputs as diag_factor_kernel (L in place with
// the upper part of the block zeroed, X = L^{-1} into block `blk` of Linv,
// info for a bad pivot), with far fewer workgroup barriers.  The block lives
// in LDS as one array of 16 x 16 lower tiles (element (r, c) of a tile at
// r * 16 + (c ^ r) so that reading a tile column is free of bank
// conflicts); a tile holds A, then L, then M = X_ii L_ij, then X, so that
// the block takes 74 KB in FP64 and two workgroups share a CU.  L leaves for
// global memory as its tiles become final.  For each tile column p:
//   1. wave 0 factors the diagonal tile and inverts it in registers,
//      column by column, exchanging values with lane shuffles (no
//      barriers); L_pp goes to global memory, X_pp to the tile;
//   2. panel phase, one tile per item: L_ip = A_ip X_pp^T (i > p; to the tile
//      and to global memory) and M_pk = X_pp L_pk (k < p, in place: L row p
//      has no other use left);
//   3. wave 0 updates and factors the next diagonal tile, the others form
//      row p of X, X_pj = -sum_{j<=k<p} M_pk X_kj, held in registers until
//      every wave has read row p's M tiles, and share out the trailing tiles
//      A_ij -= L_ip L_jp^T (p < j <= i).
// Tile products run on the 16x16x4 MFMAs.
constexpr int DK_THREADS = 512;
constexpr int NW_DK = DK_THREADS / 64;   // waves
constexpr int DK_TILES = (DB / 16) * (DB / 16 + 1) / 2;
static_assert(DB == 128, "the tile-row lookup of the diagonal kernel assumes 8 x 8 tiles");
__device__ inline int dk_tile(int I, int J) { return I * (I + 1) / 2 + J; }
__device__ inline int dk_at(int r, int c) { return r * 16 + (c ^ r); }
__device__ inline double dk_bcast(double v, int lane) {
  const unsigned long long u = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)(u & 0xffffffffull), lane);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), lane);
  return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}
__device__ inline float dk_bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
// Value of lane 16 * (lane / 16) + J (row broadcast within each group of 16
// lanes, DPP row_newbcast): no trip through the LDS unit.
template <int J>
__device__ inline float dk_rowbcast(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + J, 0xf, 0xf, false));
}
template <int J>
__device__ inline double dk_rowbcast(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffll), 0x150 + J, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), 0x150 + J, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// 1/sqrt(d) for the pivots of the wave-level factorisation: the hardware
// estimate refined by Newton steps y <- y (3/2 - d y^2 / 2) (two for FP64,
// one for FP32), a few ulp from the rounded value.
__device__ inline double dk_rsqrt(double d) {
  double y = __builtin_amdgcn_rsq(d);
  const double h = 0.5 * d;
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(y, fma(-h * y, y, 0.5), y);
  return y;
}
__device__ inline float dk_rsqrt(float d) {
  float y = __builtin_amdgcn_rsqf(d);
  const float h = 0.5f * d;
  return fmaf(y, fmaf(-h * y, y, 0.5f), y);
}

// acc += op(P) op(Q) over one 16-wide k range for the calling wave:
// P[r][k] (tile p, rows r) times Q^T (qt = 1: Q[c][k]) or Q (qt = 0: Q[k][c]).
template <typename T>
__device__ inline void dk_mma(typename Acc<T>::type& acc, const T* P, const T* Q, int qt, int lane) {
  const int r = lane & 15, kk = lane >> 4;
  T a[4], b[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = 4 * s + kk;
    a[s] = P[dk_at(r, k)];
    b[s] = qt ? Q[dk_at(r, k)] : Q[dk_at(k, r)];
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = Acc<T>::mfma(a[s], b[s], acc);
}

template <typename T>
__global__ __launch_bounds__(DK_THREADS) void diag_block_kernel(T* A, int64_t lda, int64_t sA, int k0, int b,
                                                                T* Linv, int64_t sL, int blk, int* info) {
  extern __shared__ __align__(16) unsigned char dk_lds[];
  // one array of lower tiles: tile (i, j) holds A, then L once its panel
  // step is done, then (row i's inverse step) M = X_ii L_ij, and finally X
  T* Ts = reinterpret_cast<T*>(dk_lds);
  const int64_t bz = blockIdx.x;
  T* a = A + bz * sA + (int64_t)k0 * lda + k0;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nt = b >> 4;
  typedef typename Acc<T>::type AccT;
  // load the lower tiles (upper part of diagonal tiles as zero).  Every
  // load is issued before the first LDS write.
  constexpr int LD_IT = DK_TILES * 256 / DK_THREADS;
  static_assert(LD_IT * DK_THREADS == DK_TILES * 256, "load split");
  T ld[LD_IT];
#pragma unroll
  for (int it = 0; it < LD_IT; ++it) {
    const int e = tid + it * DK_THREADS;
    const int q = e >> 8, rc = e & 255, r = rc >> 4, c = rc & 15;
    const int I = (q >= 1) + (q >= 3) + (q >= 6) + (q >= 10) + (q >= 15) + (q >= 21) + (q >= 28);
    const int J = q - I * (I + 1) / 2;
    ld[it] = (I < nt && (I != J || c <= r)) ? a[(int64_t)(16 * I + r) * lda + 16 * J + c] : T(0);
  }
#pragma unroll
  for (int it = 0; it < LD_IT; ++it) {
    const int e = tid + it * DK_THREADS;
    const int q = e >> 8, rc = e & 255, r = rc >> 4, c = rc & 15;
    Ts[q * 256 + dk_at(r, c)] = ld[it];
  }
  __syncthreads();
  int bad = 0;   // wave 0: first failing row + 1
  // wave 0: factor and invert diagonal tile p in registers.  Lane (r, g)
  // holds columns g + 4t of row r of the whole symmetric tile (both
  // triangles, updated alike, so they stay exactly equal): row j of A and X
  // reaches every lane by a row broadcast from lane j of its own group, and
  // only column j of A (one value per lane) needs a lane shuffle.  L_pp
  // goes to global memory (upper triangle zero), X_pp to tile (p, p).
  auto factor_diag = [&](int p) {
    T* Tp = Ts + dk_tile(p, p) * 256;
    const int r = lane & 15, g = lane >> 4;
    T av[4], xv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int c = g + 4 * t;
      av[t] = c <= r ? Tp[dk_at(r, c)] : Tp[dk_at(c, r)];
      xv[t] = c == r ? T(1) : T(0);
    }
    auto step = [&](auto jc) {
      constexpr int j = decltype(jc)::value;
      constexpr int tj = j >> 2, gj = j & 3;
      // Row j of A is needed in columns c > j (registers t >= tj), row j of
      // X in columns c <= j (t <= tj; it is zero to the right of j, so the
      // columns of X right of j are left as they are).
      T arow[4], xrow[4];
#pragma unroll
      for (int t = tj; t < 4; ++t) arow[t] = dk_rowbcast<j>(av[t]);   // A[j][g + 4t]
#pragma unroll
      for (int t = 0; t <= tj; ++t) xrow[t] = dk_rowbcast<j>(xv[t]);  // X[j][g + 4t]
      const T acol = __shfl(av[tj], r + 16 * gj, 64);   // A[r][j]
      T d = dk_bcast(av[tj], j + 16 * gj);
      if (!(d > T(0)) || !(d < T(3.0e38))) {
        if (bad == 0) bad = k0 + 16 * p + j + 1;
        d = T(1);
      }
      const T inv = dk_rsqrt(d);
      const T ljj = d * inv;
      const T lrj = acol * inv;
      const T lrm = r > j ? lrj : T(0);   // rows above the pivot keep their values
#pragma unroll
      for (int t = tj + 1; t < 4; ++t) av[t] = fma(-lrm, arow[t] * inv, av[t]);
      {
        const T lcm = g > gj ? arow[tj] * inv : T(0);
        const T an = fma(-lrm, lcm, av[tj]);
        av[tj] = (g == gj && r >= j) ? (r == j ? ljj : lrj) : an;
      }
#pragma unroll
      for (int t = 0; t <= tj; ++t) {
        const T xjc = xrow[t] * inv;
        xv[t] = r == j ? xjc : fma(-lrm, xjc, xv[t]);
      }
    };
    step(std::integral_constant<int, 0>{});
    step(std::integral_constant<int, 1>{});
    step(std::integral_constant<int, 2>{});
    step(std::integral_constant<int, 3>{});
    step(std::integral_constant<int, 4>{});
    step(std::integral_constant<int, 5>{});
    step(std::integral_constant<int, 6>{});
    step(std::integral_constant<int, 7>{});
    step(std::integral_constant<int, 8>{});
    step(std::integral_constant<int, 9>{});
    step(std::integral_constant<int, 10>{});
    step(std::integral_constant<int, 11>{});
    step(std::integral_constant<int, 12>{});
    step(std::integral_constant<int, 13>{});
    step(std::integral_constant<int, 14>{});
    step(std::integral_constant<int, 15>{});
    // every lane has read the tile (before the first step): it now takes X_pp
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int c = g + 4 * t;
      a[(int64_t)(16 * p + r) * lda + 16 * p + c] = c <= r ? av[t] : T(0);
      Tp[dk_at(r, c)] = xv[t];
    }
  };
  // the tile of an MFMA accumulator (lane layout of Acc) to tile slot S and,
  // if g is given, to global memory at g (leading dimension lda)
  auto put_tile = [&](const AccT& acc, T* S, T* gm, T sign) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = Acc<T>::row(lane, v), c = lane & 15;
      const T x = sign * acc[v];
      S[dk_at(r, c)] = x;
      if (gm) gm[(int64_t)r * lda + c] = x;
    }
  };
  // A_ij -= L_ip L_jp^T by the calling wave
  auto trail = [&](int p, int i, int j) {
    AccT acc = {0, 0, 0, 0};
    dk_mma<T>(acc, Ts + dk_tile(i, p) * 256, Ts + dk_tile(j, p) * 256, 1, lane);
    T* Aij = Ts + dk_tile(i, j) * 256;
#pragma unroll
    for (int v = 0; v < 4; ++v) Aij[dk_at(Acc<T>::row(lane, v), lane & 15)] -= acc[v];
  };
  // X_pj (j < p) of row p of X = L^{-1}: -sum_{j<=k<p} M_pk X_kj with
  // M_pk = X_pp L_pk (tiles (p, k) hold M by then), into registers
  auto xrow_tile = [&](int p, int j) {
    AccT acc = {0, 0, 0, 0};
    for (int k = j; k < p; ++k) dk_mma<T>(acc, Ts + dk_tile(p, k) * 256, Ts + dk_tile(k, j) * 256, 0, lane);
    return acc;
  };
  // panel phase of step p: L_ip = A_ip X_pp^T (i > p; to the tile and to
  // global memory) and M_pk = X_pp L_pk (k < p; in place), one tile per item
  auto panel = [&](int p) {
    const int nl = nt - 1 - p;
    for (int item = wv; item < nl + p; item += NW_DK) {
      AccT acc = {0, 0, 0, 0};
      if (item < nl) {
        const int i = p + 1 + item;
        T* Tip = Ts + dk_tile(i, p) * 256;
        dk_mma<T>(acc, Tip, Ts + dk_tile(p, p) * 256, 1, lane);
        put_tile(acc, Tip, a + (int64_t)(16 * i) * lda + 16 * p, T(1));
      } else {
        const int k = item - nl;
        T* Tpk = Ts + dk_tile(p, k) * 256;
        dk_mma<T>(acc, Ts + dk_tile(p, p) * 256, Tpk, 0, lane);
        put_tile(acc, Tpk, nullptr, T(1));
      }
    }
  };
  if (wv == 0) factor_diag(0);
  __syncthreads();
  for (int p = 0; p < nt; ++p) {
    panel(p);
    __syncthreads();
    if (p + 1 == nt) break;
    // wave 0: the next diagonal tile's update and factorisation
    // (lookahead); the other waves: row p of X (inputs final: M row p, X
    // rows above), heaviest tile first, held in registers until every wave
    // has read row p's M tiles, then the trailing tiles
    const int m = nt - 1 - p, ntr = m * (m + 1) / 2;
    AccT xacc = {0, 0, 0, 0};
    int xj = -1;
    if (wv == 0) {
      trail(p, p + 1, p + 1);
      __builtin_amdgcn_wave_barrier();
      factor_diag(p + 1);
    } else {
      for (int item = wv - 1; item < p + ntr - 1; item += NW_DK - 1) {
        if (item < p) {
          xacc = xrow_tile(p, item);
          xj = item;
        } else {
          const int q = item - p + 1;
          int ii = 0;
          while ((ii + 1) * (ii + 2) / 2 <= q) ++ii;
          const int jj = q - ii * (ii + 1) / 2;
          trail(p, p + 1 + ii, p + 1 + jj);
        }
      }
    }
    __syncthreads();
    if (xj >= 0) put_tile(xacc, Ts + dk_tile(p, xj) * 256, nullptr, T(-1));
    // the next panel phase reads neither row p nor the tiles written here
  }
  // row nt - 1 of X (its M tiles were formed by the last panel phase)
  {
    AccT xacc = {0, 0, 0, 0};
    int xj = -1;
    for (int j = wv; j < nt - 1; j += NW_DK) {
      xacc = xrow_tile(nt - 1, j);
      xj = j;
    }
    __syncthreads();
    if (xj >= 0) put_tile(xacc, Ts + dk_tile(nt - 1, xj) * 256, nullptr, T(-1));
    __syncthreads();
  }
  // write X (zero above the diagonal and outside the b x b block) and the
  // zero upper tiles of the L block (its lower tiles left on the way), VW
  // consecutive columns per thread (b and the tile edges are multiples of
  // 16, so a group never straddles them)
  typedef typename Vec16<T>::type V;
  constexpr int VW = 16 / sizeof(T);
  T* li = Linv + bz * sL + (int64_t)blk * DB * DB;
  const bool vec = ((lda | sA | k0) % VW) == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0;
  const bool vecl = (sL % VW) == 0 && (reinterpret_cast<uintptr_t>(Linv) & 15) == 0;
  for (int e = tid; e < DB * DB / VW; e += DK_THREADS) {
    const int row = e / (DB / VW), col = (e - row * (DB / VW)) * VW;
    const int I = row >> 4, J = col >> 4, r = row & 15;
    const bool tile = row < b && col < b && J <= I;
    V xo;
#pragma unroll
    for (int k = 0; k < VW; ++k) {
      const int c = (col + k) & 15;
      const bool in = tile && col + k <= row;
      xo[k] = in ? Ts[dk_tile(I, J) * 256 + dk_at(r, c)] : T(0);
    }
    if (vecl) {
      *reinterpret_cast<V*>(li + e * VW) = xo;
    } else {
#pragma unroll
      for (int k = 0; k < VW; ++k) li[e * VW + k] = xo[k];
    }
    if (row < b && col < b && J > I) {
      T* dst = a + (int64_t)row * lda + col;
      if (vec) {
        *reinterpret_cast<V*>(dst) = V{};
      } else {
#pragma unroll
        for (int k = 0; k < VW; ++k) dst[k] = T(0);
      }
    }
  }
  if (tid == 0 && bad && info && info[bz] == 0) info[bz] = bad;
}

// Y (nb x nb per matrix) = identity.
// Element-wise helpers of the factorisation.  With vec (leading
// dimensions, batch strides, widths and base addresses multiples of 16
// bytes) every thread moves 16-byte vectors; the grid's x dimension strides
// over one matrix, y is the batch entry.
template <typename T>
bool vec16_ok(const void* p, int64_t ld, int64_t stride, int width) {
  constexpr int VW = 16 / sizeof(T);
  return (reinterpret_cast<uintptr_t>(p) & 15) == 0 && ld % VW == 0 && stride % VW == 0 && width % VW == 0;
}
// workgroups per matrix: about 4 items per thread, at most 8192 in all
inline int helper_blocks(int64_t items, int batch) {
  const int64_t cap = std::max<int64_t>(4, 8192 / std::max(1, batch));
  return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (items + 1023) / 1024));
}

// Y[r][c] = (r == c) for r, c < nb.
template <typename T>
__global__ __launch_bounds__(256) void eye_kernel(T* Y, int64_t ldy, int64_t sY, int nb, int vec) {
  typedef typename Vec16<T>::type V;
  constexpr int VW = 16 / sizeof(T);
  T* y = Y + (int64_t)blockIdx.y * sY;
  const int64_t step = (int64_t)gridDim.x * 256;
  if (vec) {
    const int vpr = nb / VW;
    const int64_t tot = (int64_t)nb * vpr;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += step) {
      const int r = (int)(e / vpr), c = (int)(e - (int64_t)r * vpr) * VW;
      V x;
#pragma unroll
      for (int l = 0; l < VW; ++l) x[l] = c + l == r ? T(1) : T(0);
      *reinterpret_cast<V*>(y + (int64_t)r * ldy + c) = x;
    }
  } else {
    const int64_t tot = (int64_t)nb * nb;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += step) {
      const int r = (int)(e / nb), c = (int)(e - (int64_t)r * nb);
      y[(int64_t)r * ldy + c] = c == r ? T(1) : T(0);
    }
  }
}

template <typename T>
void launch_eye(hipStream_t st, T* Y, int64_t ldy, int64_t sY, int nb, int batch) {
  const int vec = vec16_ok<T>(Y, ldy, sY, nb);
  const int64_t items = (int64_t)nb * nb / (vec ? 16 / sizeof(T) : 1);
  hipLaunchKernelGGL(eye_kernel<T>, dim3(helper_blocks(items, batch), batch), dim3(256), 0, st, Y, ldy, sY, nb, vec);
}

// Y[r][c] = L[r][c] for r, c < h.
template <typename T>
__global__ __launch_bounds__(256) void copy_block_kernel(const T* __restrict__ L, int64_t ldl, int64_t sL, T* Y,
                                                          int64_t ldy, int64_t sY, int h, int vec) {
  typedef typename Vec16<T>::type V;
  constexpr int VW = 16 / sizeof(T);
  const T* l = L + (int64_t)blockIdx.y * sL;
  T* y = Y + (int64_t)blockIdx.y * sY;
  const int step = gridDim.x * 256;
  if (vec) {
    const int vpr = h / VW, tot = h * vpr;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < tot; e += step) {
      const int r = e / vpr, c = (e - r * vpr) * VW;
      *reinterpret_cast<V*>(y + (int64_t)r * ldy + c) = *reinterpret_cast<const V*>(l + (int64_t)r * ldl + c);
    }
  } else {
    for (int e = blockIdx.x * 256 + threadIdx.x; e < h * h; e += step) {
      const int r = e / h, c = e - r * h;
      y[(int64_t)r * ldy + c] = l[(int64_t)r * ldl + c];
    }
  }
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

// The same for nb a multiple of 32, by 32 x 32 tiles: the lower tile (I, J)
// is read once (coalesced) into LDS and written to (I, J) and, transposed,
// to (J, I), both coalesced, with 16-byte loads (veci) and stores (veco)
// where the layouts allow them.  One block per lower tile.
template <typename T, typename TO>
__global__ __launch_bounds__(256) void symmetrize_scale_tiled_kernel(const T* in, int64_t ldi, int64_t sI,
                                                                     TO* out, int64_t ldo, int64_t sO,
                                                                     const double* D, int64_t sD, int veci,
                                                                     int veco) {
  typedef typename Vec16<T>::type VI;
  typedef typename Vec16<TO>::type VO;
  constexpr int WI = 16 / sizeof(T), WO = 16 / sizeof(TO);
  __shared__ double tile[32][33];
  __shared__ double dI[32], dJ[32];
  const int64_t bz = blockIdx.y;
  const int q = blockIdx.x, tid = threadIdx.x;
  int I = 0;
  while ((I + 1) * (I + 2) / 2 <= q) ++I;
  const int J = q - I * (I + 1) / 2;
  const T* x = in + bz * sI + (int64_t)(32 * I) * ldi + 32 * J;
  TO* o = out + bz * sO;
  const double* d = D + bz * sD;
  if (tid < 32) dI[tid] = d[32 * I + tid];
  else if (tid < 64) dJ[tid - 32] = d[32 * J + tid - 32];
  if (veci) {
    for (int e = tid; e < 32 * 32 / WI; e += 256) {
      const int r = e / (32 / WI), c = (e - r * (32 / WI)) * WI;
      const VI v = *reinterpret_cast<const VI*>(x + (int64_t)r * ldi + c);
#pragma unroll
      for (int l = 0; l < WI; ++l) tile[r][c + l] = (double)v[l];
    }
  } else {
    for (int e = tid; e < 32 * 32; e += 256) {
      const int r = e >> 5, c = e & 31;
      tile[r][c] = (double)x[(int64_t)r * ldi + c];
    }
  }
  __syncthreads();
  // element (r, c) of tile (I, J) of D sym D, and of its mirror tile (J, I)
  auto low = [&](int r, int c) { return (I != J || c <= r ? tile[r][c] : tile[c][r]) * dI[r] * dJ[c]; };
  auto mir = [&](int r, int c) { return tile[c][r] * dJ[r] * dI[c]; };
  TO* oL = o + (int64_t)(32 * I) * ldo + 32 * J;
  TO* oU = o + (int64_t)(32 * J) * ldo + 32 * I;
  if (veco) {
    for (int e = tid; e < 32 * 32 / WO; e += 256) {
      const int r = e / (32 / WO), c = (e - r * (32 / WO)) * WO;
      VO a;
#pragma unroll
      for (int l = 0; l < WO; ++l) a[l] = (TO)low(r, c + l);
      *reinterpret_cast<VO*>(oL + (int64_t)r * ldo + c) = a;
      if (I != J) {
#pragma unroll
        for (int l = 0; l < WO; ++l) a[l] = (TO)mir(r, c + l);
        *reinterpret_cast<VO*>(oU + (int64_t)r * ldo + c) = a;
      }
    }
  } else {
    for (int e = tid; e < 32 * 32; e += 256) {
      const int r = e >> 5, c = e & 31;
      oL[(int64_t)r * ldo + c] = (TO)low(r, c);
      if (I != J) oU[(int64_t)r * ldo + c] = (TO)mir(r, c);
    }
  }
}

}  // namespace

// ---- GEMM dispatch and tile-shape autotuner -----------------------------
// Tile shapes (rows x columns, bytes of k per stage): 0 = 64x64, 1 = 128x64,
// 2 = 64x128, 3 = 128x128 (128 B); 4 = 64x64, 5 = 32x64 (512 B); 6 = 64x128,
// 7 = 128x64 (256 B).  The choice for a call is looked up by (type, TA, TB,
// mode bits, in-place kind, size classes of M, N and K, power of two of
// the batch size).  Calls that overwrite their own operand (in
// place) are limited to shapes with a single tile column (or row).  The
// table is filled by gemm_autotune(), which times every allowed shape on
// scratch matrices of the first call's size and keeps the fastest; with the
// autotuner off, calls use 64x64 (64x128 / 128x64 in place).
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
// CUTBDDC_AUTOTUNE_LOG=1 prints every tuning decision (with the time of
// each candidate) to stderr.
bool autotune_log() {
  static const bool on = [] {
    const char* e = std::getenv("CUTBDDC_AUTOTUNE_LOG");
    return e && e[0] == '1';
  }();
  return on;
}
bool autotune_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("CUTBDDC_AUTOTUNE");
    return !(e && e[0] == '0');
  }();
  return on;
}
// inplace: 0, or IN_PLACE_A (C == A: the call needs a single tile column)
// or IN_PLACE_B (C == B: a single tile row)
constexpr int IN_PLACE_A = 8, IN_PLACE_B = 16;
// Size classes of the tuning table: tile waste depends on the remainders
// of M and N modulo the tile sizes, so sizes up to 1024 are told apart in
// steps of 32 and up to 8192 in steps of 128; larger ones by powers of two.
inline int size_class(int x) {
  if (x <= 1024) return (x + 31) / 32;
  if (x <= 8192) return 32 + (x + 127) / 128;
  return 1000 + log2b(x);
}
template <typename T>
TuneKey tune_key(int TA, int TB, int M, int N, int K, int batch, int mode, int inplace) {
  return TuneKey{(int)sizeof(T), TA, TB, (mode & 7) | inplace, size_class(M), size_class(N),
                 size_class(std::max(K, 1)), log2b(batch)};
}
constexpr int GEMM_NSHAPES = 8;
const int SBM[GEMM_NSHAPES] = {64, 128, 64, 128, 64, 32, 64, 128};
const int SBN[GEMM_NSHAPES] = {64, 64, 128, 128, 64, 64, 128, 64};
bool shape_allowed(int shape, int M, int N, int inplace) {
  if (inplace == IN_PLACE_A) return SBN[shape] >= N;
  if (inplace == IN_PLACE_B) return SBM[shape] >= M;
  return true;
}

// CUTBDDC_DIAG_BLOCKED=0 selects the register-tile diagonal kernel.
bool diag_blocked_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("CUTBDDC_DIAG_BLOCKED");
    return !(e && e[0] == '0');
  }();
  return on;
}

// CUTBDDC_XCD=0 turns the XCD-contiguous tile order off (for comparison).
bool gemm_xcd_swizzle() {
  static const bool on = [] {
    const char* e = std::getenv("CUTBDDC_XCD");
    return !(e && e[0] == '0');
  }();
  return on;
}

template <typename T>
void gemm_launch(int shape, hipStream_t st, int TA, int TB, int M, int N, int K, T alpha, const T* A,
                 int64_t lda, int64_t sA, const T* B, int64_t ldb, int64_t sB, T beta, T* C, int64_t ldc,
                 int64_t sC, int batch, int mode, const GemmRows& rows = GemmRows{}) {
  // shapes: 0-3 = 64x64, 128x64, 64x128, 128x128 (128-byte k stages);
  // 4 = 64x64 and 5 = 32x64 with 512-byte stages; 6 = 64x128 and 7 = 128x64
  // with 256-byte stages
  const int BM = SBM[shape], BN = SBN[shape];
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, batch);
  constexpr int VW = 16 / sizeof(T);
  auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  const int vec = (lda % VW == 0 && ldb % VW == 0 && (batch == 1 || (sA % VW == 0 && sB % VW == 0)) && al(A) &&
                   al(B)) ? 1 : 0;
  const int swz = gemm_xcd_swizzle() ? 1 : 0;
#define GEMM_CASE(a, b, sh, bm, bn, kb)                                                                   \
  if (TA == a && TB == b && shape == sh) {                                                                 \
    hipLaunchKernelGGL((gemm_kernel<T, a, b, bm, bn, 1, kb>), grid, dim3(64 * (bm / 32) * (bn / 32)), 0, st, M, \
                       N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, mode, vec, swz, rows);       \
    return;                                                                                                \
  }
#define GEMM_SHAPES(a, b)                                                                              \
  GEMM_CASE(a, b, 0, 64, 64, 128) GEMM_CASE(a, b, 1, 128, 64, 128) GEMM_CASE(a, b, 2, 64, 128, 128)    \
  GEMM_CASE(a, b, 3, 128, 128, 128) GEMM_CASE(a, b, 4, 64, 64, 512) GEMM_CASE(a, b, 5, 32, 64, 512)    \
  GEMM_CASE(a, b, 6, 64, 128, 256) GEMM_CASE(a, b, 7, 128, 64, 256)
  GEMM_SHAPES(0, 0) GEMM_SHAPES(0, 1) GEMM_SHAPES(1, 0) GEMM_SHAPES(1, 1)
#undef GEMM_SHAPES
#undef GEMM_CASE
}
}  // namespace

template <typename T>
int gemm_autotune_impl(int TA, int TB, int M, int N, int K, int batch, int mode, int inplace);

namespace {
thread_local bool t_tuning = true;   // may gemm() tune an unseen shape on this thread
}
void gemm_set_thread_tuning(bool on) { t_tuning = on; }

template <typename T>
void gemm(hipStream_t st, int TA, int TB, int M, int N, int K, T alpha, const T* A, int64_t lda,
          int64_t sA, const T* B, int64_t ldb, int64_t sB, T beta, T* C, int64_t ldc, int64_t sC,
          int batch, int mode, const GemmRows& rows) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  // C == A: one tile column, whose tiles read only their own rows of A;
  // C == B: one tile row, whose tiles read only their own columns of B
  const int inplace = ((const T*)C == A) ? IN_PLACE_A : ((const T*)C == B) ? IN_PLACE_B : 0;
  int shape = -1;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(tune_key<T>(TA, TB, M, N, K, batch, mode, inplace));
    if (it != g_tune.end()) shape = it->second;
  }
  if (shape < 0 && autotune_enabled() && t_tuning)
    shape = gemm_autotune_impl<T>(TA, TB, M, N, K, batch, mode, inplace);
  if (shape < 0) {
    shape = 0;
    if (inplace == IN_PLACE_A) shape = N > 64 ? 2 : 0;
    if (inplace == IN_PLACE_B) shape = M > 64 ? 1 : 0;
  }
  gemm_launch<T>(shape, st, TA, TB, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, mode, rows);
}

template <typename T>
int gemm_autotune(int TA, int TB, int M, int N, int K, int batch, int mode) {
  return gemm_autotune_impl<T>(TA, TB, M, N, K, batch, mode, 0);
}

// Operands of the tuning runs: values in [-0.5, 0.5) from a hash of the
// index (the MFMA units and the memory system see data like the real
// operands', not zeros).
template <typename T>
__global__ __launch_bounds__(256) void tune_fill_kernel(T* p, int64_t n, uint32_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    uint32_t h = (uint32_t)i * 2654435761u ^ seed;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    p[i] = T((double)(h & 0xffffu) / 65536.0 - 0.5);
  }
}
template <typename T>
void tune_fill(T* p, int64_t n, uint32_t seed) {
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(4096, (n + 255) / 256));
  hipLaunchKernelGGL(tune_fill_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, nullptr, p, n, seed);
}

template <typename T>
int gemm_autotune_impl(int TA, int TB, int M, int N, int K, int batch, int mode, int inplace) {
  if (M <= 0 || N <= 0 || batch <= 0) return 0;
  const TuneKey key = tune_key<T>(TA, TB, M, N, K, batch, mode, inplace);
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
  int best = -1;
  for (int shape = 0; shape < GEMM_NSHAPES && best < 0; ++shape)
    if (shape_allowed(shape, M, N, inplace)) best = shape;
  if (best < 0) return 0;
  T *A = nullptr, *B = nullptr, *C = nullptr;
  if (hipMalloc(&A, sA * batch * sizeof(T)) != hipSuccess || hipMalloc(&B, sB * batch * sizeof(T)) != hipSuccess ||
      hipMalloc(&C, sC * batch * sizeof(T)) != hipSuccess) {
    (void)hipFree(A);
    (void)hipFree(B);
    (void)hipFree(C);
    return best;
  }
  tune_fill<T>(A, sA * batch, 1u);
  tune_fill<T>(B, sB * batch, 2u);
  tune_fill<T>(C, sC * batch, 3u);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  // work queued by the caller on other streams would run beside the
  // candidates and distort their times
  (void)hipDeviceSynchronize();
  float best_ms = 1e30f;
  // the candidates run on separate C, with the in-place call's tile
  // constraint: the same kernels, timed without the aliasing; the fastest
  // of three timed runs (after one untimed) counts
  for (int shape = 0; shape < GEMM_NSHAPES; ++shape) {
    if (!shape_allowed(shape, M, N, inplace)) continue;
    float t = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      (void)hipEventRecord(e0, nullptr);
      gemm_launch<T>(shape, nullptr, TA, TB, M, N, K, T(1), A, la, sA, B, lb, sB, T(1), C, N, sC, batch, mode);
      (void)hipEventRecord(e1, nullptr);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) t = std::min(t, ms);
    }
    if (autotune_log())
      std::fprintf(stderr, "[gemm tune] T%zu TA%d TB%d M%d N%d K%d batch%d mode%d inplace%d shape%d %.1f us\n",
                   sizeof(T), TA, TB, M, N, K, batch, mode, inplace, shape, t * 1e3f);
    if (t < best_ms) {
      best_ms = t;
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

// Factors and inverts the diagonal block of order b at (K0, K0).
template <typename T>
void diag_step(hipStream_t st, T* A, int64_t lda, int64_t sA, int K0, int b, T* Linv, int64_t sL, int blk, int batch,
               int* info) {
  if (b % 16 == 0 && diag_blocked_enabled()) {
    static const bool attr =
        hipFuncSetAttribute((const void*)diag_block_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(DK_TILES * 256 * sizeof(T))) == hipSuccess;
    (void)attr;
    hipLaunchKernelGGL(diag_block_kernel<T>, dim3(batch), dim3(DK_THREADS), DK_TILES * 256 * sizeof(T), st, A,
                       lda, sA, K0, b, Linv, sL, blk, info);
  } else {
    hipLaunchKernelGGL(diag_factor_kernel<T>, dim3(batch), dim3(DF_THREADS), 0, st, A, lda, sA, K0, b, Linv, sL, blk,
                       info);
  }
}

template <typename T>
int cholesky(hipStream_t st, T* A, int64_t lda, int64_t sA, int n, int split, int batch, T* Linv, int64_t sL,
             int* info, const AuxStreams* ax, const GemmRows* rows) {
  const GemmRows none{};
  const GemmRows& rs = rows ? *rows : none;
  // Right-looking blocked Cholesky over DB-wide diagonal blocks: the block
  // is factored and inverted in LDS, the panel below becomes
  // A_panel L_kk^{-T} (one GEMM, in place: a single 128-wide column tile
  // reads only its own rows), and the trailing matrix gets one rank-b update
  // (with ax: the next column block on st, the rest on st3, see dense.h).
  if (split <= 0 || split >= n) split = 0;
  bool far_pending = false;
  int K0 = 0;
  while (K0 < n) {
    const int lim = (split > 0 && K0 < split) ? split : n;
    const int b = std::min(DB, lim - K0);
    const int K1 = K0 + b;
    diag_step<T>(st, A, lda, sA, K0, b, Linv, sL, diag_block_index(K0, split), batch, info);
    const int rest = n - K1;
    if (rest > 0) {
      T* panel = A + (int64_t)K1 * lda + K0;
      const T* li = Linv + (int64_t)diag_block_index(K0, split) * DB * DB;
      gemm<T>(st, 0, 1, rest, b, b, T(1), panel, lda, sA, li, DB, sL, T(0), panel, lda, sA, batch, 0,
              rs.at(K1, K0, K0));
      if (!ax) {
        gemm<T>(st, 0, 1, rest, rest, b, T(-1), panel, lda, sA, panel, lda, sA, T(1), A + (int64_t)K1 * lda + K1,
                lda, sA, batch, GEMM_LOWER, rs.at(K1, K1, K0));
      } else {
        // the next step's block width (blocks end at the split)
        const int lim2 = (split > 0 && K1 < split) ? split : n;
        const int b2 = std::min(DB, lim2 - K1);
        if (hipEventRecord(ax->ev2, st) != hipSuccess) return -1;
        // column block k+1 also received the far update of step k-1
        if (far_pending && hipStreamWaitEvent(st, ax->ev3, 0) != hipSuccess) return -1;
        gemm<T>(st, 0, 1, rest, b2, b, T(-1), panel, lda, sA, panel, lda, sA, T(1), A + (int64_t)K1 * lda + K1, lda,
                sA, batch, GEMM_LOWER, rs.at(K1, K1, K0));
        far_pending = rest > b2;
        if (far_pending) {
          const int K2 = K1 + b2;
          T* pf = panel + (int64_t)b2 * lda;
          if (hipStreamWaitEvent(ax->st3, ax->ev2, 0) != hipSuccess) return -1;
          gemm<T>(ax->st3, 0, 1, rest - b2, rest - b2, b, T(-1), pf, lda, sA, pf, lda, sA, T(1),
                  A + (int64_t)K2 * lda + K2, lda, sA, batch, GEMM_LOWER, rs.at(K2, K2, K0));
          if (hipEventRecord(ax->ev3, ax->st3) != hipSuccess) return -1;
        }
      }
    }
    K0 = K1;
  }
  if (ax && far_pending && hipStreamWaitEvent(st, ax->ev3, 0) != hipSuccess) return -1;
  return 0;
}

// One block step of the triangular inverse (see tri_inverse): block row S
// = [S0, S0 + h) of Y becomes final and the rows below receive its rank-h
// update.  Reads only the diagonal-block inverse and the column block of L
// below it, both final once the Cholesky sweep has passed that block.
template <typename T>
void tri_inverse_step(hipStream_t st, const T* L, int64_t ldl, int64_t sL, int off, int nb, int split, int batch,
                      const T* Linv, int64_t sLi, T* Y, int64_t ldy, int64_t sY, int S0, int h, int row_end = -1,
                      const GemmRows& rs = GemmRows{}) {
  const int send = S0 + h;
  // rows at or past row_end have L[row, S] = 0: their update is exactly zero
  const int rend = row_end < 0 ? nb : std::min(nb, row_end);
  const int blk = diag_block_index(off + S0, split);
  const T* li = Linv + (int64_t)blk * DB * DB;
  // Y[S, 0:S0] = inv(L_SS) R_S[:, 0:S0] (in place: a single tile row reads
  // only its own columns of R_S before writing them; inv(L_SS) is lower
  // triangular, so a row tile's k loop ends at its last row).  R_S[:, S] is
  // still the identity, so Y[S, S] = inv(L_SS) is a copy (the product would
  // give the same values exactly).
  if (S0 > 0)
    gemm<T>(st, 0, 0, h, S0, h, T(1), li, DB, sLi, Y + (int64_t)S0 * ldy, ldy, sY, T(0), Y + (int64_t)S0 * ldy, ldy,
            sY, batch, GEMM_KTO_DIAG, rs.at(off + S0, off, off + S0));
  {
    T* yb = Y + (int64_t)S0 * ldy + S0;
    const int vec = vec16_ok<T>(li, DB, sLi, h) && vec16_ok<T>(yb, ldy, sY, h);
    hipLaunchKernelGGL(copy_block_kernel<T>, dim3(helper_blocks((int64_t)h * h / (vec ? 16 / sizeof(T) : 1), batch), batch),
                       dim3(256), 0, st, li, DB, sLi, yb, ldy, sY, h, vec);
  }
  const int rest = rend - send;
  if (rest > 0) {
    const T* LlS = L + (int64_t)(off + send) * ldl + (off + S0);
    gemm<T>(st, 0, 0, rest, send, h, T(-1), LlS, ldl, sL, Y + (int64_t)S0 * ldy, ldy, sY, T(1),
            Y + (int64_t)send * ldy, ldy, sY, batch, 0, rs.at(off + send, off, off + S0));
  }
}

template <typename T>
void tri_inverse(hipStream_t st, const T* L, int64_t ldl, int64_t sL, int off, int nb, int split, int batch,
                 const T* Linv, int64_t sLi, T* Y, int64_t ldy, int64_t sY, const GemmRows* rows, bool fill) {
  // Y = L_block^{-1} for the diagonal range [off, off+nb) of L (lower) by
  // block forward substitution on L Y = I over the factor's diagonal blocks
  // S: Y holds the running right-hand side R (initially I); Y[S, 0:send] =
  // inv(L_SS) R_S[:, 0:send], and the rows below get one rank-|S| update.
  if (fill) launch_eye<T>(st, Y, ldy, sY, nb, batch);
  int S0 = 0;
  while (S0 < nb) {
    const int p = off + S0;
    const int lim = (split > 0 && p < split) ? std::min(split - off, nb) : nb;
    const int h = std::min(DB, lim - S0);
    tri_inverse_step<T>(st, L, ldl, sL, off, nb, split, batch, Linv, sLi, Y, ldy, sY, S0, h, -1,
                        rows ? *rows : GemmRows{});
    S0 += h;
  }
}

template <typename T>
void fill_identity(hipStream_t st, T* Y, int64_t ldy, int64_t sY, int nb, int batch) {
  launch_eye<T>(st, Y, ldy, sY, nb, batch);
}

template <typename T>
int cholesky_inverse(hipStream_t st, const AuxStreams& ax, T* A, int64_t lda, int64_t sA, int n, int batch, T* Linv,
                     int64_t sL, int* info, T* Y, int64_t sY, const int* env) {
  // Block step k on st: diagonal block, panel, then the update of column
  // block k+1 only (after the far update of step k-1, which also covered
  // it).  The far update of step k (rows and columns right of block k+1)
  // runs on st3 beside the factorisation of block k+1: the two touch
  // disjoint parts of A and read only the panel of block k.  Step k of the
  // triangular inverse reads the final column block k and runs on st2.
  // With env, every step works only on rows below the block's envelope end
  // (the factor is zero beyond it, so the skipped updates are exact zeros).
  launch_eye<T>(st, Y, lda, sY, n, batch);
  bool far_pending = false;
  int K0 = 0;
  while (K0 < n) {
    const int b = std::min(DB, n - K0);
    const int K1 = K0 + b;
    diag_step<T>(st, A, lda, sA, K0, b, Linv, sL, diag_block_index(K0, 0), batch, info);
    const int rend = env ? std::max(K1, std::min(n, env[K0 / DB])) : n;
    const int rest = rend - K1;
    T* panel = A + (int64_t)K1 * lda + K0;
    if (rest > 0) {
      const T* li = Linv + (int64_t)diag_block_index(K0, 0) * DB * DB;
      gemm<T>(st, 0, 1, rest, b, b, T(1), panel, lda, sA, li, DB, sL, T(0), panel, lda, sA, batch, 0);
    }
    if (hipEventRecord(ax.ev2, st) != hipSuccess || hipStreamWaitEvent(ax.st2, ax.ev2, 0) != hipSuccess) return -1;
    tri_inverse_step<T>(ax.st2, A, lda, sA, 0, n, 0, batch, Linv, sL, Y, lda, sY, K0, b, rend);
    if (rest > 0) {
      const int b2 = std::min(DB, rest);
      if (far_pending && hipStreamWaitEvent(st, ax.ev3, 0) != hipSuccess) return -1;
      gemm<T>(st, 0, 1, rest, b2, b, T(-1), panel, lda, sA, panel, lda, sA, T(1), A + (int64_t)K1 * lda + K1, lda,
              sA, batch, GEMM_LOWER);
      far_pending = rest > b2;
      if (far_pending) {
        const int K2 = K1 + b2;
        T* pf = panel + (int64_t)b2 * lda;
        if (hipStreamWaitEvent(ax.st3, ax.ev2, 0) != hipSuccess) return -1;
        gemm<T>(ax.st3, 0, 1, rest - b2, rest - b2, b, T(-1), pf, lda, sA, pf, lda, sA, T(1),
                A + (int64_t)K2 * lda + K2, lda, sA, batch, GEMM_LOWER);
        if (hipEventRecord(ax.ev3, ax.st3) != hipSuccess) return -1;
      }
    }
    K0 = K1;
  }
  if (hipEventRecord(ax.ev2, ax.st2) != hipSuccess || hipStreamWaitEvent(st, ax.ev2, 0) != hipSuccess) return -1;
  if (hipEventRecord(ax.ev3, ax.st3) != hipSuccess || hipStreamWaitEvent(st, ax.ev3, 0) != hipSuccess) return -1;
  return 0;
}

template <typename T, typename TO>
void symmetrize_scale(hipStream_t st, const T* in, int64_t ldi, int64_t sI, TO* out, int64_t ldo,
                      int64_t sO, const double* D, int64_t sD, int nb, int batch) {
  if (nb % 32 == 0) {
    const int nt = nb / 32;
    const int veci = vec16_ok<T>(in, ldi, sI, 32), veco = vec16_ok<TO>(out, ldo, sO, 32);
    hipLaunchKernelGGL((symmetrize_scale_tiled_kernel<T, TO>), dim3(nt * (nt + 1) / 2, batch), dim3(256), 0, st, in,
                       ldi, sI, out, ldo, sO, D, sD, veci, veco);
    return;
  }
  hipLaunchKernelGGL((symmetrize_scale_kernel<T, TO>), dim3(nb, batch), dim3(256), 0, st, in, ldi,
                     sI, out, ldo, sO, D, sD, nb);
}

#define INST(T)                                                                                 \
  template void gemm<T>(hipStream_t, int, int, int, int, int, T, const T*, int64_t, int64_t,    \
                        const T*, int64_t, int64_t, T, T*, int64_t, int64_t, int, int,          \
                        const GemmRows&);                                                      \
  template int gemm_autotune<T>(int, int, int, int, int, int, int);                              \
  template int cholesky<T>(hipStream_t, T*, int64_t, int64_t, int, int, int, T*, int64_t, int*,   \
                           const AuxStreams*, const GemmRows*);                                  \
  template void tri_inverse<T>(hipStream_t, const T*, int64_t, int64_t, int, int, int, int, const T*, \
                               int64_t, T*, int64_t, int64_t, const GemmRows*, bool);               \
  template void fill_identity<T>(hipStream_t, T*, int64_t, int64_t, int, int);                   \
  template int cholesky_inverse<T>(hipStream_t, const AuxStreams&, T*, int64_t, int64_t, int, int, T*,  \
                                   int64_t, int*, T*, int64_t, const int*);
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
