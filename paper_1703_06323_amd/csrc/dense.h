// Batched dense linear algebra (MFMA) used by the subdomain and coarse
// factorisations.  All matrices are row-major; `s*` arguments are element
// strides between consecutive matrices of a batch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cutbddc {

enum GemmMode {
  GEMM_LOWER = 1,        // only output tiles/elements on or below the diagonal
  GEMM_KFROM_DIAG = 2,   // K loop starts at max(row0, col0) (op(A) upper-zero in K)
  GEMM_KTO_DIAG = 4      // K loop ends at row0 + 64 (op(A) lower triangular)
};

constexpr int CHOL_BLOCK = 32;

// Padded batches: matrix b of a batch is nonzero only on the index set
// [0, na[b]) u [split, split + nb[b]) of a common index space (rows, columns
// and the k of a product may be offset into it by r_off, c_off and k_off);
// outside it only the diagonal may be nonzero, and no product reads it.
// Given to gemm(), every output tile whose rows or columns miss the set, or
// whose k range does, takes no product (its C is left as is when beta = 1,
// else becomes beta C), and the k loop of the other tiles covers only the
// hull of the set's k (rounded down to a stage).  The result is exact when
// A and B vanish outside the set; an output entry with both indices outside
// it then gets beta C instead of the product of the padding diagonals.
// nb may be null (one range).  Device pointers, indexed by the batch entry.
struct GemmRows {
  const int32_t* na = nullptr;
  const int32_t* nb = nullptr;
  int32_t split = 0;
  int32_t r_off = 0, c_off = 0, k_off = 0;
  GemmRows at(int r, int c, int k) const {
    GemmRows g = *this;
    g.r_off = r;
    g.c_off = c;
    g.k_off = k;
    return g;
  }
};

// C = alpha op(A) op(B) + beta C; TA/TB = 0 plain, 1 transposed storage.
template <typename T>
void gemm(hipStream_t st, int TA, int TB, int M, int N, int K, T alpha, const T* A, int64_t lda,
          int64_t sA, const T* B, int64_t ldb, int64_t sB, T beta, T* C, int64_t ldc, int64_t sC,
          int batch, int mode, const GemmRows& rows = GemmRows{});

// Times every GEMM tile shape on scratch matrices of the bucket of
// (TA, TB, M, N, K, batch, mode) and records the fastest for later calls of
// that bucket (synchronous, default stream).  Returns the chosen shape.
template <typename T>
int gemm_autotune(int TA, int TB, int M, int N, int K, int batch, int mode);

// Diagonal blocks of the factorisations have order DB (the last block of a
// range may be smaller).  Blocks start at 0 and, when a split point is
// given, again at the split (so that the two diagonal ranges [0, split) and
// [split, n) are unions of whole blocks).
// With false, gemm() on the calling thread never runs the autotuner (which
// allocates its test operands): shapes not tuned yet use the default tile.
void gemm_set_thread_tuning(bool on);
constexpr int DB = 128;
inline int diag_blocks(int n, int split) {
  if (split <= 0 || split >= n) return (n + DB - 1) / DB;
  return (split + DB - 1) / DB + (n - split + DB - 1) / DB;
}
// Index of the diagonal block that starts at position p.
inline int diag_block_index(int p, int split) {
  if (split <= 0 || p < split) return p / DB;
  return (split + DB - 1) / DB + (p - split) / DB;
}

// In-place lower Cholesky of n x n matrices (n a multiple of CHOL_BLOCK;
// split 0 or a multiple of CHOL_BLOCK).  Linv receives, per matrix, the
// inverse of every diagonal block as a DB x DB row-major block (zero above
// the diagonal): sL >= diag_blocks(n, split) * DB * DB.  info[b] is set to
// (first row with a non-positive pivot) + 1 for matrix b; the pivot is then
// replaced by 1 so that the factorisation finishes without NaNs.
// With ax (streams and events lent by the caller, see AuxStreams), one
// block of lookahead: after the panel of block k, st updates only column
// block k+1 and goes on to factor it, while ax->st3 updates the rest of the
// trailing matrix; st waits for st3 before returning.  Returns -1 if an
// event record or wait fails.
// rows (optional): the nonzero index sets of the matrices (GemmRows with
// offsets 0; the padding outside them holds the identity): the panel and
// trailing updates skip the tiles and k stages that only meet padding.
struct AuxStreams;
template <typename T>
int cholesky(hipStream_t st, T* A, int64_t lda, int64_t sA, int n, int split, int batch, T* Linv, int64_t sL,
             int* info, const AuxStreams* ax = nullptr, const GemmRows* rows = nullptr);

// Y = inverse of the lower-triangular diagonal range [off, off+nb) of L
// (off and off+nb block starts of the same split), from the diagonal-block
// inverses written by cholesky().  rows (optional, as for cholesky(), in
// the index space of L): the updates skip padding tiles; Y is still the
// identity on the padding.  fill = false: Y already holds the identity
// (written by fill_identity on st, or on a stream that st waits for).
template <typename T>
void tri_inverse(hipStream_t st, const T* L, int64_t ldl, int64_t sL, int off, int nb, int split, int batch,
                 const T* Linv, int64_t sLi, T* Y, int64_t ldy, int64_t sY, const GemmRows* rows = nullptr,
                 bool fill = true);
// Y[b] = I (nb x nb, leading dimension ldy, matrix stride sY) for b < batch.
template <typename T>
void fill_identity(hipStream_t st, T* Y, int64_t ldy, int64_t sY, int nb, int batch);

// Streams and events lent to cholesky_inverse by the caller (default
// priority, non-blocking).  The events are recorded and waited on at every
// step, so they must outlive the work.
struct AuxStreams {
  hipStream_t st2, st3;
  hipEvent_t ev2, ev3;
};

// Cholesky of n x n matrices (no split) and Y = L^{-1} (as tri_inverse over
// the whole range, Y with leading dimension lda and stride sY), with one
// block of lookahead: after the panel of block k, st updates only column
// block k+1 and goes on to factor it, while st3 updates the rest of the
// trailing matrix; the triangular-inverse step of block k runs on st2.  st
// waits for st2 and st3 before returning.  Returns -1 if an event record or
// wait fails.
// env (host, optional): per DB-wide column block k, the end (exclusive) of
// the rows of every matrix of the batch that can be nonzero in that column
// block of L: one past the last row i whose first nonzero column in A lies
// at or before the block's last column (fill stays inside this envelope).
// Rows at or past it take only zero updates, which are skipped.
template <typename T>
int cholesky_inverse(hipStream_t st, const AuxStreams& ax, T* A, int64_t lda, int64_t sA, int n, int batch, T* Linv,
                     int64_t sL, int* info, T* Y, int64_t sY, const int* env = nullptr);

// out = D sym(lower(in)) D, full storage.
template <typename T, typename TO>
void symmetrize_scale(hipStream_t st, const T* in, int64_t ldi, int64_t sI, TO* out, int64_t ldo,
                      int64_t sO, const double* D, int64_t sD, int nb, int batch);

}  // namespace cutbddc
