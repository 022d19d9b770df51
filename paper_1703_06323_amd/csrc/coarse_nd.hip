// Coarse problem by one level of nested dissection: block gathers, the
// Schur complement of the separator and the solve (see coarse_nd.h).
#include "coarse_nd.h"

namespace cutbddc {
namespace {

constexpr int ND_T = 256;

// Sum of v over the workgroup, valid in thread 0 (lanes by shuffles, then
// the waves in order: the same order in every workgroup).
__device__ inline double nd_block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < ND_T / 64; ++i) t += sh[i];
  return t;
}

// one workgroup per octant row o * Lo + i
__global__ __launch_bounds__(ND_T) void nd_gather_kernel(NDDev nd, const double* __restrict__ Ac, int ldc,
                                                         double* __restrict__ Aoo, double* __restrict__ Aos) {
  const int row = blockIdx.x, Lo = nd.Lo, Lso = nd.Lso;
  const int o = row / Lo, i = row - o * Lo;
  const int gi = nd.oid[row];
  const int32_t* ids = nd.oid + (int64_t)o * Lo;
  const int32_t* sc = nd.sep + (int64_t)o * Lso;
  const double* arow = Ac + (int64_t)(gi < 0 ? 0 : gi) * ldc;
  double* ao = Aoo + (int64_t)row * Lo;
  double* as = Aos + (int64_t)row * Lso;
  for (int j = threadIdx.x; j < Lo; j += ND_T) {
    const int gj = ids[j];
    ao[j] = (gi >= 0 && gj >= 0) ? arow[gj] : (i == j ? 1.0 : 0.0);
  }
  for (int a = threadIdx.x; a < Lso; a += ND_T) {
    const int sa = sc[a];
    as[a] = (gi >= 0 && sa >= 0) ? arow[nd.sid[sa]] : 0.0;
  }
}

// one workgroup per separator row i (Ls rows)
__global__ __launch_bounds__(ND_T) void nd_schur_kernel(NDDev nd, const double* __restrict__ Ac, int ldc,
                                                        const double* __restrict__ So, double* __restrict__ S) {
  const int i = blockIdx.x, Ls = nd.Ls, n_s = nd.n_s, Lso = nd.Lso;
  double* srow = S + (int64_t)i * Ls;
  if (i >= n_s) {
    for (int j = threadIdx.x; j < Ls; j += ND_T) srow[j] = i == j ? 1.0 : 0.0;
    return;
  }
  int pi[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) pi[o] = nd.pos[(int64_t)o * n_s + i];
  const double* arow = Ac + (int64_t)nd.sid[i] * ldc;
  for (int j = threadIdx.x; j < Ls; j += ND_T) {
    double v = 0.0;
    if (j < n_s) {
      v = arow[nd.sid[j]];
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        const int pj = nd.pos[(int64_t)o * n_s + j];
        if (pi[o] >= 0 && pj >= 0) {
          const int hi = max(pi[o], pj), lo = min(pi[o], pj);
          v -= So[((int64_t)o * Lso + hi) * Lso + lo];
        }
      }
    }
    srow[j] = v;
  }
}

// WT[o] = W[o]^T, 32 x 32 tiles through LDS; block (32, 8)
__global__ __launch_bounds__(256) void nd_transpose_kernel(NDDev nd, const double* __restrict__ W,
                                                           double* __restrict__ WT) {
  __shared__ double tile[32][33];
  const int Lo = nd.Lo, Lso = nd.Lso;
  const int o = blockIdx.z, i0 = blockIdx.y * 32, a0 = blockIdx.x * 32;
  const double* w = W + (int64_t)o * Lo * Lso;
  double* wt = WT + (int64_t)o * Lso * Lo;
  for (int r = threadIdx.y; r < 32; r += 8) tile[r][threadIdx.x] = w[(int64_t)(i0 + r) * Lso + a0 + threadIdx.x];
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += 8) wt[(int64_t)(a0 + r) * Lo + i0 + threadIdx.x] = tile[threadIdx.x][r];
}

// t_o = Y_o r_o: one workgroup per octant row (r gathered by original id)
__global__ __launch_bounds__(ND_T) void nd_fwd_kernel(BatchDev bd, NDDev nd, const double* __restrict__ Yo,
                                                      const double* __restrict__ x, double* __restrict__ to) {
  __shared__ double sh[ND_T / 64];
  if (bd.active && !bd.active[0]) return;
  const int row = blockIdx.x, Lo = nd.Lo;
  const int o = row / Lo, i = row - o * Lo;
  const double* y = Yo + (int64_t)row * Lo;
  const int32_t* ids = nd.oid + (int64_t)o * Lo;
  double acc = 0.0;
  for (int j = threadIdx.x; j <= i; j += ND_T) {
    const int g = ids[j];
    if (g >= 0) acc += y[j] * x[g];
  }
  const double t = nd_block_sum(acc, sh);
  if (threadIdx.x == 0) to[row] = t;
}

// r_s' = r_s - sum_o W_o^T t_o: one workgroup per separator row (Ls rows)
__global__ __launch_bounds__(ND_T) void nd_sep_rhs_kernel(BatchDev bd, NDDev nd, const double* __restrict__ WT,
                                                          const double* __restrict__ to,
                                                          const double* __restrict__ x, double* __restrict__ rs) {
  __shared__ double sh[ND_T / 64];
  if (bd.active && !bd.active[0]) return;
  const int s = blockIdx.x, Lo = nd.Lo, Lso = nd.Lso, n_s = nd.n_s;
  if (s >= n_s) {
    if (threadIdx.x == 0) rs[s] = 0.0;
    return;
  }
  double acc = 0.0;
  for (int o = 0; o < 8; ++o) {
    const int a = nd.pos[(int64_t)o * n_s + s];
    if (a < 0) continue;
    const double* wt = WT + ((int64_t)o * Lso + a) * Lo;
    const double* t = to + (int64_t)o * Lo;
    for (int i = threadIdx.x; i < Lo; i += ND_T) acc += wt[i] * t[i];
  }
  const double v = nd_block_sum(acc, sh);
  if (threadIdx.x == 0) rs[s] = x[nd.sid[s]] - v;
}

// y = tril(M) x (upper = 0) or triu(M) x (upper = 1), M = Ys (Ls x Ls)
__global__ __launch_bounds__(ND_T) void nd_tri_kernel(BatchDev bd, int n, const double* __restrict__ M,
                                                      const double* __restrict__ x, double* __restrict__ y,
                                                      int upper) {
  __shared__ double sh[ND_T / 64];
  if (bd.active && !bd.active[0]) return;
  const int r = blockIdx.x;
  const double* row = M + (int64_t)r * n;
  const int lo = upper ? r : 0, hi = upper ? n - 1 : r;
  double acc = 0.0;
  for (int j = lo + threadIdx.x; j <= hi; j += ND_T) acc += row[j] * x[j];
  const double t = nd_block_sum(acc, sh);
  if (threadIdx.x == 0) y[r] = t;
}

// t_o -= W_o x_s: one workgroup per octant row
__global__ __launch_bounds__(ND_T) void nd_back_kernel(BatchDev bd, NDDev nd, const double* __restrict__ W,
                                                       const double* __restrict__ xs, double* __restrict__ to) {
  __shared__ double sh[ND_T / 64];
  if (bd.active && !bd.active[0]) return;
  const int row = blockIdx.x, Lo = nd.Lo, Lso = nd.Lso;
  const int o = row / Lo;
  const double* w = W + (int64_t)row * Lso;
  const int32_t* sc = nd.sep + (int64_t)o * Lso;
  double acc = 0.0;
  for (int a = threadIdx.x; a < Lso; a += ND_T) {
    const int sa = sc[a];
    if (sa >= 0) acc += w[a] * xs[sa];
  }
  const double v = nd_block_sum(acc, sh);
  if (threadIdx.x == 0) to[row] -= v;
}

// x_o = Y_o^T t_o scattered to the original ids (workgroups 0 .. 8 Lo - 1),
// and the separator values x_s (the n_s workgroups after them)
__global__ __launch_bounds__(ND_T) void nd_up_kernel(BatchDev bd, NDDev nd, const double* __restrict__ Yo,
                                                     const double* __restrict__ to, const double* __restrict__ xs,
                                                     double* __restrict__ y) {
  __shared__ double sh[ND_T / 64];
  if (bd.active && !bd.active[0]) return;
  const int Lo = nd.Lo, b = blockIdx.x;
  if (b >= 8 * Lo) {
    const int s = b - 8 * Lo;
    if (threadIdx.x == 0) y[nd.sid[s]] = xs[s];
    return;
  }
  const int o = b / Lo, i = b - o * Lo;
  const double* yr = Yo + (int64_t)b * Lo;
  const double* t = to + (int64_t)o * Lo;
  double acc = 0.0;
  for (int j = i + threadIdx.x; j < Lo; j += ND_T) acc += yr[j] * t[j];
  const double v = nd_block_sum(acc, sh);
  const int g = nd.oid[b];
  if (threadIdx.x == 0 && g >= 0) y[g] = v;
}

}  // namespace

void launch_nd_gather(hipStream_t st, const NDDev& nd, const double* Ac, int ldc, double* Aoo, double* Aos) {
  hipLaunchKernelGGL(nd_gather_kernel, dim3(8 * nd.Lo), dim3(ND_T), 0, st, nd, Ac, ldc, Aoo, Aos);
}

void launch_nd_schur(hipStream_t st, const NDDev& nd, const double* Ac, int ldc, const double* So, double* S) {
  hipLaunchKernelGGL(nd_schur_kernel, dim3(nd.Ls), dim3(ND_T), 0, st, nd, Ac, ldc, So, S);
}

void launch_nd_transpose(hipStream_t st, const NDDev& nd, const double* W, double* WT) {
  hipLaunchKernelGGL(nd_transpose_kernel, dim3(nd.Lso / 32, nd.Lo / 32, 8), dim3(32, 8), 0, st, nd, W, WT);
}

void launch_nd_solve(hipStream_t st, const BatchDev& b, const NDDev& nd, const double* Yo, const double* W,
                     const double* WT, const double* Ys, const double* x, double* to, double* rs, double* us,
                     double* xs, double* y) {
  hipLaunchKernelGGL(nd_fwd_kernel, dim3(8 * nd.Lo), dim3(ND_T), 0, st, b, nd, Yo, x, to);
  hipLaunchKernelGGL(nd_sep_rhs_kernel, dim3(nd.Ls), dim3(ND_T), 0, st, b, nd, WT, to, x, rs);
  hipLaunchKernelGGL(nd_tri_kernel, dim3(nd.Ls), dim3(ND_T), 0, st, b, nd.Ls, Ys, rs, us, 0);
  hipLaunchKernelGGL(nd_tri_kernel, dim3(nd.Ls), dim3(ND_T), 0, st, b, nd.Ls, Ys, us, xs, 1);
  hipLaunchKernelGGL(nd_back_kernel, dim3(8 * nd.Lo), dim3(ND_T), 0, st, b, nd, W, xs, to);
  hipLaunchKernelGGL(nd_up_kernel, dim3(8 * nd.Lo + nd.n_s), dim3(ND_T), 0, st, b, nd, Yo, to, xs, y);
}

}  // namespace cutbddc
