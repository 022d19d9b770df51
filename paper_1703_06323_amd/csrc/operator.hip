// Matrix-free operator A-bar = sum_e A_e (paper Sect. 2.2), load
// b = M_cut f, adjoint contraction and FP64 vector kernels.
//
// Vectors live on the full grid of (N+1)^3 nodes with zeros at non-DOF
// nodes, so every kernel is pure index arithmetic with coalesced access.
// Node-centric gather: the thread of node n sums the rows of the (up to 8)
// active cells around it; no atomics, fixed summation order.
#include "common.h"

#pragma clang fp contract(off)

namespace cutbddc {
namespace {

__constant__ double c_Kref[64];   // reference Q1 stiffness (kappa = 1, h = 1)
__constant__ double c_Mref[64];   // reference Q1 mass (h = 1)

template <bool MASS>
__device__ inline double node_gather(int N, int64_t I, int64_t J, int64_t K,
                                     const int32_t* __restrict__ cellinfo,
                                     const double* __restrict__ kappa,
                                     const double* __restrict__ Mat, const double* __restrict__ x,
                                     double scale) {
  const int64_t N1 = N + 1;
  double acc = 0.0;
  for (int w = 0; w < 2; ++w) {
    const int64_t ck = K - 1 + w;
    if (ck < 0 || ck >= N) continue;
    for (int v = 0; v < 2; ++v) {
      const int64_t cj = J - 1 + v;
      if (cj < 0 || cj >= N) continue;
      for (int u = 0; u < 2; ++u) {
        const int64_t ci = I - 1 + u;
        if (ci < 0 || ci >= N) continue;
        const int64_t c = ci + N * (cj + N * ck);
        const int32_t info = cellinfo[c];
        if (info == CELL_INACTIVE) continue;
        const int a = (1 - u) + 2 * (1 - v) + 4 * (1 - w);
        const int64_t n0 = ci + N1 * (cj + N1 * ck);
        const double s = MASS ? scale : kappa[c] * scale;
        double row = 0.0;
        if (info == CELL_UNCUT) {
          const double* R = MASS ? c_Mref : c_Kref;
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            const int64_t nb = n0 + (b & 1) + N1 * (((b >> 1) & 1) + N1 * ((b >> 2) & 1));
            row += R[a * 8 + b] * x[nb];
          }
        } else {
          const double* R = Mat + (int64_t)info * PACK36;
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            const int64_t nb = n0 + (b & 1) + N1 * (((b >> 1) & 1) + N1 * ((b >> 2) & 1));
            row += R[pack_index(a, b)] * x[nb];
          }
        }
        acc += s * row;
      }
    }
  }
  return acc;
}

__global__ __launch_bounds__(256) void apply_A_kernel(int N, double h,
                                                      const int32_t* __restrict__ cellinfo,
                                                      const double* __restrict__ kappa,
                                                      const double* __restrict__ Kc,
                                                      const uint8_t* __restrict__ dofmask,
                                                      const double* __restrict__ x,
                                                      double* __restrict__ y) {
  const int64_t N1 = N + 1;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N1 * N1 * N1) return;
  if (!dofmask[n]) {
    y[n] = 0.0;
    return;
  }
  const int64_t I = n % N1, J = (n / N1) % N1, K = n / (N1 * N1);
  y[n] = node_gather<false>(N, I, J, K, cellinfo, kappa, Kc, x, h);
}

__global__ __launch_bounds__(256) void load_kernel(int N, double h3,
                                                   const int32_t* __restrict__ cellinfo,
                                                   const double* __restrict__ Mc,
                                                   const uint8_t* __restrict__ outmask,
                                                   const double* __restrict__ f,
                                                   double* __restrict__ b) {
  const int64_t N1 = N + 1;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N1 * N1 * N1) return;
  if (outmask && !outmask[n]) {
    b[n] = 0.0;
    return;
  }
  const int64_t I = n % N1, J = (n / N1) % N1, K = n / (N1 * N1);
  b[n] = node_gather<true>(N, I, J, K, cellinfo, nullptr, Mc, f, h3);
}

__global__ __launch_bounds__(256) void grad_theta_kernel(int N, double h,
                                                         const int32_t* __restrict__ cellinfo,
                                                         const double* __restrict__ kappa,
                                                         const double* __restrict__ Kc,
                                                         const double* __restrict__ u,
                                                         const double* __restrict__ lam,
                                                         double* __restrict__ out) {
  const int64_t N1 = N + 1;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (int64_t)N * N * N) return;
  const int32_t info = cellinfo[c];
  if (info == CELL_INACTIVE) {
    out[c] = 0.0;
    return;
  }
  const int64_t ci = c % N, cj = (c / N) % N, ck = c / ((int64_t)N * N);
  const int64_t n0 = ci + N1 * (cj + N1 * ck);
  double ue[8], le[8];
  for (int a = 0; a < 8; ++a) {
    const int64_t na = n0 + (a & 1) + N1 * (((a >> 1) & 1) + N1 * ((a >> 2) & 1));
    ue[a] = u[na];
    le[a] = lam[na];
  }
  double acc = 0.0;
  for (int a = 0; a < 8; ++a) {
    double row = 0.0;
    for (int b = 0; b < 8; ++b) {
      const double k = info == CELL_UNCUT ? c_Kref[a * 8 + b] : Kc[(int64_t)info * PACK36 + pack_index(a, b)];
      row += k * ue[b];
    }
    acc += le[a] * row;
  }
  out[c] = -kappa[c] * h * acc;
}

__global__ void scatter_dofs_kernel(int64_t n, const int64_t* __restrict__ dof_node,
                                    const double* __restrict__ src, double* __restrict__ grid) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) grid[dof_node[i]] = src[i];
}

__global__ void gather_dofs_kernel(int64_t n, const int64_t* __restrict__ dof_node,
                                   const double* __restrict__ grid, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = grid[dof_node[i]];
}

__global__ void fill_kernel(int64_t n, double v, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// x += alpha p, r -= alpha q with alpha = S[0] / S[1] (rho / p.q)
__global__ void cg_update_xr_kernel(int64_t n, const double* __restrict__ S, const double* __restrict__ p,
                                    const double* __restrict__ q, double* __restrict__ x,
                                    double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double alpha = S[0] / S[1];
  x[i] += alpha * p[i];
  r[i] -= alpha * q[i];
}

// p = z + beta p with beta = S[3] / S[0]; the last block to finish cannot be
// known, so the rho swap S[0] = S[3] is a separate single-thread kernel.
__global__ void cg_update_p_kernel(int64_t n, const double* __restrict__ S, const double* __restrict__ z,
                                   double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double beta = S[3] / S[0];
  p[i] = z[i] + beta * p[i];
}

__global__ void cg_swap_rho_kernel(double* S) {
  if (threadIdx.x == 0 && blockIdx.x == 0) S[0] = S[3];
}

__global__ void convert_kernel(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

constexpr int DOT_BLOCKS = 512;
constexpr int DOT_THREADS = 256;

__device__ inline double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  return t;
}

__global__ __launch_bounds__(DOT_THREADS) void dot_partial_kernel(int64_t n, const double* __restrict__ x,
                                                                  const double* __restrict__ y,
                                                                  double* __restrict__ partial) {
  __shared__ double sh[DOT_THREADS / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * DOT_THREADS + threadIdx.x; i < n;
       i += (int64_t)DOT_BLOCKS * DOT_THREADS)
    acc += x[i] * y[i];
  double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(DOT_THREADS) void dot_final_kernel(const double* __restrict__ partial,
                                                                double* __restrict__ out) {
  __shared__ double sh[DOT_THREADS / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < DOT_BLOCKS; i += DOT_THREADS) acc += partial[i];
  double t = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = t;
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void set_reference_matrices(const double* Kref, const double* Mref) {
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_Kref), Kref, 64 * sizeof(double));
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_Mref), Mref, 64 * sizeof(double));
}

void launch_apply_A(hipStream_t st, GridDesc g, const int32_t* cellinfo, const double* kappa,
                    const double* Kc, const uint8_t* dofmask, const double* x, double* y) {
  const int64_t nn = (int64_t)(g.N + 1) * (g.N + 1) * (g.N + 1);
  hipLaunchKernelGGL(apply_A_kernel, dim3(nblocks(nn, 256)), dim3(256), 0, st, g.N, g.h, cellinfo,
                     kappa, Kc, dofmask, x, y);
}

void launch_load(hipStream_t st, GridDesc g, const int32_t* cellinfo, const double* Mc,
                 const uint8_t* outmask, const double* f, double* b) {
  const int64_t nn = (int64_t)(g.N + 1) * (g.N + 1) * (g.N + 1);
  hipLaunchKernelGGL(load_kernel, dim3(nblocks(nn, 256)), dim3(256), 0, st, g.N, g.h * g.h * g.h,
                     cellinfo, Mc, outmask, f, b);
}

void launch_grad_theta(hipStream_t st, GridDesc g, const int32_t* cellinfo, const double* kappa,
                       const double* Kc, const double* u, const double* lam, double* out) {
  const int64_t nc = (int64_t)g.N * g.N * g.N;
  hipLaunchKernelGGL(grad_theta_kernel, dim3(nblocks(nc, 256)), dim3(256), 0, st, g.N, g.h,
                     cellinfo, kappa, Kc, u, lam, out);
}

void launch_scatter_dofs(hipStream_t st, int64_t n, const int64_t* dof_node, const double* src,
                         double* grid) {
  if (n <= 0) return;
  hipLaunchKernelGGL(scatter_dofs_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, n, dof_node,
                     src, grid);
}

void launch_gather_dofs(hipStream_t st, int64_t n, const int64_t* dof_node, const double* grid,
                        double* dst) {
  if (n <= 0) return;
  hipLaunchKernelGGL(gather_dofs_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, n, dof_node,
                     grid, dst);
}

void launch_fill(hipStream_t st, int64_t n, double v, double* x) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, n, v, x);
}

int dot_partials() { return DOT_BLOCKS; }

void launch_cg_update_xr(hipStream_t st, int64_t n, const double* S, const double* p, const double* q, double* x,
                         double* r) {
  hipLaunchKernelGGL(cg_update_xr_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, n, S, p, q, x, r);
}

void launch_cg_update_p(hipStream_t st, int64_t n, double* S, const double* z, double* p) {
  hipLaunchKernelGGL(cg_update_p_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, n, S, z, p);
  hipLaunchKernelGGL(cg_swap_rho_kernel, dim3(1), dim3(64), 0, st, S);
}

void convert_to_float(hipStream_t st, int64_t n, const double* a, float* b) {
  if (n <= 0) return;
  hipLaunchKernelGGL(convert_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, n, a, b);
}

void launch_dot(hipStream_t st, int64_t n, const double* x, const double* y, double* partial,
                double* out) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(DOT_BLOCKS), dim3(DOT_THREADS), 0, st, n, x, y,
                     partial);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(DOT_THREADS), 0, st, partial, out);
}

}  // namespace cutbddc
