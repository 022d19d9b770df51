// Manufactured-solution accuracy (paper Sect. 5.1: the exact solution
// u = sin(5 pi |x|), strong Dirichlet data on the cube faces, Neumann or
// Nitsche-Dirichlet data on the ball surfaces, H^1 and L^2 errors).
//
// The exact solution is u = sin(k rho), rho = |x - x0|, with
// f = -Lap u = k^2 sin(k rho) - (2 k / rho) cos(k rho) and
// grad u = k cos(k rho) (x - x0) / rho.  Volume integrals use the kept
// points of the volume rule (the kept-point test of the classification,
// same expression, no contraction), surface integrals the sphere rule of
// the Nitsche terms (nitsche.hip, which adds the surface load).
//  * load: b = sum_e (volume + surface load of e) on the DOF rows, minus
//    A-bar applied to the Dirichlet lift (u at the cube-face nodes);
//  * errors: e_L2^2 = sum (h^3/512) (u - u_h)^2 and
//    e_H1^2 = sum (h^3/512) |grad u - grad u_h|^2 over kept points, with
//    u_h = the DOF values plus the lift.
// One 64-lane wave per cell; lane l owns the points l + 64 t (kx = l % 8,
// ky = l / 8, kz = t) and the wave reduces in a fixed order.
#include "manufactured.h"

#pragma clang fp contract(off)

namespace cutbddc {
namespace {

constexpr int MW = 64;

__device__ inline void exact(const MmsParams& m, const double x[3], double* u, double g[3], double* f) {
  const double d0 = x[0] - m.x0[0], d1 = x[1] - m.x0[1], d2 = x[2] - m.x0[2];
  const double rho = sqrt((d0 * d0 + d1 * d1) + d2 * d2);
  const double s = sin(m.k * rho), c = cos(m.k * rho);
  *u = s;
  const double du = m.k * c;
  g[0] = (du / rho) * d0;
  g[1] = (du / rho) * d1;
  g[2] = (du / rho) * d2;
  *f = m.k * m.k * s - 2.0 * du / rho;
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return __shfl(v, 0, 64);
}

// Points of cell c (problem d) kept by the volume rule: all 512 unless the
// cell is cut (the test of the classification).
__device__ inline bool point_kept(const ProbDev& d, const double* __restrict__ balls, bool cut, const double x[3]) {
  if (!cut) return true;
  for (int i = 0; i < d.nb; ++i) {
    const double* B = balls + 4 * (int64_t)(d.ball_off + i);
    const double dx = x[0] - B[0], dy = x[1] - B[1], dz = x[2] - B[2];
    if (!((dx * dx + dy * dy) + dz * dz > B[3])) return false;
  }
  return true;
}

__device__ inline void shape(const double xi[3], double N[8], double G[8][3]) {
  for (int a = 0; a < 8; ++a) {
    const int o0 = a & 1, o1 = (a >> 1) & 1, o2 = (a >> 2) & 1;
    const double f0 = o0 ? xi[0] : 1.0 - xi[0];
    const double f1 = o1 ? xi[1] : 1.0 - xi[1];
    const double f2 = o2 ? xi[2] : 1.0 - xi[2];
    N[a] = f0 * f1 * f2;
    G[a][0] = (o0 ? 1.0 : -1.0) * f1 * f2;
    G[a][1] = f0 * (o1 ? 1.0 : -1.0) * f2;
    G[a][2] = f0 * f1 * (o2 ? 1.0 : -1.0);
  }
}

// be[c][a] = sum over the kept points of cell c of (h^3/512) N_a f.
__global__ __launch_bounds__(MW) void mms_volume_kernel(BatchDev b, MmsParams m, const double* __restrict__ xi,
                                                        const double* __restrict__ balls,
                                                        const int32_t* __restrict__ cellinfo, int64_t n_cells,
                                                        double* __restrict__ be) {
  const int64_t c = blockIdx.x;
  if (c >= n_cells) return;
  const int lane = threadIdx.x;
  const int32_t info = cellinfo[c];
  const int p = find_segment(b.cell_off, b.P, c);
  const ProbDev& d = b.prob[p];
  const int64_t lc = c - d.cell_off, N = d.N;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (info != CELL_INACTIVE && lc < N * N * N) {
    const int64_t ci = lc % N, cj = (lc / N) % N, ck = lc / (N * N);
    const double h = 1.0 / (double)N, w = h * h * h / 512.0;
    const bool cut = info >= 0;   // cut cells with stored matrices: the kept-point test
    const int kx = lane & 7, ky = lane >> 3;
    for (int t = 0; t < 8; ++t) {
      const double x[3] = {((double)ci + xi[kx]) * h, ((double)cj + xi[ky]) * h, ((double)ck + xi[t]) * h};
      if (!point_kept(d, balls, cut, x)) continue;
      double u, g[3], f, Nv[8], G[8][3];
      exact(m, x, &u, g, &f);
      const double r[3] = {xi[kx], xi[ky], xi[t]};
      shape(r, Nv, G);
      for (int a = 0; a < 8; ++a) acc[a] += w * Nv[a] * f;
    }
  }
  for (int a = 0; a < 8; ++a) {
    const double s = wave_sum(acc[a]);
    if (lane == 0) be[c * 8 + a] = s;
  }
}

// b at the DOF nodes: sum over the node's cells (ascending cell order, all
// of them: inactive cells can hold Neumann data) of be[cell][corner]; 0
// elsewhere (everywhere when be is null).  The lift ud: u at the cube-face
// nodes.
__global__ __launch_bounds__(256) void mms_gather_kernel(BatchDev b, int64_t nn, MmsParams m,
                                                         const int32_t* __restrict__ cellinfo,
                                                         const uint8_t* __restrict__ dofmask,
                                                         const double* __restrict__ be, double* __restrict__ bg,
                                                         double* __restrict__ ud) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= nn) return;
  const int p = find_segment(b.node_off, b.P, n);
  const ProbDev& d = b.prob[p];
  const int N = d.N, N1 = N + 1;
  const int64_t l = n - d.node_off;
  double v = 0.0, lift = 0.0;
  if (l < (int64_t)N1 * N1 * N1) {
    const int I = (int)(l % N1), J = (int)((l / N1) % N1), K = (int)(l / ((int64_t)N1 * N1));
    if (be && dofmask[n]) {
      for (int w = 0; w < 2; ++w)
        for (int vv = 0; vv < 2; ++vv)
          for (int u = 0; u < 2; ++u) {
            const int ci = I - 1 + u, cj = J - 1 + vv, ck = K - 1 + w;
            if (ci < 0 || cj < 0 || ck < 0 || ci >= N || cj >= N || ck >= N) continue;
            const int64_t c = d.cell_off + ci + (int64_t)N * (cj + (int64_t)N * ck);
            const int a = (1 - u) + 2 * (1 - vv) + 4 * (1 - w);
            v += be[c * 8 + a];
          }
    }
    if (I == 0 || I == N || J == 0 || J == N || K == 0 || K == N) {
      const double x[3] = {(double)I / (double)N, (double)J / (double)N, (double)K / (double)N};
      const double d0 = x[0] - m.x0[0], d1 = x[1] - m.x0[1], d2 = x[2] - m.x0[2];
      lift = sin(m.k * sqrt((d0 * d0 + d1 * d1) + d2 * d2));
    }
  }
  bg[n] = v;
  ud[n] = lift;
}

// Per cell: (sum (h^3/512)(u - u_h)^2, sum (h^3/512)|grad u - grad u_h|^2).
__global__ __launch_bounds__(MW) void mms_error_kernel(BatchDev b, MmsParams m, const double* __restrict__ xi,
                                                       const double* __restrict__ balls,
                                                       const int32_t* __restrict__ cellinfo, int64_t n_cells,
                                                       const double* __restrict__ ug, double* __restrict__ err) {
  const int64_t c = blockIdx.x;
  if (c >= n_cells) return;
  const int lane = threadIdx.x;
  const int32_t info = cellinfo[c];
  const int p = find_segment(b.cell_off, b.P, c);
  const ProbDev& d = b.prob[p];
  const int64_t lc = c - d.cell_off, N = d.N, N1 = N + 1;
  double e0 = 0.0, e1 = 0.0;
  if (info != CELL_INACTIVE && lc < N * N * N) {
    const int64_t ci = lc % N, cj = (lc / N) % N, ck = lc / (N * N);
    double ue[8];
    for (int a = 0; a < 8; ++a)
      ue[a] = ug[d.node_off + (ci + (a & 1)) + N1 * ((cj + ((a >> 1) & 1)) + N1 * (ck + ((a >> 2) & 1)))];
    const double h = 1.0 / (double)N, w = h * h * h / 512.0;
    const int kx = lane & 7, ky = lane >> 3;
    for (int t = 0; t < 8; ++t) {
      const double x[3] = {((double)ci + xi[kx]) * h, ((double)cj + xi[ky]) * h, ((double)ck + xi[t]) * h};
      if (!point_kept(d, balls, info >= 0, x)) continue;
      double u, g[3], f, Nv[8], G[8][3];
      exact(m, x, &u, g, &f);
      const double r[3] = {xi[kx], xi[ky], xi[t]};
      shape(r, Nv, G);
      double uh = 0.0, gh[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < 8; ++a) {
        uh += Nv[a] * ue[a];
        for (int q = 0; q < 3; ++q) gh[q] += G[a][q] * ue[a];
      }
      const double du = u - uh;
      e0 += w * (du * du);
      double s2 = 0.0;
      for (int q = 0; q < 3; ++q) {
        const double dg = g[q] - gh[q] / h;
        s2 += dg * dg;
      }
      e1 += w * s2;
    }
  }
  e0 = wave_sum(e0);
  e1 = wave_sum(e1);
  if (lane == 0) {
    err[2 * c] = e0;
    err[2 * c + 1] = e1;
  }
}

// Sums the per-cell errors of every cell in order (one workgroup).
__global__ __launch_bounds__(256) void mms_error_sum_kernel(int64_t n_cells, const double* __restrict__ err,
                                                            double* __restrict__ out) {
  __shared__ double s0[256], s1[256];
  double a0 = 0.0, a1 = 0.0;
  for (int64_t c = threadIdx.x; c < n_cells; c += 256) {
    a0 += err[2 * c];
    a1 += err[2 * c + 1];
  }
  s0[threadIdx.x] = a0;
  s1[threadIdx.x] = a1;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t0 = 0.0, t1 = 0.0;
    for (int i = 0; i < 256; ++i) {
      t0 += s0[i];
      t1 += s1[i];
    }
    out[0] = t0;
    out[1] = t1;
  }
}

__global__ void mms_finish_kernel(int64_t n, const int64_t* __restrict__ dof_node, const double* __restrict__ bg,
                                  const double* __restrict__ y, double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = bg[dof_node[i]] - y[dof_node[i]];
}

}  // namespace

void launch_mms_finish(hipStream_t st, int64_t n_dof, const int64_t* dof_node, const double* bg, const double* y,
                       double* b) {
  if (n_dof <= 0) return;
  hipLaunchKernelGGL(mms_finish_kernel, dim3((unsigned)((n_dof + 255) / 256)), dim3(256), 0, st, n_dof, dof_node, bg,
                     y, b);
}

void launch_mms_volume(hipStream_t st, const BatchDev& b, const MmsParams& m, const double* xi, const double* balls,
                       const int32_t* cellinfo, int64_t n_cells, double* be) {
  if (n_cells <= 0) return;
  hipLaunchKernelGGL(mms_volume_kernel, dim3((unsigned)n_cells), dim3(MW), 0, st, b, m, xi, balls, cellinfo, n_cells,
                     be);
}

void launch_mms_gather(hipStream_t st, const BatchDev& b, int64_t nn, const MmsParams& m, const int32_t* cellinfo,
                       const uint8_t* dofmask, const double* be, double* bg, double* ud) {
  if (nn <= 0) return;
  hipLaunchKernelGGL(mms_gather_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, b, nn, m, cellinfo,
                     dofmask, be, bg, ud);
}

void launch_mms_errors(hipStream_t st, const BatchDev& b, const MmsParams& m, const double* xi, const double* balls,
                       const int32_t* cellinfo, int64_t n_cells, const double* ug, double* err, double* out) {
  if (n_cells <= 0) return;
  hipLaunchKernelGGL(mms_error_kernel, dim3((unsigned)n_cells), dim3(MW), 0, st, b, m, xi, balls, cellinfo, n_cells,
                     ug, err);
  hipLaunchKernelGGL(mms_error_sum_kernel, dim3(1), dim3(256), 0, st, n_cells, err, out);
}

}  // namespace cutbddc
