// Cell classification and cut-cell integration (paper Sect. 2.1-2.2).
//
// Each cell carries 4^3 sub-cells with a 2x2x2 Gauss rule: 8 reference
// coordinates xi_k per axis (computed once on the host), 512 points per cell,
// weight 1/512 in reference coordinates.  A point is kept when it lies
// outside every ball: (dx*dx + dy*dy) + dz*dz > r*r, evaluated in this order
// without fused multiply-adds so that the integer classification is
// reproducible.  Cells are classified per wavefront: a conservative box test
// per ball (with a 1e-12 relative margin, far above the rounding of the
// point test) skips balls that cannot touch the cell and detects balls that
// swallow it; only the remaining balls are evaluated point by point.
//
// Cut-cell integration stores the reference stiffness
//   K[a,b] = sum_{kept q} (1/512) gradN_a(xi_q) . gradN_b(xi_q)
// and mass M[a,b] = sum_{kept q} (1/512) N_a N_b (kappa = 1, h = 1) as packed
// upper triangles; the operator scales them by kappa_e h and h^3.
#include "common.h"

#pragma clang fp contract(off)

namespace cutbddc {
namespace {

constexpr int WAVE = 64;
constexpr int CELLS_PER_BLOCK = 4;

// Ball relation to the box spanned by a cell's Gauss points:
//  0: every point outside the ball, 1: some points may be inside,
//  2: every point inside the ball.
__device__ inline int ball_box_relation(const double lo[3], const double hi[3], const double* b) {
  double near2 = 0.0, far2 = 0.0;
  for (int d = 0; d < 3; ++d) {
    double c = b[d];
    double e = fmax(fmax(lo[d] - c, c - hi[d]), 0.0);
    double f = fmax(fabs(lo[d] - c), fabs(hi[d] - c));
    near2 = near2 + e * e;
    far2 = far2 + f * f;
  }
  double r2 = b[3];
  if (near2 > r2 * (1.0 + 1e-12)) return 0;
  if (far2 < r2 * (1.0 - 1e-12)) return 2;
  return 1;
}

// Evaluates the kept bits of the 8 points owned by this lane: point
// q = lane + 64 t has kx = lane % 8, ky = lane / 8, kz = t.  Returns the
// number of kept points in the cell (wave-uniform) and the lane's bits.
__device__ inline int cell_kept_bits(int N, const double* __restrict__ xi, const double* __restrict__ balls,
                                     int nb, int64_t cell, int lane, unsigned& bits) {
  const double h = 1.0 / (double)N;
  const int64_t i = cell % N, j = (cell / N) % N, k = cell / ((int64_t)N * N);
  double lo[3] = {((double)i + xi[0]) * h, ((double)j + xi[0]) * h, ((double)k + xi[0]) * h};
  double hi[3] = {((double)i + xi[7]) * h, ((double)j + xi[7]) * h, ((double)k + xi[7]) * h};
  const int kx = lane & 7, ky = lane >> 3;
  const double x = ((double)i + xi[kx]) * h;
  const double y = ((double)j + xi[ky]) * h;
  double zs[8];
  for (int t = 0; t < 8; ++t) zs[t] = ((double)k + xi[t]) * h;
  bits = 0xffu;
  bool swallowed = false;
  for (int base = 0; base < nb; base += WAVE) {
    int b = base + lane;
    int rel = 0;
    if (b < nb) rel = ball_box_relation(lo, hi, balls + 4 * b);
    unsigned long long near = __ballot(rel == 1);
    unsigned long long inside = __ballot(rel == 2);
    if (inside) {
      swallowed = true;
      break;
    }
    while (near) {
      int bit = __ffsll((long long)near) - 1;
      near &= near - 1;
      const double* B = balls + 4 * (base + bit);
      const double dx = x - B[0];
      const double dy = y - B[1];
      const double dxy = dx * dx + dy * dy;
      for (int t = 0; t < 8; ++t) {
        const double dz = zs[t] - B[2];
        const double d2 = dxy + dz * dz;
        if (!(d2 > B[3])) bits &= ~(1u << t);
      }
    }
  }
  if (swallowed) {
    bits = 0;
    return 0;
  }
  int cnt = 0;
  for (int t = 0; t < 8; ++t) cnt += __popcll(__ballot((bits >> t) & 1u));
  return cnt;
}

// Cells of all problems in one launch, 64 consecutive cells per wave.
// Each lane first tests its cell's point box against the problem's balls:
// a box inside a ball keeps no point and a box clear of every ball keeps
// all 512 (what cell_kept_bits returns in those cases); the remaining cells
// get the point-by-point test of cell_kept_bits, one after another with the
// whole wave.
__global__ __launch_bounds__(256) void classify_kernel(BatchDev bd, int64_t n_cells_total,
                                                       const double* __restrict__ xi_g,
                                                       const double* __restrict__ balls,
                                                       int32_t* __restrict__ count) {
  __shared__ double xi[8];
  if (threadIdx.x < 8) xi[threadIdx.x] = xi_g[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t wbase = ((int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE) * WAVE;
  const int64_t cell = wbase + lane;
  bool detail = false;
  if (cell < n_cells_total) {
    const ProbDev pr = bd.prob[find_segment(bd.cell_off, bd.P, cell)];
    const int64_t local = cell - pr.cell_off;
    const int N = pr.N;
    if (local >= (int64_t)N * N * N) {
      count[cell] = 0;
    } else {
      const double h = 1.0 / (double)N;
      const int64_t i = local % N, j = (local / N) % N, k = local / ((int64_t)N * N);
      const double lo[3] = {((double)i + xi[0]) * h, ((double)j + xi[0]) * h, ((double)k + xi[0]) * h};
      const double hi[3] = {((double)i + xi[7]) * h, ((double)j + xi[7]) * h, ((double)k + xi[7]) * h};
      const double* bl = balls + 4 * (int64_t)pr.ball_off;
      bool near = false, inside = false;
      for (int b = 0; b < pr.nb && !inside; ++b) {
        const int rel = ball_box_relation(lo, hi, bl + 4 * b);
        inside = rel == 2;
        near = near || rel == 1;
      }
      if (inside) count[cell] = 0;
      else if (!near) count[cell] = 512;
      else detail = true;
    }
  }
  unsigned long long todo = __ballot(detail);
  while (todo) {
    const int l = __ffsll((long long)todo) - 1;
    todo &= todo - 1;
    const int64_t c = wbase + l;
    const ProbDev pr = bd.prob[find_segment(bd.cell_off, bd.P, c)];
    unsigned bits;
    const int cnt = cell_kept_bits(pr.N, xi, balls + 4 * (int64_t)pr.ball_off, pr.nb, c - pr.cell_off, lane, bits);
    if (lane == 0) count[c] = cnt;
  }
}

// cut_cells: ids in the concatenated cell space.
__global__ __launch_bounds__(256) void integrate_cut_kernel(BatchDev bd, const double* __restrict__ xi_g,
                                                            const double* __restrict__ balls,
                                                            const int64_t* __restrict__ cut_cells,
                                                            int64_t n_cut, double* __restrict__ Kc,
                                                            double* __restrict__ Mc) {
  __shared__ double xi[8];
  __shared__ __align__(8) unsigned char keep[CELLS_PER_BLOCK][512];
  if (threadIdx.x < 8) xi[threadIdx.x] = xi_g[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int64_t idx = (int64_t)blockIdx.x * CELLS_PER_BLOCK + wv;
  const bool valid = idx < n_cut;
  unsigned bits = 0;
  if (valid) {
    const int64_t cell = cut_cells[idx];
    const int p = find_segment(bd.cell_off, bd.P, cell);
    const ProbDev pr = bd.prob[p];
    cell_kept_bits(pr.N, xi, balls + 4 * (int64_t)pr.ball_off, pr.nb, cell - pr.cell_off, lane, bits);
  }
  for (int t = 0; t < 8; ++t) keep[wv][lane + WAVE * t] = (unsigned char)((bits >> t) & 1u);
  __syncthreads();
  if (!valid || lane >= PACK36) return;
  // packed entry (a, b), a <= b
  int a = 0, rem = lane;
  while (rem >= 8 - a) {
    rem -= 8 - a;
    ++a;
  }
  const int b = a + rem;
  const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
  const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
  // Tensor-product form: with X_i = f_a(x_i) f_b(x_i) (f = p or 1 - p by the
  // corner's bit), Y_j, Z_k alike and g = +-1 the product of the two
  // derivative signs per axis, the stiffness term at point (i, j, k) is
  // gx Y_j Z_k + X_i (gy Z_k + gz Y_j) and the mass term X_i Y_j Z_k.
  double X[8], Y[8], Z[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const double p = xi[i], m = 1.0 - p;
    X[i] = (ax ? p : m) * (bx ? p : m);
    Y[i] = (ay ? p : m) * (by ? p : m);
    Z[i] = (az ? p : m) * (bz ? p : m);
  }
  const double gx = ax == bx ? 1.0 : -1.0, gy = ay == by ? 1.0 : -1.0, gz = az == bz ? 1.0 : -1.0;
  const uint64_t* kb = reinterpret_cast<const uint64_t*>(keep[wv]);
  double ks = 0.0, ms = 0.0;
  // points in ascending q = 64 k + 8 j + i; byte i of kb[8 k + j] is point q
#pragma unroll
  for (int k = 0; k < 8; ++k) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint64_t mk = kb[8 * k + j];
      if (!mk) continue;
      const double yz = Y[j] * Z[k], w = gy * Z[k] + gz * Y[j], gyz = gx * yz;
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if ((mk >> (8 * i)) & 0xffu) {
          ks += gyz + X[i] * w;
          ms += X[i] * yz;
        }
    }
  }
  Kc[idx * PACK36 + lane] = ks * (1.0 / 512.0);
  Mc[idx * PACK36 + lane] = ms * (1.0 / 512.0);
}

}  // namespace

void launch_classify(hipStream_t st, const BatchDev& b, int64_t n_cells_total, const double* xi,
                     const double* balls, int32_t* count) {
  if (n_cells_total <= 0) return;
  const int64_t blocks = (n_cells_total + 255) / 256;   // 64 cells per wave
  hipLaunchKernelGGL(classify_kernel, dim3((unsigned)blocks), dim3(256), 0, st, b, n_cells_total, xi, balls,
                     count);
}

void launch_integrate_cut(hipStream_t st, const BatchDev& b, const double* xi, const double* balls,
                          const int64_t* cut_cells, int64_t n_cut, double* Kc, double* Mc) {
  if (n_cut <= 0) return;
  const int64_t blocks = (n_cut + CELLS_PER_BLOCK - 1) / CELLS_PER_BLOCK;
  hipLaunchKernelGGL(integrate_cut_kernel, dim3((unsigned)blocks), dim3(256), 0, st, b, xi, balls, cut_cells,
                     n_cut, Kc, Mc);
}

}  // namespace cutbddc
