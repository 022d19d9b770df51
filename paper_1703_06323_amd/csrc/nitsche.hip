// Weak Dirichlet data on the ball surfaces by Nitsche's method (paper
// Sect. 2.2: the surface terms of A_e, beta_e >= C_e with C_e the largest
// eigenvalue of eq. local-eigenvals, and beta_e = 2 lambda_max).
//
// Readings (the paper omits its integration section; the oracle applies
// the same ones):
//  * Each ball carries a tensor rule on its sphere: n_t Gauss-Legendre
//    nodes in t = cos(theta), n_phi = 2 n_t midpoint nodes in phi, weight
//    r^2 w_j 2 pi / n_phi (tables built on the host, NitscheRule).
//  * Gamma_cut of a ball is the part of its sphere inside the open unit
//    cube and outside every other ball (the kept-point test of the volume
//    rule); a kept point belongs to the cell floor(x N) and counts only if
//    that cell is cut.  The outward normal of Omega points into the ball.
//  * In a cell's unit frame, S = sum w N_a N_b, T = sum w (n.grad N_a) N_b,
//    U = sum w (n.grad N_a)(n.grad N_b), summed in the order (ball, j, k);
//    lambda = largest eigenvalue of U x = lambda (K + 1e-6 K_ref) x on the
//    complement of the constants (K the cell's unit stiffness, K_ref a whole
//    cell's: the void part of the cell counted with stiffness 1e-6, which
//    bounds lambda where the kept-point rule leaves K singular there), and
//    the stored unit stiffness becomes
//    K + 2 lambda S - T - T^T (homogeneous Dirichlet data: the load is
//    unchanged).
// One 64-lane wave per cut cell: the lanes first test candidate points of
// the sphere rule in parallel and compact the kept ones into LDS in rule
// order; then lane l accumulates T[l] and, for l < 36, the packed S[l] and
// U[l] over those points in that order; lane 0 finally solves the 7x7
// eigenproblem and writes the cell's matrix.
#include "nitsche.h"
#include "manufactured.h"

#pragma clang fp contract(off)

namespace cutbddc {
namespace {

constexpr int NW = 64;          // lanes per cell
constexpr int NPTS = 512;       // kept points staged per pass

__device__ inline void shape(const double xi[3], double N[8], double G[8][3]) {
  for (int a = 0; a < 8; ++a) {
    const int o0 = a & 1, o1 = (a >> 1) & 1, o2 = (a >> 2) & 1;
    const double f0 = o0 ? xi[0] : 1.0 - xi[0];
    const double f1 = o1 ? xi[1] : 1.0 - xi[1];
    const double f2 = o2 ? xi[2] : 1.0 - xi[2];
    const double s0 = o0 ? 1.0 : -1.0, s1 = o1 ? 1.0 : -1.0, s2 = o2 ? 1.0 : -1.0;
    N[a] = f0 * f1 * f2;
    G[a][0] = s0 * f1 * f2;
    G[a][1] = f0 * s1 * f2;
    G[a][2] = f0 * f1 * s2;
  }
}

// Cyclic Jacobi eigenvalues of the symmetric 7x7 matrix C (destroyed); the
// largest one.
__device__ inline double jacobi_max(double C[7][7]) {
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < 7; ++i)
      for (int j = 0; j < 7; ++j) {
        tot += C[i][j] * C[i][j];
        if (i != j) off += C[i][j] * C[i][j];
      }
    if (!(off > 1e-32 * tot)) break;
    for (int p = 0; p < 6; ++p)
      for (int q = p + 1; q < 7; ++q) {
        if (C[p][q] == 0.0) continue;
        const double theta = (C[q][q] - C[p][p]) / (2.0 * C[p][q]);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 7; ++k) {
          const double ckp = C[k][p], ckq = C[k][q];
          C[k][p] = c * ckp - s * ckq;
          C[k][q] = s * ckp + c * ckq;
        }
        for (int k = 0; k < 7; ++k) {
          const double cpk = C[p][k], cqk = C[q][k];
          C[p][k] = c * cpk - s * cqk;
          C[q][k] = s * cpk + c * cqk;
        }
      }
  }
  double m = C[0][0];
  for (int i = 1; i < 7; ++i) m = fmax(m, C[i][i]);
  return m;
}

// 2 lambda_max of U x = lambda (K + NITSCHE_BETA_REG K_ref) x on the
// complement of the constants, from the full 8x8 K and U (both vanish on
// constants) and the whole cell's unit stiffness kref.  The complement basis is
// columns 1..7 of the Householder reflection H that maps e_0 to 1/sqrt(8).
__device__ inline double beta_from(const double K[8][8], const double U[8][8], const double* __restrict__ kref) {
  const double r8 = 1.0 / sqrt(8.0);
  double u[8];
  for (int i = 0; i < 8; ++i) u[i] = r8;
  u[0] -= 1.0;
  double nu = 0.0;
  for (int i = 0; i < 8; ++i) nu += u[i] * u[i];
  double H[8][8];
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) H[i][j] = (i == j ? 1.0 : 0.0) - 2.0 * u[i] * u[j] / nu;
  double K7[7][7], U7[7][7];
  for (int i = 0; i < 7; ++i)
    for (int j = 0; j < 7; ++j) {
      double k = 0.0, w = 0.0;
      for (int a = 0; a < 8; ++a) {
        double ka = 0.0, wa = 0.0;
        for (int b = 0; b < 8; ++b) {
          ka += (K[a][b] + NITSCHE_BETA_REG * kref[a * 8 + b]) * H[b][j + 1];
          wa += U[a][b] * H[b][j + 1];
        }
        k += H[a][i + 1] * ka;
        w += H[a][i + 1] * wa;
      }
      K7[i][j] = k;
      U7[i][j] = w;
    }
  bool any = false;
  for (int i = 0; i < 7; ++i)
    for (int j = 0; j < 7; ++j) any = any || U7[i][j] != 0.0;
  if (!any) return 0.0;
  // K7 = L L^T
  double L[7][7] = {};
  for (int j = 0; j < 7; ++j) {
    double d = K7[j][j];
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 0.0)) return -1.0;
    L[j][j] = sqrt(d);
    for (int i = j + 1; i < 7; ++i) {
      double v = K7[i][j];
      for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
      L[i][j] = v / L[j][j];
    }
  }
  // C = L^-1 U7 L^-T: W = L^-1 U7 (forward substitution per column), then
  // C = W L^-T (forward substitution per row)
  double Wm[7][7];
  for (int c = 0; c < 7; ++c)
    for (int i = 0; i < 7; ++i) {
      double v = U7[i][c];
      for (int k = 0; k < i; ++k) v -= L[i][k] * Wm[k][c];
      Wm[i][c] = v / L[i][i];
    }
  double C[7][7];
  for (int r = 0; r < 7; ++r)
    for (int i = 0; i < 7; ++i) {
      double v = Wm[r][i];
      for (int k = 0; k < i; ++k) v -= L[i][k] * C[r][k];
      C[r][i] = v / L[i][i];
    }
  for (int i = 0; i < 7; ++i)   // symmetrise the rounding
    for (int j = i + 1; j < 7; ++j) {
      const double m = 0.5 * (C[i][j] + C[j][i]);
      C[i][j] = m;
      C[j][i] = m;
    }
  return 2.0 * jacobi_max(C);
}

// MODE 0: adds the Nitsche terms to Kc (homogeneous data) and stores
// beta per cut cell.  MODE 1 / 2: adds the surface load of the exact
// solution m to be[cell] (1: Neumann data grad u . n, physical weight w,
// on every cell (cut_cells null), whatever its class; 2: Nitsche data u,
// h w_unit (beta N_a - n . grad N_a) u with the stored beta, on the cut
// cells).
template <int MODE>
__global__ __launch_bounds__(NW) void nitsche_kernel(BatchDev b, NitscheRule rule, const double* __restrict__ balls,
                                                     const int64_t* __restrict__ cut_cells, int64_t n_cut,
                                                     double* __restrict__ Kc, double* __restrict__ beta_c,
                                                     int* __restrict__ status, MmsParams mp,
                                                     double* __restrict__ be) {
  __shared__ double pts[NPTS][10];  // xi (3), n (3), unit weight, x (3)
  __shared__ int cnt;
  const int64_t e = blockIdx.x;
  if (e >= n_cut) return;
  const int lane = threadIdx.x;
  const int64_t c = cut_cells ? cut_cells[e] : e;   // no list: every cell of the context
  const int p = find_segment(b.cell_off, b.P, c);
  const ProbDev& d = b.prob[p];
  const int N = d.N;
  const int64_t lc = c - d.cell_off;
  if (lc >= (int64_t)N * N * N) return;               // alignment padding after the problem's cells
  const int ci = (int)(lc % N), cj = (int)((lc / N) % N), ck = (int)(lc / ((int64_t)N * N));
  const double h = d.h;
  const double lo[3] = {ci * h, cj * h, ck * h}, hi[3] = {(ci + 1) * h, (cj + 1) * h, (ck + 1) * h};
  const int ax = lane & 7, bx = lane >> 3;          // T entry (ax, bx) of this lane
  int sa = -1, sb = -1;                             // packed S / U entry of this lane (lane < 36)
  if (lane < 36) {
    int k = lane, r = 0;
    while (k >= 8 - r) {
      k -= 8 - r;
      ++r;
    }
    sa = r;
    sb = r + k;
  }
  double accS = 0.0, accT = 0.0, accU = 0.0, accB = 0.0;
  const double beta_cell = MODE == 2 ? beta_c[e] : 0.0;
  const double* Bp = balls + 4 * (int64_t)d.ball_off;
  const double Nd = (double)N;
  auto flush = [&](int n) {
    for (int q = 0; q < n; ++q) {
      const double xi[3] = {pts[q][0], pts[q][1], pts[q][2]};
      const double nv[3] = {pts[q][3], pts[q][4], pts[q][5]};
      const double wu = pts[q][6];
      double Nsh[8], G[8][3];
      shape(xi, Nsh, G);
      if (MODE == 0) {
        const double dna = (G[ax][0] * nv[0] + G[ax][1] * nv[1]) + G[ax][2] * nv[2];
        accT += wu * dna * Nsh[bx];
        if (sa >= 0) {
          const double dsa = (G[sa][0] * nv[0] + G[sa][1] * nv[1]) + G[sa][2] * nv[2];
          const double dsb = (G[sb][0] * nv[0] + G[sb][1] * nv[1]) + G[sb][2] * nv[2];
          accS += wu * Nsh[sa] * Nsh[sb];
          accU += wu * dsa * dsb;
        }
      } else if (lane < 8) {
        // the exact solution at the point
        const double x[3] = {pts[q][7], pts[q][8], pts[q][9]};
        const double d0 = x[0] - mp.x0[0], d1 = x[1] - mp.x0[1], d2 = x[2] - mp.x0[2];
        const double rho = sqrt((d0 * d0 + d1 * d1) + d2 * d2);
        const double u = sin(mp.k * rho), du = mp.k * cos(mp.k * rho);
        if (MODE == 1) {
          const double gn = (((du / rho) * d0) * nv[0] + ((du / rho) * d1) * nv[1]) + ((du / rho) * d2) * nv[2];
          accB += (wu / (Nd * Nd)) * Nsh[lane] * gn;
        } else {
          const double dn = (G[lane][0] * nv[0] + G[lane][1] * nv[1]) + G[lane][2] * nv[2];
          accB += h * wu * (beta_cell * Nsh[lane] - dn) * u;
        }
      }
    }
  };
  if (lane == 0) cnt = 0;
  __syncthreads();
  for (int i = 0; i < d.nb; ++i) {
    const double* B = Bp + 4 * i;
    const NitscheBall rb = rule.ball[d.ball_off + i];
    const double r = rb.r;
    // does the sphere meet the cell's box?
    double near2 = 0.0, far2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double dn = B[a] < lo[a] ? lo[a] - B[a] : (B[a] > hi[a] ? B[a] - hi[a] : 0.0);
      const double df = fmax(fabs(B[a] - lo[a]), fabs(B[a] - hi[a]));
      near2 += dn * dn;
      far2 += df * df;
    }
    if (near2 > r * r || far2 < r * r) continue;
    // rows j whose z = c_z + r t_j can lie in the cell (one more each side)
    const double* t = rule.t + rb.off_t;
    const double tmin = (lo[2] - B[2]) / r, tmax = (hi[2] - B[2]) / r;
    int j0 = 0, j1 = rb.nt - 1;
    while (j0 < rb.nt - 1 && t[j0 + 1] < tmin) ++j0;
    while (j1 > 0 && t[j1 - 1] > tmax) --j1;
    const int nphi = rb.nphi;
    const int64_t ncand = (int64_t)(j1 - j0 + 1) * nphi;
    for (int64_t base = 0; base < ncand; base += NW) {
      const int64_t q = base + lane;
      bool keep = false;
      double xv[3] = {0.0, 0.0, 0.0}, nv[3] = {0.0, 0.0, 0.0}, w = 0.0;
      if (q < ncand) {
        const int j = j0 + (int)(q / nphi), k = (int)(q % nphi);
        const double tj = t[j], st = sqrt(1.0 - tj * tj);
        const double dv[3] = {st * rule.cphi[rb.off_phi + k], st * rule.sphi[rb.off_phi + k], tj};
        keep = true;
        for (int a = 0; a < 3; ++a) {
          xv[a] = B[a] + r * dv[a];
          nv[a] = -dv[a];
          keep = keep && xv[a] > 0.0 && xv[a] < 1.0;
        }
        for (int o = 0; o < d.nb && keep; ++o) {
          if (o == i) continue;
          const double* Bo = Bp + 4 * o;
          const double dx = xv[0] - Bo[0], dy = xv[1] - Bo[1], dz = xv[2] - Bo[2];
          if (!((dx * dx + dy * dy) + dz * dz > Bo[3])) keep = false;
        }
        if (keep) {
          const int cc[3] = {ci, cj, ck};
          for (int a = 0; a < 3; ++a) {
            int m = (int)floor(xv[a] * Nd);
            if (m > N - 1) m = N - 1;
            keep = keep && m == cc[a];
          }
        }
        w = (r * r) * rule.w[rb.off_t + j] * rule.dphi[d.ball_off + i];
      }
      // compact the kept points of this chunk into LDS, in candidate order
      const unsigned long long mask = __ballot(keep);
      if (keep) {
        const int slot = cnt + __popcll(mask & ((1ull << lane) - 1ull));
        pts[slot][0] = xv[0] * Nd - (double)ci;
        pts[slot][1] = xv[1] * Nd - (double)cj;
        pts[slot][2] = xv[2] * Nd - (double)ck;
        pts[slot][3] = nv[0];
        pts[slot][4] = nv[1];
        pts[slot][5] = nv[2];
        pts[slot][6] = w * (Nd * Nd);
        pts[slot][7] = xv[0];
        pts[slot][8] = xv[1];
        pts[slot][9] = xv[2];
      }
      __syncthreads();
      if (lane == 0) cnt += __popcll(mask);
      __syncthreads();
      if (cnt > NPTS - NW) {   // room for one more chunk is kept
        flush(cnt);
        __syncthreads();
        if (lane == 0) cnt = 0;
        __syncthreads();
      }
    }
  }
  flush(cnt);
  if (MODE != 0) {
    if (lane < 8) be[c * 8 + lane] += accB;
    return;
  }
  // assemble S, T, U of the cell in LDS (reusing the point buffer)
  __syncthreads();
  double* Sm = &pts[0][0];          // [8][8]
  double* Tm = Sm + 64;             // [8][8]
  double* Um = Tm + 64;             // [8][8]
  Tm[ax * 8 + bx] = accT;
  if (sa >= 0) {
    Sm[sa * 8 + sb] = accS;
    Sm[sb * 8 + sa] = accS;
    Um[sa * 8 + sb] = accU;
    Um[sb * 8 + sa] = accU;
  }
  __syncthreads();
  if (lane == 0) {
    double* R = Kc + e * PACK36;
    double K[8][8], U[8][8];
    for (int a = 0; a < 8; ++a)
      for (int bb = 0; bb < 8; ++bb) {
        K[a][bb] = R[pack_index(a, bb)];
        U[a][bb] = Um[a * 8 + bb];
      }
    const double beta = beta_from(K, U, rule.kref);
    beta_c[e] = beta;
    if (beta < 0.0) {
      atomicAdd(status, 1);
      return;
    }
    for (int a = 0; a < 8; ++a)
      for (int bb = a; bb < 8; ++bb)
        R[pack_index(a, bb)] = K[a][bb] + beta * Sm[a * 8 + bb] - Tm[a * 8 + bb] - Tm[bb * 8 + a];
  }
}

}  // namespace

void launch_nitsche(hipStream_t st, const BatchDev& b, const NitscheRule& rule, const double* balls,
                    const int64_t* cut_cells, int64_t n_cut, double* Kc, double* beta, int* status) {
  if (n_cut <= 0) return;
  hipLaunchKernelGGL(nitsche_kernel<0>, dim3((unsigned)n_cut), dim3(NW), 0, st, b, rule, balls, cut_cells, n_cut, Kc,
                     beta, status, MmsParams{}, (double*)nullptr);
}

void launch_surface_load(hipStream_t st, const BatchDev& b, const NitscheRule& rule, const double* balls,
                         int64_t n_cells, const int64_t* cut_cells, int64_t n_cut, int nitsche, const double* beta,
                         const MmsParams& m, double* be) {
  if (nitsche ? n_cut <= 0 : n_cells <= 0) return;
  if (nitsche)
    hipLaunchKernelGGL(nitsche_kernel<2>, dim3((unsigned)n_cut), dim3(NW), 0, st, b, rule, balls, cut_cells, n_cut,
                       (double*)nullptr, const_cast<double*>(beta), (int*)nullptr, m, be);
  else
    hipLaunchKernelGGL(nitsche_kernel<1>, dim3((unsigned)n_cells), dim3(NW), 0, st, b, rule, balls,
                       (const int64_t*)nullptr, n_cells, (double*)nullptr, (double*)nullptr, (int*)nullptr, m, be);
}

}  // namespace cutbddc

namespace cutbddc {

void gauss_legendre(int n, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    // z is the i-th largest root
    x[n - 1 - i] = z;
    x[i] = -z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

}  // namespace cutbddc
