// Matrix-free operator A-bar = sum_e A_e (paper Sect. 2.2), load
// b = M_cut f, adjoint contraction and FP64 vector kernels.
//
// Vectors live on the full grid of (N+1)^3 nodes with zeros at non-DOF
// nodes, so every kernel is pure index arithmetic with coalesced access.
// Node-centric gather: the thread of node n sums the rows of the (up to 8)
// active cells around it; no atomics, fixed summation order.
#include "common.h"

#include <algorithm>

#pragma clang fp contract(off)

namespace cutbddc {
namespace {

__constant__ double c_Kref[64];   // reference Q1 stiffness (kappa = 1, h = 1)
__constant__ double c_Mref[64];   // reference Q1 mass (h = 1)

template <bool MASS, bool ONES = false>
__device__ inline double node_gather(int N, int I, int J, int K, const int32_t* __restrict__ cellinfo,
                                     const double* __restrict__ kappa, const double* __restrict__ Mat,
                                     const double* __restrict__ x, double scale) {
  const int N1 = N + 1;
  // x at the 27 nodes (I + dx - 1, J + dy - 1, K + dz - 1) around the node,
  // each loaded once (zero off the grid, where no active cell reads it)
  double xn[3][3][3];
#pragma unroll
  for (int dz = 0; dz < 3; ++dz)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int i = I + dx - 1, j = J + dy - 1, k = K + dz - 1;
        const bool in = !ONES && i >= 0 && i < N1 && j >= 0 && j < N1 && k >= 0 && k < N1;
        xn[dz][dy][dx] = in ? x[i + N1 * (j + N1 * k)] : 0.0;
      }
  double acc = 0.0;
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const int ck = K - 1 + w;
    if (ck < 0 || ck >= N) continue;
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int cj = J - 1 + v;
      if (cj < 0 || cj >= N) continue;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int ci = I - 1 + u;
        if (ci < 0 || ci >= N) continue;
        const int64_t c = ci + (int64_t)N * (cj + (int64_t)N * ck);
        const int32_t info = cellinfo[c];
        if (info == CELL_INACTIVE) continue;
        const int a = (1 - u) + 2 * (1 - v) + 4 * (1 - w);   // the node's corner in the cell
        const double s = MASS ? scale : kappa[c] * scale;
        double row = 0.0;
        if (info == CELL_UNCUT) {
          const double* R = MASS ? c_Mref : c_Kref;
#pragma unroll
          for (int b = 0; b < 8; ++b)
            row += R[a * 8 + b] * (ONES ? 1.0 : xn[w + ((b >> 2) & 1)][v + ((b >> 1) & 1)][u + (b & 1)]);
        } else {
          const double* R = Mat + (int64_t)info * PACK36;
#pragma unroll
          for (int b = 0; b < 8; ++b)
            row += R[pack_index(a, b)] * (ONES ? 1.0 : xn[w + ((b >> 2) & 1)][v + ((b >> 1) & 1)][u + (b & 1)]);
        }
        acc += s * row;
      }
    }
  }
  return acc;
}

// Sum of v over the workgroup, returned to every thread (the same order in
// every workgroup: lanes by shuffles, then the waves in order).  sh holds
// one double per wave.
__device__ inline double wg_sum_all(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += sh[i];
  __syncthreads();
  return t;
}

// Sum of part[b0, b1) by the whole workgroup, returned to every thread; all
// workgroups that call it with the same range get the same value.
__device__ inline double wg_sum_range(const double* __restrict__ part, int64_t b0, int64_t b1, double* sh) {
  double acc = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) acc += part[i];
  return wg_sum_all(acc, sh);
}

// Workgroup b runs on XCD b % 8: renumber so that each XCD runs a
// contiguous range of the G items (neighbouring blocks share their halo in
// that XCD's L2).
__device__ inline int32_t xcd_item(int32_t b, int32_t G) {
  const int32_t xcd = b & 7, k = b >> 3, base = G >> 3, rem = G & 7;
  return (xcd < rem ? xcd * (base + 1) : rem * (base + 1) + (xcd - rem) * base) + k;
}

// Cell C = u + 2 vv + 4 w around node (I, J, K) of the node-block operator kernel,
// without branches except around a cut cell's row load: a cell outside the
// grid counts as inactive (its staged code belongs to another cell), and an
// inactive one adds nothing.  cc stays inside the staged cell ranges for
// every node of the block.
template <int C>
__device__ __forceinline__ void op_cell_lin(int I, int J, int K, int N, int LC, int co, const int32_t* cs,
                                        const double* ks, const double* __restrict__ Kf,
                                        const double (&xn)[3][3][3], double& acc, bool& touched) {
  constexpr int u = C & 1, vv = (C >> 1) & 1, w = C >> 2;
  constexpr int a = 7 - C;                               // the node's corner in the cell
  const bool in = (unsigned)(I - 1 + u) < (unsigned)N && (unsigned)(J - 1 + vv) < (unsigned)N &&
                  (unsigned)(K - 1 + w) < (unsigned)N;
  const int cc = w * LC + co + u + N * vv;
  const int32_t info = in ? cs[cc] : CELL_INACTIVE;
  const bool act = info != CELL_INACTIVE;
  touched = touched || act;
  // row a of the cell matrix times x: the reference row (constant
  // operands), replaced for a cut cell by its row from the full row-major
  // copy (64 contiguous bytes)
  double row = 0.0;
#pragma unroll
  for (int b = 0; b < 8; ++b)
    row = fma(c_Kref[a * 8 + b], xn[w + ((b >> 2) & 1)][vv + ((b >> 1) & 1)][u + (b & 1)], row);
  if (info >= 0) {
    const double2* R = reinterpret_cast<const double2*>(Kf + (int64_t)info * 64 + a * 8);
    double rc = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 v2 = R[q];
      rc = fma(v2.x, xn[w + (((2 * q) >> 2) & 1)][vv + (((2 * q) >> 1) & 1)][u + ((2 * q) & 1)], rc);
      rc = fma(v2.y, xn[w + (((2 * q + 1) >> 2) & 1)][vv + (((2 * q + 1) >> 1) & 1)][u + ((2 * q + 1) & 1)], rc);
    }
    row = rc;
  }
  const double t = fma(ks[cc], row, acc);
  acc = act ? t : acc;
}

// Matrix-free A-bar x, node-block form (contexts whose meshes are all small
// enough: see op_use_boxes).  A workgroup takes a block of SEG_ALIGN consecutive
// nodes of one problem (its problem read from op_prob, no search) and first
// stages in LDS, with independent coalesced loads:
//  * x on the three node ranges that hold the blocks' neighbours in the
//    planes K-1, K, K+1: [l0 - N1 - 1, l1 + N1 + 1] + dz (N+1)^2;
//  * cell info and kappa h of the cells around the block's nodes, on two
//    ranges of the cell anchor a(l) = (I-1) + N (J-1) + N^2 (K-1) of a node:
//    [amin, amin + op_lc) + w N^2 for the layers w = 0, 1.  Along l the
//    anchor grows by one per node, stays at a row change and drops by N at
//    a plane change, so it spans at most 255 + N (256 / (N+1)^2 + 1) <=
//    511 + N over a block; amin is the smaller of a(l0) and the anchors of
//    the plane starts inside the block.
// Then each thread sums over the (up to 8) active cells around its node
// kappa_e h (row a of the cell matrix) . x_e from LDS, in the same order as
// the load's node gather; a cut cell's row comes from its full row-major
// copy Kf (one 64-byte segment per row).  DOF nodes are the interior nodes next to an
// active cell; every other node of the block gets 0.  Staged entries outside
// the problem, and cells whose coordinates leave the grid, are never used.
__global__ __launch_bounds__(SEG_ALIGN) void apply_A_lin_kernel(BatchDev bd, int32_t n_items,
                                                            const int32_t* __restrict__ cellinfo,
                                                            const double* __restrict__ kappa,
                                                            const double* __restrict__ Kf,
                                                            const double* __restrict__ x,
                                                            double* __restrict__ y, double* __restrict__ dpart) {
  extern __shared__ double op_lds[];
  __shared__ double sh[SEG_ALIGN / 64];
  const int32_t item = xcd_item((int32_t)blockIdx.x, n_items);
  const int p = bd.op_prob[item];
  if (bd.active && !bd.active[p]) return;
  const ProbDev pr = bd.prob[p];
  // local node and cell numbers fit 32 bits: N <= 1024 (setup checks it)
  const int N = pr.N, N1 = N + 1, LX = bd.op_lx, LC = bd.op_lc;
  const int plane1 = N1 * N1, nodes = plane1 * N1, ncells = N * N * N;
  const int l0 = (int)((int64_t)item * SEG_ALIGN - pr.node_off);       // first local node of the block
  const int l1 = min(l0 + SEG_ALIGN, nodes) - 1;                         // last node of the problem in it
  double* xs = op_lds;                                                   // [3][LX]
  double* ks = xs + 3 * LX;                                              // [2][LC] kappa h
  int32_t* cs = reinterpret_cast<int32_t*>(ks + 2 * LC);                 // [2][LC] cell info
  const double* xp = x + pr.node_off;
  const int32_t* cip = cellinfo + pr.cell_off;
  const double* kp = kappa + pr.cell_off;
  const int xb = l0 - N1 - 1;                                            // node of xs[1][0]
  auto anchor = [&](int l) {
    const int K = l / plane1, r = l - K * plane1;
    const int J = r / N1, I = r - J * N1;
    return (I - 1) + N * ((J - 1) + N * (K - 1));
  };
  int cb = l0 < nodes ? anchor(l0) : 0;                                  // cell of cs[0][0]
  for (int ps = (l0 / plane1 + 1) * plane1; ps <= l1; ps += plane1) cb = min(cb, anchor(ps));
  if (l0 < nodes) {
    // every load of a pass is issued before the first LDS store, so that a
    // thread waits for memory once per pass (one pass for N <= 120)
    constexpr int SV = 8;
    for (int base = 0; base < 3 * LX; base += SV * SEG_ALIGN) {
      double v[SV];
#pragma unroll
      for (int q = 0; q < SV; ++q) {
        const int t = base + q * SEG_ALIGN + (int)threadIdx.x;
        const int dz = t / LX;
        const int g = xb + (t - dz * LX) + (dz - 1) * plane1;
        v[q] = (t < 3 * LX && g >= 0 && g < nodes) ? xp[g] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < SV; ++q) {
        const int t = base + q * SEG_ALIGN + (int)threadIdx.x;
        if (t < 3 * LX) xs[t] = v[q];
      }
    }
    for (int base = 0; base < 2 * LC; base += SV * SEG_ALIGN) {
      int32_t ci[SV];
      double kv[SV];
#pragma unroll
      for (int q = 0; q < SV; ++q) {
        const int t = base + q * SEG_ALIGN + (int)threadIdx.x;
        const int w = t / LC;
        const int c = cb + (t - w * LC) + w * N * N;
        const bool ok = t < 2 * LC && c >= 0 && c < ncells;
        ci[q] = ok ? cip[c] : CELL_INACTIVE;
        kv[q] = ok ? kp[c] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < SV; ++q) {
        const int t = base + q * SEG_ALIGN + (int)threadIdx.x;
        if (t < 2 * LC) {
          cs[t] = ci[q];
          ks[t] = kv[q] * pr.h;
        }
      }
    }
  }
  __syncthreads();
  const int l = l0 + (int)threadIdx.x;
  double v = 0.0, xv0 = 0.0;
  if (l < nodes) {
    const int K = l / plane1, rr = l - K * plane1;
    const int J = rr / N1, I = rr - J * N1;
    const int xo = l - xb;                              // offset of the node itself in each x range
    const int co = anchor(l) - cb;                      // offset of its anchor cell in each cell range
    // the node's 27 neighbours (in-range LDS reads also where a neighbour
    // leaves the grid: those values only meet cells that are skipped)
    double xn[3][3][3];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) xn[dz][dy][dx] = xs[dz * LX + xo + (dx - 1) + N1 * (dy - 1)];
    xv0 = xn[1][1][1];
    // The 8 cells around the node, in the load's order (op_cell_lin<C> below,
    // one instantiation per cell so that every index is a constant)
    double acc = 0.0;
    bool touched = false;
    op_cell_lin<0>(I, J, K, N, LC, co, cs, ks, Kf, xn, acc, touched);
    op_cell_lin<1>(I, J, K, N, LC, co, cs, ks, Kf, xn, acc, touched);
    op_cell_lin<2>(I, J, K, N, LC, co, cs, ks, Kf, xn, acc, touched);
    op_cell_lin<3>(I, J, K, N, LC, co, cs, ks, Kf, xn, acc, touched);
    op_cell_lin<4>(I, J, K, N, LC, co, cs, ks, Kf, xn, acc, touched);
    op_cell_lin<5>(I, J, K, N, LC, co, cs, ks, Kf, xn, acc, touched);
    op_cell_lin<6>(I, J, K, N, LC, co, cs, ks, Kf, xn, acc, touched);
    op_cell_lin<7>(I, J, K, N, LC, co, cs, ks, Kf, xn, acc, touched);
    const bool interior = I >= 1 && I < N && J >= 1 && J < N && K >= 1 && K < N;
    v = (interior && touched) ? acc : 0.0;
  }
  // every node of the block, the alignment padding after the problem included
  y[(int64_t)item * SEG_ALIGN + threadIdx.x] = v;
  if (dpart) {
    const double t = wg_sum_all(xv0 * v, sh);
    if (threadIdx.x == 0) dpart[item] = t;
  }
}

// Cell C = u + 2 vv + 4 w around a node of the operator kernel, without
// branches except around a cut cell's row load.  cs / ks: the staged cell
// codes and kappa h of the two cell layers below (w = 0) and above (w = 1)
// the node's plane, at c0 + w cstride + vv CX + u (cells outside the grid
// are staged as inactive); an inactive cell adds nothing.
template <int C>
__device__ __forceinline__ void op_cell(const int32_t* cs, const double* ks, int c0, int cstride, int CX,
                                        const double* __restrict__ Kf, const double (&xn)[3][3][3], double& acc,
                                        bool& touched) {
  constexpr int u = C & 1, vv = (C >> 1) & 1, w = C >> 2;
  constexpr int a = 7 - C;                               // the node's corner in the cell
  const int cc = c0 + w * cstride + vv * CX + u;
  const int32_t info = cs[cc];
  const bool act = info != CELL_INACTIVE;
  touched = touched || act;
  // row a of the cell matrix times x: the reference row (constant
  // operands), replaced for a cut cell by its row from the full row-major
  // copy (64 contiguous bytes)
  double row = 0.0;
#pragma unroll
  for (int b = 0; b < 8; ++b)
    row = fma(c_Kref[a * 8 + b], xn[w + ((b >> 2) & 1)][vv + ((b >> 1) & 1)][u + (b & 1)], row);
  if (info >= 0) {
    const double2* R = reinterpret_cast<const double2*>(Kf + (int64_t)info * 64 + a * 8);
    double rc = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 v2 = R[q];
      rc = fma(v2.x, xn[w + (((2 * q) >> 2) & 1)][vv + (((2 * q) >> 1) & 1)][u + ((2 * q) & 1)], rc);
      rc = fma(v2.y, xn[w + (((2 * q + 1) >> 2) & 1)][vv + (((2 * q + 1) >> 1) & 1)][u + ((2 * q + 1) & 1)], rc);
    }
    row = rc;
  }
  const double t = fma(ks[cc], row, acc);
  acc = act ? t : acc;
}

// Matrix-free A-bar x, node-box form (contexts with large meshes).  A
// workgroup takes one node box of one problem: nx
// <= SW nodes along x, ny <= TY along y (one thread per (x, y) column) and
// nz <= ZC planes, which it marches through.  It keeps in LDS, as rings,
// three planes of x over the box's columns and their one-node halo
// ((nx + 2)(ny + 2) values each) and two layers of cell codes and kappa h
// over the (nx + 1)(ny + 1) cells around them; at each plane the loads of
// the next plane and cell layer are issued before the arithmetic, so their
// latency overlaps it.  Each thread sums over the (up to 8) active cells
// around its node kappa_e h (row a of the cell matrix) . x_e, in the same
// order as the load's node gather.  DOF nodes are the interior nodes next
// to an active cell; every other node gets 0, and the first item of a
// problem also clears the alignment padding after its nodes.
__global__ __launch_bounds__(SEG_ALIGN) void apply_A_kernel(BatchDev bd, int32_t n_items,
                                                            const int32_t* __restrict__ cellinfo,
                                                            const double* __restrict__ kappa,
                                                            const double* __restrict__ Kf,
                                                            const double* __restrict__ x,
                                                            double* __restrict__ y, double* __restrict__ dpart) {
  extern __shared__ double op_lds[];
  __shared__ double sh[SEG_ALIGN / 64];
  const int32_t item = xcd_item((int32_t)blockIdx.x, n_items);
  const int p = bd.op_prob[item];
  if (bd.active && !bd.active[p]) return;
  const ProbDev pr = bd.prob[p];
  const int32_t* gm = bd.op_geom + 8 * p;
  const int SW = gm[1], TY = gm[2], ngy = gm[3], ZC = gm[4], nzc = gm[5];
  // local node and cell numbers fit 32 bits: N <= 1024 (setup checks it)
  const int N = pr.N, N1 = N + 1;
  const int li = item - bd.op_off[p];
  const int zc = li % nzc, rest = li / nzc, gy = rest % ngy, seg = rest / ngy;
  const int x0 = seg * SW, nx = min(SW, N1 - x0);
  const int y0 = gy * TY, ny = min(TY, N1 - y0);
  const int z0 = zc * ZC, nz = min(ZC, N1 - z0);
  const int PX = nx + 2, XPL = PX * (ny + 2);            // x tile plane with its halo
  const int CX = nx + 1, CPL = CX * (ny + 1);            // cell tile layer
  const int XS = bd.op_xp, CS = bd.op_cp;                // ring slot strides
  double* xs = op_lds;                                   // [3][XS]
  double* ks = xs + 3 * XS;                              // [2][CS] kappa h
  int32_t* cs = reinterpret_cast<int32_t*>(ks + 2 * CS); // [2][CS] cell code
  const double* xp = x + pr.node_off;
  const int32_t* cip = cellinfo + pr.cell_off;
  const double* kp = kappa + pr.cell_off;
  const int t = threadIdx.x;
  const double h = pr.h;
  // staging of node plane K (x over the tile and halo) and of cell layer
  // Kc (codes and kappa h), through registers
  constexpr int RX = OP_XP_MAX / SEG_ALIGN, RC = OP_CP_MAX / SEG_ALIGN;
  double xr[RX], kr[RC];
  int32_t cr[RC];
  auto load_plane = [&](int K) {
#pragma unroll
    for (int q = 0; q < RX; ++q) {
      const int idx = t + q * SEG_ALIGN;
      const int ix = idx % PX, iy = idx / PX;
      const int gx = x0 - 1 + ix, gyy = y0 - 1 + iy;
      const bool ok = idx < XPL && (unsigned)gx < (unsigned)N1 && (unsigned)gyy < (unsigned)N1 &&
                      (unsigned)K < (unsigned)N1;
      xr[q] = ok ? xp[gx + N1 * (gyy + N1 * K)] : 0.0;
    }
  };
  auto store_plane = [&](int slot) {
#pragma unroll
    for (int q = 0; q < RX; ++q) {
      const int idx = t + q * SEG_ALIGN;
      if (idx < XPL) xs[slot * XS + idx] = xr[q];
    }
  };
  auto load_layer = [&](int Kc) {
#pragma unroll
    for (int q = 0; q < RC; ++q) {
      const int idx = t + q * SEG_ALIGN;
      const int ix = idx % CX, iy = idx / CX;
      const int gx = x0 - 1 + ix, gyy = y0 - 1 + iy;
      const bool ok = idx < CPL && (unsigned)gx < (unsigned)N && (unsigned)gyy < (unsigned)N &&
                      (unsigned)Kc < (unsigned)N;
      const int c = ok ? gx + N * (gyy + N * Kc) : 0;
      cr[q] = ok ? cip[c] : CELL_INACTIVE;
      kr[q] = ok ? kp[c] : 0.0;
    }
  };
  auto store_layer = [&](int slot) {
#pragma unroll
    for (int q = 0; q < RC; ++q) {
      const int idx = t + q * SEG_ALIGN;
      if (idx < CPL) {
        cs[slot * CS + idx] = cr[q];
        ks[slot * CS + idx] = kr[q] * h;
      }
    }
  };
  // planes z0 - 1 and z0 (slots 0, 1), cell layer z0 - 1 (slot 0); then the
  // loads of plane z0 + 1 and layer z0
  load_plane(z0 - 1);
  store_plane(0);
  load_plane(z0);
  store_plane(1);
  load_layer(z0 - 1);
  store_layer(0);
  load_plane(z0 + 1);
  load_layer(z0);
  const bool mine = t < nx * ny;
  const int tx = mine ? t % nx : 0, ty = mine ? t / nx : 0;
  const int I = x0 + tx, J = y0 + ty;
  double dot = 0.0;
  for (int k = 0; k < nz; ++k) {
    const int z = z0 + k;
    // plane z + 1 into slot (k + 2) % 3 (plane z - 2 held it), layer z into
    // slot (k + 1) % 2 (layer z - 2 held it)
    store_plane((k + 2) % 3);
    store_layer((k + 1) % 2);
    __syncthreads();
    if (k + 1 < nz) {
      load_plane(z + 2);
      load_layer(z + 1);
    }
    if (mine) {
      double xn[3][3][3];
#pragma unroll
      for (int dz = 0; dz < 3; ++dz) {
        const double* pl = xs + ((k + dz) % 3) * XS;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) xn[dz][dy][dx] = pl[(ty + dy) * PX + tx + dx];
      }
      // cell layers z - 1 (slot k % 2) and z (slot (k + 1) % 2)
      const int s0 = k & 1;
      const int c0 = s0 * CS + ty * CX + tx;
      const int cstride = s0 ? -CS : CS;
      double acc = 0.0;
      bool touched = false;
      op_cell<0>(cs, ks, c0, cstride, CX, Kf, xn, acc, touched);
      op_cell<1>(cs, ks, c0, cstride, CX, Kf, xn, acc, touched);
      op_cell<2>(cs, ks, c0, cstride, CX, Kf, xn, acc, touched);
      op_cell<3>(cs, ks, c0, cstride, CX, Kf, xn, acc, touched);
      op_cell<4>(cs, ks, c0, cstride, CX, Kf, xn, acc, touched);
      op_cell<5>(cs, ks, c0, cstride, CX, Kf, xn, acc, touched);
      op_cell<6>(cs, ks, c0, cstride, CX, Kf, xn, acc, touched);
      op_cell<7>(cs, ks, c0, cstride, CX, Kf, xn, acc, touched);
      const bool interior = I >= 1 && I < N && J >= 1 && J < N && z >= 1 && z < N;
      const double v = (interior && touched) ? acc : 0.0;
      y[pr.node_off + I + (int64_t)N1 * (J + (int64_t)N1 * z)] = v;
      dot = fma(xn[1][1][1], v, dot);
    }
    __syncthreads();
  }
  if (li == 0) {
    // the alignment padding after the problem's nodes
    const int64_t e0 = pr.node_off + (int64_t)N1 * N1 * N1, e1 = bd.node_off[p + 1];
    for (int64_t i = e0 + t; i < e1; i += SEG_ALIGN) y[i] = 0.0;
  }
  if (dpart) {
    const double tsum = wg_sum_all(dot, sh);
    if (t == 0) dpart[item] = tsum;
  }
}

__global__ __launch_bounds__(256) void load_kernel(BatchDev bd, int64_t nn,
                                                   const int32_t* __restrict__ cellinfo,
                                                   const double* __restrict__ Mc,
                                                   const uint8_t* __restrict__ outmask,
                                                   const double* __restrict__ f,
                                                   const double* const* __restrict__ f_ptrs,
                                                   double* __restrict__ b) {
  const int64_t base = (int64_t)blockIdx.x * SEG_ALIGN;
  const int64_t n = base + threadIdx.x;
  if (n >= nn) return;
  if (outmask && !outmask[n]) {
    b[n] = 0.0;
    return;
  }
  const int p = find_segment(bd.node_off, bd.P, base);
  const ProbDev pr = bd.prob[p];
  const int N1 = pr.N + 1;
  const int64_t l = n - pr.node_off;
  if (l >= (int64_t)N1 * N1 * N1) {
    b[n] = 0.0;
    return;
  }
  const int li = (int)l;
  const int I = li % N1, J = (li / N1) % N1, K = li / (N1 * N1);
  const double* fp = f_ptrs ? f_ptrs[p] : f + pr.node_off;
  const double h3 = pr.h * pr.h * pr.h;
  b[n] = fp ? node_gather<true>(pr.N, I, J, K, cellinfo + pr.cell_off, nullptr, Mc, fp, h3)
            : node_gather<true, true>(pr.N, I, J, K, cellinfo + pr.cell_off, nullptr, Mc, nullptr, h3);
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

__global__ void copy_kernel(int64_t n, const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// x += alpha p, r -= alpha q with alpha = rho / p.q of the node's problem
// (rho = r.z of the latest preconditioned residual, slot 3; p.q from the
// work-item parts of the operator kernel, also stored in slot 1); the block
// parts of the new r.r go to rr_part.  zero1 and zero2 (may be null) are
// cleared on the same nodes (the preconditioner's scratch vectors, so that
// they need no fill of their own).
__global__ __launch_bounds__(256) void cg_update_xr_kernel(BatchDev bd, int64_t nn, double* __restrict__ S,
                                                           const double* __restrict__ pq_part,
                                                           const double* __restrict__ p,
                                                           const double* __restrict__ q, double* __restrict__ x,
                                                           double* __restrict__ r, double* __restrict__ zero1,
                                                           double* __restrict__ zero2, double* __restrict__ rr_part) {
  __shared__ double sh[SEG_ALIGN / 64];
  const int64_t base = (int64_t)blockIdx.x * SEG_ALIGN;
  const int64_t i = base + threadIdx.x;
  if (base >= nn) return;
  const int pb = find_segment(bd.node_off, bd.P, base);
  if (bd.active && !bd.active[pb]) return;
  const double pq = wg_sum_range(pq_part, bd.op_off[pb], bd.op_off[pb + 1], sh);
  if (base == bd.node_off[pb] && threadIdx.x == 0) S[CG_S * pb + 1] = pq;
  const double alpha = S[CG_S * pb + 3] / pq;
  double rn = 0.0;
  if (i < nn) {
    x[i] += alpha * p[i];
    rn = r[i] - alpha * q[i];
    r[i] = rn;
    if (zero1) zero1[i] = 0.0;
    if (zero2) zero2[i] = 0.0;
  }
  const double t = wg_sum_all(rn * rn, sh);
  if (threadIdx.x == 0) rr_part[blockIdx.x] = t;
}

// p = z + beta p with beta = rho_new / rho: rho_new = r.z from the chunk
// parts of the dot kernel (also stored in slot 3), rho in slot 0 (moved
// there by the check of the iteration).
__global__ __launch_bounds__(256) void cg_update_p_kernel(BatchDev bd, int64_t nn, double* __restrict__ S,
                                                          const int32_t* __restrict__ chunk_ptr,
                                                          const double* __restrict__ rz_part,
                                                          const double* __restrict__ z, double* __restrict__ p) {
  __shared__ double sh[SEG_ALIGN / 64];
  const int64_t base = (int64_t)blockIdx.x * SEG_ALIGN;
  const int64_t i = base + threadIdx.x;
  if (base >= nn) return;
  const int pb = find_segment(bd.node_off, bd.P, base);
  if (bd.active && !bd.active[pb]) return;
  const double rz = wg_sum_range(rz_part, chunk_ptr[pb], chunk_ptr[pb + 1], sh);
  if (base == bd.node_off[pb] && threadIdx.x == 0) S[CG_S * pb + 3] = rz;
  const double beta = rz / S[CG_S * pb + 0];
  if (i < nn) p[i] = z[i] + beta * p[i];
}

__global__ void set_params_kernel(double* params, double rtol, int32_t max_iter) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    params[0] = rtol;
    params[1] = (double)max_iter;
  }
}

// Number of running problems, written by thread 0 (one block of 256) to
// n_active and, if given, to host memory.
__device__ inline void count_active(int P, const int32_t* active, int32_t* n_active, int32_t* host = nullptr) {
  __shared__ int32_t cnt[256];
  int32_t c = 0;
  for (int p = threadIdx.x; p < P; p += 256) c += active[p] ? 1 : 0;
  cnt[threadIdx.x] = c;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) cnt[threadIdx.x] += cnt[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *n_active = cnt[0];
    if (host) *host = cnt[0];
  }
}

// Start of PCG: a zero right-hand side is converged at iteration 0; with
// max_iter = 0 the problem stops at once without convergence.
__global__ __launch_bounds__(256) void cg_init_kernel(int P, const double* __restrict__ params,
                                                      double* __restrict__ S, int32_t* __restrict__ active,
                                                      int32_t* __restrict__ it, int32_t* __restrict__ status,
                                                      double* __restrict__ relres, int32_t* __restrict__ n_active) {
  const int32_t max_iter = (int32_t)params[1];
  for (int p = threadIdx.x; p < P; p += 256) {
    const double bb = S[CG_S * p + 4];
    it[p] = 0;
    if (bb == 0.0) {
      active[p] = 0;
      status[p] = 1;
      relres[p] = 0.0;
    } else if (max_iter <= 0) {
      active[p] = 0;
      status[p] = 2;
      relres[p] = 1.0;
    } else {
      active[p] = 1;
      status[p] = 0;
      relres[p] = 1.0;
    }
  }
  __syncthreads();
  count_active(P, active, n_active);
}

// After the x, r update of an iteration: count it, test |r| < rtol |b|, a
// non-finite residual, and the iteration limit (one workgroup of 256).
// r.r of a running problem is the sum of its block parts (one wave per
// problem) and goes to slot 2.  The rho of the iteration (slot 3, read by
// the x, r update) moves to slot 0, where the p update finds it after slot
// 3 receives the new r.z.  The count of running problems also goes to
// host memory (nact_host, may be null).
__global__ __launch_bounds__(256) void cg_check_kernel(int P, const int64_t* __restrict__ node_off,
                                                       const double* __restrict__ rr_part,
                                                       const double* __restrict__ params, double* __restrict__ S,
                                                       int32_t* __restrict__ active, int32_t* __restrict__ it,
                                                       int32_t* __restrict__ status, double* __restrict__ relres,
                                                       int32_t* __restrict__ n_active, int32_t* nact_host,
                                                       double* __restrict__ hist, int32_t hcap) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int p = wv; p < P; p += 4) {
    if (!active[p]) continue;
    double acc = 0.0;
    const int64_t b1 = (node_off[p + 1] + SEG_ALIGN - 1) / SEG_ALIGN;
    for (int64_t b = node_off[p] / SEG_ALIGN + lane; b < b1; b += 64) acc += rr_part[b];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) S[CG_S * p + 2] = acc;
  }
  __syncthreads();
  const double rtol = params[0];
  const int32_t max_iter = (int32_t)params[1];
  for (int p = threadIdx.x; p < P; p += 256) {
    if (!active[p]) continue;
    const int32_t k = it[p] + 1;
    if (hist && k <= hcap) {
      // alpha of this iteration (the x, r update's own quotient) and the
      // beta that formed its search direction (none for the first)
      double* hrow = hist + ((int64_t)p * hcap + (k - 1)) * 3;
      hrow[0] = S[CG_S * p + 3] / S[CG_S * p + 1];
      hrow[1] = k >= 2 ? S[CG_S * p + 3] / S[CG_S * p + 0] : 0.0;
      hrow[2] = sqrt(S[CG_S * p + 2]) / sqrt(S[CG_S * p + 4]);
    }
    S[CG_S * p + 0] = S[CG_S * p + 3];
    it[p] = k;
    const double rr = S[CG_S * p + 2];
    if (!isfinite(rr)) {
      active[p] = 0;
      status[p] = 3;
      continue;
    }
    const double rel = sqrt(rr) / sqrt(S[CG_S * p + 4]);
    relres[p] = rel;
    if (rel < rtol) {
      active[p] = 0;
      status[p] = 1;
    } else if (k >= max_iter) {
      active[p] = 0;
      status[p] = 2;
    }
  }
  __syncthreads();
  count_active(P, active, n_active, nact_host);
}

__global__ void gather_dofs_batch_kernel(int P, int64_t n, const int64_t* __restrict__ dof_off,
                                         const int64_t* __restrict__ dof_node, const double* __restrict__ grid,
                                         double* const* __restrict__ u_ptrs) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= n) return;
  const int p = find_segment(dof_off, P, d);
  u_ptrs[p][d - dof_off[p]] = grid[dof_node[d]];
}

__global__ void convert_kernel(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

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

// One block per DOT_CHUNK-sized chunk of a problem's node segment.
__global__ __launch_bounds__(DOT_THREADS) void dot_chunk_kernel(BatchDev bd, const int32_t* __restrict__ chunk_ptr,
                                                                const double* __restrict__ x,
                                                                const double* __restrict__ y,
                                                                double* __restrict__ partial) {
  __shared__ double sh[DOT_THREADS / 64];
  const int p = find_segment(chunk_ptr, bd.P, blockIdx.x);
  if (bd.active && !bd.active[p]) return;
  const ProbDev pr = bd.prob[p];
  const int64_t N1 = pr.N + 1;
  const int64_t seg_end = pr.node_off + N1 * N1 * N1;
  const int64_t start = pr.node_off + (int64_t)(blockIdx.x - chunk_ptr[p]) * DOT_CHUNK;
  const int64_t end = min(start + DOT_CHUNK, seg_end);
  double acc = 0.0;
  for (int64_t i = start + threadIdx.x; i < end; i += DOT_THREADS) acc += x[i] * y[i];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// One wave per problem sums its chunk partials in a fixed order.
__global__ __launch_bounds__(256) void dot_final_kernel(BatchDev bd, const int32_t* __restrict__ chunk_ptr,
                                                        const double* __restrict__ partial,
                                                        double* __restrict__ out, int stride) {
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (p >= bd.P) return;
  if (bd.active && !bd.active[p]) return;
  double acc = 0.0;
  for (int c = chunk_ptr[p] + lane; c < chunk_ptr[p + 1]; c += 64) acc += partial[c];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) out[(int64_t)p * stride] = acc;
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void set_reference_matrices(const double* Kref, const double* Mref) {
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_Kref), Kref, 64 * sizeof(double));
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_Mref), Mref, 64 * sizeof(double));
}

int prepare_apply_A() {
  // node blocks: 128 KB covers N up to 1024 (116 KB); node boxes: the rings
  // need at most 3 OP_XP_MAX + 2 OP_CP_MAX doubles and 2 OP_CP_MAX codes
  // (42 KB); the kernels' static LDS comes on top
  static const hipError_t e1 = hipFuncSetAttribute((const void*)apply_A_lin_kernel,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
  static const hipError_t e2 = hipFuncSetAttribute((const void*)apply_A_kernel,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
  return e1 == hipSuccess && e2 == hipSuccess ? 0 : -1;
}

OpGeom op_geometry(int N1, int64_t nodes_per_item) {
  OpGeom best{1, N1, 1, N1, 1, N1};
  double best_ratio = 1e300;
  for (int nseg = 1; nseg <= 64; ++nseg) {
    const int SW = (N1 + nseg - 1) / nseg;
    if (SW > SEG_ALIGN) continue;
    const int tymax = SEG_ALIGN / SW;
    const int ngy = (N1 + tymax - 1) / tymax;
    const int TY = (N1 + ngy - 1) / ngy;
    // at least half a workgroup of nodes per plane, when the mesh allows it
    if (2 * SW * TY < SEG_ALIGN && N1 * std::min(N1, tymax) >= SEG_ALIGN / 2) continue;
    const double ratio = (double)(SW + 2) * (TY + 2) / ((double)SW * TY);
    if (ratio < best_ratio - 1e-12) {
      best_ratio = ratio;
      best = OpGeom{(N1 + SW - 1) / SW, SW, TY, ngy, 1, N1};
    }
    if (SW <= 8) break;
  }
  const int64_t per_plane = (int64_t)best.SW * best.TY;
  const int zc = (int)std::max<int64_t>(1, std::min<int64_t>(32, (nodes_per_item + per_plane / 2) / per_plane));
  best.nzc = (N1 + zc - 1) / zc;
  best.ZC = (N1 + best.nzc - 1) / best.nzc;
  return best;
}

__global__ void expand_rows_kernel(int64_t n, const double* __restrict__ Kc, double* __restrict__ Kf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * 64) return;
  const int64_t e = i >> 6;
  const int a = (int)((i >> 3) & 7), b = (int)(i & 7);
  Kf[i] = Kc[e * PACK36 + pack_index(a, b)];
}

void launch_expand_rows(hipStream_t st, int64_t n_cut, const double* Kc, double* Kf) {
  if (n_cut <= 0) return;
  hipLaunchKernelGGL(expand_rows_kernel, dim3(nblocks(n_cut * 64, 256)), dim3(256), 0, st, n_cut, Kc, Kf);
}

void launch_apply_A(hipStream_t st, const BatchDev& b, int64_t nn, int32_t n_items, const int32_t* cellinfo,
                    const double* kappa, const double* Kf, const uint8_t* dofmask, const double* x, double* y,
                    double* dpart) {
  (void)dofmask;
  if (nn <= 0 || n_items <= 0) return;
  if (b.op_box) {
    const size_t sh = (size_t)(3 * b.op_xp + 2 * b.op_cp) * sizeof(double) + (size_t)2 * b.op_cp * sizeof(int32_t);
    hipLaunchKernelGGL(apply_A_kernel, dim3((unsigned)n_items), dim3(SEG_ALIGN), sh, st, b, n_items, cellinfo, kappa,
                       Kf, x, y, dpart);
  } else {
    const size_t sh = (size_t)(3 * b.op_lx + 2 * b.op_lc) * sizeof(double) + (size_t)2 * b.op_lc * sizeof(int32_t);
    hipLaunchKernelGGL(apply_A_lin_kernel, dim3((unsigned)n_items), dim3(SEG_ALIGN), sh, st, b, n_items, cellinfo,
                       kappa, Kf, x, y, dpart);
  }
}

void launch_load(hipStream_t st, const BatchDev& b, int64_t nn, const int32_t* cellinfo,
                 const double* Mc, const uint8_t* outmask, const double* f,
                 const double* const* f_ptrs, double* out) {
  if (nn <= 0) return;
  hipLaunchKernelGGL(load_kernel, dim3(nblocks(nn, SEG_ALIGN)), dim3(SEG_ALIGN), 0, st, b, nn, cellinfo, Mc,
                     outmask, f, f_ptrs, out);
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

void launch_copy(hipStream_t st, int64_t n, const double* src, double* dst) {
  if (n <= 0) return;
  hipLaunchKernelGGL(copy_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, n, src, dst);
}

void launch_cg_update_xr(hipStream_t st, const BatchDev& b, int64_t nn, double* S, const double* pq_part,
                         const double* p, const double* q, double* x, double* r, double* zero1, double* zero2,
                         double* rr_part) {
  hipLaunchKernelGGL(cg_update_xr_kernel, dim3(nblocks(nn, SEG_ALIGN)), dim3(SEG_ALIGN), 0, st, b, nn, S, pq_part,
                     p, q, x, r, zero1, zero2, rr_part);
}

void launch_cg_update_p(hipStream_t st, const BatchDev& b, int64_t nn, double* S, const int32_t* chunk_ptr,
                        const double* rz_part, const double* z, double* p) {
  hipLaunchKernelGGL(cg_update_p_kernel, dim3(nblocks(nn, SEG_ALIGN)), dim3(SEG_ALIGN), 0, st, b, nn, S, chunk_ptr,
                     rz_part, z, p);
}

void launch_set_params(hipStream_t st, double* params, double rtol, int32_t max_iter) {
  hipLaunchKernelGGL(set_params_kernel, dim3(1), dim3(64), 0, st, params, rtol, max_iter);
}

void launch_cg_init(hipStream_t st, int P, const double* params, double* S, int32_t* active, int32_t* it,
                    int32_t* status, double* relres, int32_t* n_active) {
  hipLaunchKernelGGL(cg_init_kernel, dim3(1), dim3(256), 0, st, P, params, S, active, it, status, relres,
                     n_active);
}

void launch_cg_check(hipStream_t st, int P, const int64_t* node_off, const double* rr_part, const double* params,
                     double* S, int32_t* active, int32_t* it, int32_t* status, double* relres, int32_t* n_active,
                     int32_t* nact_host, double* hist, int32_t hcap) {
  hipLaunchKernelGGL(cg_check_kernel, dim3(1), dim3(256), 0, st, P, node_off, rr_part, params, S, active, it,
                     status, relres, n_active, nact_host, hist, hcap);
}

void launch_gather_dofs_batch(hipStream_t st, int P, int64_t n_dof_total, const int64_t* dof_off,
                              const int64_t* dof_node, const double* grid, double* const* u_ptrs) {
  if (n_dof_total <= 0) return;
  hipLaunchKernelGGL(gather_dofs_batch_kernel, dim3(nblocks(n_dof_total, 256)), dim3(256), 0, st, P,
                     n_dof_total, dof_off, dof_node, grid, u_ptrs);
}

void convert_to_float(hipStream_t st, int64_t n, const double* a, float* b) {
  if (n <= 0) return;
  hipLaunchKernelGGL(convert_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, n, a, b);
}

void launch_dot_chunks(hipStream_t st, const BatchDev& b, const int32_t* chunk_ptr, int32_t n_chunks, const double* x,
                       const double* y, double* partial) {
  if (n_chunks <= 0) return;
  hipLaunchKernelGGL(dot_chunk_kernel, dim3(n_chunks), dim3(DOT_THREADS), 0, st, b, chunk_ptr, x, y, partial);
}

void launch_dot(hipStream_t st, const BatchDev& b, const int32_t* chunk_ptr, int32_t n_chunks,
                const double* x, const double* y, double* partial, double* out, int stride) {
  if (n_chunks <= 0) return;
  hipLaunchKernelGGL(dot_chunk_kernel, dim3(n_chunks), dim3(DOT_THREADS), 0, st, b, chunk_ptr, x, y, partial);
  hipLaunchKernelGGL(dot_final_kernel, dim3(nblocks(b.P, 4)), dim3(256), 0, st, b, chunk_ptr, partial, out,
                     stride);
}

}  // namespace cutbddc
