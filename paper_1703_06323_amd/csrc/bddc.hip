// BDDC kernels (paper Sect. 3.1-3.4 and 4.3): sub-assembly of the local
// Neumann matrices, weights, coarse basis, coarse matrix assembly and the
// pieces of the preconditioner apply M r.
//
// Local layout per subdomain omega (padded to NIp + NGp rows): interior DOFs
// first (rows [0, nI)), interface DOFs at rows [NIp, NIp + nG); padding rows
// carry the identity.  The constrained Neumann problem is posed on the
// augmented matrix K = A_omega + C^T R C with R = diag(rho_lambda),
// rho_lambda = sum of A_omega's diagonal over lambda: on the constraint
// subspace C v = 0 it equals A_omega, so its constrained inverse is that of
// A_omega.  K is Jacobi scaled before the Cholesky factorisation.
//
// With L the Cholesky factor of K ([I; G] ordering), L_II factors A_II and
// L_GG the Schur complement K_S = S_A + C^T R C of K on the interface
// (S_A the Schur complement of A_omega).  The apply uses
//   P   = A_II^{-1}                          (Dirichlet solves, E and I0 A0^-1 I0^T)
//   G   = K_S^{-1} C^T,  S_c = C G,  Phi = G S_c^{-1}   (coarse basis on the interface)
//   Kt  = K_S^{-1} - Phi G^T                  (constrained Neumann solve on the interface)
//   A_c^omega = Phi^T S_A Phi = S_c^{-1} - R  (local coarse matrix)
#include "bddc.h"
#include "dense.h"

#include <algorithm>
#include <cstdlib>
#include <type_traits>

#pragma clang fp contract(off)

namespace cutbddc {
namespace {

__constant__ double c_Kref_b[64];

__device__ inline void object_members(const SubDev& sd, int w, int* ptr, int* mem);
__device__ inline void object_members_get(const SubDev& sd, int w, int* ptr, int* mem);

// The s^3 cells of block (Bx, By, Bz) into LDS: cell info and kappa h (0 on
// inactive cells), indexed cx + s (cy + s cz).  Caller synchronises.
__device__ inline void load_block_cells(const GridDev& g, const ProbDev& pr, int Bx, int By, int Bz, int* cinfo,
                                        double* ckh) {
  const int s = g.s, n = s * s * s;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int cx = e % s, cy = (e / s) % s, cz = e / (s * s);
    const int64_t c = (int64_t)(Bx * s + cx) + (int64_t)pr.N * ((By * s + cy) + (int64_t)pr.N * (Bz * s + cz));
    const int32_t info = g.cellinfo[pr.cell_off + c];
    cinfo[e] = info;
    ckh[e] = info == CELL_INACTIVE ? 0.0 : g.kappa[pr.cell_off + c] * pr.h;
  }
}

template <typename T> struct RowVec;   // 16 bytes of T
template <> struct RowVec<float> {
  typedef float __attribute__((ext_vector_type(4))) type;
};
template <> struct RowVec<double> {
  typedef double __attribute__((ext_vector_type(2))) type;
};

// Kernel 1: per subdomain, the unscaled diagonal of A_omega, rho per coarse
// object, the Jacobi scaling, and the scaled padded matrix
// K = D (A_omega + C^T R C) D (identity on padding rows).  The diagonal and
// rho come first (one thread per row / object); then each wave builds whole
// rows in LDS: 27 lanes each sum one neighbour of the row's node over the
// cells around it (fixed order), lanes over the object's slots add the
// C^T R C term, and the row is written out with coalesced stores.
// Large subdomains (BIG: the padded row buffers and vectors would not fit
// in LDS) keep the diagonal and the scaling in Dscale, where the scaling
// ends up anyway, and build only row_waves rows at a time.
constexpr int ASM_WAVES = 8;   // rows in flight per subdomain (one per wave)
template <typename T, bool BIG>
__global__ __launch_bounds__(64 * ASM_WAVES) void assemble_local_kernel(SubDev sd, GridDev g, T* Kmat,
                                                                       double* diagA_G, double* Dscale,
                                                                       double* __restrict__ st_val,
                                                                       int32_t* __restrict__ st_col,
                                                                       int row_waves) {
  extern __shared__ double smem[];
  const int w = blockIdx.x;
  const int NIp = sd.NIp, NGp = sd.NGp, NCp = sd.NCp, nt = NIp + NGp;
  const int s = g.s, s3 = s * s * s;
  double* diag = BIG ? Dscale + (int64_t)w * nt : smem;   // [nt]
  double* Ds = BIG ? diag : diag + nt;                     // [nt] (in place of diag when BIG)
  double* rho = BIG ? smem : Ds + nt;                      // [NCp]: rho_t / |t|^2
  double* ckh = rho + NCp;          // [s^3]: kappa h per block cell
  int* optr = reinterpret_cast<int*>(ckh + s3);    // [NCp + 1]
  int* omem = optr + NCp + 1;                      // [NGp]
  int* cinfo = omem + NGp;                         // [s^3]
  T* rows = reinterpret_cast<T*>(ckh + s3 + 2 * ((NCp + 1 + NGp + s3 + 3) / 4));   // [row_waves][nt]
  const int nI = sd.nI[w], nG = sd.nG[w], nC = sd.nC[w];
  const ProbDev pr = g.prob[sd.sub_prob[w]];
  const int m = pr.m, N1 = pr.N + 1;
  const int blk = sd.sub_blk[w];
  const int Bx = blk % m, By = (blk / m) % m, Bz = blk / (m * m);
  const int s1 = s + 1;
  const int* loc = sd.bloc + (int64_t)w * s1 * s1 * s1;
  const int* gobj = sd.G_obj + (int64_t)w * NGp;
  T* K = Kmat + (int64_t)w * nt * nt;
  const int tid = threadIdx.x;
  load_block_cells(g, pr, Bx, By, Bz, cinfo, ckh);
  __syncthreads();

  // local block coordinates of the node of row r (false for padding rows)
  auto row_xyz = [&](int r, int& lx, int& ly, int& lz) -> bool {
    int64_t n;
    if (r < NIp) {
      if (r >= nI) return false;
      n = sd.I_idx[(int64_t)w * NIp + r];
    } else {
      if (r - NIp >= nG) return false;
      n = sd.G_idx[(int64_t)w * NGp + (r - NIp)];
    }
    const int l = (int)(n - pr.node_off);
    lx = l % N1 - Bx * s;
    ly = (l / N1) % N1 - By * s;
    lz = l / (N1 * N1) - Bz * s;
    return true;
  };
  // phase 0: diagonal of A_omega
  for (int r = tid; r < nt; r += 64 * ASM_WAVES) {
    int lx, ly, lz;
    double d = 0.0;
    if (row_xyz(r, lx, ly, lz)) {
      for (int u = 0; u < 8; ++u) {
        const int cx = lx - 1 + (u & 1), cy = ly - 1 + ((u >> 1) & 1), cz = lz - 1 + ((u >> 2) & 1);
        if (cx < 0 || cy < 0 || cz < 0 || cx >= s || cy >= s || cz >= s) continue;
        const int lc = cx + s * (cy + s * cz);
        const int32_t info = cinfo[lc];
        if (info == CELL_INACTIVE) continue;
        const int a = (lx - cx) + 2 * (ly - cy) + 4 * (lz - cz);
        const double kaa = info == CELL_UNCUT ? c_Kref_b[a * 9] : g.Kc[(int64_t)info * PACK36 + pack_index(a, a)];
        d += ckh[lc] * kaa;
      }
    }
    diag[r] = d;
    if (r >= NIp) diagA_G[(int64_t)w * NGp + (r - NIp)] = d;
  }
  object_members_get(sd, w, optr, omem);   // ends with a barrier
  // phase 1: rho_t / |t|^2 with rho_t the sum of the diagonal over object t
  for (int t = tid; t < NCp; t += 64 * ASM_WAVES) {
    double sr = 0.0;
    const int b0 = optr[t], b1 = optr[t + 1];
    for (int q = b0; q < b1; ++q) sr += diag[NIp + omem[q]];
    rho[t] = (t < nC && b1 > b0) ? sr / ((double)(b1 - b0) * (double)(b1 - b0)) : 0.0;
  }
  __syncthreads();
  for (int r = tid; r < nt; r += 64 * ASM_WAVES) {
    int lx, ly, lz;
    const bool real = row_xyz(r, lx, ly, lz);
    double dk = diag[r];
    if (r >= NIp && real) {
      const int t = gobj[r - NIp];
      if (t >= 0) dk += rho[t];
    }
    const double dr = real ? 1.0 / sqrt(dk) : 1.0;
    Ds[r] = dr;
    if (!BIG) Dscale[(int64_t)w * nt + r] = dr;
  }
  __syncthreads();
  // phase 2: rows, one wave per row (the first row_waves waves)
  const int lane = tid & 63, wv = tid >> 6;
  T* rb = rows + wv * nt;
  typedef typename RowVec<T>::type V;
  constexpr int VW = 16 / sizeof(T);
  for (int r = wv; wv < row_waves && r < nt; r += row_waves) {
    for (int c = lane * VW; c < nt; c += 64 * VW) *reinterpret_cast<V*>(rb + c) = V{};
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    int lx, ly, lz;
    const int64_t so = ((int64_t)w * nt + r) * STENCIL;
    if (!row_xyz(r, lx, ly, lz)) {
      if (lane == 0) rb[r] = T(1);
      if (st_val && lane < STENCIL) {
        st_val[so + lane] = 0.0;
        st_col[so + lane] = -1;
      }
    } else {
      if (lane < 27) {
        const int dx = lane % 3 - 1, dy = (lane / 3) % 3 - 1, dz = lane / 9 - 1;
        const int bx = lx + dx, by = ly + dy, bz = lz + dz;
        int col = -1;
        if (bx >= 0 && by >= 0 && bz >= 0 && bx <= s && by <= s && bz <= s) col = loc[bx + s1 * (by + s1 * bz)];
        if (col >= 0) {
          double v = 0.0;
          for (int u = 0; u < 8; ++u) {
            const int cx = lx - 1 + (u & 1), cy = ly - 1 + ((u >> 1) & 1), cz = lz - 1 + ((u >> 2) & 1);
            if (cx < 0 || cy < 0 || cz < 0 || cx >= s || cy >= s || cz >= s) continue;
            // the neighbour must be a corner of this cell too
            const int ox = bx - cx, oy = by - cy, oz = bz - cz;
            if (ox < 0 || ox > 1 || oy < 0 || oy > 1 || oz < 0 || oz > 1) continue;
            const int lc = cx + s * (cy + s * cz);
            const int32_t info = cinfo[lc];
            if (info == CELL_INACTIVE) continue;
            const int a = (lx - cx) + 2 * (ly - cy) + 4 * (lz - cz);
            const int bb = ox + 2 * oy + 4 * oz;
            const double kab = info == CELL_UNCUT ? c_Kref_b[a * 8 + bb]
                                                  : g.Kc[(int64_t)info * PACK36 + pack_index(a, bb)];
            v += ckh[lc] * kab;
          }
          rb[col] = (T)(v * Ds[r] * Ds[col]);
          if (st_val) st_val[so + lane] = v;
        } else if (st_val) {
          st_val[so + lane] = 0.0;
        }
        if (st_col) st_col[so + lane] = col;
      }
      if (r >= NIp) {
        const int t = gobj[r - NIp];
        if (t >= 0) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          const double add = rho[t] * Ds[r];
          for (int q = optr[t] + lane; q < optr[t + 1]; q += 64) {
            const int col = NIp + omem[q];
            rb[col] = (T)((double)rb[col] + add * Ds[col]);
          }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // Only the columns up to the end of the row's diagonal block of the
    // blocked Cholesky (blocks of DB rows from 0 to NIp, then from NIp) are
    // stored: the factorisation reads the lower triangle and whole diagonal
    // blocks, never the rest of the upper triangle.
    const int cend = r < NIp ? min(NIp, (r / DB + 1) * DB) : min(nt, NIp + ((r - NIp) / DB + 1) * DB);
    T* Kr = K + (int64_t)r * nt;
    for (int c = lane * VW; c < cend; c += 64 * VW) *reinterpret_cast<V*>(Kr + c) = *reinterpret_cast<const V*>(rb + c);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// Kernel 2: weights per interface DOF, summed over its subdomains in
// ascending order: stiffness A^w_xx / sum A^w'_xx, or 1/|S(x)|.
__global__ void weights_kernel(int64_t n_iface, const int64_t* __restrict__ if_ptr,
                               const int32_t* __restrict__ if_sub, const int32_t* __restrict__ if_slot,
                               int NGp, const double* __restrict__ diagA_G, int stiffness,
                               double* __restrict__ Dw) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_iface) return;
  const int64_t b = if_ptr[q], e = if_ptr[q + 1];
  double tot = 0.0;
  for (int64_t z = b; z < e; ++z) tot += diagA_G[(int64_t)if_sub[z] * NGp + if_slot[z]];
  for (int64_t z = b; z < e; ++z) {
    const int64_t k = (int64_t)if_sub[z] * NGp + if_slot[z];
    Dw[k] = stiffness ? diagA_G[k] / tot : 1.0 / (double)(e - b);
  }
}

// Kernel 3b: Y[r][t] = sum_c A_omega[r][c] X[c][t] for the local rows r in
// [r0, r0 + nrows) (unscaled FP64 local Neumann matrix; X, Y are nt x NCp
// per subdomain), from the stencil rows stored by the assembly.  One block
// per (LA_ROWS-row chunk, subdomain): the chunk's stencil rows go to LDS,
// then all threads stream X along its rows (entries summed in slot order).
constexpr int LA_ROWS = 64;
template <bool SKIP>
__global__ __launch_bounds__(256) void local_apply_kernel(SubDev sd, const double* __restrict__ st_val,
                                                          const int32_t* __restrict__ st_col,
                                                          const double* __restrict__ X, double* __restrict__ Y,
                                                          int r0, int nrows, int xfrom) {
  __shared__ double sval[LA_ROWS * STENCIL];
  __shared__ int scol[LA_ROWS * STENCIL];
  const int w = blockIdx.y;
  const int NIp = sd.NIp, NGp = sd.NGp, NCp = sd.NCp, nt = NIp + NGp;
  const int rb = r0 + blockIdx.x * LA_ROWS;
  const int tid = threadIdx.x;
  const int R = min(LA_ROWS, r0 + nrows - rb);
  const int64_t so = ((int64_t)w * nt + rb) * STENCIL;
  for (int e = tid; e < R * STENCIL; e += 256) {
    sval[e] = st_val[so + e];
    scol[e] = st_col[so + e];
  }
  __syncthreads();
  const double* x = X + (int64_t)w * nt * NCp;
  double* y = Y + (int64_t)w * nt * NCp;
  const int nI = sd.nI[w], nG = sd.nG[w], nC = sd.nC[w];
  for (int e = tid; e < R * NCp; e += 256) {
    const int rr = e / NCp, t = e - rr * NCp;
    // padding rows (empty stencils) and padding columns of X (zero) give 0
    const int r = rb + rr;
    if (t >= nC || r >= NIp + nG || (r >= nI && r < NIp)) {
      y[(int64_t)r * NCp + t] = 0.0;
      continue;
    }
    // An empty slot holds the value 0 (and column -1): its load goes to
    // column 0 and adds 0, so all 27 loads issue together.  Columns below
    // xfrom hold zeros in X: those lanes skip the load and add 0 as well.
    double xv[STENCIL];
#pragma unroll
    for (int k = 0; k < STENCIL; ++k) {
      const int c = max(scol[rr * STENCIL + k], 0);
      xv[k] = (!SKIP || c >= xfrom) ? x[(int64_t)c * NCp + t] : 0.0;
    }
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < STENCIL; ++k) acc += sval[rr * STENCIL + k] * xv[k];
    y[(int64_t)(rb + rr) * NCp + t] = acc;
  }
}

// Interface slots of each local object of subdomain w, grouped by object:
// members of object t at mem[ptr[t] .. ptr[t+1]), ascending (eq.
// coarse-dofs: the coarse DOF of object t is the mean over these slots).
__device__ inline void object_members(const SubDev& sd, int w, int* ptr, int* mem) {
  const int NGp = sd.NGp, NCp = sd.NCp;
  const int nG = sd.nG[w], nC = sd.nC[w];
  const int* obj = sd.G_obj + (int64_t)w * NGp;
  for (int t = threadIdx.x; t < NCp; t += blockDim.x) {
    int c = 0;
    if (t < nC)
      for (int j = 0; j < nG; ++j) c += obj[j] == t ? 1 : 0;
    ptr[t + 1] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    ptr[0] = 0;
    for (int t = 0; t < NCp; ++t) ptr[t + 1] += ptr[t];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nC; t += blockDim.x) {
    int q = ptr[t];
    for (int j = 0; j < nG; ++j)
      if (obj[j] == t) mem[q++] = j;
  }
  __syncthreads();
}

// The same lists from sd.optr / sd.omem when they have been built.
__device__ inline void object_members_get(const SubDev& sd, int w, int* ptr, int* mem) {
  if (!sd.optr) {
    object_members(sd, w, ptr, mem);
    return;
  }
  const int NGp = sd.NGp, NCp = sd.NCp;
  for (int t = threadIdx.x; t <= NCp; t += blockDim.x) ptr[t] = sd.optr[(int64_t)w * (NCp + 1) + t];
  for (int j = threadIdx.x; j < NGp; j += blockDim.x) mem[j] = sd.omem[(int64_t)w * NGp + j];
  __syncthreads();
}

// One workgroup per subdomain: its object lists to optr / omem (member
// slots beyond the last object's are -1).
__global__ __launch_bounds__(256) void object_lists_kernel(SubDev sd, int32_t* __restrict__ optr,
                                                           int32_t* __restrict__ omem) {
  extern __shared__ int smem_i[];
  const int w = blockIdx.x;
  const int NGp = sd.NGp, NCp = sd.NCp;
  int* ptr = smem_i;
  int* mem = smem_i + NCp + 1;
  object_members(sd, w, ptr, mem);
  const int used = ptr[NCp];
  for (int t = threadIdx.x; t <= NCp; t += blockDim.x) optr[(int64_t)w * (NCp + 1) + t] = ptr[t];
  for (int j = threadIdx.x; j < NGp; j += blockDim.x) omem[(int64_t)w * NGp + j] = j < used ? mem[j] : -1;
}

// Kernel 3c: Gt = (K_S^{-1} C^T)^T without forming C: since K_S^{-1} is
// symmetric, row t of Gt is the mean of the rows of K_S^{-1} over the slots
// of object t, so every row of K_S^{-1} is read once and coalesced.  One
// block per (CC_COLS-column chunk, subdomain): lane l of wave v owns column
// chunk + l and the objects t = v, v + 4, ...; four partial sums keep four
// row loads in flight per wave.  Gt is NCp x NGp.
constexpr int CC_COLS = 64;
__device__ inline int packed_offset(int r, int c, int vw);
__global__ __launch_bounds__(256) void constraint_cols_kernel(SubDev sd, const double* __restrict__ KS,
                                                              double* __restrict__ Gt) {
  extern __shared__ int smem_i[];
  const int w = blockIdx.y;
  const int NGp = sd.NGp, NCp = sd.NCp;
  int* ptr = smem_i;
  int* mem = smem_i + NCp + 1;
  object_members_get(sd, w, ptr, mem);
  const double* ks = KS + (int64_t)w * NGp * NGp;
  double* gt = Gt + (int64_t)w * NCp * NGp;
  const int i = blockIdx.x * CC_COLS + (threadIdx.x & 63);
  if (i >= NGp) return;
  for (int t = threadIdx.x >> 6; t < NCp; t += 4) {
    const int b = ptr[t], en = ptr[t + 1];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int q = b;
    for (; q + 4 <= en; q += 4) {
      a0 += ks[(int64_t)mem[q] * NGp + i];
      a1 += ks[(int64_t)mem[q + 1] * NGp + i];
      a2 += ks[(int64_t)mem[q + 2] * NGp + i];
      a3 += ks[(int64_t)mem[q + 3] * NGp + i];
    }
    for (; q < en; ++q) a0 += ks[(int64_t)mem[q] * NGp + i];
    gt[(int64_t)t * NGp + i] = en > b ? ((a0 + a1) + (a2 + a3)) / (double)(en - b) : 0.0;
  }
}

// Kernel 3d: S_c = C G: S_c[t][u] is the mean of Gt[u][j] over the slots j
// of object t (NCp x NCp per subdomain).
__global__ __launch_bounds__(256) void constraint_rows_kernel(SubDev sd, const double* __restrict__ Gt,
                                                              double* __restrict__ Sc) {
  extern __shared__ int smem_i[];
  const int w = blockIdx.x;
  const int NGp = sd.NGp, NCp = sd.NCp;
  int* ptr = smem_i;
  int* mem = smem_i + NCp + 1;
  object_members_get(sd, w, ptr, mem);
  const double* gt = Gt + (int64_t)w * NCp * NGp;
  double* sc = Sc + (int64_t)w * NCp * NCp;
  for (int e = threadIdx.x; e < NCp * NCp; e += 256) {
    const int t = e / NCp, u = e - t * NCp;
    const int b = ptr[t], en = ptr[t + 1];
    double acc = 0.0;
    for (int q = b; q < en; ++q) acc += gt[(int64_t)u * NGp + mem[q]];
    sc[e] = en > b ? acc / (double)(en - b) : 0.0;
  }
}

// The same with one row u of Gt per wave, staged in LDS by coalesced loads;
// lane t then averages the staged row over the slots of object t (the same
// terms in the same order as above).  Block (CR_W waves) rows blockIdx.x *
// CR_W + wave; LDS: the member lists, then one row buffer per wave.
__global__ __launch_bounds__(256) void constraint_rows_staged_kernel(SubDev sd, const double* __restrict__ Gt,
                                                                     double* __restrict__ Sc) {
  extern __shared__ int smem_i[];
  const int w = blockIdx.y;
  const int NGp = sd.NGp, NCp = sd.NCp;
  int* ptr = smem_i;
  int* mem = smem_i + NCp + 1;
  double* buf = reinterpret_cast<double*>(smem_i + ((NCp + 1 + NGp + 1) & ~1));
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int u = blockIdx.x * (blockDim.x >> 6) + wave;
  double* row = buf + (int64_t)wave * NGp;
  if (u < NCp) {
    const double* gt = Gt + ((int64_t)w * NCp + u) * NGp;
    for (int j = lane; j < NGp; j += 64) row[j] = gt[j];
  }
  object_members_get(sd, w, ptr, mem);   // ends with a barrier
  if (u >= NCp) return;
  double* sc = Sc + (int64_t)w * NCp * NCp;
  for (int t = lane; t < NCp; t += 64) {
    const int b = ptr[t], en = ptr[t + 1];
    double acc = 0.0;
    for (int q = b; q < en; ++q) acc += row[mem[q]];
    sc[(int64_t)t * NCp + u] = en > b ? acc / (double)(en - b) : 0.0;
  }
}

// Kernel 3e: in-place inverse of the SPD matrices S_c (NCp x NCp, identity
// on padded rows) by Gauss-Jordan elimination in LDS.
__global__ __launch_bounds__(256) void small_spd_inverse_kernel(SubDev sd, double* __restrict__ Sm, int* info) {
  extern __shared__ double S[];
  const int w = blockIdx.x;
  const int NCp = sd.NCp, nC = sd.nC[w];
  double* g = Sm + (int64_t)w * NCp * NCp;
  const int tid = threadIdx.x;
  for (int e = tid; e < NCp * NCp; e += 256) {
    const int t = e / NCp, u = e % NCp;
    S[e] = (t < nC && u < nC) ? g[e] : (t == u ? 1.0 : 0.0);
  }
  __syncthreads();
  __shared__ double piv;
  // the padding rows and columns are an identity block that no step changes
  for (int k = 0; k < nC; ++k) {
    if (tid == 0) {
      const double p = S[k * NCp + k];
      if (!(p > 0.0) && info) atomicMax(info, 1);
      piv = (p > 0.0) ? p : 1.0;
    }
    __syncthreads();
    const double p = piv;
    for (int j = tid; j < NCp; j += 256)
      if (j != k) S[k * NCp + j] /= p;
    __syncthreads();
    for (int e = tid; e < NCp * NCp; e += 256) {
      const int i = e / NCp, j = e % NCp;
      if (i == k || j == k) continue;
      S[e] -= S[i * NCp + k] * S[k * NCp + j];
    }
    __syncthreads();
    for (int i = tid; i < NCp; i += 256)
      if (i != k) S[i * NCp + k] = -S[i * NCp + k] / p;
    __syncthreads();
    if (tid == 0) S[k * NCp + k] = 1.0 / p;
    __syncthreads();
  }
  for (int e = tid; e < NCp * NCp; e += 256) g[e] = S[e];
}

// Kernel 4: row c of problem p's coarse matrix = sum over the subdomains
// touching coarse DOF c (ascending) of the matching row of A_c^w.
// One workgroup per padded row: the row is accumulated in LDS by one wave
// (the entries of one subdomain go to distinct columns; the subdomains
// follow one another in program order, so every entry is summed in
// ascending subdomain order) and then written whole, zeros included, to Ac
// and, if given, to keep.  Padding rows are identity rows.
template <bool IN_LDS>
__global__ __launch_bounds__(256) void coarse_assemble_kernel(BatchDev bd, const int64_t* __restrict__ prow_off,
                                                              const int64_t* __restrict__ cs_ptr,
                                                              const int32_t* __restrict__ cs_sub,
                                                              const int32_t* __restrict__ cs_row, SubDev sd,
                                                              const double* __restrict__ AcLoc, double* Ac,
                                                              double* __restrict__ keep) {
  extern __shared__ double crow_lds[];
  const int64_t q = (int64_t)blockIdx.x + (int64_t)gridDim.x * blockIdx.y;
  if (q >= prow_off[bd.P]) return;
  const int p = find_segment(prow_off, bd.P, q);
  const ProbDev pr = bd.prob[p];
  const int lr = (int)(q - prow_off[p]);
  const int ldc = pr.ldc, tid = threadIdx.x;
  const int64_t off = pr.ac_off + (int64_t)lr * ldc;
  double* crow = IN_LDS ? crow_lds : Ac + off;   // rows too long for LDS are built in place
  for (int i = tid; i < ldc; i += 256) crow[i] = i == lr && lr >= pr.nc ? 1.0 : 0.0;
  __syncthreads();
  if (lr < pr.nc && tid < 64) {
    const int NCp = sd.NCp;
    const int c = pr.coarse_off + lr;
    for (int64_t z = cs_ptr[c]; z < cs_ptr[c + 1]; ++z) {
      const int w = cs_sub[z], t = cs_row[z];
      const int nC = sd.nC[w];
      const double* src = AcLoc + ((int64_t)w * NCp + t) * NCp;
      const int32_t* ids = sd.C_ids + (int64_t)w * NCp;
      for (int u = tid; u < nC; u += 64) crow[ids[u] - pr.coarse_off] += src[u];
    }
  }
  __syncthreads();
  for (int i = tid; i < ldc; i += 256) {
    const double v = crow[i];
    if (IN_LDS) Ac[off + i] = v;
    if (keep) keep[off + i] = v;
  }
}

// ---- apply ----------------------------------------------------------------

// ---- symmetric operators in packed lower-block storage --------------------
// A symmetric n x n operator (n a multiple of SB) is kept as its lower SB x SB
// blocks (I, J), J <= I, in row-major block order; block q = I (I + 1) / 2 + J
// holds SB*SB values in the order in which the apply kernel's lanes read
// them: lane l = r + 32 h (row r, column half h) reads its 16 values of row
// r, columns 16 h + [0, 16), as 16-byte vectors k; vector (k, l) sits at
// (k * 64 + l) * 16 bytes, so each wave-wide load reads 1 KB contiguously.
__device__ inline int packed_offset(int r, int c, int vw) {
  const int h = c >> 4, cc = c & 15;
  return ((cc / vw) * 64 + r + 32 * h) * vw + (cc % vw);
}

// out (packed) = D sym(in) D where sym(in)[i][j] = in[max(i,j)][min(i,j)]
// (only the lower triangle of in is read); D may be null (identity).  One
// block per lower SB x SB block: the block is read into LDS (16-byte loads
// with veci) and leaves in the packed order, one 16-byte vector per store.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void pack_lower_kernel(const TI* __restrict__ in, int64_t ldi, int64_t sI,
                                                         const double* __restrict__ D, int64_t sD,
                                                         TO* __restrict__ out, int nbk, int veci) {
  typedef TI __attribute__((ext_vector_type(16 / sizeof(TI)))) VI;
  typedef TO __attribute__((ext_vector_type(16 / sizeof(TO)))) VO;
  constexpr int VW = 16 / sizeof(TO), WI = 16 / sizeof(TI);
  __shared__ double tile[SB][SB + 1];
  __shared__ double dI[SB], dJ[SB];
  const int64_t w = blockIdx.y;
  const int q = blockIdx.x, tid = threadIdx.x;
  int I = 0;
  while ((I + 1) * (I + 2) / 2 <= q) ++I;
  const int J = q - I * (I + 1) / 2;
  const TI* x = in + w * sI + (int64_t)(SB * I) * ldi + SB * J;
  const double* d = D ? D + w * sD : nullptr;
  if (tid < SB) dI[tid] = d ? d[SB * I + tid] : 1.0;
  else if (tid < 2 * SB) dJ[tid - SB] = d ? d[SB * J + tid - SB] : 1.0;
  if (veci) {
    for (int e = tid; e < SB * SB / WI; e += 256) {
      const int r = e / (SB / WI), c = (e - r * (SB / WI)) * WI;
      const VI v = *reinterpret_cast<const VI*>(x + (int64_t)r * ldi + c);
#pragma unroll
      for (int l = 0; l < WI; ++l) tile[r][c + l] = (double)v[l];
    }
  } else {
    for (int e = tid; e < SB * SB; e += 256) {
      const int r = e / SB, c = e % SB;
      tile[r][c] = (double)x[(int64_t)r * ldi + c];
    }
  }
  __syncthreads();
  // vector p = k * 64 + r + 32 h of the block holds row r, columns
  // 16 h + k VW + [0, VW) (packed_offset)
  TO* o = out + (w * nbk + q) * (int64_t)(SB * SB);
  for (int p = tid; p < SB * SB / VW; p += 256) {
    const int k = p >> 6, r = p & 31, h = (p >> 5) & 1;
    VO a;
#pragma unroll
    for (int l = 0; l < VW; ++l) {
      const int c = 16 * h + k * VW + l;
      const double v = (I != J || c <= r) ? tile[r][c] : tile[c][r];
      a[l] = (TO)(v * dI[r] * dJ[c]);
    }
    *reinterpret_cast<VO*>(o + (int64_t)p * VW) = a;
  }
}

// ys[0, nbu*SB) = P xs for one packed symmetric operator P with nb block rows,
// of which the first nbu hold active rows (blocks beyond are skipped: xs is
// zero there).  Run by the whole workgroup; each wave takes whole blocks:
// the row part of block (I, J) goes to rowp, for I != J the transposed part
// (P_IJ^T x_I) to colp, through a butterfly transpose-reduce within each
// 32-lane half.  The partials are summed per row in a fixed order, so the
// result does not depend on the wave schedule.
// gather() fills xs (with a barrier after it); it runs after the first
// operator block of every wave has been requested, so that the two overlap.
template <typename TM, typename Gather>
__device__ inline void symv_packed(const TM* __restrict__ Pk, int nbu, Gather&& gather, const double* xs,
                                   double* rowp, double* colp, double* ys) {
  typedef typename std::conditional<sizeof(TM) == 4, float __attribute__((ext_vector_type(4))),
                                    double __attribute__((ext_vector_type(2)))>::type V;
  constexpr int VW = 16 / sizeof(TM), NV = 16 / VW;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int r = lane & 31, h = lane >> 5;
  const int nq = nbu * (nbu + 1) / 2;
  // the next block of this wave is loaded before the current one is
  // reduced, so that the wave keeps a block's loads in flight throughout
  V nxt[NV];
  auto fetch = [&](int q) {
    const V* src = reinterpret_cast<const V*>(Pk + (int64_t)q * SB * SB) + lane;
#pragma unroll
    for (int k = 0; k < NV; ++k) nxt[k] = src[k * 64];
  };
  if (wv < nq) fetch(wv);
  gather();
  __syncthreads();
  int I = 0;
  for (int q = wv; q < nq; q += nw) {
    while ((I + 1) * (I + 2) / 2 <= q) ++I;
    const int J = q - I * (I + 1) / 2;
    double v[16];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const V x = nxt[k];
#pragma unroll
      for (int e = 0; e < VW; ++e) v[k * VW + e] = (double)x[e];
    }
    if (q + nw < nq) fetch(q + nw);
    const double* xj = xs + SB * J + 16 * h;
    double rs = 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c) rs += v[c] * xj[c];
    rs += __shfl_xor(rs, 32, 64);
    if (h == 0) rowp[q * SB + r] = rs;
    if (I != J) {
      const double xi = xs[SB * I + r];
#pragma unroll
      for (int c = 0; c < 16; ++c) v[c] *= xi;
      // sum over the 32 rows of each of the 16 columns: after the halving
      // steps lane r holds column (r >> 1) of its half
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const bool up = (r & 16) != 0;
        const double send = up ? v[k] : v[k + 8];
        const double keep = up ? v[k + 8] : v[k];
        v[k] = keep + __shfl_xor(send, 16, 64);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool up = (r & 8) != 0;
        const double send = up ? v[k] : v[k + 4];
        const double keep = up ? v[k + 4] : v[k];
        v[k] = keep + __shfl_xor(send, 8, 64);
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const bool up = (r & 4) != 0;
        const double send = up ? v[k] : v[k + 2];
        const double keep = up ? v[k + 2] : v[k];
        v[k] = keep + __shfl_xor(send, 4, 64);
      }
      {
        const bool up = (r & 2) != 0;
        const double send = up ? v[0] : v[1];
        const double keep = up ? v[1] : v[0];
        v[0] = keep + __shfl_xor(send, 2, 64);
      }
      v[0] += __shfl_xor(v[0], 1, 64);
      if ((r & 1) == 0) colp[q * SB + 16 * h + (r >> 1)] = v[0];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nbu * SB; i += blockDim.x) {
    const int Ib = i / SB, ri = i % SB;
    double acc = 0.0;
    for (int Jb = 0; Jb <= Ib; ++Jb) acc += rowp[(Ib * (Ib + 1) / 2 + Jb) * SB + ri];
    for (int Kb = Ib + 1; Kb < nbu; ++Kb) acc += colp[(Kb * (Kb + 1) / 2 + Ib) * SB + ri];
    ys[i] = acc;
  }
  __syncthreads();
}

// Block-row form of the packed symmetric products, for operators whose
// per-block partial sums would not fit in LDS: one workgroup of SYMV_ROWS_T
// threads per (block row I, subdomain) forms
//   y_I = sum_{J <= I} P_IJ x_J + sum_{K > I} P_KI^T x_K
// (every block is read twice, once for its row and once for its column).
// Thread (r, p) (r = t % 32, p = t / 32) sums the columns c = p + 8 k of
// every block in block order; the 8 partial sums of row r are then added
// in order of p.  Returns y_I[r] in threads r < 32.
constexpr int SYMV_ROWS_T = 256;
template <typename TM>
__device__ inline double symv_block_row(const TM* __restrict__ Pk, int nbu, int I, const double* xs, double* red) {
  constexpr int VW = 16 / sizeof(TM);
  const int t = threadIdx.x, r = t & 31, p = t >> 5;
  double acc = 0.0;
  for (int J = 0; J <= I; ++J) {
    const TM* B = Pk + (int64_t)(I * (I + 1) / 2 + J) * SB * SB;
#pragma unroll
    for (int k = 0; k < SB / 8; ++k) {
      const int c = p + 8 * k;
      acc += (double)B[packed_offset(r, c, VW)] * xs[J * SB + c];
    }
  }
  for (int K = I + 1; K < nbu; ++K) {
    const TM* B = Pk + (int64_t)(K * (K + 1) / 2 + I) * SB * SB;
#pragma unroll
    for (int k = 0; k < SB / 8; ++k) {
      const int c = p + 8 * k;
      acc += (double)B[packed_offset(c, r, VW)] * xs[K * SB + c];
    }
  }
  red[t] = acc;
  __syncthreads();
  double y = 0.0;
  if (t < SB)
    for (int q = 0; q < SYMV_ROWS_T / SB; ++q) y += red[q * SB + t];
  return y;
}

// apply_interior_kernel in block-row form: grid (NIp / SB, ns).
template <typename TM>
__global__ __launch_bounds__(SYMV_ROWS_T) void apply_interior_rows_kernel(SubDev sd, const TM* __restrict__ P,
                                                                      const double* __restrict__ a,
                                                                      const double* __restrict__ b,
                                                                      double* __restrict__ out) {
  extern __shared__ double lds[];
  const int I = blockIdx.x, w = blockIdx.y;
  if (sd.active && !sd.active[sd.sub_prob[w]]) return;
  const int NIp = sd.NIp, nbk = (NIp / SB) * (NIp / SB + 1) / 2;
  const int nI = sd.nI[w], nbu = (nI + SB - 1) / SB;
  if (I >= nbu) return;
  double* xs = lds;                 // [NIp]
  double* red = xs + NIp;           // [SYMV_ROWS_T]
  const int64_t* idx = sd.I_idx + (int64_t)w * NIp;
  for (int j = threadIdx.x; j < NIp; j += blockDim.x) {
    double v = 0.0;
    if (j < nI) {
      const int64_t n = idx[j];
      v = a[n] - (b ? b[n] : 0.0);
    }
    xs[j] = v;
  }
  __syncthreads();
  const double y = symv_block_row<TM>(P + (int64_t)w * nbk * SB * SB, nbu, I, xs, red);
  const int j = I * SB + threadIdx.x;
  if (threadIdx.x < SB && j < nI) out[idx[j]] = y;
}

// apply_neumann_kernel in block-row form: grid (NGp / SB, ns); block row 0
// also forms the coarse restriction cloc_w = Phi_w^T g_w.
template <typename TM, typename TP>
__global__ __launch_bounds__(SYMV_ROWS_T) void apply_neumann_rows_kernel(SubDev sd, const TM* __restrict__ Kt,
                                                                     const TP* __restrict__ Phi,
                                                                     const double* __restrict__ Dw,
                                                                     const double* __restrict__ r,
                                                                     const double* __restrict__ t,
                                                                     double* __restrict__ z,
                                                                     double* __restrict__ cloc) {
  extern __shared__ double lds[];
  const int I = blockIdx.x, w = blockIdx.y;
  if (sd.active && !sd.active[sd.sub_prob[w]]) return;
  const int NGp = sd.NGp, NCp = sd.NCp, nbk = (NGp / SB) * (NGp / SB + 1) / 2;
  const int nG = sd.nG[w], nC = sd.nC[w], nbu = (nG + SB - 1) / SB;
  const int tid = threadIdx.x;
  if (I >= nbu) {
    if (tid < SB) z[(int64_t)w * NGp + I * SB + tid] = 0.0;
    return;
  }
  double* gs = lds;                 // [NGp]
  double* red = gs + NGp;           // [SYMV_ROWS_T]
  const int64_t* idx = sd.G_idx + (int64_t)w * NGp;
  for (int j = tid; j < NGp; j += blockDim.x) {
    double v = 0.0;
    if (j < nG) {
      const int64_t n = idx[j];
      v = Dw[(int64_t)w * NGp + j] * (r[n] - t[n]);
    }
    gs[j] = v;
  }
  __syncthreads();
  if (I == 0) {
    const TP* ph = Phi + (int64_t)w * NGp * NCp;
    for (int u = tid; u < NCp; u += blockDim.x) {
      double acc = 0.0;
      if (u < nC)
        for (int j = 0; j < nG; ++j) acc += (double)ph[(int64_t)j * NCp + u] * gs[j];
      cloc[(int64_t)w * NCp + u] = acc;
    }
  }
  const double y = symv_block_row<TM>(Kt + (int64_t)w * nbk * SB * SB, nbu, I, gs, red);
  const int j = I * SB + tid;
  if (tid < SB) z[(int64_t)w * NGp + j] = j < nG ? y : 0.0;
}

// Threads per workgroup of the packed apply kernels: with two subdomains
// per CU, 512 threads keep 4 waves per SIMD streaming operator blocks.
constexpr int APPLY_T = 512;

// out[node(I_idx)] = P_w (a - b)[I_idx] (b may be null), one workgroup per
// subdomain, P_w = A_II^{-1} in packed storage.
template <typename TM>
__global__ __launch_bounds__(APPLY_T) void apply_interior_kernel(SubDev sd, const TM* __restrict__ P,
                                                             const double* __restrict__ a,
                                                             const double* __restrict__ b,
                                                             double* __restrict__ out) {
  extern __shared__ double lds[];
  const int w = blockIdx.x;
  if (sd.active && !sd.active[sd.sub_prob[w]]) return;
  const int NIp = sd.NIp, nbk = (NIp / SB) * (NIp / SB + 1) / 2;
  const int nI = sd.nI[w];
  const int nbu = (nI + SB - 1) / SB;
  double* xs = lds;                 // [NIp]
  double* ys = xs + NIp;            // [NIp]
  double* rowp = ys + NIp;          // [nbk * SB]
  double* colp = rowp + nbk * SB;   // [nbk * SB]
  const int64_t* idx = sd.I_idx + (int64_t)w * NIp;
  auto gather = [&]() {
    for (int j = threadIdx.x; j < NIp; j += blockDim.x) {
      double v = 0.0;
      if (j < nI) {
        const int64_t n = idx[j];
        v = a[n] - (b ? b[n] : 0.0);
      }
      xs[j] = v;
    }
  };
  symv_packed<TM>(P + (int64_t)w * nbk * SB * SB, nbu, gather, xs, rowp, colp, ys);
  for (int j = threadIdx.x; j < nI; j += blockDim.x) out[idx[j]] = ys[j];
}

// z_w = Kt_w g_w with g_w[j] = Dw[j] (r - t)[G_idx[j]] (Kt_w packed);
// cloc_w = Phi_w^T g_w.
template <typename TM, typename TP>
__global__ __launch_bounds__(APPLY_T) void apply_neumann_kernel(SubDev sd, const TM* __restrict__ Kt,
                                                            const TP* __restrict__ Phi,
                                                            const double* __restrict__ Dw,
                                                            const double* __restrict__ r,
                                                            const double* __restrict__ t,
                                                            double* __restrict__ z, double* __restrict__ cloc) {
  extern __shared__ double lds[];
  const int w = blockIdx.x;
  if (sd.active && !sd.active[sd.sub_prob[w]]) return;
  const int NGp = sd.NGp, NCp = sd.NCp, nbk = (NGp / SB) * (NGp / SB + 1) / 2;
  const int nG = sd.nG[w], nC = sd.nC[w];
  const int nbu = (nG + SB - 1) / SB;
  double* gs = lds;                 // [NGp]
  double* ys = gs + NGp;            // [NGp]
  double* rowp = ys + NGp;          // [nbk * SB]
  double* colp = rowp + nbk * SB;   // [nbk * SB]
  const int64_t* idx = sd.G_idx + (int64_t)w * NGp;
  // the coarse restriction needs only g_w: it is formed right after the
  // gather, while the first operator blocks are in flight
  auto gather = [&]() {
    for (int j = threadIdx.x; j < NGp; j += blockDim.x) {
      double v = 0.0;
      if (j < nG) {
        const int64_t n = idx[j];
        v = Dw[(int64_t)w * NGp + j] * (r[n] - t[n]);
      }
      gs[j] = v;
    }
    __syncthreads();
    // coarse right-hand side cloc_w = Phi_w^T g_w: thread t takes column
    // u = t % nu of the rows j = t / nu + G k (G = blockDim / nu row groups),
    // so that consecutive threads read consecutive entries of a row; the G
    // partial sums of a column are added in a fixed order
    double* part = colp + nbk * SB;   // [blockDim]
    const TP* ph = Phi + (int64_t)w * NGp * NCp;
    const int tid = threadIdx.x;
    for (int u0 = 0; u0 < NCp; u0 += blockDim.x) {
      const int nu = min(NCp - u0, (int)blockDim.x), G = blockDim.x / nu;
      const int u = u0 + tid % nu, gq = tid / nu;
      double acc = 0.0;
      if (gq < G && u < nC)
        for (int j = gq; j < nG; j += G) acc += (double)ph[(int64_t)j * NCp + u] * gs[j];
      part[tid] = acc;
      __syncthreads();
      if (tid < nu) {
        double sum = 0.0;
        for (int q = 0; q < G; ++q) sum += part[q * nu + tid];
        cloc[(int64_t)w * NCp + u0 + tid] = sum;
      }
      __syncthreads();
    }
  };
  symv_packed<TM>(Kt + (int64_t)w * nbk * SB * SB, nbu, gather, gs, rowp, colp, ys);
  for (int j = threadIdx.x; j < NGp; j += blockDim.x) z[(int64_t)w * NGp + j] = j < nG ? ys[j] : 0.0;
}

__global__ void coarse_rhs_kernel(int nc, const int64_t* __restrict__ cs_ptr, const int32_t* __restrict__ cs_sub,
                                  const int32_t* __restrict__ cs_row, int NCp, const double* __restrict__ cloc,
                                  double* __restrict__ c) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  double acc = 0.0;
  for (int64_t z = cs_ptr[q]; z < cs_ptr[q + 1]; ++z) acc += cloc[(int64_t)cs_sub[z] * NCp + cs_row[z]];
  c[q] = acc;
}

// One triangular half of the coarse solve, one workgroup per global coarse
// row (rows differ in length, and workgroups balance them): y[c] = sum over
// j in [lo, hi] of M_p[r][j] x[j], r the problem-local row, [lo, hi] =
// [0, r] (lower) or [r, nc_p - 1] (upper).
constexpr int CT_T = 256;
__global__ __launch_bounds__(CT_T) void coarse_tri_kernel(BatchDev bd, const int32_t* __restrict__ coarse_prob,
                                                          const double* __restrict__ A,
                                                          const double* __restrict__ x, double* __restrict__ y,
                                                          int upper) {
  __shared__ double sh[CT_T / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int c = blockIdx.x;
  const int p = coarse_prob[c];
  if (bd.active && !bd.active[p]) return;
  const ProbDev pr = bd.prob[p];
  const int r = c - pr.coarse_off;
  const double* row = A + pr.ac_off + (int64_t)r * pr.ldc;
  const double* xp = x + pr.coarse_off;
  const int lo = upper ? r : 0, hi = upper ? pr.nc - 1 : r;
  double acc = 0.0;
  if (((reinterpret_cast<uintptr_t>(row) | reinterpret_cast<uintptr_t>(xp)) & 15) == 0) {
    // 16-byte loads of the pairs (j, j + 1), j even; a pair's element below
    // lo is dropped, and a pair reaching past hi loads only j
    for (int j = (lo & ~1) + 2 * tid; j <= hi; j += 2 * CT_T) {
      if (j + 1 <= hi) {
        const double2 a = *reinterpret_cast<const double2*>(row + j);
        const double2 b = *reinterpret_cast<const double2*>(xp + j);
        if (j >= lo) acc += a.x * b.x;
        acc += a.y * b.y;
      } else {
        acc += row[j] * xp[j];   // j = hi >= lo here
      }
    }
  } else {
    for (int j = lo + tid; j <= hi; j += CT_T) acc += row[j] * xp[j];
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) sh[wv] = acc;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int i = 0; i < CT_T / 64; ++i) t += sh[i];
    y[c] = t;
  }
}

// u~_w[j] = z_w[j] + sum_t Phi_w[j][t] u_c[C_ids[t]]  (in place in z)
template <typename TP>
__global__ __launch_bounds__(256) void add_coarse_kernel(SubDev sd, const TP* __restrict__ Phi,
                                                         const double* __restrict__ uc, double* __restrict__ z) {
  extern __shared__ double ul[];
  const int w = blockIdx.x;
  if (sd.active && !sd.active[sd.sub_prob[w]]) return;
  const int NGp = sd.NGp, NCp = sd.NCp;
  const int nG = sd.nG[w], nC = sd.nC[w];
  for (int t = threadIdx.x; t < NCp; t += 256) ul[t] = t < nC ? uc[sd.C_ids[(int64_t)w * NCp + t]] : 0.0;
  __syncthreads();
  const TP* ph = Phi + (int64_t)w * NGp * NCp;
  for (int j = threadIdx.x; j < nG; j += 256) {
    double acc = z[(int64_t)w * NGp + j];
    for (int t = 0; t < nC; ++t) acc += (double)ph[(int64_t)j * NCp + t] * ul[t];
    z[(int64_t)w * NGp + j] = acc;
  }
}

// u_G[node] = sum over the DOF's subdomains (ascending) of Dw u~_w.
__global__ void iface_average_kernel(int64_t n_iface, const int64_t* __restrict__ iface_node,
                                     const int64_t* __restrict__ if_ptr, const int32_t* __restrict__ if_sub,
                                     const int32_t* __restrict__ if_slot, int NGp,
                                     const double* __restrict__ Dw, const double* __restrict__ z,
                                     double* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_iface) return;
  double acc = 0.0;
  for (int64_t e = if_ptr[q]; e < if_ptr[q + 1]; ++e) {
    const int64_t k = (int64_t)if_sub[e] * NGp + if_slot[e];
    acc += Dw[k] * z[k];
  }
  out[iface_node[q]] = acc;
}

}  // namespace

void bddc_set_reference(const double* Kref) {
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_Kref_b), Kref, 64 * sizeof(double));
}

inline int packed_blocks(int n) { return (n / SB) * (n / SB + 1) / 2; }

// Dynamic LDS bytes of the per-subdomain kernels, from the padded sizes.
// The assembly keeps its diagonal and scaling vectors in LDS and builds
// ASM_WAVES rows at a time when that fits; otherwise (big) it keeps them in
// global memory and builds as many rows at a time as fit (asm_row_waves).
size_t lds_assemble_fixed(int NGp, int NCp, int s) {
  const int s3 = s * s * s;
  return (size_t)(NCp + s3 + 2 * ((NCp + 1 + NGp + s3 + 3) / 4)) * sizeof(double);
}
size_t lds_assemble_local(int NIp, int NGp, int NCp, int s, size_t elem) {
  const int nt = NIp + NGp;
  return lds_assemble_fixed(NGp, NCp, s) + (size_t)2 * nt * sizeof(double) + (size_t)ASM_WAVES * nt * elem;
}
// rows in flight of the big assembly (0: even one row does not fit)
int asm_row_waves(int NIp, int NGp, int NCp, int s, size_t elem) {
  const size_t fixed = lds_assemble_fixed(NGp, NCp, s), row = (size_t)(NIp + NGp) * elem;
  if (fixed + row > LDS_BYTES) return 0;
  return (int)std::min<size_t>(ASM_WAVES, (LDS_BYTES - fixed) / row);
}
bool asm_big(int NIp, int NGp, int NCp, int s, size_t elem) {
  return lds_assemble_local(NIp, NGp, NCp, s, elem) > LDS_BYTES;
}
// The packed applies hold the vectors and the partial sums of every block in
// LDS; larger operators take the block-row form (x and one partial per
// thread in LDS).
size_t lds_apply_interior(int NIp) { return (size_t)(2 * NIp + 2 * packed_blocks(NIp) * SB) * sizeof(double); }
size_t lds_apply_neumann(int NGp) {
  return (size_t)(2 * NGp + 2 * packed_blocks(NGp) * SB + APPLY_T) * sizeof(double);
}
size_t lds_apply_rows(int n) { return (size_t)(n + SYMV_ROWS_T) * sizeof(double); }
size_t lds_small_spd_inverse(int NCp) { return (size_t)NCp * NCp * sizeof(double); }

size_t bddc_lds_need(int NIp, int NGp, int NCp, int s, int fp32_local) {
  const size_t elem = fp32_local ? sizeof(float) : sizeof(double);
  const size_t as = asm_big(NIp, NGp, NCp, s, elem)
                        ? (asm_row_waves(NIp, NGp, NCp, s, elem) > 0 ? lds_assemble_fixed(NGp, NCp, s) +
                                                                             (size_t)(NIp + NGp) * elem
                                                                       : (size_t)-1)
                        : lds_assemble_local(NIp, NGp, NCp, s, elem);
  const size_t ai = lds_apply_interior(NIp) <= LDS_BYTES ? lds_apply_interior(NIp) : lds_apply_rows(NIp);
  const size_t an = lds_apply_neumann(NGp) <= LDS_BYTES ? lds_apply_neumann(NGp) : lds_apply_rows(NGp);
  return std::max(std::max(as, ai), std::max(an, lds_small_spd_inverse(NCp)));
}

template <typename T>
void launch_assemble_local(hipStream_t st, const SubDev& sd, const GridDev& g, int ns, T* K,
                           double* diagA_G, double* Dscale, double* st_val, int32_t* st_col) {
  static const bool attr =
      hipFuncSetAttribute((const void*)assemble_local_kernel<T, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)LDS_BYTES) == hipSuccess &&
      hipFuncSetAttribute((const void*)assemble_local_kernel<T, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)LDS_BYTES) == hipSuccess;
  (void)attr;
  if (!asm_big(sd.NIp, sd.NGp, sd.NCp, g.s, sizeof(T))) {
    const size_t sh = lds_assemble_local(sd.NIp, sd.NGp, sd.NCp, g.s, sizeof(T));
    hipLaunchKernelGGL((assemble_local_kernel<T, false>), dim3(ns), dim3(64 * ASM_WAVES), sh, st, sd, g, K, diagA_G,
                       Dscale, st_val, st_col, ASM_WAVES);
  } else {
    // setup has checked that one row fits (bddc_lds_need)
    const int rw = asm_row_waves(sd.NIp, sd.NGp, sd.NCp, g.s, sizeof(T));
    const size_t sh = lds_assemble_fixed(sd.NGp, sd.NCp, g.s) + (size_t)rw * (sd.NIp + sd.NGp) * sizeof(T);
    hipLaunchKernelGGL((assemble_local_kernel<T, true>), dim3(ns), dim3(64 * ASM_WAVES), sh, st, sd, g, K, diagA_G,
                       Dscale, st_val, st_col, rw);
  }
}
template void launch_assemble_local<double>(hipStream_t, const SubDev&, const GridDev&, int, double*,
                                            double*, double*, double*, int32_t*);
template void launch_assemble_local<float>(hipStream_t, const SubDev&, const GridDev&, int, float*,
                                           double*, double*, double*, int32_t*);

void launch_weights(hipStream_t st, int64_t n_iface, const int64_t* if_ptr, const int32_t* if_sub,
                    const int32_t* if_slot, int NGp, const double* diagA_G, int stiffness, double* Dw) {
  if (n_iface <= 0) return;
  hipLaunchKernelGGL(weights_kernel, dim3((unsigned)((n_iface + 255) / 256)), dim3(256), 0, st, n_iface,
                     if_ptr, if_sub, if_slot, NGp, diagA_G, stiffness, Dw);
}

void launch_object_lists(hipStream_t st, const SubDev& sd, int ns, int32_t* optr, int32_t* omem) {
  if (ns <= 0) return;
  hipLaunchKernelGGL(object_lists_kernel, dim3(ns), dim3(256), (size_t)(sd.NCp + 1 + sd.NGp) * sizeof(int), st, sd,
                     optr, omem);
}

void launch_local_apply(hipStream_t st, const SubDev& sd, int ns, const double* st_val, const int32_t* st_col,
                        const double* X, double* Y, int r0, int nrows, int xfrom) {
  if (nrows <= 0 || ns <= 0) return;
  dim3 grid((nrows + LA_ROWS - 1) / LA_ROWS, ns);
  if (xfrom > 0)
    hipLaunchKernelGGL(local_apply_kernel<true>, grid, dim3(256), 0, st, sd, st_val, st_col, X, Y, r0, nrows, xfrom);
  else
    hipLaunchKernelGGL(local_apply_kernel<false>, grid, dim3(256), 0, st, sd, st_val, st_col, X, Y, r0, nrows, 0);
}

void launch_constraint_cols(hipStream_t st, const SubDev& sd, int ns, const double* KS, double* Gt) {
  if (ns <= 0) return;
  dim3 grid((sd.NGp + CC_COLS - 1) / CC_COLS, ns);
  hipLaunchKernelGGL(constraint_cols_kernel, grid, dim3(256), (size_t)(sd.NCp + 1 + sd.NGp) * sizeof(int), st, sd,
                     KS, Gt);
}

void launch_constraint_rows(hipStream_t st, const SubDev& sd, int ns, const double* Gt, double* Sc) {
  if (ns <= 0) return;
  // staged form while the member lists and four row buffers fit in 64 KB
  const size_t ints = (size_t)((sd.NCp + 1 + sd.NGp + 1) & ~1) * sizeof(int);
  const size_t rowb = (size_t)sd.NGp * sizeof(double);
  constexpr int CR_W = 4;
  if (ints + CR_W * rowb <= 65536) {
    hipLaunchKernelGGL(constraint_rows_staged_kernel, dim3((sd.NCp + CR_W - 1) / CR_W, ns), dim3(64 * CR_W),
                       ints + CR_W * rowb, st, sd, Gt, Sc);
    return;
  }
  hipLaunchKernelGGL(constraint_rows_kernel, dim3(ns), dim3(256), (size_t)(sd.NCp + 1 + sd.NGp) * sizeof(int), st,
                     sd, Gt, Sc);
}


void launch_small_spd_inverse(hipStream_t st, const SubDev& sd, int ns, double* S, int* info) {
  hipLaunchKernelGGL(small_spd_inverse_kernel, dim3(ns), dim3(256), lds_small_spd_inverse(sd.NCp), st, sd, S,
                     info);
}

void launch_coarse_assemble(hipStream_t st, const BatchDev& b, const int64_t* prow_off, int64_t n_prows, int max_ldc,
                            const int64_t* cs_ptr, const int32_t* cs_sub, const int32_t* cs_row, const SubDev& sd,
                            const double* AcLoc, double* Ac, double* keep) {
  if (n_prows <= 0) return;
  const int64_t gx = std::min<int64_t>(n_prows, 65535);
  const dim3 grid((unsigned)gx, (unsigned)((n_prows + gx - 1) / gx));
  // CUTBDDC_COARSE_ROW_LDS lowers the longest row built in LDS (read at
  // every call, so that the global-memory path can be tested on small
  // problems)
  int lim = COARSE_ASSEMBLE_LDS_LDC;
  if (const char* e = std::getenv("CUTBDDC_COARSE_ROW_LDS")) lim = std::max(0, std::min(lim, std::atoi(e)));
  if (max_ldc <= lim) {
    static const bool attr = hipFuncSetAttribute((const void*)coarse_assemble_kernel<true>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)(COARSE_ASSEMBLE_LDS_LDC * sizeof(double))) == hipSuccess;
    (void)attr;
    hipLaunchKernelGGL(coarse_assemble_kernel<true>, grid, dim3(256), (size_t)max_ldc * sizeof(double), st, b,
                       prow_off, cs_ptr, cs_sub, cs_row, sd, AcLoc, Ac, keep);
  } else {
    hipLaunchKernelGGL(coarse_assemble_kernel<false>, grid, dim3(256), 0, st, b, prow_off, cs_ptr, cs_sub, cs_row,
                       sd, AcLoc, Ac, keep);
  }
}

template <typename TI, typename TO>
void launch_pack_lower(hipStream_t st, int n, int ns, const TI* in, int64_t ldi, int64_t sI, const double* D,
                       int64_t sD, TO* out) {
  if (ns <= 0 || n <= 0) return;
  constexpr int WI = 16 / sizeof(TI);
  const int veci = (reinterpret_cast<uintptr_t>(in) & 15) == 0 && ldi % WI == 0 && sI % WI == 0;
  hipLaunchKernelGGL((pack_lower_kernel<TI, TO>), dim3(packed_blocks(n), ns), dim3(256), 0, st, in, ldi, sI, D, sD,
                     out, packed_blocks(n), veci);
}
template void launch_pack_lower<float, float>(hipStream_t, int, int, const float*, int64_t, int64_t, const double*,
                                              int64_t, float*);
template void launch_pack_lower<double, double>(hipStream_t, int, int, const double*, int64_t, int64_t,
                                                const double*, int64_t, double*);
template void launch_pack_lower<double, float>(hipStream_t, int, int, const double*, int64_t, int64_t,
                                               const double*, int64_t, float*);

template <typename TM>
void launch_apply_interior(hipStream_t st, const SubDev& sd, int ns, const TM* P, const double* a,
                           const double* b, double* out) {
  const size_t sh = lds_apply_interior(sd.NIp);
  if (sh > LDS_BYTES) {
    static const bool attr_rows = hipFuncSetAttribute((const void*)apply_interior_rows_kernel<TM>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                                      (int)LDS_BYTES) == hipSuccess;
    (void)attr_rows;
    hipLaunchKernelGGL(apply_interior_rows_kernel<TM>, dim3(sd.NIp / SB, ns), dim3(SYMV_ROWS_T),
                       lds_apply_rows(sd.NIp), st, sd, P, a, b, out);
    return;
  }
  static bool attr = (hipFuncSetAttribute((const void*)apply_interior_kernel<TM>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) == hipSuccess);
  (void)attr;
  hipLaunchKernelGGL(apply_interior_kernel<TM>, dim3(ns), dim3(APPLY_T), sh, st, sd, P, a, b, out);
}
template void launch_apply_interior<double>(hipStream_t, const SubDev&, int, const double*, const double*,
                                            const double*, double*);
template void launch_apply_interior<float>(hipStream_t, const SubDev&, int, const float*, const double*,
                                           const double*, double*);

template <typename TM, typename TP>
void launch_apply_neumann(hipStream_t st, const SubDev& sd, int ns, const TM* Kt, const TP* Phi,
                          const double* Dw, const double* r, const double* t, double* z, double* cloc) {
  const size_t sh = lds_apply_neumann(sd.NGp);
  if (sh > LDS_BYTES) {
    static const bool attr_rows = hipFuncSetAttribute((const void*)apply_neumann_rows_kernel<TM, TP>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                                      (int)LDS_BYTES) == hipSuccess;
    (void)attr_rows;
    hipLaunchKernelGGL((apply_neumann_rows_kernel<TM, TP>), dim3(sd.NGp / SB, ns), dim3(SYMV_ROWS_T),
                       lds_apply_rows(sd.NGp), st, sd, Kt, Phi, Dw, r, t, z, cloc);
    return;
  }
  static bool attr = (hipFuncSetAttribute((const void*)apply_neumann_kernel<TM, TP>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) == hipSuccess);
  (void)attr;
  hipLaunchKernelGGL((apply_neumann_kernel<TM, TP>), dim3(ns), dim3(APPLY_T), sh, st, sd, Kt, Phi, Dw, r, t, z,
                     cloc);
}
template void launch_apply_neumann<double, double>(hipStream_t, const SubDev&, int, const double*, const double*,
                                                   const double*, const double*, const double*, double*, double*);
template void launch_apply_neumann<float, float>(hipStream_t, const SubDev&, int, const float*, const float*,
                                                 const double*, const double*, const double*, double*, double*);

void launch_coarse_rhs(hipStream_t st, int nc, const int64_t* cs_ptr, const int32_t* cs_sub,
                       const int32_t* cs_row, int NCp, const double* cloc, double* c) {
  if (nc <= 0) return;
  hipLaunchKernelGGL(coarse_rhs_kernel, dim3((nc + 255) / 256), dim3(256), 0, st, nc, cs_ptr, cs_sub, cs_row,
                     NCp, cloc, c);
}

void launch_coarse_gemv(hipStream_t st, const BatchDev& b, int nc_total, const int32_t* coarse_prob,
                        const double* M, const double* x, double* t, double* y) {
  if (nc_total <= 0) return;
  hipLaunchKernelGGL(coarse_tri_kernel, dim3(nc_total), dim3(CT_T), 0, st, b, coarse_prob, M, x, t, 0);
  hipLaunchKernelGGL(coarse_tri_kernel, dim3(nc_total), dim3(CT_T), 0, st, b, coarse_prob, M, t, y, 1);
}

template <typename TP>
void launch_add_coarse(hipStream_t st, const SubDev& sd, int ns, const TP* Phi, const double* uc, double* z) {
  hipLaunchKernelGGL(add_coarse_kernel<TP>, dim3(ns), dim3(256), sd.NCp * sizeof(double), st, sd, Phi, uc, z);
}
template void launch_add_coarse<double>(hipStream_t, const SubDev&, int, const double*, const double*, double*);
template void launch_add_coarse<float>(hipStream_t, const SubDev&, int, const float*, const double*, double*);

void launch_iface_average(hipStream_t st, int64_t n_iface, const int64_t* iface_node, const int64_t* if_ptr,
                          const int32_t* if_sub, const int32_t* if_slot, int NGp, const double* Dw,
                          const double* z, double* out) {
  if (n_iface <= 0) return;
  hipLaunchKernelGGL(iface_average_kernel, dim3((unsigned)((n_iface + 255) / 256)), dim3(256), 0, st,
                     n_iface, iface_node, if_ptr, if_sub, if_slot, NGp, Dw, z, out);
}

}  // namespace cutbddc
