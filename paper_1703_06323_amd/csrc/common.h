// Shared declarations for the cutbddc device kernels and their host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace cutbddc {

// Cell encoding used by every grid kernel:
//   cellinfo[c] = -2 inactive, -1 active and integrated as uncut (reference
//   matrices), >= 0 index of the cut cell's stored matrices.
constexpr int32_t CELL_INACTIVE = -2;
constexpr int32_t CELL_UNCUT = -1;

constexpr int PACK36 = 36;   // packed upper triangle of an 8x8 matrix

struct GridDesc {
  int32_t N;                 // cells per axis
  double h;                  // 1/N
};

// A context holds P >= 1 independent meshes.  Their cell, node, DOF,
// subdomain and coarse arrays are concatenated in problem order; every cell
// and node segment starts at a multiple of SEG_ALIGN, so a block of
// SEG_ALIGN consecutive entries never spans two problems.
constexpr int SEG_ALIGN = 256;

struct ProbDev {
  int32_t N, s, m;           // cells per axis, cells per subdomain side, subdomains per axis
  int32_t nb, ball_off;      // balls of the level set and the first one in the ball array
  double h;                  // 1/N
  int64_t cell_off, node_off, dof_off;
  int32_t sub_off, coarse_off;
  int32_t nc, ldc;           // coarse DOFs, order of the padded coarse block
  int64_t ac_off;            // element offset of the coarse block (ldc x ldc)
};

struct BatchDev {
  int32_t P;
  const ProbDev* prob;       // [P]
  const int64_t* cell_off;   // [P+1]
  const int64_t* node_off;   // [P+1]
  const int32_t* active;     // [P] problems whose PCG still runs, or null (all)
  // Work items of the matrix-free operator, problem p owning items
  // [op_off[p], op_off[p+1]), op_prob[item] = p, in one of two forms:
  //  * op_box = 0, node blocks: the blocks of SEG_ALIGN consecutive nodes
  //    (op_off = node_off / SEG_ALIGN); op_lx, op_lc: lengths of the LDS
  //    ranges of x and of the cell data per block (SEG_ALIGN + 2 (N+1) + 2
  //    and 2 SEG_ALIGN + 2 N + 2 for the largest N of the context);
  //  * op_box = 1, node boxes: SW along x, TY along y, ZC along z (SW TY <=
  //    SEG_ALIGN threads, one node each per plane, marching over the ZC
  //    planes); op_geom[8 p ..] = {nseg, SW, TY, ngy, ZC, nzc}: nseg
  //    x-segments, ngy y-groups and nzc z-chunks, the item's local number
  //    being (seg ngy + gy) nzc + zc; op_xp, op_cp: the largest tile plane
  //    of x with its halo, (SW + 2)(TY + 2), and of cells, (SW + 1)(TY + 1).
  const int32_t* op_off;     // [P+1]
  const int32_t* op_prob;    // [items]
  const int32_t* op_geom;    // [8 P] (boxes)
  int32_t op_box;
  int32_t op_lx, op_lc;      // (blocks)
  int32_t op_xp, op_cp;      // (boxes)
};

// Operator node-box geometry of a problem with N1 = N + 1 nodes per axis
// (host): x-segments and y-groups whose (SW + 2)(TY + 2) / (SW TY) halo
// ratio is smallest with at least half a workgroup of nodes per plane, and
// ZC planes per item so that an item holds about nodes_per_item nodes.
// Boxes stage each x value about 1.3 times against about 4 (9 for a
// 256-node block inside one row) for node blocks, but keep fewer threads
// busy on small meshes; contexts whose meshes all have at least
// OP_BOX_MIN_N cells per axis use them (environment CUTBDDC_OPERATOR =
// box or block forces one form).
struct OpGeom {
  int32_t nseg, SW, TY, ngy, ZC, nzc;
};
OpGeom op_geometry(int N1, int64_t nodes_per_item);
constexpr int OP_BOX_MIN_N = 128;
constexpr int OP_XP_MAX = 4 * SEG_ALIGN;   // staging registers per thread: 4 x values
constexpr int OP_CP_MAX = 3 * SEG_ALIGN;   // and 3 cells


// Largest p in [0, P) with off[p] <= i (off ascending, off[0] = 0).
template <typename I>
__host__ __device__ inline int find_segment(const I* off, int P, int64_t i) {
  int lo = 0, hi = P - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int64_t)off[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Index of entry (a, b) of a symmetric 8x8 matrix in its packed upper
// triangle (row by row).
__host__ __device__ inline int pack_index(int a, int b) {
  int r = a < b ? a : b;
  int c = a < b ? b : a;
  return r * 8 - (r * (r - 1)) / 2 + (c - r);
}

// Records msg as the thread's last error (cb_last_error) and returns code.
int report_error(int code, const std::string& msg);

// ---- launchers (defined in the .hip files) --------------------------------
// integrate.hip (cells: concatenated cell space of n_cells_total entries)
void launch_classify(hipStream_t st, const BatchDev& b, int64_t n_cells_total, const double* xi,
                     const double* balls, int32_t* count);
void launch_integrate_cut(hipStream_t st, const BatchDev& b, const double* xi, const double* balls,
                          const int64_t* cut_cells, int64_t n_cut, double* Kc, double* Mc);
// operator.hip (nodes: concatenated node space of nn entries)
void set_reference_matrices(const double* Kref, const double* Mref);
// Raises the operator kernel's dynamic LDS limit (call outside stream
// capture, before its first launch); 0 on success.
int prepare_apply_A();
// y = A x on the node space (n_items = b.op_off[P] work items); with dpart,
// dpart[item] = the work item's part of x.y.
// Kf: the cut cells' unit stiffness as full row-major 8x8 matrices
// (launch_expand_rows).
void launch_apply_A(hipStream_t st, const BatchDev& b, int64_t nn, int32_t n_items, const int32_t* cellinfo,
                    const double* kappa, const double* Kf, const uint8_t* dofmask, const double* x,
                    double* y, double* dpart = nullptr);
// Kf[e] (64 values, row-major) = the packed matrix Kc[e] (36 values), for n cut cells.
void launch_expand_rows(hipStream_t st, int64_t n_cut, const double* Kc, double* Kf);
// b = M_cut f.  f is read per problem from f_ptrs[p] (local node numbering;
// a null entry means f = 1) when f_ptrs is given, else from the
// concatenated vector f.  outmask null: every node of a segment is written.
void launch_load(hipStream_t st, const BatchDev& b, int64_t nn, const int32_t* cellinfo,
                 const double* Mc, const uint8_t* outmask, const double* f,
                 const double* const* f_ptrs, double* out);
void launch_grad_theta(hipStream_t st, GridDesc g, const int32_t* cellinfo, const double* kappa,
                       const double* Kc, const double* u, const double* lam, double* out);
void launch_scatter_dofs(hipStream_t st, int64_t n, const int64_t* dof_node, const double* src,
                         double* grid);
void launch_gather_dofs(hipStream_t st, int64_t n, const int64_t* dof_node, const double* grid,
                        double* dst);
void launch_fill(hipStream_t st, int64_t n, double v, double* x);
void launch_copy(hipStream_t st, int64_t n, const double* src, double* dst);
// Per-problem dot products over the node segments, in a fixed order:
// out[p * stride] = x_p . y_p.  chunk_ptr[p] = first DOT_CHUNK-sized chunk of
// problem p (chunk_ptr[P] = total); partial holds one value per chunk.
constexpr int DOT_CHUNK = 1024;
void launch_dot(hipStream_t st, const BatchDev& b, const int32_t* chunk_ptr, int32_t n_chunks,
                const double* x, const double* y, double* partial, double* out, int stride);
// only the chunk parts of launch_dot (partial[chunk])
void launch_dot_chunks(hipStream_t st, const BatchDev& b, const int32_t* chunk_ptr, int32_t n_chunks, const double* x,
                       const double* y, double* partial);
// PCG scalars per problem p at S[8p + k]: 0 rho of the previous iteration,
// 1 p.q, 2 r.r, 3 rho = r.z of the latest preconditioned residual, 4 b.b.
// State per problem: it (iterations), status (0 running, 1 converged,
// 2 iteration limit, 3 breakdown), relres; n_active[0] = number of running
// problems.  params = {rtol, max_iter}.
constexpr int CG_S = 8;
void launch_cg_init(hipStream_t st, int P, const double* params, double* S, int32_t* active, int32_t* it,
                    int32_t* status, double* relres, int32_t* n_active);
// Convergence test after the x, r update: r.r of each running problem from
// the block parts rr_part (blocks of SEG_ALIGN nodes; node_off [P+1]) into
// slot 2; moves slot 3 to slot 0; writes the count of running problems to
// n_active and to host memory nact_host (may be null).
// hist (may be null): per problem p and iteration k <= hcap, the triple
// (alpha_k, beta that formed p_k (0 for k = 1), |r_k| / |b|) at
// hist[(p hcap + k - 1) 3].
void launch_cg_check(hipStream_t st, int P, const int64_t* node_off, const double* rr_part, const double* params,
                     double* S, int32_t* active, int32_t* it, int32_t* status, double* relres, int32_t* n_active,
                     int32_t* nact_host, double* hist, int32_t hcap);
// x, r update (alpha = S[3] / p.q, p.q = sum of the problem's work-item
// parts pq_part of the operator, stored in slot 1); the block parts of the new r.r go to rr_part;
// zero1 and zero2 (may be null) are cleared on the same nodes.
void launch_cg_update_xr(hipStream_t st, const BatchDev& b, int64_t nn, double* S, const double* pq_part,
                         const double* p, const double* q, double* x, double* r, double* zero1, double* zero2,
                         double* rr_part);
// p update (beta = r.z / S[0], r.z = sum of the problem's chunk parts
// rz_part from launch_dot_chunks, stored in slot 3).
void launch_cg_update_p(hipStream_t st, const BatchDev& b, int64_t nn, double* S, const int32_t* chunk_ptr,
                        const double* rz_part, const double* z, double* p);
void launch_set_params(hipStream_t st, double* params, double rtol, int32_t max_iter);
// u_p[d] = grid[dof_node[dof_off[p] + d]] for every problem (u_ptrs: device
// array of P output pointers), or dst[d] = grid[dof_node[d]] if u_ptrs is null.
void launch_gather_dofs_batch(hipStream_t st, int P, int64_t n_dof_total, const int64_t* dof_off,
                              const int64_t* dof_node, const double* grid, double* const* u_ptrs);
void convert_to_float(hipStream_t st, int64_t n, const double* a, float* b);

}  // namespace cutbddc
