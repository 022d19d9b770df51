// Device descriptors and launchers of the BDDC kernels.
#pragma once

#include "common.h"

namespace cutbddc {

// Per-subdomain index data (device pointers), padded sizes.
struct SubDev {
  int NIp, NGp, NCp;              // padded interior / interface / coarse counts
  const int32_t* nI;              // [ns]
  const int32_t* nG;              // [ns]
  const int32_t* nC;              // [ns]
  const int64_t* I_idx;           // [ns*NIp] grid node of each interior row (-1 pad)
  const int64_t* G_idx;           // [ns*NGp] grid node of each interface row (-1 pad)
  const int32_t* G_obj;           // [ns*NGp] local coarse row of each interface row or -1
  const int32_t* C_ids;           // [ns*NCp] global coarse id of each local coarse row (-1 pad)
  const int32_t* bloc;            // [ns*(s+1)^3] block node -> local row or -1
  const int32_t* sub_prob;        // [ns] problem of each subdomain
  const int32_t* sub_blk;         // [ns] subdomain index within its problem
  const int32_t* active;          // [P] problems whose PCG still runs, or null
  // Interface slots of each local object, grouped by object (see
  // launch_object_lists), or null: kernels that need them then build them.
  const int32_t* optr;            // [ns*(NCp+1)] start of object t's members
  const int32_t* omem;            // [ns*NGp] member slots, ascending per object
};

// Grid data of all problems (concatenated cell arrays).
struct GridDev {
  const ProbDev* prob;            // [P]
  int s;                          // cells per subdomain side (common to the batch)
  const int32_t* cellinfo;        // concatenated cells
  const double* kappa;
  const double* Kc;               // [n_cut_total*36]
};

void bddc_set_reference(const double* Kref);

// optr/omem of every subdomain (sizes as in SubDev), built once so that the
// assembly and the constraint kernels need not scan the interface for them.
void launch_object_lists(hipStream_t st, const SubDev& sd, int ns, int32_t* optr, int32_t* omem);

// Stencil rows of A_omega kept for the Gram-matrix products: for row r of
// subdomain w, slot k (neighbour offset (k%3-1, k/3%3-1, k/9-1)) holds the
// unscaled entry and its column (-1: none), at [(w nt + r) 27 + k].
constexpr int STENCIL = 27;
// Also writes the stencil rows (st_val, st_col) when they are non-null.
template <typename T>
void launch_assemble_local(hipStream_t st, const SubDev& sd, const GridDev& g, int ns, T* K,
                           double* diagA_G, double* Dscale, double* st_val, int32_t* st_col);
void launch_weights(hipStream_t st, int64_t n_iface, const int64_t* if_ptr, const int32_t* if_sub,
                    const int32_t* if_slot, int NGp, const double* diagA_G, int stiffness, double* Dw);
// Rows [r0, r0 + nrows) of Y = A_omega X (FP64, nt x NCp blocks), from the
// stencil rows written by launch_assemble_local.  The caller states that
// rows [0, xfrom) of X are zero: their terms are not loaded.
void launch_local_apply(hipStream_t st, const SubDev& sd, int ns, const double* st_val, const int32_t* st_col,
                        const double* X, double* Y, int r0, int nrows, int xfrom = 0);
// Gt = (K_S^{-1} C^T)^T (NCp x NGp) and S_c = C G with C the object-mean
// constraints.
void launch_constraint_cols(hipStream_t st, const SubDev& sd, int ns, const double* KS, double* Gt);
void launch_constraint_rows(hipStream_t st, const SubDev& sd, int ns, const double* Gt, double* Sc);
void launch_small_spd_inverse(hipStream_t st, const SubDev& sd, int ns, double* S, int* info);
// Coarse matrix of every problem p as its own ldc_p x ldc_p block at
// Ac + ac_off_p (identity on the padding rows; every entry written);
// prow_off[p] = first padded row of problem p in the launch, prow_off[P] =
// n_prows.  keep (may be null) receives the same values.  max_ldc = largest
// ldc_p: rows up to COARSE_ASSEMBLE_LDS_LDC long (or the smaller limit in
// the environment variable CUTBDDC_COARSE_ROW_LDS) are built in LDS, longer
// ones in place in Ac (the same sums in the same order).
constexpr int COARSE_ASSEMBLE_LDS_LDC = 16384;
void launch_coarse_assemble(hipStream_t st, const BatchDev& b, const int64_t* prow_off, int64_t n_prows, int max_ldc,
                            const int64_t* cs_ptr, const int32_t* cs_sub, const int32_t* cs_row, const SubDev& sd,
                            const double* AcLoc, double* Ac, double* keep);
// Symmetric operators in packed lower-block storage: SB x SB blocks (I, J),
// J <= I, packed_blocks(n) blocks of SB*SB values per subdomain.
constexpr int SB = 32;
inline int packed_elems(int n) { return (n / SB) * (n / SB + 1) / 2 * SB * SB; }
// out[w] = D_w sym(in_w) D_w in packed storage (only the lower triangle of
// in_w is read; D may be null).  n a multiple of SB.
template <typename TI, typename TO>
void launch_pack_lower(hipStream_t st, int n, int ns, const TI* in, int64_t ldi, int64_t sI, const double* D,
                       int64_t sD, TO* out);
// P, Kt: packed storage.
template <typename TM>
void launch_apply_interior(hipStream_t st, const SubDev& sd, int ns, const TM* P, const double* a,
                           const double* b, double* out);
// Phi in the storage type TP (FP64; FP32 on the FP32-local path).
template <typename TM, typename TP>
void launch_apply_neumann(hipStream_t st, const SubDev& sd, int ns, const TM* Kt, const TP* Phi,
                          const double* Dw, const double* r, const double* t, double* z, double* cloc);
// Largest dynamic LDS request in bytes of the per-subdomain kernels (local
// assembly, packed applies, coarse-basis Gram inverse) for padded orders
// NIp, NGp, NCp and subdomain side s; it must not exceed LDS_BYTES.
constexpr size_t LDS_BYTES = 160 * 1024;
size_t bddc_lds_need(int NIp, int NGp, int NCp, int s, int fp32_local);
void launch_coarse_rhs(hipStream_t st, int nc, const int64_t* cs_ptr, const int32_t* cs_sub,
                       const int32_t* cs_row, int NCp, const double* cloc, double* c);
// Coarse solve y = A_c^{-1} x = Y^T (Y x) per problem, Y = L^{-1} of the
// coarse Cholesky factor, from M_p (ldc_p x ldc_p at ac_off_p) holding Y in
// its lower triangle and Y^T in its upper one (the diagonal is shared):
// t = tril(M) x, then y = triu(M) t, one workgroup per global coarse row c
// (p = coarse_prob[c]).  t has nc_total entries.
void launch_coarse_gemv(hipStream_t st, const BatchDev& b, int nc_total, const int32_t* coarse_prob,
                        const double* M, const double* x, double* t, double* y);
template <typename TP>
void launch_add_coarse(hipStream_t st, const SubDev& sd, int ns, const TP* Phi, const double* uc, double* z);
void launch_iface_average(hipStream_t st, int64_t n_iface, const int64_t* iface_node, const int64_t* if_ptr,
                          const int32_t* if_sub, const int32_t* if_slot, int NGp, const double* Dw,
                          const double* z, double* out);

}  // namespace cutbddc
