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
};

struct GridDev {
  int N, s;
  double h;
  const int32_t* cellinfo;        // [N^3]
  const double* kappa;            // [N^3]
  const double* Kc;               // [n_cut*36]
};

void bddc_set_reference(const double* Kref);

template <typename T>
void launch_assemble_local(hipStream_t st, const SubDev& sd, const GridDev& g, int ns, T* K,
                           double* diagA_G, double* Dscale);
void launch_weights(hipStream_t st, int64_t n_iface, const int64_t* if_ptr, const int32_t* if_sub,
                    const int32_t* if_slot, int NGp, const double* diagA_G, int stiffness, double* Dw);
void launch_local_apply(hipStream_t st, const SubDev& sd, const GridDev& g, int ns, const double* X, double* Y);
void launch_build_constraints(hipStream_t st, const SubDev& sd, int ns, double* Cm);
void launch_small_spd_inverse(hipStream_t st, const SubDev& sd, int ns, double* S, int* info);
void launch_coarse_assemble(hipStream_t st, int nc, int ldc, const int64_t* cs_ptr, const int32_t* cs_sub,
                            const int32_t* cs_row, const SubDev& sd, const double* AcLoc, double* Ac);
template <typename TM>
void launch_apply_interior(hipStream_t st, const SubDev& sd, int ns, const TM* P, const double* a,
                           const double* b, double* out);
template <typename TM>
void launch_apply_neumann(hipStream_t st, const SubDev& sd, int ns, const TM* Kt, const double* Phi,
                          const double* Dw, const double* r, const double* t, double* z, double* cloc);
void launch_coarse_rhs(hipStream_t st, int nc, const int64_t* cs_ptr, const int32_t* cs_sub,
                       const int32_t* cs_row, int NCp, const double* cloc, double* c);
void launch_gemv(hipStream_t st, int n, int ld, const double* A, const double* x, double* y);
void launch_add_coarse(hipStream_t st, const SubDev& sd, int ns, const double* Phi, const double* uc,
                       double* z);
void launch_iface_average(hipStream_t st, int64_t n_iface, const int64_t* iface_node, const int64_t* if_ptr,
                          const int32_t* if_sub, const int32_t* if_slot, int NGp, const double* Dw,
                          const double* z, double* out);

}  // namespace cutbddc
