// Shared declarations for the cutbddc device kernels and their host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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

// Index of entry (a, b) of a symmetric 8x8 matrix in its packed upper
// triangle (row by row).
__host__ __device__ inline int pack_index(int a, int b) {
  int r = a < b ? a : b;
  int c = a < b ? b : a;
  return r * 8 - (r * (r - 1)) / 2 + (c - r);
}

// ---- launchers (defined in the .hip files) --------------------------------
// integrate.hip
void launch_classify(hipStream_t st, int N, const double* xi, const double* balls, int nb,
                     int32_t* count);
void launch_integrate_cut(hipStream_t st, int N, const double* xi, const double* balls, int nb,
                          const int64_t* cut_cells, int64_t n_cut, double* Kc, double* Mc);
// operator.hip
void set_reference_matrices(const double* Kref, const double* Mref);
void launch_apply_A(hipStream_t st, GridDesc g, const int32_t* cellinfo, const double* kappa,
                    const double* Kc, const uint8_t* dofmask, const double* x, double* y);
void launch_load(hipStream_t st, GridDesc g, const int32_t* cellinfo, const double* Mc,
                 const uint8_t* outmask, const double* f, double* b);
void launch_grad_theta(hipStream_t st, GridDesc g, const int32_t* cellinfo, const double* kappa,
                       const double* Kc, const double* u, const double* lam, double* out);
void launch_scatter_dofs(hipStream_t st, int64_t n, const int64_t* dof_node, const double* src,
                         double* grid);
void launch_gather_dofs(hipStream_t st, int64_t n, const int64_t* dof_node, const double* grid,
                        double* dst);
void launch_fill(hipStream_t st, int64_t n, double v, double* x);
// deterministic dot product: result written to out (device)
void launch_dot(hipStream_t st, int64_t n, const double* x, const double* y, double* partial,
                double* out);
int dot_partials();
void launch_cg_update_xr(hipStream_t st, int64_t n, const double* S, const double* p, const double* q, double* x,
                         double* r);
void launch_cg_update_p(hipStream_t st, int64_t n, double* S, const double* z, double* p);
void convert_to_float(hipStream_t st, int64_t n, const double* a, float* b);

}  // namespace cutbddc
