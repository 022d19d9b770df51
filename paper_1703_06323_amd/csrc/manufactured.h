// Manufactured-solution accuracy (paper Sect. 5.1): the load of the exact
// solution u = sin(k |x - x0|) and the H^1 / L^2 errors of a discrete
// solution (manufactured.hip); the surface load comes from nitsche.hip.
#pragma once

#include "common.h"

namespace cutbddc {

struct MmsParams {
  double x0[3];   // centre of the radial solution
  double k;       // wave number (5 pi in the paper)
};

// be[c][a] (8 per cell of the concatenated cell space) = the volume load of
// cell c: sum over its kept points of (h^3/512) N_a f.
void launch_mms_volume(hipStream_t st, const BatchDev& b, const MmsParams& m, const double* xi, const double* balls,
                       const int32_t* cellinfo, int64_t n_cells, double* be);
// bg = the cell loads gathered at the DOF nodes (0 elsewhere, and 0
// everywhere when be is null); ud = u at the cube-face nodes (the Dirichlet
// lift, 0 elsewhere).
void launch_mms_gather(hipStream_t st, const BatchDev& b, int64_t nn, const MmsParams& m, const int32_t* cellinfo,
                       const uint8_t* dofmask, const double* be, double* bg, double* ud);
// out[0], out[1] = the squared L2 and H1-seminorm errors of the grid vector
// ug (DOF values plus the lift); err: 2 per cell of scratch.
void launch_mms_errors(hipStream_t st, const BatchDev& b, const MmsParams& m, const double* xi, const double* balls,
                       const int32_t* cellinfo, int64_t n_cells, const double* ug, double* err, double* out);
// b[i] = bg[dof_node[i]] - y[dof_node[i]].
void launch_mms_finish(hipStream_t st, int64_t n_dof, const int64_t* dof_node, const double* bg, const double* y,
                       double* b);

}  // namespace cutbddc
