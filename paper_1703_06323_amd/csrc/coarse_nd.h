// Coarse problem by one level of nested dissection (paper Sect. 3.4: the
// coarse matrix couples two coarse DOFs only through a subdomain that holds
// both).  The subdomain grid is cut into its 8 octants; a coarse DOF held
// only by subdomains of octant o is interior to o, every other one belongs
// to the separator.  Interior DOFs of different octants never share a
// subdomain, so with the interior DOFs first, octant by octant,
//   A_c = [A_oo  A_os; A_so  A_ss],  A_oo block diagonal (one block per octant).
// With A_oo,o = L_o L_o^T, Y_o = L_o^{-1}, W_o = Y_o A_os,o and the Schur
// complement S = A_ss - sum_o W_o^T W_o = L_s L_s^T, Y_s = L_s^{-1}:
//   A_c^{-1} r:  t_o = Y_o r_o,  r_s' = r_s - sum_o W_o^T t_o,
//               x_s = Y_s^T Y_s r_s',  x_o = Y_o^T (t_o - W_o x_s).
// The octant blocks are factored as one batch, so the chain of dependent
// block steps is that of the largest octant plus that of the separator
// instead of that of the whole coarse matrix.
//
// Device layouts (row-major, octants padded to a common order):
//   oid  [8][Lo]       original coarse id of octant row i (-1: padding)
//   sid  [n_s]         original coarse id of separator row s
//   sep  [8][Lso]      separator row coupled to octant column a (-1: padding)
//   pos  [8][n_s]      column of separator row s in octant o (-1: not coupled)
//   Yo   [8][Lo][Lo]   Y_o in the lower triangle, Y_o^T in the strict upper one
//   W    [8][Lo][Lso]  W_o;  WT [8][Lso][Lo] its transpose
//   Ys   [Ls][Ls]      Y_s lower, Y_s^T strict upper (identity on padding rows)
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"

namespace cutbddc {

struct NDDev {
  int Lo = 0, Lso = 0, Ls = 0, n_s = 0;
  const int32_t* oid = nullptr;
  const int32_t* sid = nullptr;
  const int32_t* sep = nullptr;
  const int32_t* pos = nullptr;
};

// Aoo[o] = A_c on octant o's rows and columns (identity on padding), Aos[o]
// = A_c on octant o's rows and its coupled separator columns (zero on
// padding), from the full ldc x ldc matrix Ac.
void launch_nd_gather(hipStream_t st, const NDDev& nd, const double* Ac, int ldc, double* Aoo, double* Aos);
// S = A_ss - sum_o So[o] (So[o] = W_o^T W_o, lower triangle read; the
// octants summed in order 0..7), identity on padding, full storage.
void launch_nd_schur(hipStream_t st, const NDDev& nd, const double* Ac, int ldc, const double* So, double* S);
// WT[o] = W[o]^T for the 8 octant blocks (Lo and Lso multiples of 32).
void launch_nd_transpose(hipStream_t st, const NDDev& nd, const double* W, double* WT);
// y = A_c^{-1} x by the formulas above (x and y in original coarse ids; to,
// rs, us, xs: scratch of 8 Lo, Ls, Ls and Ls values).  Skipped, like the
// other preconditioner kernels, when b.active says the problem has stopped.
void launch_nd_solve(hipStream_t st, const BatchDev& b, const NDDev& nd, const double* Yo, const double* W,
                     const double* WT, const double* Ys, const double* x, double* to, double* rs, double* us,
                     double* xs, double* y);

}  // namespace cutbddc
