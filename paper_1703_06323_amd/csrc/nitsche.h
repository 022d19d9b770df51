// Nitsche's weak Dirichlet condition on the ball surfaces (paper Sect. 2.2,
// eq. local-eigenvals): the sphere rule of every ball and the launcher that
// adds the surface terms to the stored unit stiffness of the cut cells.
#pragma once

#include "common.h"

namespace cutbddc {

// Stiffness of a cut cell's void part in the eigenproblem, relative to a
// whole cell's: it bounds lambda_max where the kept-point rule leaves the
// volume form singular on the complement of the constants.
constexpr double NITSCHE_BETA_REG = 1e-6;

struct NitscheBall {
  double r;                 // radius
  int32_t nt, nphi;         // Gauss-Legendre nodes in cos(theta), midpoint nodes in phi
  int32_t off_t, off_phi;   // offsets into t / w and cphi / sphi
};

// Device tables of the sphere rules of all balls of a context (in the
// order of the ball array).
struct NitscheRule {
  const NitscheBall* ball;
  const double* t;      // nodes in [-1, 1], ascending
  const double* w;      // Gauss-Legendre weights
  const double* cphi;   // cos(2 pi (k + 1/2) / nphi)
  const double* sphi;   // sin(...)
  const double* dphi;   // 2 pi / nphi per ball
  const double* kref;   // unit stiffness of a whole cell, 8x8 row-major
};

// Nodes and weights of the n-point Gauss-Legendre rule on [-1, 1],
// ascending (Newton iteration on the Legendre recurrence).
void gauss_legendre(int n, double* x, double* w);

// Adds the Nitsche terms with homogeneous data to the unit stiffness Kc of
// each cut cell (packed, cut cells in cut_cells order); status receives the
// number of cells whose eigenproblem broke down.
// beta receives beta_e (unit frame) of every cut cell.
void launch_nitsche(hipStream_t st, const BatchDev& b, const NitscheRule& rule, const double* balls,
                    const int64_t* cut_cells, int64_t n_cut, double* Kc, double* beta, int* status);

struct MmsParams;
// Adds to be[cell][a] the surface load of the exact solution m: Neumann
// data grad u . n on every one of the n_cells cells that holds a kept
// sphere point (nitsche = 0), or the Nitsche data terms
// h w_unit (beta_e N_a - n . grad N_a) u on the n_cut cut cells (nitsche =
// 1, beta from launch_nitsche).
void launch_surface_load(hipStream_t st, const BatchDev& b, const NitscheRule& rule, const double* balls,
                         int64_t n_cells, const int64_t* cut_cells, int64_t n_cut, int nitsche, const double* beta,
                         const MmsParams& m, double* be);

}  // namespace cutbddc
