// Device indexing of the cut-cell BDDC method for every problem of a
// context at once: DOF numbering, subdomain sets S(xi), interface objects
// and their types (Sect. 3.2), the variant-1 splitting of cut coarse edges
// (Sect. 4.4), coarse numbering and the per-subdomain index maps consumed
// by the assembly, factorisation and preconditioner kernels.
//
// Everything is indexed by the concatenated node space of the context
// (problem segments aligned to SEG_ALIGN).  Within a problem, ascending node
// id is ascending DOF id, so "smallest DOF of an object" is its smallest
// node, which is the root that the union-find passes converge to.
#pragma once

#include "common.h"

namespace cutbddc {

enum ObjKind : int8_t { KIND_CORNER = 0, KIND_EDGE = 1, KIND_FACE = 2 };

// Four 32-bit counters scanned together.
struct Count4 {
  int32_t x, y, z, w;
};

// Per-node work arrays of the device indexing (nn entries each unless noted).
struct IndexWork {
  uint8_t* smask;     // S(xi) as bits over the 2x2x2 blocks around the node; 0: not a DOF
  uint8_t* link;      // bits 0-2: link to the +axis neighbour; bits 3-5: that FE edge is cut
  uint8_t* face;      // at pass-1 object roots: the object holds a subdomain face
  uint8_t* cutdof;    // DOF incident to a cut FE edge of an edge object
  uint8_t* ground;    // at floating-check roots: the component touches the cube boundary
  int32_t* par0;      // union-find over DOF nodes joined by active cells (floating check)
  int32_t* par1;      // objects before the variant-1 split
  int32_t* par2;      // objects after it
  int32_t* size1;     // members per pass-1 root
  int32_t* size2;     // members per final root
  int32_t* gif;       // global interface index of an interface DOF, else -1
  int32_t* gifp;      // offset of its (subdomain, slot) list
  int32_t* oidx;      // at final roots: global object index
  int32_t* ocid;      // at selected final roots: global coarse id, else -1
  int32_t* ocsp;      // at selected final roots: offset of its (subdomain, row) list
  Count4* bsum;       // scan block sums (scan_blocks(max(n_cells, nn)) entries)
  // per-problem results ([P+1] each; entry P holds the totals)
  Count4* seg_cells;  // active cells, geometrically cut cells, cut cells with stored matrices
  Count4* seg_nodes;  // DOFs, interface DOFs, interface list length
  Count4* seg_obj;    // objects, coarse DOFs, coarse list length
  int32_t* floating;  // [P] 1 if an active component touches no Dirichlet node
};

int64_t index_scan_blocks(int64_t n);

// Cell pass: cellinfo (inactive / uncut / cut-matrix index), the list of
// stored cut cells (global cell ids, cut_cells sized n_cells_total) and the
// per-problem cell counts.  store_cut = 0: every active cell is integrated
// as uncut.
void launch_index_cells(hipStream_t st, const BatchDev& b, int64_t n_cells_total, const int32_t* count,
                        int store_cut, const IndexWork& w, int32_t* cellinfo, int64_t* cut_cells);

// Inputs of the variant-2 split (Sect. 4.5): the cell data and integrated
// cut-cell matrices, and the diagonal of the uncut reference stiffness
// (device, 8 values); stiffness = 0 (topological weights, constant on every
// object) leaves the standard objects.
struct V2Inputs {
  int stiffness;
  const int32_t* cellinfo;
  const double* kappa;
  const double* Kc;
  const double* kdiag;
};
// "The same weighting coefficient, up to machine precision" (Sect. 4.5):
// coefficients lie in [0, 1].
constexpr double V2_TOL = 1e-12;

// Node passes up to the per-subdomain counts: DOFs, S sets, the floating
// check, objects, variant 1 (variant = 1; problems without balls have no
// cut FE edges) or variant 2 (variant = 2: the cell info and cut-cell
// matrices of v2 must be complete), coarse selection (objects = 0: every
// object; 1: corners and edges).  Writes
// dofmask [nn], dof_node [n_dof] (global node ids; sized nn), and per
// subdomain nI, nG, nC.
void launch_index_nodes(hipStream_t st, const BatchDev& b, int64_t n_cells_total, int64_t nn, int ns,
                        const int32_t* sub_off, const int32_t* count, const double* balls, int variant, int objects,
                        const V2Inputs& v2, const IndexWork& w, uint8_t* dofmask, int64_t* dof_node, int32_t* nI,
                        int32_t* nG, int32_t* nC);

// Per-subdomain index maps with padded sizes NIp, NGp, NCp (see SubDev) and
// the interface / coarse lists:
//   if_ptr [n_iface+1], if_sub/if_slot [interface list length],
//   iface_node [n_iface], cs_ptr [n_coarse+1], cs_sub/cs_row [coarse list
//   length], coarse_prob [n_coarse], sub_prob/sub_blk [ns].
struct IndexMaps {
  int NIp, NGp, NCp;
  int64_t* I_idx;
  int64_t* G_idx;
  int32_t* G_obj;
  int32_t* C_ids;
  int32_t* bloc;
  int64_t* if_ptr;
  int32_t* if_sub;
  int32_t* if_slot;
  int64_t* iface_node;
  int64_t* cs_ptr;
  int32_t* cs_sub;
  int32_t* cs_row;
  int32_t* coarse_prob;
  int32_t* sub_prob;
  int32_t* sub_blk;
};
void launch_index_fill(hipStream_t st, const BatchDev& b, int ns, int s, const int32_t* sub_off,
                       const IndexWork& w, const IndexMaps& m);

}  // namespace cutbddc
