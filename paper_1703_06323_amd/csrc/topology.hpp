// Host-side indexing of the cut-cell BDDC method: DOF numbering, subdomain
// node sets, interface objects (Sect. 3.2), variant-1 splitting of cut coarse
// edges (Sect. 4.4), coarse numbering and the per-subdomain index maps that
// the device kernels consume.  Pure C++ (no HIP), integer work except the
// exact segment/ball tests of variant 1, which are compiled without FP
// contraction so that their results are reproducible.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace cutbddc {

enum ObjType : int8_t { OBJ_CORNER = 0, OBJ_EDGE = 1, OBJ_FACE = 2 };

struct Geometry {
  int N = 0;                     // cells per axis
  int s = 0;                     // subdomain block size (cells)
  std::vector<double> centres;   // [nb*3]
  std::vector<double> radii;     // [nb]
  int objects = 0;               // 0 cef, 1 ce
  int variant = 1;               // 0 standard, 1 split cut edges
};

struct Topology {
  int N = 0, s = 0, m = 0;
  int64_t n_nodes = 0;           // (N+1)^3
  int64_t n_dof = 0;
  std::vector<int32_t> dof_of_node;   // [(N+1)^3], -1 if not a DOF
  std::vector<int64_t> dof_node;      // [n_dof]
  std::vector<int32_t> S;             // [n_dof*8] ascending subdomain ids, -1 padded
  std::vector<uint8_t> card;          // [n_dof]

  // objects, ordered by smallest DOF id
  std::vector<int64_t> obj_ptr;       // [n_obj+1]
  std::vector<int64_t> obj_dofs;      // DOF ids, ascending within an object
  std::vector<int8_t> obj_type;
  std::vector<int32_t> coarse_of_obj; // -1 if not selected
  int32_t n_coarse = 0;
  int32_t n_iface = 0;

  // per subdomain (m^3): interior / interface DOF lists as grid node ids
  int32_t n_sub = 0;
  std::vector<int32_t> nI, nG, nC;    // counts
  int32_t maxI = 0, maxG = 0, maxC = 0;
  std::vector<int64_t> I_ptr, G_ptr;  // CSR into I_nodes / G_nodes
  std::vector<int64_t> I_nodes, G_nodes;
  std::vector<int64_t> C_ptr;         // coarse ids per subdomain (ascending)
  std::vector<int32_t> C_ids;
  std::vector<int32_t> G_obj;         // per (subdomain, interface slot): local coarse row or -1

  // interface DOF -> (subdomain, interface slot), ascending subdomain
  std::vector<int64_t> iface_node;    // [n_iface] grid node ids (ascending)
  std::vector<int64_t> if_ptr;        // [n_iface+1]
  std::vector<int32_t> if_sub, if_slot;
  // coarse DOF -> (subdomain, local coarse row), ascending subdomain
  std::vector<int64_t> cs_ptr;        // [n_coarse+1]
  std::vector<int32_t> cs_sub, cs_row;
};

// Builds the full indexing from per-cell kept-point counts (count > 0 means
// active).  Returns 0 on success; on failure a negative code and a message.
//   -2: an active component without Dirichlet node (singular operator)
int build_topology(const Geometry& g, const int32_t* cell_count, Topology& t,
                   std::string& err);

// Empties every array of t but keeps their capacity for the next build.
void reset_topology(Topology& t);

// Runs f(begin, end) over chunks of [0, n) on the indexing thread pool.
void parallel_rows(int64_t n, const std::function<void(int64_t, int64_t)>& f);

// On the calling thread, run the loops of build_topology inline (for
// threads that each index one problem of a batch concurrently).
void set_serial_indexing(bool serial);

// Threads of the indexing pool (including the caller).
int indexing_threads();

// Exact class of the FE edge from grid node (I,J,K) to (I,J,K)+e_axis:
// 0 interior (edge inside Omega), 1 exterior (edge misses Omega), 2 cut.
int segment_class(int N, const int64_t ijk[3], int axis, const std::vector<double>& centres,
                  const std::vector<double>& radii);

}  // namespace cutbddc
