// Host-side indexing for cut-cell BDDC (see topology.hpp).
//
// Readings of the paper (which gives no algorithm for these steps), applied
// identically wherever the indexing is built:
//  * DOFs: grid nodes (I,J,K), 1 <= I,J,K <= N-1, touched by an active cell,
//    numbered by ascending node id (strong Dirichlet on the cube faces,
//    Sect. 5.1).
//  * S(xi): ascending ids of the subdomains owning an active cell that
//    contains node xi; interior DOF iff |S| = 1 (Sect. 3.2 classification by
//    the set of subdomains containing an entity).
//  * Objects: connected components of links between axis-adjacent interface
//    DOFs a, b with S(a) = S(b) such that every subdomain of S(a) has an
//    active cell containing the FE edge (a, b).  Corner if one DOF; face if
//    it holds the 4 DOFs of a mesh face whose two cells are active and lie in
//    the two subdomains of S; edge otherwise.  Ordered by smallest DOF id.
//  * Variant 1 (Sect. 4.4): every DOF of a cut FE edge of an edge object is a
//    corner; the other DOFs form sub-edges through non-cut FE edges; a
//    one-DOF sub-edge is a corner.  FE edges are classified exactly against
//    the balls (segment distance for "inside Omega", chord coverage for
//    "outside Omega").
#include "topology.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <utility>

#pragma clang fp contract(off)
#pragma STDC FP_CONTRACT OFF

namespace cutbddc {
namespace {

// Disjoint sets over [0, n): union by size with path halving; every root
// also records the smallest member of its set.
struct UnionFind {
  std::vector<int32_t> p, sz, mn;
  explicit UnionFind(int64_t n) : p(n), sz(n, 1), mn(n) {
    std::iota(p.begin(), p.end(), 0);
    std::iota(mn.begin(), mn.end(), 0);
  }
  int32_t find(int32_t x) {
    while (p[x] != x) {
      p[x] = p[p[x]];
      x = p[x];
    }
    return x;
  }
  void unite(int32_t a, int32_t b) {
    a = find(a);
    b = find(b);
    if (a == b) return;
    if (sz[a] < sz[b]) std::swap(a, b);
    p[b] = a;
    sz[a] += sz[b];
    mn[a] = std::min(mn[a], mn[b]);
  }
  int32_t smallest(int32_t x) { return mn[find(x)]; }
};

inline bool same_set(const int32_t* a, const int32_t* b) {
  for (int t = 0; t < 8; ++t)
    if (a[t] != b[t]) return false;
  return true;
}

}  // namespace

int segment_class(int N, const int64_t ijk[3], int axis, const std::vector<double>& centres,
                  const std::vector<double>& radii) {
  const double h = 1.0 / (double)N;
  double p[3] = {(double)ijk[0] * h, (double)ijk[1] * h, (double)ijk[2] * h};
  const double a = p[axis];
  const double b = (double)(ijk[axis] + 1) * h;
  int o1 = axis == 0 ? 1 : 0;
  int o2 = axis == 2 ? 1 : 2;
  bool interior = true;
  std::vector<std::pair<double, double>> chords;
  const size_t nb = radii.size();
  for (size_t i = 0; i < nb; ++i) {
    const double* c = &centres[3 * i];
    const double r2 = radii[i] * radii[i];
    const double dy = p[o1] - c[o1];
    const double dz = p[o2] - c[o2];
    const double dy2 = dy * dy;
    const double dz2 = dz * dz;
    const double p2 = dy2 + dz2;
    const double t = std::min(std::max(c[axis], a), b);
    const double dd = t - c[axis];
    const double dd2 = dd * dd;
    const double dist2 = p2 + dd2;
    if (!(dist2 > r2)) interior = false;
    if (p2 <= r2) {
      const double half = std::sqrt(r2 - p2);
      chords.emplace_back(c[axis] - half, c[axis] + half);
    }
  }
  if (interior) return 0;
  std::sort(chords.begin(), chords.end());
  double cur = a;
  for (auto& ch : chords) {
    if (ch.first > cur) break;
    cur = std::max(cur, ch.second);
    if (cur >= b) return 1;
  }
  return 2;
}

int build_topology(const Geometry& g, const int32_t* cell_count, Topology& t, std::string& err) {
  const int N = g.N, s = g.s, m = N / s;
  const int64_t N1 = N + 1;
  const int64_t ncell = (int64_t)N * N * N;
  const int64_t nnode = N1 * N1 * N1;
  t = Topology();
  t.N = N;
  t.s = s;
  t.m = m;
  t.n_nodes = nnode;
  t.n_sub = m * m * m;
  auto cell_id = [&](int64_t i, int64_t j, int64_t k) { return i + N * (j + N * k); };
  auto node_id = [&](int64_t I, int64_t J, int64_t K) { return I + N1 * (J + N1 * K); };
  std::vector<int32_t> blk(N);   // block index of each cell layer (avoids divisions)
  for (int i = 0; i < N; ++i) blk[i] = i / s;
  auto sub_of = [&](int64_t i, int64_t j, int64_t k) {
    return (int32_t)(blk[i] + m * (blk[j] + m * blk[k]));
  };
  auto active = [&](int64_t c) { return cell_count[c] > 0; };

  // ---- DOFs ------------------------------------------------------------
  std::vector<uint8_t> touched(nnode, 0);
  for (int64_t k = 0; k < N; ++k)
    for (int64_t j = 0; j < N; ++j)
      for (int64_t i = 0; i < N; ++i) {
        if (!active(cell_id(i, j, k))) continue;
        for (int a = 0; a < 8; ++a)
          touched[node_id(i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1))] = 1;
      }
  t.dof_of_node.assign(nnode, -1);
  for (int64_t K = 1; K < N; ++K)
    for (int64_t J = 1; J < N; ++J)
      for (int64_t I = 1; I < N; ++I) {
        int64_t nd = node_id(I, J, K);
        if (touched[nd]) {
          t.dof_of_node[nd] = (int32_t)t.dof_node.size();
          t.dof_node.push_back(nd);
        }
      }
  // dof_node must be ascending in node id: the loops above run K, J, I
  // outermost to innermost, which is ascending node id order.
  const int64_t nd = (int64_t)t.dof_node.size();
  t.n_dof = nd;

  // ---- floating components ---------------------------------------------
  {
    UnionFind uf(nd);
    std::vector<uint8_t> grounded(nd, 0);
    for (int64_t k = 0; k < N; ++k)
      for (int64_t j = 0; j < N; ++j)
        for (int64_t i = 0; i < N; ++i) {
          if (!active(cell_id(i, j, k))) continue;
          int64_t first = -1;
          bool face = (i == 0 || j == 0 || k == 0 || i == N - 1 || j == N - 1 || k == N - 1);
          for (int a = 0; a < 8; ++a) {
            int32_t d = t.dof_of_node[node_id(i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1))];
            if (d < 0) continue;
            if (first < 0) first = d;
            else uf.unite(first, d);
          }
          if (face && first >= 0) grounded[first] = 1;
        }
    std::vector<uint8_t> rg(nd, 0);
    for (int64_t d = 0; d < nd; ++d)
      if (grounded[d]) rg[uf.find((int32_t)d)] = 1;
    for (int64_t d = 0; d < nd; ++d)
      if (!rg[uf.find((int32_t)d)]) {
        err = "an active component touches no Dirichlet node (singular operator)";
        return -2;
      }
  }

  // ---- subdomain sets S(xi) ----------------------------------------------
  // per DOF node: subdomains of the active cells among its 8 neighbours,
  // ascending (the cells are visited in ascending subdomain order up to
  // duplicates, which are merged by insertion)
  t.S.assign(nd * 8, -1);
  t.card.assign(nd, 0);
  for (int64_t K = 1; K < N; ++K)
    for (int64_t J = 1; J < N; ++J)
      for (int64_t I = 1; I < N; ++I) {
    const int32_t d = t.dof_of_node[node_id(I, J, K)];
    if (d < 0) continue;
    int32_t* Sd = &t.S[(int64_t)d * 8];
    int c = 0;
    for (int u = 0; u < 8; ++u) {
      const int64_t ci = I - 1 + (u & 1), cj = J - 1 + ((u >> 1) & 1), ck = K - 1 + ((u >> 2) & 1);
      if (!active(cell_id(ci, cj, ck))) continue;
      const int32_t w = sub_of(ci, cj, ck);
      bool found = false;
      for (int q = 0; q < c; ++q)
        if (Sd[q] == w) found = true;
      if (found) continue;
      int q = c;
      while (q > 0 && Sd[q - 1] > w) {
        Sd[q] = Sd[q - 1];
        --q;
      }
      Sd[q] = w;
      ++c;
    }
    t.card[d] = (uint8_t)c;
      }

  // ---- links and objects -------------------------------------------------
  UnionFind uf(nd);
  struct Link {
    int32_t a, b;
    int8_t axis;
  };
  std::vector<Link> links;
  for (int64_t K = 1; K < N; ++K)
    for (int64_t J = 1; J < N; ++J)
      for (int64_t I = 1; I < N; ++I) {
    const int64_t node = node_id(I, J, K);
    const int32_t a = t.dof_of_node[node];
    if (a < 0 || t.card[a] < 2) continue;
    int64_t ijk[3] = {I, J, K};
    for (int axis = 0; axis < 3; ++axis) {
      int64_t step = axis == 0 ? 1 : (axis == 1 ? N1 : N1 * N1);
      if (ijk[axis] + 1 > N) continue;
      int32_t b = t.dof_of_node[node + step];
      if (b < 0 || t.card[b] < 2) continue;
      if (!same_set(&t.S[(int64_t)a * 8], &t.S[(int64_t)b * 8])) continue;
      int o1 = axis == 0 ? 1 : 0;
      int o2 = axis == 2 ? 1 : 2;
      int32_t St[4];
      int nst = 0;
      for (int u = -1; u <= 0; ++u)
        for (int v = -1; v <= 0; ++v) {
          int64_t c3[3] = {I, J, K};
          c3[o1] += u;
          c3[o2] += v;
          if (c3[0] < 0 || c3[1] < 0 || c3[2] < 0 || c3[0] >= N || c3[1] >= N || c3[2] >= N)
            continue;
          if (!active(cell_id(c3[0], c3[1], c3[2]))) continue;
          St[nst++] = sub_of(c3[0], c3[1], c3[2]);
        }
      bool full = true;
      for (int q = 0; q < t.card[a]; ++q) {
        int32_t w = t.S[(int64_t)a * 8 + q];
        bool present = false;
        for (int z = 0; z < nst; ++z)
          if (St[z] == w) present = true;
        if (!present) full = false;
      }
      if (!full) continue;
      links.push_back({(int32_t)a, b, (int8_t)axis});
      uf.unite((int32_t)a, b);
    }
      }
  // component root = smallest DOF id of the component
  std::vector<int32_t> comp_of(nd, -1);
  std::vector<int64_t> roots;
  for (int64_t a = 0; a < nd; ++a) {
    if (t.card[a] < 2) continue;
    if (uf.smallest((int32_t)a) == a) {
      comp_of[a] = (int32_t)roots.size();
      roots.push_back(a);
    }
  }
  for (int64_t a = 0; a < nd; ++a)
    if (t.card[a] >= 2) comp_of[a] = comp_of[uf.smallest((int32_t)a)];
  const int64_t ncomp = (int64_t)roots.size();
  std::vector<uint8_t> is_face(ncomp, 0);
  for (int axis = 0; axis < 3; ++axis) {
    int o1 = axis == 0 ? 1 : 0;
    int o2 = axis == 2 ? 1 : 2;
    // cells lo on the last layer of a block, hi across the block boundary
    for (int64_t plane = s - 1; plane + 1 < N; plane += s)
      for (int64_t v = 0; v < N; ++v)
        for (int64_t u = 0; u < N; ++u) {
          int64_t c3[3];
          c3[axis] = plane;
          c3[o1] = u;
          c3[o2] = v;
          const int64_t i = c3[0], j = c3[1], k = c3[2];
          int64_t lo = cell_id(i, j, k);
          int64_t h3[3] = {i, j, k};
          h3[axis] += 1;
          int64_t hi = cell_id(h3[0], h3[1], h3[2]);
          if (!active(lo) || !active(hi)) continue;
          int32_t fd[4];
          int q = 0;
          bool ok = true;
          for (int u = 0; u <= 1; ++u)
            for (int v = 0; v <= 1; ++v) {
              int64_t n3[3] = {i, j, k};
              n3[axis] += 1;
              n3[o1] += u;
              n3[o2] += v;
              int32_t d = t.dof_of_node[node_id(n3[0], n3[1], n3[2])];
              if (d < 0 || t.card[d] < 2) ok = false;
              fd[q++] = d;
            }
          if (!ok) continue;
          int32_t o = comp_of[fd[0]];
          if (comp_of[fd[1]] != o || comp_of[fd[2]] != o || comp_of[fd[3]] != o) continue;
          const int32_t* Sf = &t.S[(int64_t)fd[0] * 8];
          if (t.card[fd[0]] != 2) continue;
          int32_t w1 = sub_of(i, j, k), w2 = sub_of(h3[0], h3[1], h3[2]);
          if (std::min(w1, w2) == Sf[0] && std::max(w1, w2) == Sf[1]) is_face[o] = 1;
        }
  }
  // members per component (ascending DOF ids)
  std::vector<int64_t> cptr(ncomp + 1, 0);
  for (int64_t a = 0; a < nd; ++a)
    if (comp_of[a] >= 0) cptr[comp_of[a] + 1]++;
  for (int64_t c = 0; c < ncomp; ++c) cptr[c + 1] += cptr[c];
  std::vector<int64_t> cmem(cptr[ncomp]);
  {
    std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
    for (int64_t a = 0; a < nd; ++a)
      if (comp_of[a] >= 0) cmem[fill[comp_of[a]]++] = a;
  }
  struct Obj {
    std::vector<int64_t> dofs;
    int8_t type;
  };
  std::vector<Obj> objs;
  objs.reserve(ncomp);
  const bool v1 = g.variant == 1 && !g.radii.empty();
  // links grouped per component (for variant 1)
  std::vector<int64_t> lptr, lidx;
  if (v1) {
    lptr.assign(ncomp + 1, 0);
    for (auto& L : links) lptr[comp_of[L.a] + 1]++;
    for (int64_t c = 0; c < ncomp; ++c) lptr[c + 1] += lptr[c];
    lidx.resize(links.size());
    std::vector<int64_t> fill(lptr.begin(), lptr.end() - 1);
    for (int64_t e = 0; e < (int64_t)links.size(); ++e) lidx[fill[comp_of[links[e].a]]++] = e;
  }
  for (int64_t c = 0; c < ncomp; ++c) {
    std::vector<int64_t> dofs(cmem.begin() + cptr[c], cmem.begin() + cptr[c + 1]);
    int8_t type = dofs.size() == 1 ? OBJ_CORNER : (is_face[c] ? OBJ_FACE : OBJ_EDGE);
    if (!(v1 && type == OBJ_EDGE)) {
      objs.push_back({std::move(dofs), type});
      continue;
    }
    // variant 1: classify the component's FE edges
    std::vector<int8_t> cls;
    bool any_cut = false;
    for (int64_t q = lptr[c]; q < lptr[c + 1]; ++q) {
      const Link& L = links[lidx[q]];
      int64_t node = t.dof_node[L.a];
      int64_t ijk[3] = {node % N1, (node / N1) % N1, node / (N1 * N1)};
      int8_t k = (int8_t)segment_class(N, ijk, L.axis, g.centres, g.radii);
      cls.push_back(k);
      if (k == 2) any_cut = true;
    }
    if (!any_cut) {
      objs.push_back({std::move(dofs), type});
      continue;
    }
    std::vector<int64_t> cut_dofs;
    for (int64_t q = lptr[c]; q < lptr[c + 1]; ++q)
      if (cls[q - lptr[c]] == 2) {
        cut_dofs.push_back(links[lidx[q]].a);
        cut_dofs.push_back(links[lidx[q]].b);
      }
    std::sort(cut_dofs.begin(), cut_dofs.end());
    cut_dofs.erase(std::unique(cut_dofs.begin(), cut_dofs.end()), cut_dofs.end());
    for (int64_t x : cut_dofs) objs.push_back({{x}, OBJ_CORNER});
    std::vector<int64_t> rest;
    for (int64_t x : dofs)
      if (!std::binary_search(cut_dofs.begin(), cut_dofs.end(), x)) rest.push_back(x);
    if (rest.empty()) continue;
    UnionFind lu((int64_t)rest.size());
    auto pos = [&](int64_t x) -> int64_t {
      auto it = std::lower_bound(rest.begin(), rest.end(), x);
      return (it != rest.end() && *it == x) ? (int64_t)(it - rest.begin()) : -1;
    };
    for (int64_t q = lptr[c]; q < lptr[c + 1]; ++q) {
      if (cls[q - lptr[c]] == 2) continue;
      int64_t pa = pos(links[lidx[q]].a), pb = pos(links[lidx[q]].b);
      if (pa >= 0 && pb >= 0) lu.unite((int32_t)pa, (int32_t)pb);
    }
    std::vector<std::vector<int64_t>> parts;
    std::vector<int64_t> part_of(rest.size(), -1);
    for (int64_t r = 0; r < (int64_t)rest.size(); ++r) {
      int64_t root = lu.find((int32_t)r);
      if (part_of[root] < 0) {
        part_of[root] = (int64_t)parts.size();
        parts.emplace_back();
      }
      parts[part_of[root]].push_back(rest[r]);
    }
    for (auto& pdofs : parts) {
      int8_t ty = pdofs.size() == 1 ? OBJ_CORNER : OBJ_EDGE;
      objs.push_back({std::move(pdofs), ty});
    }
  }
  std::sort(objs.begin(), objs.end(),
            [](const Obj& x, const Obj& y) { return x.dofs[0] < y.dofs[0]; });
  const int64_t nobj = (int64_t)objs.size();
  t.obj_ptr.assign(nobj + 1, 0);
  t.obj_type.resize(nobj);
  t.coarse_of_obj.assign(nobj, -1);
  std::vector<int32_t> obj_of_dof(nd, -1);
  for (int64_t o = 0; o < nobj; ++o) {
    t.obj_ptr[o + 1] = t.obj_ptr[o] + (int64_t)objs[o].dofs.size();
    t.obj_type[o] = objs[o].type;
    for (int64_t x : objs[o].dofs) {
      t.obj_dofs.push_back(x);
      obj_of_dof[x] = (int32_t)o;
    }
    bool selected = (g.objects == 0) || objs[o].type != OBJ_FACE;
    if (selected) t.coarse_of_obj[o] = t.n_coarse++;
  }

  // ---- per-subdomain lists ---------------------------------------------
  const int32_t ns = t.n_sub;
  t.nI.assign(ns, 0);
  t.nG.assign(ns, 0);
  t.nC.assign(ns, 0);
  int64_t n_iface = 0;
  for (int64_t a = 0; a < nd; ++a) {
    if (t.card[a] == 1) t.nI[t.S[a * 8]]++;
    else {
      n_iface++;
      for (int q = 0; q < t.card[a]; ++q) t.nG[t.S[a * 8 + q]]++;
    }
  }
  t.n_iface = (int32_t)n_iface;
  t.I_ptr.assign(ns + 1, 0);
  t.G_ptr.assign(ns + 1, 0);
  for (int32_t w = 0; w < ns; ++w) {
    t.I_ptr[w + 1] = t.I_ptr[w] + t.nI[w];
    t.G_ptr[w + 1] = t.G_ptr[w] + t.nG[w];
    t.maxI = std::max(t.maxI, t.nI[w]);
    t.maxG = std::max(t.maxG, t.nG[w]);
  }
  t.I_nodes.resize(t.I_ptr[ns]);
  t.G_nodes.resize(t.G_ptr[ns]);
  t.G_obj.assign(t.G_ptr[ns], -1);
  t.iface_node.resize(n_iface);
  t.if_ptr.assign(n_iface + 1, 0);
  t.if_sub.reserve(t.G_ptr[ns]);
  t.if_slot.reserve(t.G_ptr[ns]);
  {
    std::vector<int64_t> fi(t.I_ptr.begin(), t.I_ptr.end() - 1);
    std::vector<int64_t> fg(t.G_ptr.begin(), t.G_ptr.end() - 1);
    int64_t q = 0;
    for (int64_t a = 0; a < nd; ++a) {
      if (t.card[a] == 1) {
        t.I_nodes[fi[t.S[a * 8]]++] = t.dof_node[a];
      } else {
        t.iface_node[q] = t.dof_node[a];
        for (int z = 0; z < t.card[a]; ++z) {
          int32_t w = t.S[a * 8 + z];
          int64_t slot = fg[w]++;
          t.G_nodes[slot] = t.dof_node[a];
          t.if_sub.push_back(w);
          t.if_slot.push_back((int32_t)(slot - t.G_ptr[w]));
        }
        t.if_ptr[q + 1] = (int64_t)t.if_sub.size();
        ++q;
      }
    }
  }
  // coarse DOFs per subdomain (ascending coarse id) and the local row of
  // each interface slot
  std::vector<std::vector<int32_t>> sub_c(ns);
  for (int64_t o = 0; o < nobj; ++o) {
    int32_t cid = t.coarse_of_obj[o];
    if (cid < 0) continue;
    int64_t d0 = objs[o].dofs[0];
    for (int z = 0; z < t.card[d0]; ++z) sub_c[t.S[d0 * 8 + z]].push_back(cid);
  }
  t.C_ptr.assign(ns + 1, 0);
  for (int32_t w = 0; w < ns; ++w) {
    std::sort(sub_c[w].begin(), sub_c[w].end());
    t.nC[w] = (int32_t)sub_c[w].size();
    t.maxC = std::max(t.maxC, t.nC[w]);
    t.C_ptr[w + 1] = t.C_ptr[w] + t.nC[w];
    for (int32_t c : sub_c[w]) t.C_ids.push_back(c);
  }
  for (int32_t w = 0; w < ns; ++w) {
    for (int64_t j = t.G_ptr[w]; j < t.G_ptr[w + 1]; ++j) {
      int32_t dof = t.dof_of_node[t.G_nodes[j]];
      int32_t o = obj_of_dof[dof];
      int32_t cid = t.coarse_of_obj[o];
      if (cid < 0) continue;
      auto b = t.C_ids.begin() + t.C_ptr[w], e = t.C_ids.begin() + t.C_ptr[w + 1];
      auto it = std::lower_bound(b, e, cid);
      t.G_obj[j] = (int32_t)(it - b);
    }
  }
  // coarse DOF -> (subdomain, row), ascending subdomain
  t.cs_ptr.assign(t.n_coarse + 1, 0);
  for (int32_t w = 0; w < ns; ++w)
    for (int64_t q = t.C_ptr[w]; q < t.C_ptr[w + 1]; ++q) t.cs_ptr[t.C_ids[q] + 1]++;
  for (int32_t c = 0; c < t.n_coarse; ++c) t.cs_ptr[c + 1] += t.cs_ptr[c];
  t.cs_sub.resize(t.cs_ptr[t.n_coarse]);
  t.cs_row.resize(t.cs_ptr[t.n_coarse]);
  {
    std::vector<int64_t> fill(t.cs_ptr.begin(), t.cs_ptr.end() - 1);
    for (int32_t w = 0; w < ns; ++w)
      for (int64_t q = t.C_ptr[w]; q < t.C_ptr[w + 1]; ++q) {
        int32_t c = t.C_ids[q];
        t.cs_sub[fill[c]] = w;
        t.cs_row[fill[c]] = (int32_t)(q - t.C_ptr[w]);
        fill[c]++;
      }
  }
  return 0;
}

}  // namespace cutbddc
