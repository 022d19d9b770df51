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
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <numeric>
#include <thread>
#include <utility>

#pragma clang fp contract(off)
#pragma STDC FP_CONTRACT OFF

namespace cutbddc {
namespace {

// Disjoint sets over [0, n): union by size with path halving; every root
// also records the smallest member of its set.
struct UnionFind {
  std::vector<int32_t> p, sz, mn;
  UnionFind() = default;
  explicit UnionFind(int64_t n) { reset(n); }
  void reset(int64_t n) {
    p.resize(n);
    sz.assign(n, 1);
    mn.resize(n);
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

// Fixed pool of worker threads for the data-parallel loops of the indexing
// (created once per process; at most 16 workers).  Each run has a
// generation number; tasks are claimed and counted under the mutex, and only
// while the claimer's generation is the current one, so every task of a run
// is executed exactly once and the completion count of a run ends at its
// task count.
class Pool {
 public:
  static Pool& get() {
    static Pool* p = new Pool();   // intentionally leaked at exit
    return *p;
  }
  int size() const { return (int)workers_.size() + 1; }
  // Runs f(task) for task in [0, ntasks) on the workers and the caller.
  void run(int ntasks, const std::function<void(int)>& f) {
    if (ntasks <= 1 || workers_.empty()) {
      for (int t = 0; t < ntasks; ++t) f(t);
      return;
    }
    std::lock_guard<std::mutex> one_run(run_mu_);
    uint64_t g;
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = &f;
      ntasks_ = ntasks;
      next_ = 0;
      done_ = 0;
      g = ++gen_;
    }
    cv_.notify_all();
    work(g);
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [&] { return done_ == ntasks_; });
    job_ = nullptr;
  }

 private:
  Pool() {
    int hw = (int)std::thread::hardware_concurrency();
    int n = std::max(0, std::min(hw, 16) - 1);
    for (int i = 0; i < n; ++i) workers_.emplace_back([this] { loop(); });
    for (auto& w : workers_) w.detach();
  }
  void work(uint64_t g) {
    std::unique_lock<std::mutex> lk(mu_);
    while (gen_ == g && next_ < ntasks_) {
      const int t = next_++;
      const std::function<void(int)>* job = job_;
      lk.unlock();
      (*job)(t);
      lk.lock();
      if (++done_ == ntasks_) done_cv_.notify_all();
    }
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return gen_ != seen; });
        seen = gen_;
      }
      work(seen);
    }
  }
  std::vector<std::thread> workers_;
  std::mutex run_mu_;   // one run at a time
  std::mutex mu_;       // guards everything below
  std::condition_variable cv_, done_cv_;
  const std::function<void(int)>* job_ = nullptr;
  int ntasks_ = 0, next_ = 0, done_ = 0;
  uint64_t gen_ = 0;
};

// Set on threads that each index a whole problem of a batch: their loops run
// inline instead of on the shared pool.
thread_local bool t_serial = false;

// f(begin, end) over [0, n) split into contiguous chunks.
template <typename F>
void parallel_for(int64_t n, F&& f) {
  if (n <= 0) return;
  if (t_serial) {
    f(0, n);
    return;
  }
  const int chunks = (int)std::min<int64_t>(n, 4 * Pool::get().size());
  std::function<void(int)> task = [&](int c) {
    const int64_t b = n * c / chunks, e = n * (c + 1) / chunks;
    if (b < e) f(b, e);
  };
  Pool::get().run(chunks, task);
}

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

void reset_topology(Topology& t) {
  // sizes back to zero, capacities kept (repeated builds reuse the memory)
  t.N = t.s = t.m = 0;
  t.n_nodes = t.n_dof = 0;
  t.n_coarse = t.n_iface = 0;
  t.n_sub = 0;
  t.maxI = t.maxG = t.maxC = 0;
  for (auto* v : {&t.dof_node, &t.obj_ptr, &t.obj_dofs, &t.I_ptr, &t.G_ptr, &t.I_nodes, &t.G_nodes, &t.C_ptr,
                  &t.iface_node, &t.if_ptr, &t.cs_ptr})
    v->clear();
  for (auto* v : {&t.dof_of_node, &t.S, &t.coarse_of_obj, &t.nI, &t.nG, &t.nC, &t.C_ids, &t.G_obj, &t.if_sub,
                  &t.if_slot, &t.cs_sub, &t.cs_row})
    v->clear();
  t.card.clear();
  t.obj_type.clear();
}

int build_topology(const Geometry& g, const int32_t* cell_count, Topology& t, std::string& err) {
  const int N = g.N, s = g.s, m = N / s;
  const int64_t N1 = N + 1;
  const int64_t nnode = N1 * N1 * N1;
  const int s1 = s + 1;
  const int64_t nbn = (int64_t)s1 * s1 * s1;   // nodes of one block
  reset_topology(t);
  t.N = N;
  t.s = s;
  t.m = m;
  t.n_nodes = nnode;
  t.n_sub = m * m * m;
  const int32_t ns = t.n_sub;
  auto cell_id = [&](int64_t i, int64_t j, int64_t k) { return i + N * (j + N * k); };
  auto node_id = [&](int64_t I, int64_t J, int64_t K) { return I + N1 * (J + N1 * K); };
  std::vector<int32_t> blk(N);   // block index of each cell layer (avoids divisions)
  for (int i = 0; i < N; ++i) blk[i] = i / s;
  auto sub_of = [&](int64_t i, int64_t j, int64_t k) {
    return (int32_t)(blk[i] + m * (blk[j] + m * blk[k]));
  };
  auto active = [&](int64_t c) { return cell_count[c] > 0; };
  auto active_at = [&](int64_t i, int64_t j, int64_t k) {
    return i >= 0 && j >= 0 && k >= 0 && i < N && j < N && k < N && cell_count[cell_id(i, j, k)] > 0;
  };

  // ---- DOFs: interior nodes touched by an active cell, ascending ---------
  t.dof_of_node.assign(nnode, -1);
  std::vector<int64_t> slab_count(N1 + 1, 0);
  auto is_dof = [&](int64_t I, int64_t J, int64_t K) {
    if (I < 1 || J < 1 || K < 1 || I > N - 1 || J > N - 1 || K > N - 1) return false;
    for (int u = 0; u < 8; ++u)
      if (active_at(I - 1 + (u & 1), J - 1 + ((u >> 1) & 1), K - 1 + ((u >> 2) & 1))) return true;
    return false;
  };
  parallel_for(N1, [&](int64_t kb, int64_t ke) {
    for (int64_t K = kb; K < ke; ++K) {
      int64_t c = 0;
      for (int64_t J = 0; J <= N; ++J)
        for (int64_t I = 0; I <= N; ++I)
          if (is_dof(I, J, K)) {
            t.dof_of_node[node_id(I, J, K)] = 1;
            ++c;
          }
      slab_count[K + 1] = c;
    }
  });
  for (int64_t K = 0; K < N1; ++K) slab_count[K + 1] += slab_count[K];
  const int64_t nd = slab_count[N1];
  t.n_dof = nd;
  t.dof_node.resize(nd);
  parallel_for(N1, [&](int64_t kb, int64_t ke) {
    for (int64_t K = kb; K < ke; ++K) {
      int64_t d = slab_count[K];
      for (int64_t J = 0; J <= N; ++J)
        for (int64_t I = 0; I <= N; ++I) {
          const int64_t n = node_id(I, J, K);
          if (t.dof_of_node[n] == 1) {
            t.dof_of_node[n] = (int32_t)d;
            t.dof_node[d] = n;
            ++d;
          } else {
            t.dof_of_node[n] = -1;
          }
        }
    }
  });

  // ---- subdomain sets S(xi) (node-parallel) -------------------------------
  t.S.assign(nd * 8, -1);
  t.card.assign(nd, 0);
  // slab by slab in node order (DOF nodes are interior: their 8 cells exist)
  parallel_for(N1, [&](int64_t kb, int64_t ke) {
    for (int64_t K = std::max<int64_t>(kb, 1); K < std::min<int64_t>(ke, N); ++K)
      for (int64_t J = 1; J < N; ++J)
        for (int64_t I = 1; I < N; ++I) {
      const int32_t d = t.dof_of_node[node_id(I, J, K)];
      if (d < 0) continue;
      int32_t* Sd = &t.S[(int64_t)d * 8];
      if (I % s != 0 && J % s != 0 && K % s != 0) {
        // strictly inside a block: all 8 cells are in it, one of them active
        Sd[0] = sub_of(I - 1, J - 1, K - 1);
        t.card[d] = 1;
        continue;
      }
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
  });

  // ---- floating components ---------------------------------------------
  // Active cells are joined through shared DOF nodes.  Per subdomain block
  // (in parallel): union-find over the block's nodes, giving numbered local
  // components and whether they hold a cell on the cube boundary.  Then one
  // small union-find over all local components, joined through the DOF
  // nodes shared by several blocks.
  {
    std::vector<int32_t> lcomp, nlc, base;   // plain locals: the lambdas below run on pool threads
    std::vector<uint8_t> lground;
    lcomp.assign((size_t)ns * nbn, -1);                    // local component id per block node
    lground.assign((size_t)ns * nbn, 0);                  // per (block, local component)
    nlc.assign(ns + 1, 0);
    parallel_for(ns, [&](int64_t wb, int64_t we) {
      std::vector<int32_t> p(nbn), id(nbn);
      std::vector<uint8_t> used(nbn), gr(nbn);
      for (int64_t w = wb; w < we; ++w) {
        const int Bx = (int)(w % m), By = (int)((w / m) % m), Bz = (int)(w / (m * m));
        // a block whose cells are all active is one component (neighbouring
        // cells always share a DOF node when N > 1)
        bool full = N > 1, face_any = false;
        for (int cz = 0; cz < s && full; ++cz)
          for (int cy = 0; cy < s && full; ++cy)
            for (int cx = 0; cx < s; ++cx) {
              const int64_t i = (int64_t)Bx * s + cx, j = (int64_t)By * s + cy, k = (int64_t)Bz * s + cz;
              if (!active(cell_id(i, j, k))) {
                full = false;
                break;
              }
              if (i == 0 || j == 0 || k == 0 || i == N - 1 || j == N - 1 || k == N - 1) face_any = true;
            }
        if (full) {
          int32_t nc = 0;
          for (int lz = 0; lz <= s; ++lz)
            for (int ly = 0; ly <= s; ++ly)
              for (int lx = 0; lx <= s; ++lx)
                if (t.dof_of_node[node_id((int64_t)Bx * s + lx, (int64_t)By * s + ly, (int64_t)Bz * s + lz)] >= 0) {
                  lcomp[w * nbn + lx + s1 * (ly + s1 * lz)] = 0;
                  nc = 1;
                }
          if (nc && face_any) lground[w * nbn] = 1;
          nlc[w + 1] = nc;
          continue;
        }
        std::iota(p.begin(), p.end(), 0);
        std::fill(used.begin(), used.end(), 0);
        std::fill(gr.begin(), gr.end(), 0);
        auto find = [&](int32_t x) {
          while (p[x] != x) {
            p[x] = p[p[x]];
            x = p[x];
          }
          return x;
        };
        for (int cz = 0; cz < s; ++cz)
          for (int cy = 0; cy < s; ++cy)
            for (int cx = 0; cx < s; ++cx) {
              const int64_t i = (int64_t)Bx * s + cx, j = (int64_t)By * s + cy, k = (int64_t)Bz * s + cz;
              if (!active(cell_id(i, j, k))) continue;
              const bool face = (i == 0 || j == 0 || k == 0 || i == N - 1 || j == N - 1 || k == N - 1);
              int32_t first = -1;
              for (int a = 0; a < 8; ++a) {
                const int lx = cx + (a & 1), ly = cy + ((a >> 1) & 1), lz = cz + ((a >> 2) & 1);
                if (t.dof_of_node[node_id((int64_t)Bx * s + lx, (int64_t)By * s + ly, (int64_t)Bz * s + lz)] < 0)
                  continue;
                const int32_t ln = lx + s1 * (ly + s1 * lz);
                used[ln] = 1;
                if (first < 0) {
                  first = ln;
                } else {
                  const int32_t ra = find(first), rb = find(ln);
                  if (ra != rb) p[std::max(ra, rb)] = std::min(ra, rb);
                }
              }
              if (face && first >= 0) gr[first] = 1;
            }
        int32_t nc = 0;
        std::fill(id.begin(), id.end(), -1);
        for (int32_t ln = 0; ln < nbn; ++ln) {
          if (!used[ln]) continue;
          const int32_t r = find(ln);
          if (id[r] < 0) id[r] = nc++;
          lcomp[w * nbn + ln] = id[r];
        }
        for (int32_t ln = 0; ln < nbn; ++ln)
          if (used[ln] && gr[ln]) lground[w * nbn + lcomp[w * nbn + ln]] = 1;
        nlc[w + 1] = nc;
      }
    });
    base.assign(ns + 1, 0);
    for (int32_t w = 0; w < ns; ++w) base[w + 1] = base[w] + nlc[w + 1];
    const int32_t ncomp_all = base[ns];
    UnionFind guf(ncomp_all);
    std::vector<int32_t> bx0(ns), by0(ns), bz0(ns);   // block origins (node coordinates)
    for (int32_t w = 0; w < ns; ++w) {
      bx0[w] = (w % m) * s;
      by0[w] = ((w / m) % m) * s;
      bz0[w] = (w / (m * m)) * s;
    }
    for (int64_t K = 1; K < N; ++K)
      for (int64_t J = 1; J < N; ++J)
        for (int64_t I = 1; I < N; ++I) {
          const int32_t d = t.dof_of_node[node_id(I, J, K)];
          if (d < 0 || t.card[d] < 2) continue;
          int32_t first = -1;
          for (int q = 0; q < t.card[d]; ++q) {
            const int32_t w = t.S[(int64_t)d * 8 + q];
            const int ln = (int)(I - bx0[w]) + s1 * ((int)(J - by0[w]) + s1 * (int)(K - bz0[w]));
            const int32_t idg = base[w] + lcomp[w * nbn + ln];
            if (first < 0) first = idg;
            else guf.unite(first, idg);
          }
        }
    std::vector<uint8_t> rg(ncomp_all, 0);
    for (int32_t w = 0; w < ns; ++w)
      for (int32_t c = 0; c < nlc[w + 1]; ++c)
        if (lground[w * nbn + c]) rg[guf.find(base[w] + c)] = 1;
    for (int32_t e = 0; e < ncomp_all; ++e)
      if (!rg[guf.find(e)]) {
        err = "an active component touches no Dirichlet node (singular operator)";
        return -2;
      }
  }

  // ---- links between axis-adjacent interface DOFs -------------------------
  struct Link {
    int32_t a, b;
    int8_t axis;
  };
  std::vector<std::vector<Link>> tlinks(N1);
  parallel_for(N1, [&](int64_t kb, int64_t ke) {
    for (int64_t K = kb; K < ke; ++K) {
      auto& out = tlinks[K];
      for (int64_t J = 1; J < N; ++J)
        for (int64_t I = 1; I < N; ++I) {
          const int64_t node = node_id(I, J, K);
          const int32_t a = t.dof_of_node[node];
          if (a < 0 || t.card[a] < 2) continue;
          const int64_t ijk[3] = {I, J, K};
          for (int axis = 0; axis < 3; ++axis) {
            const int64_t step = axis == 0 ? 1 : (axis == 1 ? N1 : N1 * N1);
            if (ijk[axis] + 1 > N) continue;
            const int32_t b = t.dof_of_node[node + step];
            if (b < 0 || t.card[b] < 2) continue;
            if (!same_set(&t.S[(int64_t)a * 8], &t.S[(int64_t)b * 8])) continue;
            const int o1 = axis == 0 ? 1 : 0;
            const int o2 = axis == 2 ? 1 : 2;
            int32_t St[4];
            int nst = 0;
            for (int u = -1; u <= 0; ++u)
              for (int v = -1; v <= 0; ++v) {
                int64_t c3[3] = {I, J, K};
                c3[o1] += u;
                c3[o2] += v;
                if (!active_at(c3[0], c3[1], c3[2])) continue;
                St[nst++] = sub_of(c3[0], c3[1], c3[2]);
              }
            bool full = true;
            for (int q = 0; q < t.card[a]; ++q) {
              const int32_t w = t.S[(int64_t)a * 8 + q];
              bool present = false;
              for (int z = 0; z < nst; ++z)
                if (St[z] == w) present = true;
              if (!present) full = false;
            }
            if (full) out.push_back({a, b, (int8_t)axis});
          }
        }
    }
  });
  std::vector<Link> links;
  for (auto& v : tlinks) links.insert(links.end(), v.begin(), v.end());
  UnionFind uf(nd);
  for (auto& L : links) uf.unite(L.a, L.b);

  // ---- objects ----------------------------------------------------------
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
  {
    // cells lo on the last layer of a block, hi across the block boundary
    std::vector<std::vector<int32_t>> faces_found(3 * std::max(1, m - 1));
    parallel_for(3 * std::max(0, m - 1), [&](int64_t pb, int64_t pe) {
      for (int64_t pl = pb; pl < pe; ++pl) {
        const int axis = (int)(pl / (m - 1));
        const int64_t plane = (pl % (m - 1)) * s + (s - 1);
        const int o1 = axis == 0 ? 1 : 0;
        const int o2 = axis == 2 ? 1 : 2;
        for (int64_t v = 0; v < N; ++v)
          for (int64_t u = 0; u < N; ++u) {
            int64_t c3[3];
            c3[axis] = plane;
            c3[o1] = u;
            c3[o2] = v;
            int64_t h3[3] = {c3[0], c3[1], c3[2]};
            h3[axis] += 1;
            if (!active(cell_id(c3[0], c3[1], c3[2])) || !active(cell_id(h3[0], h3[1], h3[2]))) continue;
            int32_t fd[4];
            int q = 0;
            bool ok = true;
            for (int uu = 0; uu <= 1; ++uu)
              for (int vv = 0; vv <= 1; ++vv) {
                int64_t n3[3] = {c3[0], c3[1], c3[2]};
                n3[axis] += 1;
                n3[o1] += uu;
                n3[o2] += vv;
                const int32_t d = t.dof_of_node[node_id(n3[0], n3[1], n3[2])];
                if (d < 0 || t.card[d] < 2) ok = false;
                fd[q++] = d;
              }
            if (!ok) continue;
            const int32_t o = comp_of[fd[0]];
            if (comp_of[fd[1]] != o || comp_of[fd[2]] != o || comp_of[fd[3]] != o) continue;
            if (t.card[fd[0]] != 2) continue;
            const int32_t* Sf = &t.S[(int64_t)fd[0] * 8];
            const int32_t w1 = sub_of(c3[0], c3[1], c3[2]), w2 = sub_of(h3[0], h3[1], h3[2]);
            if (std::min(w1, w2) == Sf[0] && std::max(w1, w2) == Sf[1]) faces_found[pl].push_back(o);
          }
      }
    });
    for (auto& v : faces_found)
      for (int32_t o : v) is_face[o] = 1;
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
      const int64_t node = t.dof_node[L.a];
      const int64_t ijk[3] = {node % N1, (node / N1) % N1, node / (N1 * N1)};
      const int8_t k = (int8_t)segment_class(N, ijk, L.axis, g.centres, g.radii);
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
      const int64_t pa = pos(links[lidx[q]].a), pb = pos(links[lidx[q]].b);
      if (pa >= 0 && pb >= 0) lu.unite((int32_t)pa, (int32_t)pb);
    }
    std::vector<std::vector<int64_t>> parts;
    std::vector<int64_t> part_of(rest.size(), -1);
    for (int64_t r = 0; r < (int64_t)rest.size(); ++r) {
      const int64_t root = lu.find((int32_t)r);
      if (part_of[root] < 0) {
        part_of[root] = (int64_t)parts.size();
        parts.emplace_back();
      }
      parts[part_of[root]].push_back(rest[r]);
    }
    for (auto& pdofs : parts) {
      const int8_t ty = pdofs.size() == 1 ? OBJ_CORNER : OBJ_EDGE;
      objs.push_back({std::move(pdofs), ty});
    }
  }
  std::sort(objs.begin(), objs.end(), [](const Obj& x, const Obj& y) { return x.dofs[0] < y.dofs[0]; });
  const int64_t nobj = (int64_t)objs.size();
  t.obj_ptr.assign(nobj + 1, 0);
  t.obj_type.resize(nobj);
  t.coarse_of_obj.assign(nobj, -1);
  std::vector<int32_t> obj_of_dof(nd, -1);
  for (int64_t o = 0; o < nobj; ++o) t.obj_ptr[o + 1] = t.obj_ptr[o] + (int64_t)objs[o].dofs.size();
  t.obj_dofs.resize(t.obj_ptr[nobj]);
  for (int64_t o = 0; o < nobj; ++o) {
    t.obj_type[o] = objs[o].type;
    int64_t q = t.obj_ptr[o];
    for (int64_t x : objs[o].dofs) {
      t.obj_dofs[q++] = x;
      obj_of_dof[x] = (int32_t)o;
    }
    const bool selected = (g.objects == 0) || objs[o].type != OBJ_FACE;
    if (selected) t.coarse_of_obj[o] = t.n_coarse++;
  }

  // ---- per-subdomain lists (subdomain-parallel) ---------------------------
  // Interface numbering of the DOFs (ascending) and its CSR of subdomains.
  std::vector<int32_t> iface_of(nd, -1);
  int64_t n_iface = 0;
  t.if_ptr.assign(1, 0);
  for (int64_t a = 0; a < nd; ++a)
    if (t.card[a] >= 2) {
      iface_of[a] = (int32_t)n_iface++;
      t.if_ptr.push_back(t.if_ptr.back() + t.card[a]);
    }
  t.n_iface = (int32_t)n_iface;
  t.iface_node.resize(n_iface);
  t.if_sub.resize(t.if_ptr.back());
  t.if_slot.resize(t.if_ptr.back());
  t.nI.assign(ns, 0);
  t.nG.assign(ns, 0);
  t.nC.assign(ns, 0);
  // coarse DOFs per subdomain
  std::vector<std::vector<int32_t>> sub_c(ns);
  for (int64_t o = 0; o < nobj; ++o) {
    const int32_t cid = t.coarse_of_obj[o];
    if (cid < 0) continue;
    const int64_t d0 = objs[o].dofs[0];
    for (int z = 0; z < t.card[d0]; ++z) sub_c[t.S[d0 * 8 + z]].push_back(cid);
  }
  // count pass: nodes of each block in ascending node order
  auto block_nodes = [&](int32_t w, auto&& fn) {
    const int Bx = w % m, By = (w / m) % m, Bz = w / (m * m);
    for (int lz = 0; lz <= s; ++lz)
      for (int ly = 0; ly <= s; ++ly) {
        const bool inner_yz = lz > 0 && lz < s && ly > 0 && ly < s;
        int64_t n = node_id((int64_t)Bx * s, (int64_t)By * s + ly, (int64_t)Bz * s + lz);
        for (int lx = 0; lx <= s; ++lx, ++n) {
          const int32_t d = t.dof_of_node[n];
          if (d < 0) continue;
          if (inner_yz && lx > 0 && lx < s) {   // interior node of this block: S = {w}
            fn(n, d, 0);
            continue;
          }
          const int32_t* Sd = &t.S[(int64_t)d * 8];
          int k = -1;
          for (int q = 0; q < t.card[d]; ++q)
            if (Sd[q] == w) k = q;
          if (k < 0) continue;
          fn(n, d, k);
        }
      }
  };
  parallel_for(ns, [&](int64_t wb, int64_t we) {
    for (int64_t w = wb; w < we; ++w) {
      int32_t ci = 0, cg = 0;
      block_nodes((int32_t)w, [&](int64_t, int32_t d, int) {
        if (t.card[d] == 1) ++ci;
        else ++cg;
      });
      t.nI[w] = ci;
      t.nG[w] = cg;
      std::sort(sub_c[w].begin(), sub_c[w].end());
      t.nC[w] = (int32_t)sub_c[w].size();
    }
  });
  t.I_ptr.assign(ns + 1, 0);
  t.G_ptr.assign(ns + 1, 0);
  t.C_ptr.assign(ns + 1, 0);
  for (int32_t w = 0; w < ns; ++w) {
    t.I_ptr[w + 1] = t.I_ptr[w] + t.nI[w];
    t.G_ptr[w + 1] = t.G_ptr[w] + t.nG[w];
    t.C_ptr[w + 1] = t.C_ptr[w] + t.nC[w];
    t.maxI = std::max(t.maxI, t.nI[w]);
    t.maxG = std::max(t.maxG, t.nG[w]);
    t.maxC = std::max(t.maxC, t.nC[w]);
  }
  t.I_nodes.resize(t.I_ptr[ns]);
  t.G_nodes.resize(t.G_ptr[ns]);
  t.G_obj.assign(t.G_ptr[ns], -1);
  t.C_ids.resize(t.C_ptr[ns]);
  parallel_for(ns, [&](int64_t wb, int64_t we) {
    for (int64_t w = wb; w < we; ++w) {
      int64_t qi = t.I_ptr[w], qg = t.G_ptr[w];
      std::copy(sub_c[w].begin(), sub_c[w].end(), t.C_ids.begin() + t.C_ptr[w]);
      const auto cb = t.C_ids.begin() + t.C_ptr[w], ce = t.C_ids.begin() + t.C_ptr[w + 1];
      block_nodes((int32_t)w, [&](int64_t n, int32_t d, int k) {
        if (t.card[d] == 1) {
          t.I_nodes[qi++] = n;
          return;
        }
        const int32_t slot = (int32_t)(qg - t.G_ptr[w]);
        t.G_nodes[qg] = n;
        const int32_t cid = t.coarse_of_obj[obj_of_dof[d]];
        if (cid >= 0) t.G_obj[qg] = (int32_t)(std::lower_bound(cb, ce, cid) - cb);
        ++qg;
        const int32_t q = iface_of[d];
        t.if_sub[t.if_ptr[q] + k] = (int32_t)w;
        t.if_slot[t.if_ptr[q] + k] = slot;
        if (k == 0) t.iface_node[q] = n;   // written once, by the first subdomain of S
      });
    }
  });
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
        const int32_t c = t.C_ids[q];
        t.cs_sub[fill[c]] = w;
        t.cs_row[fill[c]] = (int32_t)(q - t.C_ptr[w]);
        fill[c]++;
      }
  }
  return 0;
}

void parallel_rows(int64_t n, const std::function<void(int64_t, int64_t)>& f) { parallel_for(n, f); }

void set_serial_indexing(bool serial) { t_serial = serial; }

int indexing_threads() { return Pool::get().size(); }

}  // namespace cutbddc
