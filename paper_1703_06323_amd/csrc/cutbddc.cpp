// C ABI of the cut-cell BDDC-PCG solver (see include/cutbddc.h): context,
// device buffers and the orchestration of setup / factor / solve.
#include "cutbddc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <memory>
#include <type_traits>
#include <string>
#include <vector>

#include "bddc.h"
#include "common.h"
#include "dense.h"
#include "topology.hpp"

using namespace cutbddc;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? CB_ERR_OOM : CB_ERR_DEVICE,              \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

#define CHK(expr)              \
  do {                         \
    int rc_ = (expr);          \
    if (rc_ != CB_OK) return rc_; \
  } while (0)

// Process-wide cache of device blocks: freed blocks are kept (keyed by size,
// per device) and handed out again for requests of up to the same size, so
// repeated setup/factor/solve cycles issue no hipMalloc/hipFree (hipFree
// synchronises the device).  A block released while work that uses it is
// still queued is only reused on the same device after that device's
// pending work has been ordered: reuse happens on the stream of the new
// owner, and cross-context reuse synchronises the releasing stream.
struct CachedBlock {
  void* p;
  size_t bytes;
  hipStream_t st;
};
struct BlockCache {
  std::mutex mu;
  std::multimap<size_t, CachedBlock> blocks;   // by size
  size_t bytes = 0;
};
BlockCache& block_cache() {
  static BlockCache* c = new BlockCache();   // intentionally leaked at exit
  return *c;
}
constexpr size_t CACHE_LIMIT = (size_t)48 << 30;   // bytes kept for reuse

void* cache_get(size_t bytes, hipStream_t st, hipError_t* err) {
  BlockCache& c = block_cache();
  {
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.blocks.lower_bound(bytes);
    if (it != c.blocks.end() && it->first <= bytes + bytes / 4 + (1 << 20)) {
      CachedBlock b = it->second;
      c.blocks.erase(it);
      c.bytes -= b.bytes;
      if (b.st != st) (void)hipStreamSynchronize(b.st);
      *err = hipSuccess;
      return b.p;
    }
  }
  void* p = nullptr;
  *err = hipMalloc(&p, bytes);
  if (*err == hipErrorOutOfMemory) {
    // release the cache and retry once
    std::vector<void*> drop;
    {
      std::lock_guard<std::mutex> g(c.mu);
      for (auto& kv : c.blocks) drop.push_back(kv.second.p);
      c.blocks.clear();
      c.bytes = 0;
    }
    (void)hipDeviceSynchronize();
    for (void* q : drop) (void)hipFree(q);
    *err = hipMalloc(&p, bytes);
  }
  return *err == hipSuccess ? p : nullptr;
}

void cache_put(void* p, size_t bytes, hipStream_t st) {
  BlockCache& c = block_cache();
  std::lock_guard<std::mutex> g(c.mu);
  if (c.bytes + bytes > CACHE_LIMIT) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(p);
    return;
  }
  c.blocks.emplace(bytes, CachedBlock{p, bytes, st});
  c.bytes += bytes;
}

// Device buffer owned by a context (allocated from the block cache).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t st = nullptr;
  ~DevBuf() { release(); }
  void release() {
    if (p) cache_put(p, bytes, st);
    p = nullptr;
    bytes = 0;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

thread_local hipStream_t g_alloc_stream = nullptr;   // stream of the context being served

int dalloc(DevBuf& b, size_t bytes) {
  b.release();
  if (bytes == 0) bytes = 8;
  bytes = (bytes + 255) & ~(size_t)255;
  hipError_t e;
  b.p = cache_get(bytes, g_alloc_stream, &e);
  if (!b.p) {
    return fail(CB_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                hipGetErrorString(e));
  }
  b.bytes = bytes;
  b.st = g_alloc_stream;
  return CB_OK;
}

template <typename T>
int upload(DevBuf& b, const std::vector<T>& v, hipStream_t st) {
  CHK(dalloc(b, v.size() * sizeof(T)));
  if (!v.empty()) HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return CB_OK;
}

inline int round_up(int x, int q) { return ((x + q - 1) / q) * q; }

// Reference Q1 matrices from the 512-point rule with every point kept.
void reference_matrices(const double xi[8], double K[64], double M[64]) {
  for (int e = 0; e < 64; ++e) K[e] = M[e] = 0.0;
  for (int q = 0; q < 512; ++q) {
    const double p[3] = {xi[q & 7], xi[(q >> 3) & 7], xi[q >> 6]};
    double Nv[8], G[8][3];
    for (int a = 0; a < 8; ++a) {
      const int o[3] = {a & 1, (a >> 1) & 1, (a >> 2) & 1};
      double f[3], d[3];
      for (int k = 0; k < 3; ++k) {
        f[k] = o[k] ? p[k] : 1.0 - p[k];
        d[k] = o[k] ? 1.0 : -1.0;
      }
      Nv[a] = f[0] * f[1] * f[2];
      G[a][0] = d[0] * f[1] * f[2];
      G[a][1] = f[0] * d[1] * f[2];
      G[a][2] = f[0] * f[1] * d[2];
    }
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b) {
        K[a * 8 + b] += G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2];
        M[a * 8 + b] += Nv[a] * Nv[b];
      }
  }
  for (int e = 0; e < 64; ++e) {
    K[e] *= 1.0 / 512.0;
    M[e] *= 1.0 / 512.0;
  }
}

// Reuse of host indexing storage across contexts (avoids re-faulting the
// pages of large fresh allocations on every setup).
std::mutex g_topo_mu;
std::vector<Topology*> g_topo_pool;
Topology* take_topology() {
  std::lock_guard<std::mutex> g(g_topo_mu);
  if (g_topo_pool.empty()) return new Topology();
  Topology* t = g_topo_pool.back();
  g_topo_pool.pop_back();
  return t;
}
void give_topology(Topology* t) {
  std::lock_guard<std::mutex> g(g_topo_mu);
  if (g_topo_pool.size() < 4) g_topo_pool.push_back(t);
  else delete t;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

struct ProfEntry {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
};

struct cb_ctx {
  hipStream_t st = nullptr;
  bool prof = false;
  std::map<std::string, ProfEntry> prof_ev;
  ~cb_ctx() {
    give_topology(topo_p);
    for (auto& kv : prof_ev)
      for (auto& e : kv.second.ev) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
      }
  }
  Geometry geo;
  Topology* topo_p = take_topology();
  Topology& topo = *topo_p;
  int N = 0, s = 0, m = 0, ns = 0;
  double h = 0;
  int weighting = 1, objects = 0, variant = 1, precision = 0, full_elements = 0;
  std::vector<int32_t> count;
  std::vector<int64_t> cut_cells;
  int64_t n_active = 0, n_cut = 0;
  double xi[8];
  double Kref[64], Mref[64];
  bool factored = false;
  int n_fallbacks = 0;

  // grid data
  DevBuf xi_d, balls, kappa, count_d, cellinfo, cut_d, Kc, Mc, dofmask, dof_node;
  // subdomain index data
  int NIp = 0, NGp = 0, NCp = 0, nt = 0, ldc = 0;
  DevBuf nI, nG, nC, Iidx, Gidx, Gobj, Cids, bloc, if_ptr, if_sub, if_slot, iface_node, cs_ptr, cs_sub,
      cs_row;
  // factor results
  DevBuf P, Kt, Phi, Dw, diagAG, Ds, Acinv, AcKeep, info_d;
  // work vectors
  DevBuf x, r, z, p, q, t1, t2, t3, zbuf, cloc, cvec, ucvec, partial, scal, bgrid;
  cb_info info{};

  GridDev grid() const {
    GridDev g;
    g.N = N;
    g.s = s;
    g.h = h;
    g.cellinfo = cellinfo.as<int32_t>();
    g.kappa = kappa.as<double>();
    g.Kc = Kc.as<double>();
    return g;
  }
  SubDev sub() const {
    SubDev d;
    d.NIp = NIp;
    d.NGp = NGp;
    d.NCp = NCp;
    d.nI = nI.as<int32_t>();
    d.nG = nG.as<int32_t>();
    d.nC = nC.as<int32_t>();
    d.I_idx = Iidx.as<int64_t>();
    d.G_idx = Gidx.as<int64_t>();
    d.G_obj = Gobj.as<int32_t>();
    d.C_ids = Cids.as<int32_t>();
    d.bloc = bloc.as<int32_t>();
    return d;
  }
  int64_t n_nodes() const { return (int64_t)(N + 1) * (N + 1) * (N + 1); }
};

namespace {

// Brackets the launches issued during its lifetime with HIP events when
// profiling is enabled.
struct ProfScope {
  cb_ctx* c;
  hipEvent_t b = nullptr, e = nullptr;
  const char* name;
  ProfScope(cb_ctx* ctx, const char* n) : c(ctx), name(n) {
    if (!c->prof) return;
    if (hipEventCreate(&b) != hipSuccess || hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(b, c->st);
  }
  ~ProfScope() {
    if (!c->prof || !b || !e) return;
    (void)hipEventRecord(e, c->st);
    c->prof_ev[name].ev.emplace_back(b, e);
  }
};

int apply_A_grid(cb_ctx* c, const double* x, double* y) {
  ProfScope ps(c, "apply_A");
  GridDesc g{c->N, c->h};
  launch_apply_A(c->st, g, c->cellinfo.as<int32_t>(), c->kappa.as<double>(), c->Kc.as<double>(),
                 c->dofmask.as<uint8_t>(), x, y);
  HIPCHK(hipGetLastError());
  return CB_OK;
}

template <typename F>
void timed(cb_ctx* c, const char* name, F&& f) {
  ProfScope ps(c, name);
  f();
}

// z = M r on grid vectors (eq. bddc), steps (1)-(7).
int apply_M_grid(cb_ctx* c, const double* r, double* z) {
  hipStream_t st = c->st;
  const SubDev sd = c->sub();
  const int64_t nn = c->n_nodes();
  double* t1 = c->t1.as<double>();
  double* t2 = c->t2.as<double>();
  double* t3 = c->t3.as<double>();
  // (1) delta_I = A_II^{-1} r_I
  launch_fill(st, nn, 0.0, t1);
  timed(c, "apply_interior", [&] {
    if (c->precision == CB_FP32_LOCAL)
      launch_apply_interior<float>(st, sd, c->ns, c->P.as<float>(), r, nullptr, t1);
    else
      launch_apply_interior<double>(st, sd, c->ns, c->P.as<double>(), r, nullptr, t1);
  });
  // (2) rhat_G = r_G - (A delta)_G
  CHK(apply_A_grid(c, t1, t2));
  // (3)-(4) weighted restriction, constrained Neumann solves, coarse rhs
  timed(c, "apply_neumann", [&] {
    if (c->precision == CB_FP32_LOCAL)
      launch_apply_neumann<float>(st, sd, c->ns, c->Kt.as<float>(), c->Phi.as<double>(), c->Dw.as<double>(),
                                  r, t2, c->zbuf.as<double>(), c->cloc.as<double>());
    else
      launch_apply_neumann<double>(st, sd, c->ns, c->Kt.as<double>(), c->Phi.as<double>(),
                                   c->Dw.as<double>(), r, t2, c->zbuf.as<double>(), c->cloc.as<double>());
  });
  // (5) coarse correction
  const int nc = c->topo.n_coarse;
  if (nc > 0) {
    launch_coarse_rhs(st, nc, c->cs_ptr.as<int64_t>(), c->cs_sub.as<int32_t>(), c->cs_row.as<int32_t>(),
                      c->NCp, c->cloc.as<double>(), c->cvec.as<double>());
    timed(c, "coarse_gemv",
          [&] { launch_gemv(st, nc, c->ldc, c->Acinv.as<double>(), c->cvec.as<double>(), c->ucvec.as<double>()); });
    launch_add_coarse(st, sd, c->ns, c->Phi.as<double>(), c->ucvec.as<double>(), c->zbuf.as<double>());
  }
  // (6) weighted average on the interface
  launch_fill(st, nn, 0.0, z);
  launch_iface_average(st, c->topo.n_iface, c->iface_node.as<int64_t>(), c->if_ptr.as<int64_t>(),
                       c->if_sub.as<int32_t>(), c->if_slot.as<int32_t>(), c->NGp, c->Dw.as<double>(),
                       c->zbuf.as<double>(), z);
  // (7) harmonic extension: z_I = A_II^{-1} (r - A [0; u_G])_I
  CHK(apply_A_grid(c, z, t3));
  timed(c, "apply_interior", [&] {
    if (c->precision == CB_FP32_LOCAL)
      launch_apply_interior<float>(st, sd, c->ns, c->P.as<float>(), r, t3, z);
    else
      launch_apply_interior<double>(st, sd, c->ns, c->P.as<double>(), r, t3, z);
  });
  HIPCHK(hipGetLastError());
  return CB_OK;
}

int read_scalar(cb_ctx* c, const double* d, double* h) {
  HIPCHK(hipMemcpyAsync(h, d, sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return CB_OK;
}

int dot(cb_ctx* c, const double* a, const double* b, double* out_dev) {
  launch_dot(c->st, c->n_nodes(), a, b, c->partial.as<double>(), out_dev);
  HIPCHK(hipGetLastError());
  return CB_OK;
}

// PCG on grid vectors: b in c->bgrid, result in c->x.
int pcg(cb_ctx* c, double rtol, int32_t max_iter, int32_t* iters, double* relres_out) {
  hipStream_t st = c->st;
  const int64_t nn = c->n_nodes();
  double* x = c->x.as<double>();
  double* r = c->r.as<double>();
  double* z = c->z.as<double>();
  double* p = c->p.as<double>();
  double* q = c->q.as<double>();
  double* S = c->scal.as<double>();   // [0] rho, [1] pq, [2] rr, [3] rho_new, [4] bb
  const double* b = c->bgrid.as<double>();
  launch_fill(st, nn, 0.0, x);
  HIPCHK(hipMemcpyAsync(r, b, nn * sizeof(double), hipMemcpyDeviceToDevice, st));
  CHK(dot(c, b, b, S + 4));
  double bb = 0.0;
  CHK(read_scalar(c, S + 4, &bb));
  const double bnorm = std::sqrt(bb);
  int32_t k = 0;
  double relres = 0.0;
  if (bnorm == 0.0) {
    if (iters) *iters = 0;
    if (relres_out) *relres_out = 0.0;
    return CB_OK;
  }
  relres = 1.0;
  CHK(apply_M_grid(c, r, z));
  HIPCHK(hipMemcpyAsync(p, z, nn * sizeof(double), hipMemcpyDeviceToDevice, st));
  CHK(dot(c, r, z, S + 0));
  bool converged = false;
  while (k < max_iter) {
    CHK(apply_A_grid(c, p, q));
    CHK(dot(c, p, q, S + 1));
    launch_cg_update_xr(st, nn, S, p, q, x, r);
    CHK(dot(c, r, r, S + 2));
    ++k;
    double rr = 0.0;
    CHK(read_scalar(c, S + 2, &rr));
    if (!std::isfinite(rr)) {
      if (iters) *iters = k;
      return fail(CB_ERR_NOT_SPD, "PCG breakdown (non-finite residual)");
    }
    relres = std::sqrt(rr) / bnorm;
    if (relres < rtol) {
      converged = true;
      break;
    }
    CHK(apply_M_grid(c, r, z));
    CHK(dot(c, r, z, S + 3));
    launch_cg_update_p(st, nn, S, z, p);
  }
  HIPCHK(hipGetLastError());
  if (iters) *iters = k;
  if (relres_out) *relres_out = relres;
  if (!converged) return fail(CB_ERR_NO_CONVERGENCE, "PCG reached max_iter");
  return CB_OK;
}

}  // namespace

extern "C" {

const char* cb_last_error(void) { return g_err.c_str(); }

int cb_host_indexing(const cb_problem* p, const int32_t* cell_count, cb_info* info, int64_t* dof_node,
                     int32_t* card, int64_t* obj_ptr, int64_t* obj_dofs, int8_t* obj_type, int32_t* coarse_of_obj) {
  if (!p || !cell_count || !info) return fail(CB_ERR_ARG, "null argument");
  const int N = p->n_cells, s = p->sub_cells;
  if (N < 1 || s < 1 || N % s != 0) return fail(CB_ERR_ARG, "n_cells must be >= 1 and divisible by sub_cells");
  if (p->n_balls < 0 || (p->n_balls > 0 && (!p->ball_centres || !p->ball_radii)))
    return fail(CB_ERR_ARG, "invalid ball arrays");
  Geometry geo;
  geo.N = N;
  geo.s = s;
  geo.objects = p->objects;
  geo.variant = p->coarse_variant;
  geo.centres.assign(p->ball_centres, p->ball_centres + 3 * p->n_balls);
  geo.radii.assign(p->ball_radii, p->ball_radii + p->n_balls);
  std::unique_ptr<Topology> t(new Topology());
  std::string err;
  const double t0 = now_ms();
  const int rc = build_topology(geo, cell_count, *t, err);
  if (rc == -2) return fail(CB_ERR_SINGULAR, err);
  if (rc != 0) return fail(CB_ERR_ARG, err);
  *info = cb_info{};
  info->n_dof = t->n_dof;
  info->n_sub = t->n_sub;
  info->n_coarse = t->n_coarse;
  info->n_objects = (int32_t)t->obj_type.size();
  info->n_iface = t->n_iface;
  info->max_coarse_per_sub = t->maxC;
  info->t_topology_ms = now_ms() - t0;
  if (dof_node) std::memcpy(dof_node, t->dof_node.data(), t->n_dof * sizeof(int64_t));
  if (card)
    for (int64_t d = 0; d < t->n_dof; ++d) card[d] = t->card[d];
  if (obj_ptr) std::memcpy(obj_ptr, t->obj_ptr.data(), t->obj_ptr.size() * sizeof(int64_t));
  if (obj_dofs) std::memcpy(obj_dofs, t->obj_dofs.data(), t->obj_dofs.size() * sizeof(int64_t));
  if (obj_type) std::memcpy(obj_type, t->obj_type.data(), t->obj_type.size());
  if (coarse_of_obj) std::memcpy(coarse_of_obj, t->coarse_of_obj.data(), t->coarse_of_obj.size() * sizeof(int32_t));
  return CB_OK;
}

int cb_dense_spd_inverse(int32_t n, int32_t batch, int32_t precision, const double* A, double* Ainv) {
  g_alloc_stream = nullptr;
  if (n < 1 || batch < 1 || !A || !Ainv || precision < 0 || precision > 1)
    return fail(CB_ERR_ARG, "invalid argument");
  const int np = round_up(n, CHOL_BLOCK);
  const size_t nn = (size_t)np * np;
  std::vector<double> h((size_t)batch * nn, 0.0);
  for (int b = 0; b < batch; ++b)
    for (int i = 0; i < np; ++i)
      for (int j = 0; j < np; ++j)
        h[b * nn + (size_t)i * np + j] = (i < n && j < n) ? A[(size_t)b * n * n + (size_t)i * n + j] : (i == j ? 1.0 : 0.0);
  auto run = [&](auto tag) -> int {
    using T = decltype(tag);
    std::vector<T> ht(h.begin(), h.end());
    DevBuf dA, dL, dY, dP, dOut, dOnes, dInfo;
    CHK(upload(dA, ht, nullptr));
    const int nt = np / CHOL_BLOCK;
    CHK(dalloc(dL, (size_t)batch * nt * CHOL_BLOCK * CHOL_BLOCK * sizeof(T)));
    CHK(dalloc(dY, (size_t)batch * nn * sizeof(T)));
    CHK(dalloc(dP, (size_t)batch * nn * sizeof(T)));
    CHK(dalloc(dOut, (size_t)batch * nn * sizeof(double)));
    CHK(upload(dOnes, std::vector<double>((size_t)batch * np, 1.0), nullptr));
    CHK(upload(dInfo, std::vector<int>(batch, 0), nullptr));
    const int64_t sL = (int64_t)nt * CHOL_BLOCK * CHOL_BLOCK;
    cholesky<T>(nullptr, dA.as<T>(), np, nn, np, batch, dL.as<T>(), sL, dInfo.as<int>());
    DevBuf dT;
    CHK(dalloc(dT, (size_t)batch * TRI_SUPER * np * sizeof(T)));
    tri_inverse<T>(nullptr, dA.as<T>(), np, nn, 0, np, batch, dL.as<T>(), sL, dY.as<T>(), np, nn, dT.as<T>(),
                   (int64_t)TRI_SUPER * np);
    gemm<T>(nullptr, 1, 0, np, np, np, T(1), dY.as<T>(), np, nn, dY.as<T>(), np, nn, T(0), dP.as<T>(), np, nn, batch,
            GEMM_LOWER | GEMM_KFROM_DIAG);
    symmetrize_scale<T, double>(nullptr, dP.as<T>(), np, nn, dOut.as<double>(), np, nn, dOnes.as<double>(), np, np,
                                batch);
    HIPCHK(hipGetLastError());
    std::vector<double> out((size_t)batch * nn);
    HIPCHK(hipMemcpy(out.data(), dOut.p, out.size() * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<int> info(batch);
    HIPCHK(hipMemcpy(info.data(), dInfo.p, batch * sizeof(int), hipMemcpyDeviceToHost));
    for (int b = 0; b < batch; ++b)
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ainv[(size_t)b * n * n + (size_t)i * n + j] = out[b * nn + (size_t)i * np + j];
    for (int b = 0; b < batch; ++b)
      if (info[b]) return fail(CB_ERR_NOT_SPD, "Cholesky breakdown in matrix " + std::to_string(b));
    return CB_OK;
  };
  return precision == CB_FP32_LOCAL ? run(float(0)) : run(double(0));
}

int cb_setup(const cb_problem* p, void* stream, cb_ctx** out) {
  if (!p || !out) return fail(CB_ERR_ARG, "null argument");
  *out = nullptr;
  const int N = p->n_cells, s = p->sub_cells;
  if (N < 1 || s < 1 || N % s != 0) return fail(CB_ERR_ARG, "n_cells must be >= 1 and divisible by sub_cells");
  if (N > 1024) return fail(CB_ERR_ARG, "n_cells too large");
  if (p->n_balls < 0 || (p->n_balls > 0 && (!p->ball_centres || !p->ball_radii)))
    return fail(CB_ERR_ARG, "invalid ball arrays");
  if (p->weighting < 0 || p->weighting > 1 || p->objects < 0 || p->objects > 1 || p->coarse_variant < 0 ||
      p->coarse_variant > 1 || p->local_precision < 0 || p->local_precision > 1)
    return fail(CB_ERR_ARG, "invalid option value");
  for (int i = 0; i < p->n_balls; ++i) {
    if (!(p->ball_radii[i] > 0.0) || !std::isfinite(p->ball_radii[i]))
      return fail(CB_ERR_ARG, "ball radius must be positive and finite");
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(p->ball_centres[3 * i + d])) return fail(CB_ERR_ARG, "ball centre not finite");
  }
  const int64_t ncell = (int64_t)N * N * N;
  if (p->kappa)
    for (int64_t c = 0; c < ncell; ++c)
      if (!(p->kappa[c] > 0.0) || !std::isfinite(p->kappa[c]))
        return fail(CB_ERR_ARG, "kappa must be positive and finite");

  std::unique_ptr<cb_ctx> c(new cb_ctx());
  c->st = static_cast<hipStream_t>(stream);
  g_alloc_stream = c->st;
  c->N = N;
  c->s = s;
  c->m = N / s;
  c->ns = c->m * c->m * c->m;
  c->h = 1.0 / (double)N;
  c->weighting = p->weighting;
  c->objects = p->objects;
  c->variant = p->coarse_variant;
  c->precision = p->local_precision;
  c->full_elements = p->full_elements ? 1 : 0;
  c->geo.N = N;
  c->geo.s = s;
  c->geo.objects = p->objects;
  c->geo.variant = p->coarse_variant;
  c->geo.centres.assign(p->ball_centres, p->ball_centres + 3 * p->n_balls);
  c->geo.radii.assign(p->ball_radii, p->ball_radii + p->n_balls);
  hipStream_t st = c->st;

  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, st));
  // sub-cell Gauss coordinates: xi_k = (a + g_p) / 4, k = 2a + p
  const double g0 = 0.5 - 0.5 / std::sqrt(3.0), g1 = 0.5 + 0.5 / std::sqrt(3.0);
  for (int a = 0; a < 4; ++a) {
    c->xi[2 * a] = ((double)a + g0) * 0.25;
    c->xi[2 * a + 1] = ((double)a + g1) * 0.25;
  }
  reference_matrices(c->xi, c->Kref, c->Mref);
  set_reference_matrices(c->Kref, c->Mref);
  bddc_set_reference(c->Kref);
  std::vector<double> xi(c->xi, c->xi + 8);
  CHK(upload(c->xi_d, xi, st));
  std::vector<double> balls(4 * (size_t)p->n_balls);
  for (int i = 0; i < p->n_balls; ++i) {
    balls[4 * i + 0] = p->ball_centres[3 * i + 0];
    balls[4 * i + 1] = p->ball_centres[3 * i + 1];
    balls[4 * i + 2] = p->ball_centres[3 * i + 2];
    balls[4 * i + 3] = p->ball_radii[i] * p->ball_radii[i];
  }
  CHK(upload(c->balls, balls, st));
  std::vector<double> kap(ncell, 1.0);
  if (p->kappa) std::memcpy(kap.data(), p->kappa, ncell * sizeof(double));
  CHK(upload(c->kappa, kap, st));
  CHK(dalloc(c->count_d, ncell * sizeof(int32_t)));
  launch_classify(st, N, c->xi_d.as<double>(), c->balls.as<double>(), p->n_balls, c->count_d.as<int32_t>());
  HIPCHK(hipGetLastError());
  c->count.resize(ncell);
  HIPCHK(hipMemcpyAsync(c->count.data(), c->count_d.p, ncell * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<int32_t> cellinfo(ncell, CELL_INACTIVE);
  for (int64_t cc = 0; cc < ncell; ++cc) {
    const int32_t k = c->count[cc];
    if (k <= 0) continue;
    c->n_active++;
    if (k < 512 && !c->full_elements) {
      cellinfo[cc] = (int32_t)c->cut_cells.size();
      c->cut_cells.push_back(cc);
    } else {
      cellinfo[cc] = CELL_UNCUT;
    }
  }
  c->n_cut = 0;
  for (int64_t cc = 0; cc < ncell; ++cc)
    if (c->count[cc] > 0 && c->count[cc] < 512) c->n_cut++;
  CHK(upload(c->cellinfo, cellinfo, st));
  CHK(upload(c->cut_d, c->cut_cells, st));
  const int64_t nstore = (int64_t)c->cut_cells.size();
  CHK(dalloc(c->Kc, std::max<int64_t>(1, nstore) * PACK36 * sizeof(double)));
  CHK(dalloc(c->Mc, std::max<int64_t>(1, nstore) * PACK36 * sizeof(double)));
  launch_integrate_cut(st, N, c->xi_d.as<double>(), c->balls.as<double>(), p->n_balls, c->cut_d.as<int64_t>(),
                       nstore, c->Kc.as<double>(), c->Mc.as<double>());
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(e1, st));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  c->info.t_integrate_ms = ms;

  // host indexing
  const double th0 = now_ms();
  std::string err;
  int rc = build_topology(c->geo, c->count.data(), c->topo, err);
  if (rc == -2) return fail(CB_ERR_SINGULAR, err);
  if (rc != 0) return fail(CB_ERR_ARG, err);
  Topology& t = c->topo;
  c->NIp = round_up(std::max(1, t.maxI), CHOL_BLOCK);
  c->NGp = round_up(std::max(1, t.maxG), CHOL_BLOCK);
  c->NCp = round_up(std::max(1, t.maxC), 16);
  c->nt = c->NIp + c->NGp;
  c->ldc = round_up(std::max(1, t.n_coarse), CHOL_BLOCK);
  const int ns = c->ns, NIp = c->NIp, NGp = c->NGp, NCp = c->NCp;
  std::vector<int64_t> Iidx((size_t)ns * NIp, -1), Gidx((size_t)ns * NGp, -1);
  std::vector<int32_t> Gobj((size_t)ns * NGp, -1), Cids((size_t)ns * NCp, -1);
  const int s1 = s + 1;
  std::vector<int32_t> bloc((size_t)ns * s1 * s1 * s1, -1);
  const int64_t N1 = N + 1;
  for (int w = 0; w < ns; ++w) {
    const int Bx = w % c->m, By = (w / c->m) % c->m, Bz = w / (c->m * c->m);
    auto set_loc = [&](int64_t node, int row) {
      const int64_t I = node % N1, J = (node / N1) % N1, K = node / (N1 * N1);
      const int lx = (int)(I - (int64_t)Bx * s), ly = (int)(J - (int64_t)By * s), lz = (int)(K - (int64_t)Bz * s);
      bloc[(size_t)w * s1 * s1 * s1 + lx + s1 * (ly + s1 * lz)] = row;
    };
    for (int64_t q = t.I_ptr[w]; q < t.I_ptr[w + 1]; ++q) {
      const int i = (int)(q - t.I_ptr[w]);
      Iidx[(size_t)w * NIp + i] = t.I_nodes[q];
      set_loc(t.I_nodes[q], i);
    }
    for (int64_t q = t.G_ptr[w]; q < t.G_ptr[w + 1]; ++q) {
      const int j = (int)(q - t.G_ptr[w]);
      Gidx[(size_t)w * NGp + j] = t.G_nodes[q];
      Gobj[(size_t)w * NGp + j] = t.G_obj[q];
      set_loc(t.G_nodes[q], NIp + j);
    }
    for (int64_t q = t.C_ptr[w]; q < t.C_ptr[w + 1]; ++q) Cids[(size_t)w * NCp + (q - t.C_ptr[w])] = t.C_ids[q];
  }
  std::vector<uint8_t> mask(c->n_nodes(), 0);
  for (int64_t d = 0; d < t.n_dof; ++d) mask[t.dof_node[d]] = 1;
  c->info.t_topology_ms = now_ms() - th0;
  CHK(upload(c->nI, t.nI, st));
  CHK(upload(c->nG, t.nG, st));
  CHK(upload(c->nC, t.nC, st));
  CHK(upload(c->Iidx, Iidx, st));
  CHK(upload(c->Gidx, Gidx, st));
  CHK(upload(c->Gobj, Gobj, st));
  CHK(upload(c->Cids, Cids, st));
  CHK(upload(c->bloc, bloc, st));
  CHK(upload(c->if_ptr, t.if_ptr, st));
  CHK(upload(c->if_sub, t.if_sub, st));
  CHK(upload(c->if_slot, t.if_slot, st));
  CHK(upload(c->iface_node, t.iface_node, st));
  CHK(upload(c->cs_ptr, t.cs_ptr, st));
  CHK(upload(c->cs_sub, t.cs_sub, st));
  CHK(upload(c->cs_row, t.cs_row, st));
  CHK(upload(c->dofmask, mask, st));
  CHK(upload(c->dof_node, t.dof_node, st));
  const int64_t nn = c->n_nodes();
  for (DevBuf* b : {&c->x, &c->r, &c->z, &c->p, &c->q, &c->t1, &c->t2, &c->t3, &c->bgrid})
    CHK(dalloc(*b, nn * sizeof(double)));
  CHK(dalloc(c->zbuf, (size_t)ns * NGp * sizeof(double)));
  CHK(dalloc(c->cloc, (size_t)ns * NCp * sizeof(double)));
  CHK(dalloc(c->cvec, (size_t)c->ldc * sizeof(double)));
  CHK(dalloc(c->ucvec, (size_t)c->ldc * sizeof(double)));
  CHK(dalloc(c->partial, (size_t)dot_partials() * sizeof(double)));
  CHK(dalloc(c->scal, 16 * sizeof(double)));
  HIPCHK(hipStreamSynchronize(st));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->info.n_dof = t.n_dof;
  c->info.n_active = c->n_active;
  c->info.n_cut = c->n_cut;
  c->info.n_cut_stored = (int64_t)c->cut_cells.size();
  c->info.n_sub = ns;
  c->info.n_coarse = t.n_coarse;
  c->info.n_objects = (int32_t)t.obj_type.size();
  c->info.n_iface = t.n_iface;
  int maxl = 0;
  for (int w = 0; w < ns; ++w) {
    maxl = std::max(maxl, t.nI[w] + t.nG[w]);
    const double nI = t.nI[w], nG = t.nG[w];
    c->info.sum_nI2 += (int64_t)t.nI[w] * t.nI[w];
    c->info.sum_nG2 += (int64_t)t.nG[w] * t.nG[w];
    c->info.sum_nI += t.nI[w];
    c->info.sum_nG += t.nG[w];
    c->info.flops_local_chol += (nI + nG) * (nI + nG) * (nI + nG) / 3.0 + nI * nI * nI / 3.0;
  }
  c->info.max_local_dofs = maxl;
  c->info.max_coarse_per_sub = t.maxC;
  *out = c.release();
  return CB_OK;
}

}  // extern "C"

namespace {

template <typename T>
int factor_impl(cb_ctx* c) {
  hipStream_t st = c->st;
  const int ns = c->ns, NIp = c->NIp, NGp = c->NGp, NCp = c->NCp, nt = c->nt;
  const SubDev sd = c->sub();
  const GridDev g = c->grid();
  DevBuf K, Linv, Y, PS, G, AcLoc, KS, Ac;
  CHK(dalloc(K, (size_t)ns * nt * nt * sizeof(T)));
  const int ntiles = nt / CHOL_BLOCK;
  CHK(dalloc(Linv, (size_t)ns * ntiles * CHOL_BLOCK * CHOL_BLOCK * sizeof(T)));
  const int nbig = std::max(NIp, NGp);
  CHK(dalloc(Y, (size_t)ns * nbig * nbig * sizeof(T)));
  CHK(dalloc(PS, (size_t)ns * nbig * nbig * sizeof(T)));
  DevBuf Tmp;
  const int64_t sT = (int64_t)TRI_SUPER * nbig;
  CHK(dalloc(Tmp, (size_t)ns * sT * sizeof(T)));
  CHK(dalloc(c->diagAG, (size_t)ns * NGp * sizeof(double)));
  CHK(dalloc(c->Ds, (size_t)ns * nt * sizeof(double)));
  CHK(dalloc(c->Dw, (size_t)ns * NGp * sizeof(double)));
  CHK(dalloc(c->info_d, (size_t)(ns + 2) * sizeof(int)));
  HIPCHK(hipMemsetAsync(c->info_d.p, 0, (size_t)(ns + 2) * sizeof(int), st));
  HIPCHK(hipMemsetAsync(c->Dw.p, 0, (size_t)ns * NGp * sizeof(double), st));
  launch_assemble_local<T>(st, sd, g, ns, K.as<T>(), c->diagAG.as<double>(), c->Ds.as<double>());
  HIPCHK(hipGetLastError());
  launch_weights(st, c->topo.n_iface, c->if_ptr.as<int64_t>(), c->if_sub.as<int32_t>(), c->if_slot.as<int32_t>(),
                 NGp, c->diagAG.as<double>(), c->weighting == CB_W_STIFFNESS, c->Dw.as<double>());
  const int64_t sK = (int64_t)nt * nt;
  const int64_t sL = (int64_t)ntiles * CHOL_BLOCK * CHOL_BLOCK;
  timed(c, "local_cholesky", [&] { cholesky<T>(st, K.as<T>(), nt, sK, nt, ns, Linv.as<T>(), sL, c->info_d.as<int>()); });
  HIPCHK(hipGetLastError());
  // P = A_II^{-1} = D_I (Y_I^T Y_I) D_I
  const int64_t sY = (int64_t)nbig * nbig;
  timed(c, "local_inverse", [&] {
    tri_inverse<T>(st, K.as<T>(), nt, sK, 0, NIp, ns, Linv.as<T>(), sL, Y.as<T>(), NIp, sY, Tmp.as<T>(), sT);
    gemm<T>(st, 1, 0, NIp, NIp, NIp, T(1), Y.as<T>(), NIp, sY, Y.as<T>(), NIp, sY, T(0), PS.as<T>(), NIp, sY, ns,
            GEMM_LOWER | GEMM_KFROM_DIAG);
  });
  CHK(dalloc(c->P, (size_t)ns * NIp * NIp * sizeof(T)));
  symmetrize_scale<T, T>(st, PS.as<T>(), NIp, sY, c->P.as<T>(), NIp, (int64_t)NIp * NIp, c->Ds.as<double>(), nt,
                         NIp, ns);
  // FP64 copy of A_II^{-1} for the harmonic extension of the coarse basis
  DevBuf Pd64;
  const double* Pd = nullptr;
  if (std::is_same<T, double>::value) {
    Pd = reinterpret_cast<const double*>(c->P.p);
  } else {
    CHK(dalloc(Pd64, (size_t)ns * NIp * NIp * sizeof(double)));
    symmetrize_scale<T, double>(st, PS.as<T>(), NIp, sY, Pd64.as<double>(), NIp, (int64_t)NIp * NIp,
                                c->Ds.as<double>(), nt, NIp, ns);
    Pd = Pd64.as<double>();
  }
  HIPCHK(hipGetLastError());
  // K_S^{-1} = D_G (Y_G^T Y_G) D_G, kept in FP64 for the coarse basis
  timed(c, "local_inverse", [&] {
    tri_inverse<T>(st, K.as<T>(), nt, sK, NIp, NGp, ns, Linv.as<T>(), sL, Y.as<T>(), NGp, sY, Tmp.as<T>(), sT);
    gemm<T>(st, 1, 0, NGp, NGp, NGp, T(1), Y.as<T>(), NGp, sY, Y.as<T>(), NGp, sY, T(0), PS.as<T>(), NGp, sY, ns,
            GEMM_LOWER | GEMM_KFROM_DIAG);
  });
  CHK(dalloc(KS, (size_t)ns * NGp * NGp * sizeof(double)));
  symmetrize_scale<T, double>(st, PS.as<T>(), NGp, sY, KS.as<double>(), NGp, (int64_t)NGp * NGp,
                              c->Ds.as<double>() + NIp, nt, NGp, ns);
  HIPCHK(hipGetLastError());
  K.release();
  Y.release();
  PS.release();
  Linv.release();
  Tmp.release();
  // coarse basis on the interface: G = K_S^{-1} C^T, S_c = C G,
  // Phi_G = G S_c^{-1} (C Phi_G = I, energy-minimising for S_A)
  CHK(dalloc(G, (size_t)ns * NGp * NCp * sizeof(double)));
  CHK(dalloc(c->Phi, (size_t)ns * NGp * NCp * sizeof(double)));
  CHK(dalloc(AcLoc, (size_t)ns * NCp * NCp * sizeof(double)));
  {
    DevBuf Cm, Sc;
    const int64_t sG = (int64_t)NGp * NCp, sC = (int64_t)NCp * NCp;
    CHK(dalloc(Cm, (size_t)ns * NCp * NGp * sizeof(double)));
    CHK(dalloc(Sc, (size_t)ns * sC * sizeof(double)));
    launch_build_constraints(st, sd, ns, Cm.as<double>());
    gemm<double>(st, 0, 1, NGp, NCp, NGp, 1.0, KS.as<double>(), NGp, (int64_t)NGp * NGp, Cm.as<double>(), NGp,
                 (int64_t)NCp * NGp, 0.0, G.as<double>(), NCp, sG, ns, 0);
    gemm<double>(st, 0, 0, NCp, NCp, NGp, 1.0, Cm.as<double>(), NGp, (int64_t)NCp * NGp, G.as<double>(), NCp, sG,
                 0.0, Sc.as<double>(), NCp, sC, ns, 0);
    launch_small_spd_inverse(st, sd, ns, Sc.as<double>(), c->info_d.as<int>() + ns);
    gemm<double>(st, 0, 0, NGp, NCp, NCp, 1.0, G.as<double>(), NCp, sG, Sc.as<double>(), NCp, sC, 0.0,
                 c->Phi.as<double>(), NCp, sG, ns, 0);
    HIPCHK(hipGetLastError());
  }
  {
    // full coarse basis Phi = [-A_II^{-1} A_IG Phi_G; Phi_G] and the local
    // coarse matrix as the FP64 Gram matrix Phi^T A_omega Phi
    DevBuf PhiF, V;
    const int64_t sF = (int64_t)nt * NCp;
    CHK(dalloc(PhiF, (size_t)ns * sF * sizeof(double)));
    CHK(dalloc(V, (size_t)ns * sF * sizeof(double)));
    launch_fill(st, (int64_t)ns * sF, 0.0, PhiF.as<double>());
    HIPCHK(hipMemcpy2DAsync(PhiF.as<double>() + (int64_t)NIp * NCp, sF * sizeof(double), c->Phi.p,
                            (size_t)NGp * NCp * sizeof(double), (size_t)NGp * NCp * sizeof(double), ns,
                            hipMemcpyDeviceToDevice, st));
    launch_local_apply(st, sd, g, ns, PhiF.as<double>(), V.as<double>());
    gemm<double>(st, 0, 0, NIp, NCp, NIp, -1.0, Pd, NIp, (int64_t)NIp * NIp, V.as<double>(), NCp, sF, 0.0,
                 PhiF.as<double>(), NCp, sF, ns, 0);
    launch_local_apply(st, sd, g, ns, PhiF.as<double>(), V.as<double>());
    gemm<double>(st, 1, 0, NCp, NCp, nt, 1.0, PhiF.as<double>(), NCp, sF, V.as<double>(), NCp, sF, 0.0,
                 AcLoc.as<double>(), NCp, (int64_t)NCp * NCp, ns, 0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
  }
  Pd64.release();
  // Kt = K_S^{-1} - Phi G^T
  gemm<double>(st, 0, 1, NGp, NGp, NCp, -1.0, c->Phi.as<double>(), NCp, (int64_t)NGp * NCp, G.as<double>(), NCp,
               (int64_t)NGp * NCp, 1.0, KS.as<double>(), NGp, (int64_t)NGp * NGp, ns, 0);
  HIPCHK(hipGetLastError());
  if (std::is_same<T, float>::value) {
    CHK(dalloc(c->Kt, (size_t)ns * NGp * NGp * sizeof(float)));
    convert_to_float(st, (int64_t)ns * NGp * NGp, KS.as<double>(), c->Kt.as<float>());
    HIPCHK(hipStreamSynchronize(st));
    KS.release();
  } else {
    c->Kt.p = KS.p;
    c->Kt.bytes = KS.bytes;
    KS.p = nullptr;
    KS.bytes = 0;
  }
  G.release();
  // coarse matrix and its inverse (FP64)
  const int nc = c->topo.n_coarse, ldc = c->ldc;
  if (nc > 0) {
    CHK(dalloc(Ac, (size_t)ldc * ldc * sizeof(double)));
    launch_fill(st, (int64_t)ldc * ldc, 0.0, Ac.as<double>());
    launch_coarse_assemble(st, nc, ldc, c->cs_ptr.as<int64_t>(), c->cs_sub.as<int32_t>(), c->cs_row.as<int32_t>(),
                           sd, AcLoc.as<double>(), Ac.as<double>());
    HIPCHK(hipGetLastError());
    CHK(dalloc(c->AcKeep, (size_t)ldc * ldc * sizeof(double)));
    HIPCHK(hipMemcpyAsync(c->AcKeep.p, Ac.p, (size_t)ldc * ldc * sizeof(double), hipMemcpyDeviceToDevice, st));
    DevBuf Lc, Yc, PSc, ones;
    const int nct = ldc / CHOL_BLOCK;
    CHK(dalloc(Lc, (size_t)nct * CHOL_BLOCK * CHOL_BLOCK * sizeof(double)));
    ProfScope cps(c, "coarse_factor");
    cholesky<double>(st, Ac.as<double>(), ldc, 0, ldc, 1, Lc.as<double>(), 0, c->info_d.as<int>() + ns + 1);
    CHK(dalloc(Yc, (size_t)ldc * ldc * sizeof(double)));
    DevBuf Tc;
    CHK(dalloc(Tc, (size_t)TRI_SUPER * ldc * sizeof(double)));
    tri_inverse<double>(st, Ac.as<double>(), ldc, 0, 0, ldc, 1, Lc.as<double>(), 0, Yc.as<double>(), ldc, 0,
                        Tc.as<double>(), 0);
    CHK(dalloc(PSc, (size_t)ldc * ldc * sizeof(double)));
    gemm<double>(st, 1, 0, ldc, ldc, ldc, 1.0, Yc.as<double>(), ldc, 0, Yc.as<double>(), ldc, 0, 0.0,
                 PSc.as<double>(), ldc, 0, 1, GEMM_LOWER | GEMM_KFROM_DIAG);
    std::vector<double> one(ldc, 1.0);
    CHK(upload(ones, one, st));
    CHK(dalloc(c->Acinv, (size_t)ldc * ldc * sizeof(double)));
    symmetrize_scale<double, double>(st, PSc.as<double>(), ldc, 0, c->Acinv.as<double>(), ldc, 0,
                                     ones.as<double>(), 0, ldc, 1);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
  }
  std::vector<int> info(ns + 2);
  HIPCHK(hipMemcpyAsync(info.data(), c->info_d.p, (ns + 2) * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int w = 0; w < ns; ++w)
    if (info[w] != 0)
      return fail(CB_ERR_NOT_SPD, "local Cholesky failed in subdomain " + std::to_string(w) + " at row " +
                                      std::to_string(info[w] - 1));
  if (info[ns] != 0) return fail(CB_ERR_NOT_SPD, "singular local coarse matrix");
  if (info[ns + 1] != 0) return fail(CB_ERR_NOT_SPD, "coarse Cholesky failed");
  return CB_OK;
}

}  // namespace

extern "C" {

int cb_factor(cb_ctx* c) {
  if (!c) return fail(CB_ERR_ARG, "null context");
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, c->st));
  c->factored = false;
  g_alloc_stream = c->st;
  int rc = c->precision == CB_FP32_LOCAL ? factor_impl<float>(c) : factor_impl<double>(c);
  if (rc != CB_OK) return rc;
  HIPCHK(hipEventRecord(e1, c->st));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  c->info.t_factor_ms = ms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->factored = true;
  c->info.factored = 1;
  return CB_OK;
}

static int solve_common(cb_ctx* c, double* u_dev, double rtol, int32_t max_iter, int32_t* iters,
                        double* relres) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, c->st));
  int rc = pcg(c, rtol, max_iter, iters, relres);
  if (rc == CB_OK || rc == CB_ERR_NO_CONVERGENCE) {
    launch_gather_dofs(c->st, c->topo.n_dof, c->dof_node.as<int64_t>(), c->x.as<double>(), u_dev);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipEventRecord(e1, c->st));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  c->info.t_solve_ms = ms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int cb_solve(cb_ctx* c, const double* f_nodes_dev, double* u_dev, double rtol, int32_t max_iter,
             int32_t* iters, double* final_relres) {
  if (!c || !u_dev) return fail(CB_ERR_ARG, "null argument");
  if (!c->factored) return fail(CB_ERR_STATE, "cb_solve before cb_factor");
  if (!(rtol > 0.0) || max_iter < 0) return fail(CB_ERR_ARG, "rtol must be > 0 and max_iter >= 0");
  const int64_t nn = c->n_nodes();
  const double* f = f_nodes_dev;
  if (!f) {
    launch_fill(c->st, nn, 1.0, c->t1.as<double>());
    f = c->t1.as<double>();
  }
  GridDesc g{c->N, c->h};
  launch_load(c->st, g, c->cellinfo.as<int32_t>(), c->Mc.as<double>(), c->dofmask.as<uint8_t>(), f,
              c->bgrid.as<double>());
  HIPCHK(hipGetLastError());
  return solve_common(c, u_dev, rtol, max_iter, iters, final_relres);
}

int cb_solve_rhs(cb_ctx* c, const double* b_dev, double* u_dev, double rtol, int32_t max_iter, int32_t* iters,
                 double* final_relres) {
  if (!c || !u_dev || !b_dev) return fail(CB_ERR_ARG, "null argument");
  if (!c->factored) return fail(CB_ERR_STATE, "cb_solve_rhs before cb_factor");
  if (!(rtol > 0.0) || max_iter < 0) return fail(CB_ERR_ARG, "rtol must be > 0 and max_iter >= 0");
  launch_fill(c->st, c->n_nodes(), 0.0, c->bgrid.as<double>());
  launch_scatter_dofs(c->st, c->topo.n_dof, c->dof_node.as<int64_t>(), b_dev, c->bgrid.as<double>());
  HIPCHK(hipGetLastError());
  return solve_common(c, u_dev, rtol, max_iter, iters, final_relres);
}

int cb_apply_operator(cb_ctx* c, const double* x_dev, double* y_dev) {
  if (!c || !x_dev || !y_dev) return fail(CB_ERR_ARG, "null argument");
  const int64_t nn = c->n_nodes();
  launch_fill(c->st, nn, 0.0, c->x.as<double>());
  launch_scatter_dofs(c->st, c->topo.n_dof, c->dof_node.as<int64_t>(), x_dev, c->x.as<double>());
  CHK(apply_A_grid(c, c->x.as<double>(), c->q.as<double>()));
  launch_gather_dofs(c->st, c->topo.n_dof, c->dof_node.as<int64_t>(), c->q.as<double>(), y_dev);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->st));
  return CB_OK;
}

int cb_apply_preconditioner(cb_ctx* c, const double* r_dev, double* z_dev) {
  if (!c || !r_dev || !z_dev) return fail(CB_ERR_ARG, "null argument");
  if (!c->factored) return fail(CB_ERR_STATE, "preconditioner applied before cb_factor");
  const int64_t nn = c->n_nodes();
  launch_fill(c->st, nn, 0.0, c->r.as<double>());
  launch_scatter_dofs(c->st, c->topo.n_dof, c->dof_node.as<int64_t>(), r_dev, c->r.as<double>());
  CHK(apply_M_grid(c, c->r.as<double>(), c->z.as<double>()));
  launch_gather_dofs(c->st, c->topo.n_dof, c->dof_node.as<int64_t>(), c->z.as<double>(), z_dev);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->st));
  return CB_OK;
}

int cb_load(cb_ctx* c, const double* f_nodes_dev, double* b_dev) {
  if (!c || !b_dev) return fail(CB_ERR_ARG, "null argument");
  const int64_t nn = c->n_nodes();
  const double* f = f_nodes_dev;
  if (!f) {
    launch_fill(c->st, nn, 1.0, c->t1.as<double>());
    f = c->t1.as<double>();
  }
  GridDesc g{c->N, c->h};
  launch_load(c->st, g, c->cellinfo.as<int32_t>(), c->Mc.as<double>(), c->dofmask.as<uint8_t>(), f,
              c->bgrid.as<double>());
  launch_gather_dofs(c->st, c->topo.n_dof, c->dof_node.as<int64_t>(), c->bgrid.as<double>(), b_dev);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->st));
  return CB_OK;
}

int cb_grad(cb_ctx* c, const double* u_dev, const double* lam_dev, double* dJ_dtheta_dev, double* dJ_df_dev) {
  if (!c || !u_dev || !lam_dev) return fail(CB_ERR_ARG, "null argument");
  const int64_t nn = c->n_nodes();
  double* ug = c->t1.as<double>();
  double* lg = c->t2.as<double>();
  launch_fill(c->st, nn, 0.0, ug);
  launch_fill(c->st, nn, 0.0, lg);
  launch_scatter_dofs(c->st, c->topo.n_dof, c->dof_node.as<int64_t>(), u_dev, ug);
  launch_scatter_dofs(c->st, c->topo.n_dof, c->dof_node.as<int64_t>(), lam_dev, lg);
  GridDesc g{c->N, c->h};
  if (dJ_dtheta_dev)
    launch_grad_theta(c->st, g, c->cellinfo.as<int32_t>(), c->kappa.as<double>(), c->Kc.as<double>(), ug, lg,
                      dJ_dtheta_dev);
  if (dJ_df_dev)
    launch_load(c->st, g, c->cellinfo.as<int32_t>(), c->Mc.as<double>(), nullptr, lg, dJ_df_dev);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->st));
  return CB_OK;
}

int cb_query(const cb_ctx* c, cb_info* out) {
  if (!c || !out) return fail(CB_ERR_ARG, "null argument");
  *out = c->info;
  out->n_fp64_fallbacks = c->n_fallbacks;
  out->factored = c->factored ? 1 : 0;
  return CB_OK;
}

int cb_export_indexing(const cb_ctx* c, uint8_t* cell_status, int32_t* cell_count, int64_t* dof_node,
                       int32_t* card, int64_t* obj_ptr, int64_t* obj_dofs, int8_t* obj_type,
                       int32_t* coarse_of_obj) {
  if (!c) return fail(CB_ERR_ARG, "null context");
  const Topology& t = c->topo;
  const int64_t ncell = (int64_t)c->N * c->N * c->N;
  if (cell_status)
    for (int64_t i = 0; i < ncell; ++i)
      cell_status[i] = c->count[i] == 0 ? 0 : (c->count[i] == 512 ? 2 : 1);
  if (cell_count) std::memcpy(cell_count, c->count.data(), ncell * sizeof(int32_t));
  if (dof_node) std::memcpy(dof_node, t.dof_node.data(), t.n_dof * sizeof(int64_t));
  if (card)
    for (int64_t d = 0; d < t.n_dof; ++d) card[d] = t.card[d];
  if (obj_ptr) std::memcpy(obj_ptr, t.obj_ptr.data(), t.obj_ptr.size() * sizeof(int64_t));
  if (obj_dofs) std::memcpy(obj_dofs, t.obj_dofs.data(), t.obj_dofs.size() * sizeof(int64_t));
  if (obj_type) std::memcpy(obj_type, t.obj_type.data(), t.obj_type.size());
  if (coarse_of_obj) std::memcpy(coarse_of_obj, t.coarse_of_obj.data(), t.coarse_of_obj.size() * sizeof(int32_t));
  return CB_OK;
}

int cb_export_cut_matrices(const cb_ctx* c, double* K, double* M, int64_t* cut_cells) {
  if (!c) return fail(CB_ERR_ARG, "null context");
  const int64_t n = (int64_t)c->cut_cells.size();
  if (K && n) HIPCHK(hipMemcpy(K, c->Kc.p, n * PACK36 * sizeof(double), hipMemcpyDeviceToHost));
  if (M && n) HIPCHK(hipMemcpy(M, c->Mc.p, n * PACK36 * sizeof(double), hipMemcpyDeviceToHost));
  if (cut_cells && n) std::memcpy(cut_cells, c->cut_cells.data(), n * sizeof(int64_t));
  return CB_OK;
}

int cb_export_coarse(const cb_ctx* c, double* Ac) {
  if (!c || !Ac) return fail(CB_ERR_ARG, "null argument");
  if (!c->factored) return fail(CB_ERR_STATE, "coarse matrix requested before cb_factor");
  const int nc = c->topo.n_coarse, ldc = c->ldc;
  if (nc == 0) return CB_OK;
  HIPCHK(hipMemcpy2D(Ac, nc * sizeof(double), c->AcKeep.p, ldc * sizeof(double), nc * sizeof(double), nc,
                     hipMemcpyDeviceToHost));
  return CB_OK;
}

int cb_profile(cb_ctx* c, int32_t enable) {
  if (!c) return fail(CB_ERR_ARG, "null context");
  c->prof = enable != 0;
  return CB_OK;
}

int cb_profile_time(cb_ctx* c, const char* name, double* total_ms, int64_t* launches) {
  if (!c || !name) return fail(CB_ERR_ARG, "null argument");
  HIPCHK(hipStreamSynchronize(c->st));
  double tot = 0.0;
  int64_t n = 0;
  auto it = c->prof_ev.find(name);
  if (it != c->prof_ev.end())
    for (auto& e : it->second.ev) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e.first, e.second));
      tot += ms;
      ++n;
    }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = n;
  return CB_OK;
}

void cb_destroy(cb_ctx* c) {
  if (!c) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  else (void)hipDeviceSynchronize();
  delete c;
}

}  // extern "C"
