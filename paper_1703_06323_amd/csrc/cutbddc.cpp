// C ABI of the cut-cell BDDC-PCG solver (see include/cutbddc.h): context,
// device buffers and the orchestration of setup / factor / solve.
#include "cutbddc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <memory>
#include <numeric>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "bddc.h"
#include "coarse_nd.h"
#include "common.h"
#include "dense.h"
#include "indexing.h"
#include "manufactured.h"
#include "nitsche.h"
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

// Streams, events and pinned staging blocks of finished calls and destroyed
// contexts, kept for later ones: creating and destroying them costs about
// 0.2 ms per context, as much as a small solver step.  Kept per device;
// whatever comes back is idle (a context synchronises its streams before it
// hands them back, a call's timing events have completed or are re-recorded
// before any read).  The pool lives until the process ends.
struct HandlePool {
  std::mutex mu;
  std::map<int, std::vector<hipStream_t>> streams;      // non-blocking, default priority
  std::map<int, std::vector<hipEvent_t>> sync_events;   // timing disabled
  std::map<int, std::vector<hipEvent_t>> time_events;   // timing enabled
  std::map<int, std::vector<std::pair<size_t, void*>>> pinned;
};
HandlePool& handle_pool() {
  static HandlePool* p = new HandlePool;
  return *p;
}
int current_device() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d;
}
template <typename H>
bool pool_take(std::map<int, std::vector<H>>& m, int dev, H* out) {
  std::lock_guard<std::mutex> g(handle_pool().mu);
  auto& v = m[dev];
  if (v.empty()) return false;
  *out = v.back();
  v.pop_back();
  return true;
}
template <typename H>
void pool_put(std::map<int, std::vector<H>>& m, int dev, H h) {
  std::lock_guard<std::mutex> g(handle_pool().mu);
  m[dev].push_back(h);
}
hipError_t pooled_stream(hipStream_t* s) {
  if (pool_take(handle_pool().streams, current_device(), s)) return hipSuccess;
  return hipStreamCreateWithFlags(s, hipStreamNonBlocking);
}
hipError_t pooled_sync_event(hipEvent_t* e) {
  if (pool_take(handle_pool().sync_events, current_device(), e)) return hipSuccess;
  return hipEventCreateWithFlags(e, hipEventDisableTiming);
}
hipError_t pooled_time_event(hipEvent_t* e) {
  if (pool_take(handle_pool().time_events, current_device(), e)) return hipSuccess;
  return hipEventCreate(e);
}
// pinned block of at least `bytes` (its capacity in *cap)
hipError_t pooled_pinned(void** p, size_t bytes, size_t* cap) {
  {
    std::lock_guard<std::mutex> g(handle_pool().mu);
    auto& v = handle_pool().pinned[current_device()];
    for (size_t i = 0; i < v.size(); ++i)
      if (v[i].first >= bytes) {
        *cap = v[i].first;
        *p = v[i].second;
        v.erase(v.begin() + (std::ptrdiff_t)i);
        return hipSuccess;
      }
  }
  *cap = std::max<size_t>(bytes, 4096);
  return hipHostMalloc(p, *cap, hipHostMallocDefault);
}

// Two timing events owned by one call, handed back on every exit (error
// returns included).
struct EventPair {
  hipEvent_t* a;
  hipEvent_t* b;
  ~EventPair() {
    const int dev = current_device();
    if (*a) pool_put(handle_pool().time_events, dev, *a);
    if (*b) pool_put(handle_pool().time_events, dev, *b);
  }
};

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
constexpr int32_t HIST_CAP = 1024;                   // PCG iterations recorded per problem

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

// Opt-in poison mode (environment CUTBDDC_POISON=1): every buffer handed
// out is filled with 0xFF bytes first (NaN in every float, -1 in every
// signed integer), so a read of data that nothing wrote shows up in the
// results instead of reusing what an earlier owner of the block left.
bool poison_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("CUTBDDC_POISON");
    return e && e[0] == '1';
  }();
  return on;
}

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
  if (poison_enabled()) {
    // finished before the call returns, whichever stream then uses the block
    HIPCHK(hipMemsetAsync(b.p, 0xFF, bytes, g_alloc_stream));
    HIPCHK(hipStreamSynchronize(g_alloc_stream));
  }
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
double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Pinned host staging for the large setup copies (cell counts down, cell
// info and cut-cell lists up), kept per host thread and grown on demand.
// A setup call synchronises its stream before it returns, so the next call
// on the same thread may reuse the buffer.
struct PinnedStage {
  void* p = nullptr;
  size_t bytes = 0;
  ~PinnedStage() {
    if (p) (void)hipHostFree(p);
  }
  void* get(size_t need) {
    if (need > bytes) {
      if (p) (void)hipHostFree(p);
      p = nullptr;
      bytes = 0;
      const size_t want = std::max<size_t>(need, (size_t)1 << 20);
      if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) return nullptr;
      bytes = want;
    }
    return p;
  }
};
thread_local PinnedStage t_stage;

}  // namespace

struct ProfEntry {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
};

// Host data of one problem of a context.
struct ProbHost {
  int N = 0, m = 0, ns = 0;
  double h = 0;
  int nb = 0, ball_off = 0;
  int64_t n_active = 0, n_cut = 0, n_cut_stored = 0;
  int64_t n_dof = 0, n_iface = 0;
  int32_t n_obj = 0, n_coarse = 0, maxC = 0;
  int64_t cell_off = 0, node_off = 0, dof_off = 0, cut_off = 0, obj_off = 0;
  int32_t sub_off = 0, coarse_off = 0, ldc = 0, chunk_off = 0;
  int64_t ac_off = 0, prow_off = 0;
  int64_t iface_off = 0;
  cb_info info{};
};

// Problems of equal padded coarse order, factored as one batch.
struct CoarseGroup {
  int ldc = 0;
  int64_t ac_off = 0;
  std::vector<int> probs;   // problem ids, in block order
};

struct cb_ctx {
  hipStream_t st = nullptr;
  bool prof = false;
  std::map<std::string, ProfEntry> prof_ev;
  int P = 0;
  std::vector<ProbHost> pb;
  int s = 0;
  int weighting = 1, objects = 0, variant = 1, precision = 0, full_elements = 0;
  bool nitsche = false;       // Nitsche's weak Dirichlet condition on the ball surfaces
  bool kappa_given = false;   // some problem brought its own kappa
  std::vector<double> radii_h;   // ball radii, in the order of the ball array
  // sphere rules of the balls (built on first use) and beta_e of every
  // stored cut cell (Nitsche only)
  DevBuf sr_ball, sr_t, sr_w, sr_c, sr_s, sr_d, sr_k, beta_d;
  bool sr_ready = false;
  NitscheRule sr{};
  int64_t n_cells_tot = 0, nn = 0, n_dof_tot = 0, n_iface_tot = 0, n_cut_tot = 0;
  int ns = 0, nc_tot = 0;
  int32_t n_chunks = 0;
  int64_t n_prows = 0, ac_total = 0;
  std::vector<CoarseGroup> groups;
  double xi[8];
  double Kref[64], Mref[64];
  bool factored = false;
  int n_fallbacks = 0;

  // per-problem device tables
  DevBuf kdiag_d;            // diagonal of the uncut reference stiffness (variant 2)
  DevBuf op_off_d, op_prob_d, op_geom_d;   // operator work items (BatchDev::op_off, op_prob, op_geom)
  int32_t op_items = 0, op_box = 0, op_lx = 0, op_lc = 0, op_xp = 0, op_cp = 0;
  DevBuf prob_d, cell_off_d, node_off_d, sub_off_d, dof_off_d, chunk_ptr_d, prow_off_d, coarse_prob_d, sub_prob_d,
      sub_blk_d;
  // device indexing work arrays (kept for the index export)
  DevBuf iwork;
  IndexWork iw{};
  // grid data (concatenated)
  DevBuf xi_d, balls, kappa, count_d, cellinfo, cut_d, Kc, Mc, Kf, dofmask, dof_node;
  // subdomain index data
  int NIp = 0, NGp = 0, NCp = 0, nt = 0;
  DevBuf nI, nG, nC, Iidx, Gidx, Gobj, Cids, bloc, if_ptr, if_sub, if_slot, iface_node, cs_ptr, cs_sub,
      cs_row;
  // factor results
  DevBuf P_, Kt, Phi, Dw, diagAG, Ds, Acinv, AcKeep, info_d;
  DevBuf Phi32;   // FP32 copy of Phi for the products of the FP32-local path
  // coarse problem by one level of nested dissection (coarse_nd.h), chosen
  // at each cb_factor for single-problem contexts; Acinv is then unused
  struct {
    bool on = false;
    int Lo = 0, Lso = 0, Ls = 0, n_s = 0, n_o_max = 0;
    DevBuf oid, sid, sep, pos, Yo, W, WT, Ys, to, rs, us, xs, info;
    NDDev dev() const {
      NDDev d;
      d.Lo = Lo;
      d.Lso = Lso;
      d.Ls = Ls;
      d.n_s = n_s;
      d.oid = oid.as<int32_t>();
      d.sid = sid.as<int32_t>();
      d.sep = sep.as<int32_t>();
      d.pos = pos.as<int32_t>();
      return d;
    }
  } nd;
  DevBuf optr_d, omem_d;   // object member lists per subdomain (built at factorisation)
  // work vectors and PCG state
  DevBuf x, r, z, p, q, t1, t2, t3, zbuf, cloc, cvec, tcvec, ucvec, partial, scal, bgrid;
  DevBuf pq_part, rr_part;   // per node block (SEG_ALIGN nodes): parts of p.q and r.r
  DevBuf hist;               // PCG coefficients per problem and iteration (launch_cg_check)
  bool solved = false;
  DevBuf params, active, itc, status, relres_d, nact_d, fptrs, uptrs;
  // pinned host staging: [0] n_active, then P iterations, P statuses, P relres, 2P pointers
  void* pin = nullptr;
  size_t pin_cap = 0;
  int dev = 0;                       // device of the context's streams, events and pinned block
  int32_t* pin_nact_dev = nullptr;   // device address of pin_nact()
  // second and third streams for work that overlaps the coarse factorisation
  hipStream_t aux_st = nullptr, aux_st3 = nullptr;
  hipEvent_t aux_ev = nullptr, aux_ev3 = nullptr;
  hipEvent_t fill_ev = nullptr;   // identity fills of the local inverses done
  hipEvent_t nact_ev = nullptr;   // readback of the running-problem count
  // captured PCG iteration
  hipStream_t cap_st = nullptr;
  hipGraphExec_t graph = nullptr;
  bool graph_failed = false;
  cb_info info{};

  ~cb_ctx() {
    if (graph) (void)hipGraphExecDestroy(graph);
    // streams, events and the pinned block go back to the handle pool, idle
    HandlePool& hp = handle_pool();
    for (hipStream_t s : {cap_st, aux_st, aux_st3})
      if (s && hipStreamSynchronize(s) == hipSuccess) pool_put(hp.streams, dev, s);
      else if (s) (void)hipStreamDestroy(s);
    for (hipEvent_t e : {aux_ev, aux_ev3, fill_ev, nact_ev})
      if (e) pool_put(hp.sync_events, dev, e);
    if (pin) pool_put(hp.pinned, dev, std::make_pair(pin_cap, pin));
    for (auto& kv : prof_ev)
      for (auto& e : kv.second.ev) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
      }
  }
  int32_t* pin_nact() const { return static_cast<int32_t*>(pin); }
  int32_t* pin_it() const { return static_cast<int32_t*>(pin) + 2; }
  int32_t* pin_status() const { return pin_it() + P; }
  double* pin_relres() const {
    const size_t off = (((size_t)(2 + 2 * P) * sizeof(int32_t)) + 7) & ~(size_t)7;
    return reinterpret_cast<double*>(static_cast<char*>(pin) + off);
  }
  const double** pin_fptrs() const { return reinterpret_cast<const double**>(pin_relres() + P); }
  double** pin_uptrs() const { return reinterpret_cast<double**>(pin_relres() + 2 * P); }
  size_t pin_bytes() const {
    return ((((size_t)(2 + 2 * P) * sizeof(int32_t)) + 7) & ~(size_t)7) + (size_t)3 * P * sizeof(double);
  }

  BatchDev batch(bool masked) const {
    BatchDev b;
    b.P = P;
    b.prob = prob_d.as<ProbDev>();
    b.cell_off = cell_off_d.as<int64_t>();
    b.node_off = node_off_d.as<int64_t>();
    b.active = masked ? active.as<int32_t>() : nullptr;
    b.op_off = op_off_d.as<int32_t>();
    b.op_prob = op_prob_d.as<int32_t>();
    b.op_geom = op_geom_d.as<int32_t>();
    b.op_box = op_box;
    b.op_lx = op_lx;
    b.op_lc = op_lc;
    b.op_xp = op_xp;
    b.op_cp = op_cp;
    return b;
  }
  GridDev grid() const {
    GridDev g;
    g.prob = prob_d.as<ProbDev>();
    g.s = s;
    g.cellinfo = cellinfo.as<int32_t>();
    g.kappa = kappa.as<double>();
    g.Kc = Kc.as<double>();
    return g;
  }
  // Subdomain data starting at subdomain w0.
  SubDev sub(int w0 = 0, bool masked = false) const {
    const int s1 = s + 1;
    SubDev d;
    d.NIp = NIp;
    d.NGp = NGp;
    d.NCp = NCp;
    d.nI = nI.as<int32_t>() + w0;
    d.nG = nG.as<int32_t>() + w0;
    d.nC = nC.as<int32_t>() + w0;
    d.I_idx = Iidx.as<int64_t>() + (int64_t)w0 * NIp;
    d.G_idx = Gidx.as<int64_t>() + (int64_t)w0 * NGp;
    d.G_obj = Gobj.as<int32_t>() + (int64_t)w0 * NGp;
    d.C_ids = Cids.as<int32_t>() + (int64_t)w0 * NCp;
    d.bloc = bloc.as<int32_t>() + (int64_t)w0 * s1 * s1 * s1;
    d.sub_prob = sub_prob_d.as<int32_t>() + w0;
    d.sub_blk = sub_blk_d.as<int32_t>() + w0;
    d.active = masked ? active.as<int32_t>() : nullptr;
    d.optr = optr_d.p ? optr_d.as<int32_t>() + (int64_t)w0 * (NCp + 1) : nullptr;
    d.omem = omem_d.p ? omem_d.as<int32_t>() + (int64_t)w0 * NGp : nullptr;
    return d;
  }
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
    if (!c->prof) return;
    if (!b || !e) {
      if (b) (void)hipEventDestroy(b);
      return;
    }
    (void)hipEventRecord(e, c->st);
    c->prof_ev[name].ev.emplace_back(b, e);
  }
};

template <typename F>
void timed(cb_ctx* c, const char* name, F&& f) {
  ProfScope ps(c, name);
  f();
}

int apply_A_grid(cb_ctx* c, const double* x, double* y, bool masked, double* dpart = nullptr) {
  ProfScope ps(c, "apply_A");
  launch_apply_A(c->st, c->batch(masked), c->nn, c->op_items, c->cellinfo.as<int32_t>(), c->kappa.as<double>(),
                 c->Kf.as<double>(), c->dofmask.as<uint8_t>(), x, y, dpart);
  return CB_OK;
}

// z = M r on grid vectors (eq. bddc), steps (1)-(7), for every problem (or,
// masked, for the problems whose PCG still runs).
int apply_M_grid(cb_ctx* c, const double* r, double* z, bool masked, bool cleared = false) {
  hipStream_t st = c->st;
  const SubDev sd = c->sub(0, masked);
  const int64_t nn = c->nn;
  double* t1 = c->t1.as<double>();
  double* t2 = c->t2.as<double>();
  double* t3 = c->t3.as<double>();
  // (1) delta_I = A_II^{-1} r_I (t1 and z start at zero: cleared here or,
  // within a PCG iteration, by the x, r update)
  if (!cleared) launch_fill(st, nn, 0.0, t1);
  timed(c, "apply_interior", [&] {
    if (c->precision == CB_FP32_LOCAL)
      launch_apply_interior<float>(st, sd, c->ns, c->P_.as<float>(), r, nullptr, t1);
    else
      launch_apply_interior<double>(st, sd, c->ns, c->P_.as<double>(), r, nullptr, t1);
  });
  // (2) rhat_G = r_G - (A delta)_G
  CHK(apply_A_grid(c, t1, t2, masked));
  // (3)-(4) weighted restriction, constrained Neumann solves, coarse rhs
  timed(c, "apply_neumann", [&] {
    if (c->precision == CB_FP32_LOCAL)
      launch_apply_neumann<float, float>(st, sd, c->ns, c->Kt.as<float>(), c->Phi32.as<float>(), c->Dw.as<double>(),
                                  r, t2, c->zbuf.as<double>(), c->cloc.as<double>());
    else
      launch_apply_neumann<double, double>(st, sd, c->ns, c->Kt.as<double>(), c->Phi.as<double>(),
                                   c->Dw.as<double>(), r, t2, c->zbuf.as<double>(), c->cloc.as<double>());
  });
  // (5) coarse correction
  if (c->nc_tot > 0) {
    launch_coarse_rhs(st, c->nc_tot, c->cs_ptr.as<int64_t>(), c->cs_sub.as<int32_t>(), c->cs_row.as<int32_t>(),
                      c->NCp, c->cloc.as<double>(), c->cvec.as<double>());
    timed(c, "coarse_gemv", [&] {
      if (c->nd.on)
        launch_nd_solve(st, c->batch(masked), c->nd.dev(), c->nd.Yo.as<double>(), c->nd.W.as<double>(),
                        c->nd.WT.as<double>(), c->nd.Ys.as<double>(), c->cvec.as<double>(), c->nd.to.as<double>(),
                        c->nd.rs.as<double>(), c->nd.us.as<double>(), c->nd.xs.as<double>(),
                        c->ucvec.as<double>());
      else
        launch_coarse_gemv(st, c->batch(masked), c->nc_tot, c->coarse_prob_d.as<int32_t>(), c->Acinv.as<double>(),
                           c->cvec.as<double>(), c->tcvec.as<double>(), c->ucvec.as<double>());
    });
    if (c->precision == CB_FP32_LOCAL)
      launch_add_coarse<float>(st, sd, c->ns, c->Phi32.as<float>(), c->ucvec.as<double>(), c->zbuf.as<double>());
    else
      launch_add_coarse<double>(st, sd, c->ns, c->Phi.as<double>(), c->ucvec.as<double>(), c->zbuf.as<double>());
  }
  // (6) weighted average on the interface
  if (!cleared) launch_fill(st, nn, 0.0, z);
  launch_iface_average(st, c->n_iface_tot, c->iface_node.as<int64_t>(), c->if_ptr.as<int64_t>(),
                       c->if_sub.as<int32_t>(), c->if_slot.as<int32_t>(), c->NGp, c->Dw.as<double>(),
                       c->zbuf.as<double>(), z);
  // (7) harmonic extension: z_I = A_II^{-1} (r - A [0; u_G])_I
  CHK(apply_A_grid(c, z, t3, masked));
  timed(c, "apply_interior", [&] {
    if (c->precision == CB_FP32_LOCAL)
      launch_apply_interior<float>(st, sd, c->ns, c->P_.as<float>(), r, t3, z);
    else
      launch_apply_interior<double>(st, sd, c->ns, c->P_.as<double>(), r, t3, z);
  });
  return CB_OK;
}

void dot(cb_ctx* c, const double* a, const double* b, int slot, bool masked) {
  launch_dot(c->st, c->batch(masked), c->chunk_ptr_d.as<int32_t>(), c->n_chunks, a, b, c->partial.as<double>(),
             c->scal.as<double>() + slot, CG_S);
}

// One PCG iteration for every running problem: q = A p (with the block
// parts of p.q), x and r update (which also clears the preconditioner's
// scratch vectors and forms the block parts of r.r), convergence test,
// z = M r, chunk parts of r.z, p update (which sums them).
int pcg_body(cb_ctx* c) {
  hipStream_t st = c->st;
  double* S = c->scal.as<double>();
  const BatchDev bm = c->batch(true);
  CHK(apply_A_grid(c, c->p.as<double>(), c->q.as<double>(), true, c->pq_part.as<double>()));
  launch_cg_update_xr(st, bm, c->nn, S, c->pq_part.as<double>(), c->p.as<double>(), c->q.as<double>(),
                      c->x.as<double>(), c->r.as<double>(), c->t1.as<double>(), c->z.as<double>(),
                      c->rr_part.as<double>());
  launch_cg_check(st, c->P, c->node_off_d.as<int64_t>(), c->rr_part.as<double>(), c->params.as<double>(), S,
                  c->active.as<int32_t>(), c->itc.as<int32_t>(), c->status.as<int32_t>(), c->relres_d.as<double>(),
                  c->nact_d.as<int32_t>(), c->pin_nact_dev, c->hist.as<double>(), HIST_CAP);
  CHK(apply_M_grid(c, c->r.as<double>(), c->z.as<double>(), true, true));
  launch_dot_chunks(st, bm, c->chunk_ptr_d.as<int32_t>(), c->n_chunks, c->r.as<double>(), c->z.as<double>(),
                    c->partial.as<double>());
  launch_cg_update_p(st, bm, c->nn, S, c->chunk_ptr_d.as<int32_t>(), c->partial.as<double>(), c->z.as<double>(),
                     c->p.as<double>());
  return CB_OK;
}

bool graphs_enabled() {
  const char* e = std::getenv("CUTBDDC_GRAPH");
  return !(e && e[0] == '0');
}

// Captures pcg_body into an executable graph (once per factorisation).  The
// capture runs on a private stream; replays go to the context's stream.
int capture_body(cb_ctx* c) {
  if (c->graph || c->graph_failed) return CB_OK;
  if (!c->cap_st) HIPCHK(pooled_stream(&c->cap_st));
  hipStream_t user = c->st;
  c->st = c->cap_st;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(c->cap_st, hipStreamCaptureModeThreadLocal);
  int rc = CB_OK;
  if (e == hipSuccess) {
    rc = pcg_body(c);
    e = hipStreamEndCapture(c->cap_st, &g);
  }
  c->st = user;
  if (rc != CB_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e == hipSuccess && g) e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    // fall back to issuing the iteration eagerly
    (void)hipGetLastError();
    c->graph = nullptr;
    c->graph_failed = true;
  }
  return CB_OK;
}

// PCG on grid vectors for all problems at once: b in c->bgrid, x in c->x.
// Per-problem results land in the pinned staging arrays.  A problem whose
// residual meets the tolerance stops; the others continue.  Returns the
// number of iteration sweeps run.
int pcg(cb_ctx* c, double rtol, int32_t max_iter, int* sweeps) {
  hipStream_t st = c->st;
  const int64_t nn = c->nn;
  double* S = c->scal.as<double>();
  launch_set_params(st, c->params.as<double>(), rtol, max_iter);
  launch_fill(st, nn, 0.0, c->x.as<double>());
  launch_copy(st, nn, c->bgrid.as<double>(), c->r.as<double>());
  dot(c, c->bgrid.as<double>(), c->bgrid.as<double>(), 4, false);
  launch_cg_init(st, c->P, c->params.as<double>(), S, c->active.as<int32_t>(), c->itc.as<int32_t>(),
                 c->status.as<int32_t>(), c->relres_d.as<double>(), c->nact_d.as<int32_t>());
  HIPCHK(hipGetLastError());
  // The count of running problems after the initial check is read back
  // through an event while the first preconditioner apply is queued and the
  // iteration graph captured: with no running problem that apply is masked
  // by the device's active flags and the loop is skipped.  Without any DOF
  // (where some grids would be empty) the apply waits for the count.
  if (!c->nact_ev) HIPCHK(pooled_sync_event(&c->nact_ev));
  HIPCHK(hipMemcpyAsync(c->pin_nact(), c->nact_d.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipEventRecord(c->nact_ev, st));
  const bool use_graph = graphs_enabled() && !c->prof;
  auto first_apply = [&]() -> int {
    CHK(apply_M_grid(c, c->r.as<double>(), c->z.as<double>(), true));
    launch_copy(st, nn, c->z.as<double>(), c->p.as<double>());
    dot(c, c->r.as<double>(), c->z.as<double>(), 3, true);
    HIPCHK(hipGetLastError());
    if (use_graph) CHK(capture_body(c));
    return CB_OK;
  };
  const bool early = c->n_dof_tot > 0;
  if (early) CHK(first_apply());
  HIPCHK(hipEventSynchronize(c->nact_ev));
  int32_t n_active = *static_cast<volatile int32_t*>(c->pin_nact());
  int k = 0;
  if (n_active > 0) {
    if (!early) CHK(first_apply());
    auto issue = [&]() -> int {
      if (use_graph && c->graph) HIPCHK(hipGraphLaunch(c->graph, st));
      else CHK(pcg_body(c));
      HIPCHK(hipGetLastError());
      ++k;
      return CB_OK;
    };
    // the check kernel of every iteration writes the count of running
    // problems straight to pinned host memory; the event marks the end of
    // an iteration (a later iteration may already have lowered the count,
    // which only ends the loop with work that is queued anyway)
    auto queue_read = [&]() -> int {
      HIPCHK(hipEventRecord(c->nact_ev, st));
      return CB_OK;
    };
    // One iteration stays queued ahead of the host's convergence readback:
    // the readback after iteration k overlaps iteration k+1, which is a
    // masked no-op for every problem that has stopped (the device stops a
    // problem at its own max_iter, so the loop always ends).
    CHK(issue());
    CHK(queue_read());
    for (;;) {
      const bool ahead = k <= max_iter;
      if (ahead) CHK(issue());
      HIPCHK(hipEventSynchronize(c->nact_ev));
      n_active = *static_cast<volatile int32_t*>(c->pin_nact());
      if (n_active == 0 || !ahead) break;
      CHK(queue_read());
    }
  }
  HIPCHK(hipMemcpyAsync(c->pin_it(), c->itc.p, c->P * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(c->pin_status(), c->status.p, c->P * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(c->pin_relres(), c->relres_d.p, c->P * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (sweeps) *sweeps = k;
  return CB_OK;
}

// Status of problem p after pcg().
int pcg_status(cb_ctx* c, int p) {
  const int s = c->pin_status()[p];
  if (s == 3) return fail(CB_ERR_NOT_SPD, "PCG breakdown (non-finite residual) in problem " + std::to_string(p));
  if (s != 1) return fail(CB_ERR_NO_CONVERGENCE, "PCG reached max_iter in problem " + std::to_string(p));
  return CB_OK;
}

int validate_problem(const cb_problem* p) {
  const int N = p->n_cells, s = p->sub_cells;
  if (N < 1 || s < 1 || N % s != 0) return fail(CB_ERR_ARG, "n_cells must be >= 1 and divisible by sub_cells");
  if (N > 1024) return fail(CB_ERR_ARG, "n_cells too large");
  if (p->n_balls < 0 || (p->n_balls > 0 && (!p->ball_centres || !p->ball_radii)))
    return fail(CB_ERR_ARG, "invalid ball arrays");
  if (p->weighting < 0 || p->weighting > 1 || p->objects < 0 || p->objects > 1 || p->coarse_variant < 0 ||
      p->coarse_variant > 2 || p->local_precision < 0 || p->local_precision > 1 || p->cut_boundary < 0 ||
      p->cut_boundary > 1)
    return fail(CB_ERR_ARG, "invalid option value");
  for (int i = 0; i < p->n_balls; ++i) {
    if (!(p->ball_radii[i] > 0.0) || !std::isfinite(p->ball_radii[i]))
      return fail(CB_ERR_ARG, "ball radius must be positive and finite");
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(p->ball_centres[3 * i + d])) return fail(CB_ERR_ARG, "ball centre not finite");
  }
  {
    // the per-subdomain kernels hold padded local vectors and partial sums in
    // LDS: reject block sizes whose uncut subdomain (interior (s-1)^3 nodes,
    // interface (s+1)^3 - (s-1)^3, 26 coarse DOFs) would not fit
    const int nI = (s - 1) * (s - 1) * (s - 1), nG = (s + 1) * (s + 1) * (s + 1) - nI;
    const size_t need = bddc_lds_need(round_up(std::max(1, nI), CHOL_BLOCK), round_up(nG, CHOL_BLOCK), 32, s,
                                      p->local_precision);
    if (need > LDS_BYTES)
      return fail(CB_ERR_ARG, "sub_cells = " + std::to_string(s) + " needs " + std::to_string(need) +
                                  " bytes of LDS per subdomain workgroup (limit " + std::to_string(LDS_BYTES) + ")");
  }
  const int64_t ncell = (int64_t)N * N * N;
  if (p->kappa)
    for (int64_t c = 0; c < ncell; ++c)
      if (!(p->kappa[c] > 0.0) || !std::isfinite(p->kappa[c]))
        return fail(CB_ERR_ARG, "kappa must be positive and finite");
  return CB_OK;
}

inline int64_t align_seg(int64_t x) { return ((x + SEG_ALIGN - 1) / SEG_ALIGN) * SEG_ALIGN; }

// Tensor rules of every ball's sphere (Gauss-Legendre in cos theta,
// midpoint in phi, n_t = max(8, ceil(4 pi r / h)) from the problem's h),
// uploaded once per context.
int build_sphere_rules(cb_ctx* c) {
  if (c->sr_ready) return CB_OK;
  hipStream_t st = c->st;
  std::vector<NitscheBall> rb;
  std::vector<double> t, w, cph, sph, dph;
  const double two_pi = 6.283185307179586476925286766559;
  for (int k = 0; k < c->P; ++k) {
    const ProbHost& h = c->pb[k];
    for (int i = 0; i < h.nb; ++i) {
      const double r = c->radii_h[h.ball_off + i];
      const int nt = std::max(8, (int)std::ceil(4.0 * 3.14159265358979323846 * r / h.h));
      const int nphi = 2 * nt;
      NitscheBall b{r, nt, nphi, (int32_t)t.size(), (int32_t)cph.size()};
      rb.push_back(b);
      t.resize(t.size() + nt);
      w.resize(w.size() + nt);
      gauss_legendre(nt, t.data() + b.off_t, w.data() + b.off_t);
      for (int q = 0; q < nphi; ++q) {
        const double phi = two_pi * (q + 0.5) / nphi;
        cph.push_back(std::cos(phi));
        sph.push_back(std::sin(phi));
      }
      dph.push_back(two_pi / nphi);
    }
  }
  if (rb.empty()) rb.push_back(NitscheBall{});   // keeps every table non-empty
  for (std::vector<double>* v : {&t, &w, &cph, &sph, &dph})
    if (v->empty()) v->push_back(0.0);
  CHK(dalloc(c->sr_ball, rb.size() * sizeof(NitscheBall)));
  HIPCHK(hipMemcpyAsync(c->sr_ball.p, rb.data(), rb.size() * sizeof(NitscheBall), hipMemcpyHostToDevice, st));
  CHK(upload(c->sr_t, t, st));
  CHK(upload(c->sr_w, w, st));
  CHK(upload(c->sr_c, cph, st));
  CHK(upload(c->sr_s, sph, st));
  CHK(upload(c->sr_d, dph, st));
  CHK(upload(c->sr_k, std::vector<double>(c->Kref, c->Kref + 64), st));
  // the host tables must outlive the copies
  HIPCHK(hipStreamSynchronize(st));
  c->sr = NitscheRule{c->sr_ball.as<NitscheBall>(), c->sr_t.as<double>(), c->sr_w.as<double>(),
                      c->sr_c.as<double>(),        c->sr_s.as<double>(), c->sr_d.as<double>(),
                      c->sr_k.as<double>()};
  c->sr_ready = true;
  return CB_OK;
}

// Nitsche's surface terms (homogeneous Dirichlet data on the ball surfaces)
// added to the unit stiffness of the n_cut stored cut cells, and beta_e of
// each kept for the surface load of given data.
int add_nitsche_terms(cb_ctx* c, int64_t n_cut) {
  hipStream_t st = c->st;
  CHK(build_sphere_rules(c));
  CHK(dalloc(c->beta_d, std::max<int64_t>(1, n_cut) * sizeof(double)));
  if (n_cut <= 0) return CB_OK;
  DevBuf d_status;
  CHK(upload(d_status, std::vector<int>(1, 0), st));
  launch_nitsche(st, c->batch(false), c->sr, c->balls.as<double>(), c->cut_d.as<int64_t>(), n_cut, c->Kc.as<double>(),
                 c->beta_d.as<double>(), d_status.as<int>());
  HIPCHK(hipGetLastError());
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, d_status.p, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (bad) return fail(CB_ERR_NOT_SPD, std::to_string(bad) + " cut cells: the Nitsche eigenproblem broke down");
  return CB_OK;
}

// Setup of P problems: cell classification, indexing and cut-cell
// integration on the GPU, with one readback of the per-problem counts (the
// host sizes the index maps and groups the coarse problems).
int setup_impl(const cb_problem* ps, int P, void* stream, cb_ctx** out) {
  if (!ps || !out || P < 1) return fail(CB_ERR_ARG, "null argument or empty batch");
  *out = nullptr;
  for (int k = 0; k < P; ++k) {
    const int rc = validate_problem(&ps[k]);
    if (rc != CB_OK) return P > 1 ? fail(rc, "problem " + std::to_string(k) + ": " + g_err) : rc;
    const cb_problem& a = ps[k];
    const cb_problem& b = ps[0];
    if (a.sub_cells != b.sub_cells || a.weighting != b.weighting || a.objects != b.objects ||
        a.coarse_variant != b.coarse_variant || a.local_precision != b.local_precision ||
        (a.full_elements != 0) != (b.full_elements != 0) || a.cut_boundary != b.cut_boundary)
      return fail(CB_ERR_ARG, "problems of a batch must share sub_cells and every option");
  }
  std::unique_ptr<cb_ctx> c(new cb_ctx());
  c->dev = current_device();
  c->st = static_cast<hipStream_t>(stream);
  g_alloc_stream = c->st;
  c->P = P;
  c->s = ps[0].sub_cells;
  c->weighting = ps[0].weighting;
  c->objects = ps[0].objects;
  c->variant = ps[0].coarse_variant;
  c->precision = ps[0].local_precision;
  c->full_elements = ps[0].full_elements ? 1 : 0;
  c->nitsche = ps[0].cut_boundary == 1 && !c->full_elements;
  hipStream_t st = c->st;
  const int s = c->s;

  hipEvent_t e0 = nullptr, e1 = nullptr;
  EventPair ev01{&e0, &e1};
  HIPCHK(pooled_time_event(&e0));
  HIPCHK(pooled_time_event(&e1));
  HIPCHK(hipEventRecord(e0, st));

  // problem segments
  c->pb.resize(P);
  int64_t cell_off = 0, node_off = 0;
  int ball_off = 0, sub_off = 0;
  for (int k = 0; k < P; ++k) {
    ProbHost& h = c->pb[k];
    const int N = ps[k].n_cells;
    h.N = N;
    h.m = N / s;
    h.ns = h.m * h.m * h.m;
    h.h = 1.0 / (double)N;
    h.nb = ps[k].n_balls;
    h.ball_off = ball_off;
    h.cell_off = cell_off;
    h.node_off = node_off;
    h.sub_off = sub_off;
    cell_off += align_seg((int64_t)N * N * N);
    node_off += align_seg((int64_t)(N + 1) * (N + 1) * (N + 1));
    ball_off += h.nb;
    sub_off += h.ns;
  }
  c->n_cells_tot = cell_off;
  c->nn = node_off;
  c->ns = sub_off;

  // sub-cell Gauss coordinates: xi_k = (a + g_p) / 4, k = 2a + p
  const double g0 = 0.5 - 0.5 / std::sqrt(3.0), g1 = 0.5 + 0.5 / std::sqrt(3.0);
  for (int a = 0; a < 4; ++a) {
    c->xi[2 * a] = ((double)a + g0) * 0.25;
    c->xi[2 * a + 1] = ((double)a + g1) * 0.25;
  }
  reference_matrices(c->xi, c->Kref, c->Mref);
  set_reference_matrices(c->Kref, c->Mref);
  bddc_set_reference(c->Kref);
  const std::vector<double> xiv(c->xi, c->xi + 8);
  CHK(upload(c->xi_d, xiv, st));
  std::vector<double> balls(4 * (size_t)std::max(1, ball_off));
  for (int k = 0; k < P; ++k) {
    const ProbHost& h = c->pb[k];
    for (int i = 0; i < h.nb; ++i) {
      double* B = &balls[4 * (size_t)(h.ball_off + i)];
      B[0] = ps[k].ball_centres[3 * i + 0];
      B[1] = ps[k].ball_centres[3 * i + 1];
      B[2] = ps[k].ball_centres[3 * i + 2];
      B[3] = ps[k].ball_radii[i] * ps[k].ball_radii[i];
    }
  }
  CHK(upload(c->balls, balls, st));
  c->radii_h.assign((size_t)std::max(1, ball_off), 0.0);
  for (int k = 0; k < P; ++k)
    for (int i = 0; i < c->pb[k].nb; ++i) c->radii_h[c->pb[k].ball_off + i] = ps[k].ball_radii[i];
  for (int k = 0; k < P; ++k) c->kappa_given = c->kappa_given || ps[k].kappa != nullptr;
  // kappa: 1 on the device, then the given per-cell values
  CHK(dalloc(c->kappa, c->n_cells_tot * sizeof(double)));
  launch_fill(st, c->n_cells_tot, 1.0, c->kappa.as<double>());
  for (int k = 0; k < P; ++k)
    if (ps[k].kappa)
      HIPCHK(hipMemcpyAsync(c->kappa.as<double>() + c->pb[k].cell_off, ps[k].kappa,
                            (size_t)c->pb[k].N * c->pb[k].N * c->pb[k].N * sizeof(double), hipMemcpyHostToDevice,
                            st));
  // preliminary problem table for the grid kernels
  // (uploaded host vectors stay alive until the stream is synchronised)
  auto prob_table = [&](bool indexed) {
    std::vector<ProbDev> t(P);
    for (int k = 0; k < P; ++k) {
      const ProbHost& h = c->pb[k];
      ProbDev d{};
      d.N = h.N;
      d.s = s;
      d.m = h.m;
      d.nb = h.nb;
      d.ball_off = h.ball_off;
      d.h = h.h;
      d.cell_off = h.cell_off;
      d.node_off = h.node_off;
      d.dof_off = h.dof_off;
      d.sub_off = h.sub_off;
      d.coarse_off = h.coarse_off;
      d.nc = indexed ? h.n_coarse : 0;
      d.ldc = h.ldc;
      d.ac_off = h.ac_off;
      t[k] = d;
    }
    return t;
  };
  std::vector<int64_t> cell_offs(P + 1), node_offs(P + 1);
  for (int k = 0; k < P; ++k) {
    cell_offs[k] = c->pb[k].cell_off;
    node_offs[k] = c->pb[k].node_off;
  }
  cell_offs[P] = c->n_cells_tot;
  node_offs[P] = c->nn;
  const std::vector<ProbDev> table0 = prob_table(false);
  CHK(upload(c->prob_d, table0, st));
  CHK(upload(c->cell_off_d, cell_offs, st));
  CHK(upload(c->node_off_d, node_offs, st));
  std::vector<int32_t> sub_offs(P + 1);
  for (int k = 0; k < P; ++k) sub_offs[k] = c->pb[k].sub_off;
  sub_offs[P] = c->ns;
  CHK(upload(c->sub_off_d, sub_offs, st));
  // operator work items: node boxes (every mesh large) or node blocks
  {
    int minN = 1 << 30, maxN = 1;
    int64_t all_nodes = 0;
    for (int k = 0; k < P; ++k) {
      minN = std::min(minN, c->pb[k].N);
      maxN = std::max(maxN, c->pb[k].N);
      all_nodes += (int64_t)(c->pb[k].N + 1) * (c->pb[k].N + 1) * (c->pb[k].N + 1);
    }
    // CUTBDDC_OPERATOR = block, box or box:<nodes per box> overrides the choice
    const char* mode = std::getenv("CUTBDDC_OPERATOR");
    int64_t per_item_forced = 0;
    if (mode && std::strncmp(mode, "box", 3) == 0) {
      c->op_box = 1;
      if (mode[3] == ':') per_item_forced = std::max<long long>(1, std::atoll(mode + 4));
    } else {
      c->op_box = mode && std::strcmp(mode, "block") == 0 ? 0 : (minN >= OP_BOX_MIN_N ? 1 : 0);
    }
    std::vector<int32_t> op_offs(P + 1, 0), op_prob, geom((size_t)8 * P, 0);
    c->op_lx = SEG_ALIGN + 2 * (maxN + 1) + 2;
    c->op_lc = 2 * SEG_ALIGN + 2 * maxN + 2;
    c->op_xp = c->op_cp = 1;
    if (c->op_box) {
      // about 2048 boxes in the context, of at most 2048 nodes each
      const int64_t per_item = per_item_forced ? per_item_forced
                                               : std::min<int64_t>(2048, std::max<int64_t>(1, all_nodes / 2048));
      for (int k = 0; k < P; ++k) {
        const OpGeom g = op_geometry(c->pb[k].N + 1, per_item);
        int32_t* gk = &geom[(size_t)8 * k];
        gk[0] = g.nseg, gk[1] = g.SW, gk[2] = g.TY, gk[3] = g.ngy, gk[4] = g.ZC, gk[5] = g.nzc;
        const int32_t items = g.nseg * g.ngy * g.nzc;
        op_offs[k + 1] = op_offs[k] + items;
        op_prob.insert(op_prob.end(), (size_t)items, k);
        c->op_xp = std::max(c->op_xp, (g.SW + 2) * (g.TY + 2));
        c->op_cp = std::max(c->op_cp, (g.SW + 1) * (g.TY + 1));
      }
      if (c->op_xp > OP_XP_MAX || c->op_cp > OP_CP_MAX)
        return fail(CB_ERR_ARG, "operator node box exceeds its staging registers");
    } else {
      op_prob.resize((size_t)(c->nn / SEG_ALIGN));
      for (int k = 0; k < P; ++k) {
        op_offs[k + 1] = (int32_t)(node_offs[k + 1] / SEG_ALIGN);
        for (int32_t it = op_offs[k]; it < op_offs[k + 1]; ++it) op_prob[it] = k;
      }
    }
    c->op_items = op_offs[P];
    CHK(upload(c->op_off_d, op_offs, st));
    CHK(upload(c->op_prob_d, op_prob, st));
    CHK(upload(c->op_geom_d, geom, st));
    if (prepare_apply_A() != 0) return fail(CB_ERR_DEVICE, "setting the operator kernels' LDS limits failed");
  }
  const int64_t nn = c->nn, ncell = c->n_cells_tot;
  const int ns = c->ns;
  CHK(dalloc(c->count_d, ncell * sizeof(int32_t)));
  launch_classify(st, c->batch(false), ncell, c->xi_d.as<double>(), c->balls.as<double>(),
                  c->count_d.as<int32_t>());
  HIPCHK(hipGetLastError());
  hipEvent_t ea = nullptr, eb = nullptr;
  EventPair ev_ab{&ea, &eb};
  HIPCHK(pooled_time_event(&ea));
  HIPCHK(pooled_time_event(&eb));
  HIPCHK(hipEventRecord(ea, st));

  // ---- device indexing (one readback of the counts) ----------------------
  {
    const size_t nbs = (size_t)index_scan_blocks(std::max(ncell, nn));
    const size_t al = 256;
    auto up = [&](size_t x) { return (x + al - 1) / al * al; };
    const size_t u8 = up((size_t)nn), i32 = up((size_t)nn * 4), sg = up((size_t)(P + 1) * sizeof(Count4));
    const size_t total = 5 * u8 + 10 * i32 + up(nbs * sizeof(Count4)) + 3 * sg + up((size_t)P * 4);
    CHK(dalloc(c->iwork, total));
    char* q = static_cast<char*>(c->iwork.p);
    IndexWork& w = c->iw;
    // the per-problem results first: one contiguous readback
    w.seg_cells = reinterpret_cast<Count4*>(q), q += sg;
    w.seg_nodes = reinterpret_cast<Count4*>(q), q += sg;
    w.seg_obj = reinterpret_cast<Count4*>(q), q += sg;
    w.floating = reinterpret_cast<int32_t*>(q), q += up((size_t)P * 4);
    for (uint8_t** u : {&w.smask, &w.link, &w.face, &w.cutdof, &w.ground}) *u = reinterpret_cast<uint8_t*>(q), q += u8;
    for (int32_t** v : {&w.par0, &w.par1, &w.par2, &w.size1, &w.size2, &w.gif, &w.gifp, &w.oidx, &w.ocid, &w.ocsp})
      *v = reinterpret_cast<int32_t*>(q), q += i32;
    w.bsum = reinterpret_cast<Count4*>(q);
  }
  const size_t sgb = ((size_t)(P + 1) * sizeof(Count4) + 255) / 256 * 256;
  const size_t small_bytes = 3 * sgb + (size_t)P * 4;
  CHK(dalloc(c->cellinfo, ncell * sizeof(int32_t)));
  CHK(dalloc(c->cut_d, ncell * sizeof(int64_t)));
  launch_index_cells(st, c->batch(false), ncell, c->count_d.as<int32_t>(), c->full_elements ? 0 : 1, c->iw,
                     c->cellinfo.as<int32_t>(), c->cut_d.as<int64_t>());
  // Variant 2 compares weighting coefficients built from the cut-cell
  // matrices, so those are integrated before the node passes (one extra
  // readback: the number of stored cut cells); otherwise after them.
  const bool integrate_first = c->variant == 2 || c->nitsche;
  auto integrate = [&](int64_t n_cut) -> int {
    CHK(dalloc(c->Kc, std::max<int64_t>(1, n_cut) * PACK36 * sizeof(double)));
    CHK(dalloc(c->Mc, std::max<int64_t>(1, n_cut) * PACK36 * sizeof(double)));
    launch_integrate_cut(st, c->batch(false), c->xi_d.as<double>(), c->balls.as<double>(), c->cut_d.as<int64_t>(),
                         n_cut, c->Kc.as<double>(), c->Mc.as<double>());
    HIPCHK(hipGetLastError());
    return CB_OK;
  };
  if (integrate_first) {
    Count4 tot{};
    HIPCHK(hipMemcpyAsync(&tot, c->iw.seg_cells + P, sizeof(Count4), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    CHK(integrate(tot.z));
    if (c->nitsche) CHK(add_nitsche_terms(c.get(), tot.z));
    std::vector<double> kd(8);
    for (int a = 0; a < 8; ++a) kd[a] = c->Kref[a * 8 + a];
    CHK(upload(c->kdiag_d, kd, st));
  }
  const V2Inputs v2in{c->weighting == CB_W_STIFFNESS ? 1 : 0, c->cellinfo.as<int32_t>(), c->kappa.as<double>(),
                      c->Kc.as<double>(), c->kdiag_d.as<double>()};
  CHK(dalloc(c->dofmask, nn));
  CHK(dalloc(c->dof_node, nn * sizeof(int64_t)));
  CHK(dalloc(c->nI, (size_t)ns * sizeof(int32_t)));
  CHK(dalloc(c->nG, (size_t)ns * sizeof(int32_t)));
  CHK(dalloc(c->nC, (size_t)ns * sizeof(int32_t)));
  launch_index_nodes(st, c->batch(false), ncell, nn, ns, c->sub_off_d.as<int32_t>(), c->count_d.as<int32_t>(),
                     c->balls.as<double>(), c->variant, c->objects, v2in, c->iw, c->dofmask.as<uint8_t>(),
                     c->dof_node.as<int64_t>(), c->nI.as<int32_t>(), c->nG.as<int32_t>(), c->nC.as<int32_t>());
  HIPCHK(hipGetLastError());
  char* stage = static_cast<char*>(t_stage.get(small_bytes + 3 * (size_t)ns * sizeof(int32_t) + 256));
  if (!stage) return fail(CB_ERR_OOM, "pinned staging allocation failed");
  int32_t* nIh = reinterpret_cast<int32_t*>(stage + ((small_bytes + 255) / 256) * 256);
  int32_t* nGh = nIh + ns;
  int32_t* nCh = nGh + ns;
  HIPCHK(hipMemcpyAsync(stage, c->iw.seg_cells, small_bytes, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(nIh, c->nI.p, (size_t)ns * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(nGh, c->nG.p, (size_t)ns * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(nCh, c->nC.p, (size_t)ns * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const Count4* segc = reinterpret_cast<const Count4*>(stage);
  const Count4* segn = reinterpret_cast<const Count4*>(stage + sgb);
  const Count4* sego = reinterpret_cast<const Count4*>(stage + 2 * sgb);
  const int32_t* floating = reinterpret_cast<const int32_t*>(stage + 3 * sgb);
  for (int k = 0; k < P; ++k)
    if (floating[k]) {
      const std::string where = P > 1 ? "problem " + std::to_string(k) + ": " : std::string();
      return fail(CB_ERR_SINGULAR, where + "an active component touches no Dirichlet node (singular operator)");
    }
  int maxI = 1, maxG = 1, maxC = 1;
  int32_t chunk_off = 0;
  for (int k = 0; k < P; ++k) {
    ProbHost& h = c->pb[k];
    h.n_active = segc[k + 1].x - segc[k].x;
    h.n_cut = segc[k + 1].y - segc[k].y;
    h.n_cut_stored = segc[k + 1].z - segc[k].z;
    h.cut_off = segc[k].z;
    h.dof_off = segn[k].x;
    h.n_dof = segn[k + 1].x - segn[k].x;
    h.iface_off = segn[k].y;
    h.n_iface = segn[k + 1].y - segn[k].y;
    h.obj_off = sego[k].x;
    h.n_obj = sego[k + 1].x - sego[k].x;
    h.coarse_off = sego[k].y;
    h.n_coarse = sego[k + 1].y - sego[k].y;
    h.maxC = 0;
    for (int b = h.sub_off; b < h.sub_off + h.ns; ++b) {
      maxI = std::max(maxI, nIh[b]);
      maxG = std::max(maxG, nGh[b]);
      h.maxC = std::max(h.maxC, nCh[b]);
    }
    maxC = std::max(maxC, h.maxC);
    h.chunk_off = chunk_off;
    chunk_off += (int32_t)(((int64_t)(h.N + 1) * (h.N + 1) * (h.N + 1) + DOT_CHUNK - 1) / DOT_CHUNK);
  }
  c->n_cut_tot = segc[P].z;
  c->n_dof_tot = segn[P].x;
  c->n_iface_tot = segn[P].y;
  c->nc_tot = sego[P].y;
  const int64_t if_len = segn[P].z, cs_len = sego[P].z;
  c->n_chunks = chunk_off;
  c->NIp = round_up(maxI, CHOL_BLOCK);
  c->NGp = round_up(maxG, CHOL_BLOCK);
  c->NCp = round_up(maxC, 16);
  {
    const size_t need = bddc_lds_need(c->NIp, c->NGp, c->NCp, s, c->precision);
    if (need > LDS_BYTES)
      return fail(CB_ERR_ARG, "padded local orders (interior " + std::to_string(c->NIp) + ", interface " +
                                  std::to_string(c->NGp) + ", coarse " + std::to_string(c->NCp) + ") need " +
                                  std::to_string(need) + " bytes of LDS per subdomain workgroup (limit " +
                                  std::to_string(LDS_BYTES) + ")");
  }
  c->nt = c->NIp + c->NGp;
  const int NIp = c->NIp, NGp = c->NGp, NCp = c->NCp;
  const int s1 = s + 1;

  // coarse blocks: problems grouped by padded coarse order (within 25%)
  {
    std::vector<int> co(P);
    std::iota(co.begin(), co.end(), 0);
    std::stable_sort(co.begin(), co.end(), [&](int a, int b) { return c->pb[a].n_coarse < c->pb[b].n_coarse; });
    int64_t ac = 0;
    size_t i = 0;
    while (i < co.size()) {
      const int nc0 = c->pb[co[i]].n_coarse;
      if (nc0 == 0) {
        c->pb[co[i]].ldc = 0;
        ++i;
        continue;
      }
      const int l0 = round_up(nc0, CHOL_BLOCK);
      size_t j = i;
      int L = l0;
      while (j < co.size()) {
        const int l = round_up(c->pb[co[j]].n_coarse, CHOL_BLOCK);
        if (l > l0 + l0 / 4) break;
        L = l;
        ++j;
      }
      CoarseGroup g;
      g.ldc = L;
      g.ac_off = ac;
      for (size_t q = i; q < j; ++q) {
        ProbHost& h = c->pb[co[q]];
        h.ldc = L;
        h.ac_off = ac;
        ac += (int64_t)L * L;
        g.probs.push_back(co[q]);
      }
      c->groups.push_back(std::move(g));
      i = j;
    }
    c->ac_total = ac;
    int64_t prow = 0;
    for (int k = 0; k < P; ++k) {
      c->pb[k].prow_off = prow;
      prow += c->pb[k].ldc;
    }
    c->n_prows = prow;
  }

  // per-subdomain index maps and interface / coarse lists
  CHK(dalloc(c->Iidx, (size_t)ns * NIp * sizeof(int64_t)));
  CHK(dalloc(c->Gidx, (size_t)ns * NGp * sizeof(int64_t)));
  CHK(dalloc(c->Gobj, (size_t)ns * NGp * sizeof(int32_t)));
  CHK(dalloc(c->Cids, (size_t)ns * NCp * sizeof(int32_t)));
  CHK(dalloc(c->bloc, (size_t)ns * s1 * s1 * s1 * sizeof(int32_t)));
  CHK(dalloc(c->if_ptr, (size_t)(c->n_iface_tot + 1) * sizeof(int64_t)));
  CHK(dalloc(c->if_sub, (size_t)std::max<int64_t>(1, if_len) * sizeof(int32_t)));
  CHK(dalloc(c->if_slot, (size_t)std::max<int64_t>(1, if_len) * sizeof(int32_t)));
  CHK(dalloc(c->iface_node, (size_t)std::max<int64_t>(1, c->n_iface_tot) * sizeof(int64_t)));
  CHK(dalloc(c->cs_ptr, (size_t)(c->nc_tot + 1) * sizeof(int64_t)));
  CHK(dalloc(c->cs_sub, (size_t)std::max<int64_t>(1, cs_len) * sizeof(int32_t)));
  CHK(dalloc(c->cs_row, (size_t)std::max<int64_t>(1, cs_len) * sizeof(int32_t)));
  CHK(dalloc(c->coarse_prob_d, (size_t)std::max(1, c->nc_tot) * sizeof(int32_t)));
  CHK(dalloc(c->sub_prob_d, (size_t)ns * sizeof(int32_t)));
  CHK(dalloc(c->sub_blk_d, (size_t)ns * sizeof(int32_t)));
  IndexMaps mp;
  mp.NIp = NIp;
  mp.NGp = NGp;
  mp.NCp = NCp;
  mp.I_idx = c->Iidx.as<int64_t>();
  mp.G_idx = c->Gidx.as<int64_t>();
  mp.G_obj = c->Gobj.as<int32_t>();
  mp.C_ids = c->Cids.as<int32_t>();
  mp.bloc = c->bloc.as<int32_t>();
  mp.if_ptr = c->if_ptr.as<int64_t>();
  mp.if_sub = c->if_sub.as<int32_t>();
  mp.if_slot = c->if_slot.as<int32_t>();
  mp.iface_node = c->iface_node.as<int64_t>();
  mp.cs_ptr = c->cs_ptr.as<int64_t>();
  mp.cs_sub = c->cs_sub.as<int32_t>();
  mp.cs_row = c->cs_row.as<int32_t>();
  mp.coarse_prob = c->coarse_prob_d.as<int32_t>();
  mp.sub_prob = c->sub_prob_d.as<int32_t>();
  mp.sub_blk = c->sub_blk_d.as<int32_t>();
  launch_index_fill(st, c->batch(false), ns, s, c->sub_off_d.as<int32_t>(), c->iw, mp);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(eb, st));

  // cut-cell integration
  if (!integrate_first) CHK(integrate(c->n_cut_tot));
  // full row-major copies of the cut cells' stiffness for the operator
  CHK(dalloc(c->Kf, std::max<int64_t>(1, c->n_cut_tot) * 64 * sizeof(double)));
  launch_expand_rows(st, c->n_cut_tot, c->Kc.as<double>(), c->Kf.as<double>());
  HIPCHK(hipEventRecord(e1, st));

  std::vector<int64_t> dof_offs(P + 1), prow_offs(P + 1);
  std::vector<int32_t> chunk_ptr(P + 1);
  for (int k = 0; k < P; ++k) {
    dof_offs[k] = c->pb[k].dof_off;
    prow_offs[k] = c->pb[k].prow_off;
    chunk_ptr[k] = c->pb[k].chunk_off;
  }
  dof_offs[P] = c->n_dof_tot;
  prow_offs[P] = c->n_prows;
  chunk_ptr[P] = c->n_chunks;
  const std::vector<ProbDev> table1 = prob_table(true);
  CHK(upload(c->prob_d, table1, st));
  CHK(upload(c->dof_off_d, dof_offs, st));
  CHK(upload(c->prow_off_d, prow_offs, st));
  CHK(upload(c->chunk_ptr_d, chunk_ptr, st));
  for (DevBuf* b : {&c->x, &c->r, &c->z, &c->p, &c->q, &c->t1, &c->t2, &c->t3, &c->bgrid})
    CHK(dalloc(*b, nn * sizeof(double)));
  CHK(dalloc(c->zbuf, (size_t)ns * NGp * sizeof(double)));
  CHK(dalloc(c->cloc, (size_t)ns * NCp * sizeof(double)));
  CHK(dalloc(c->cvec, (size_t)std::max(1, c->nc_tot) * sizeof(double)));
  CHK(dalloc(c->ucvec, (size_t)std::max(1, c->nc_tot) * sizeof(double)));
  CHK(dalloc(c->tcvec, (size_t)std::max(1, c->nc_tot) * sizeof(double)));
  CHK(dalloc(c->partial, (size_t)std::max(1, c->n_chunks) * sizeof(double)));
  const size_t n_blk = std::max<size_t>(1, (size_t)((c->nn + SEG_ALIGN - 1) / SEG_ALIGN));
  CHK(dalloc(c->pq_part, (size_t)std::max(1, c->op_items) * sizeof(double)));
  CHK(dalloc(c->rr_part, n_blk * sizeof(double)));
  CHK(dalloc(c->hist, (size_t)P * HIST_CAP * 3 * sizeof(double)));
  CHK(dalloc(c->scal, (size_t)P * CG_S * sizeof(double)));
  CHK(dalloc(c->params, 2 * sizeof(double)));
  CHK(dalloc(c->active, (size_t)P * sizeof(int32_t)));
  CHK(dalloc(c->itc, (size_t)P * sizeof(int32_t)));
  CHK(dalloc(c->status, (size_t)P * sizeof(int32_t)));
  CHK(dalloc(c->relres_d, (size_t)P * sizeof(double)));
  CHK(dalloc(c->nact_d, sizeof(int32_t)));
  CHK(dalloc(c->fptrs, (size_t)P * sizeof(double*)));
  CHK(dalloc(c->uptrs, (size_t)P * sizeof(double*)));
  HIPCHK(pooled_pinned(&c->pin, c->pin_bytes(), &c->pin_cap));
  {
    void* dp = nullptr;
    HIPCHK(hipHostGetDevicePointer(&dp, c->pin, 0));
    c->pin_nact_dev = static_cast<int32_t*>(dp);
  }
  HIPCHK(hipStreamSynchronize(st));
  {
    float m0 = 0.f, m1 = 0.f, m2 = 0.f;
    HIPCHK(hipEventElapsedTime(&m0, e0, ea));
    HIPCHK(hipEventElapsedTime(&m1, ea, eb));
    HIPCHK(hipEventElapsedTime(&m2, eb, e1));
    c->info.t_integrate_ms = m0 + m2;
    c->info.t_topology_ms = m1;
  }


  // per-problem and total counts
  cb_info& tot = c->info;
  int maxl = 0, maxc = 0;
  for (int k = 0; k < P; ++k) {
    ProbHost& h = c->pb[k];
    cb_info& in = h.info;
    in.n_dof = h.n_dof;
    in.n_active = h.n_active;
    in.n_cut = h.n_cut;
    in.n_cut_stored = h.n_cut_stored;
    in.n_sub = h.ns;
    in.n_coarse = h.n_coarse;
    in.n_objects = h.n_obj;
    in.n_iface = h.n_iface;
    in.max_coarse_per_sub = h.maxC;
    int ml = 0;
    for (int b = h.sub_off; b < h.sub_off + h.ns; ++b) {
      ml = std::max(ml, nIh[b] + nGh[b]);
      const double nI = nIh[b], nG = nGh[b];
      in.sum_nI2 += (int64_t)nIh[b] * nIh[b];
      in.sum_nG2 += (int64_t)nGh[b] * nGh[b];
      in.sum_nI += nIh[b];
      in.sum_nG += nGh[b];
      in.sum_nGnC += (int64_t)nGh[b] * nCh[b];
      in.flops_local_chol += (nI + nG) * (nI + nG) * (nI + nG) / 3.0 + nI * nI * nI / 3.0;
    }
    in.max_local_dofs = ml;
    maxl = std::max(maxl, ml);
    maxc = std::max(maxc, h.maxC);
    tot.n_dof += in.n_dof;
    tot.n_active += in.n_active;
    tot.n_cut += in.n_cut;
    tot.n_cut_stored += in.n_cut_stored;
    tot.n_sub += in.n_sub;
    tot.n_coarse += in.n_coarse;
    tot.n_objects += in.n_objects;
    tot.n_iface += in.n_iface;
    tot.sum_nI2 += in.sum_nI2;
    tot.sum_nG2 += in.sum_nG2;
    tot.sum_nI += in.sum_nI;
    tot.sum_nG += in.sum_nG;
    tot.sum_nGnC += in.sum_nGnC;
    in.n_nodes = (int64_t)(h.N + 1) * (h.N + 1) * (h.N + 1);
    tot.n_nodes += in.n_nodes;
    tot.flops_local_chol += in.flops_local_chol;
  }
  tot.max_local_dofs = maxl;
  tot.max_coarse_per_sub = maxc;
  *out = c.release();
  return CB_OK;
}

size_t factor_work_budget() {
  const char* e = std::getenv("CUTBDDC_FACTOR_WORK_GB");
  double gb = e ? std::atof(e) : 16.0;
  if (!(gb > 0.0)) gb = 16.0;
  return (size_t)(gb * (double)(1ull << 30));
}

// Work buffers of the local factorisation for a chunk of subdomains, in the
// compute type T of the local Cholesky and inverses.
template <typename T>
struct FactorWork {
  int chunk = 0;
  DevBuf K, Linv, Y, PS, YI, PSI, Pd64, KSw, G, Sc, PhiF, V, StV, StC;
  static size_t per_sub(const cb_ctx* c) {
    const int nt = c->nt, NIp = c->NIp, NGp = c->NGp, NCp = c->NCp, nbig = std::max(NIp, NGp);
    return (size_t)nt * nt * sizeof(T) + (size_t)diag_blocks(nt, NIp) * DB * DB * sizeof(T) +
           2 * (size_t)nbig * nbig * sizeof(T) + 2 * (size_t)NIp * NIp * sizeof(T) + (size_t)NIp * NIp * 8 +
           (size_t)NGp * NGp * 8 +
           (size_t)(NGp * NCp + NCp * NCp + 2 * nt * NCp) * sizeof(double) +
           (size_t)nt * STENCIL * (sizeof(double) + sizeof(int32_t));
  }
  int alloc(const cb_ctx* c, int n) {
    chunk = n;
    const int nt = c->nt, NIp = c->NIp, NGp = c->NGp, NCp = c->NCp, nbig = std::max(NIp, NGp);
    const size_t sF = (size_t)nt * NCp;
    CHK(dalloc(K, (size_t)n * nt * nt * sizeof(T)));
    CHK(dalloc(Linv, (size_t)n * diag_blocks(nt, NIp) * DB * DB * sizeof(T)));
    CHK(dalloc(Y, (size_t)n * nbig * nbig * sizeof(T)));
    CHK(dalloc(PS, (size_t)n * nbig * nbig * sizeof(T)));
    CHK(dalloc(YI, (size_t)n * NIp * NIp * sizeof(T)));
    CHK(dalloc(PSI, (size_t)n * NIp * NIp * sizeof(T)));
    CHK(dalloc(Pd64, (size_t)n * NIp * NIp * sizeof(double)));
    CHK(dalloc(KSw, (size_t)n * NGp * NGp * sizeof(double)));
    CHK(dalloc(G, (size_t)n * NGp * NCp * sizeof(double)));
    CHK(dalloc(Sc, (size_t)n * NCp * NCp * sizeof(double)));
    CHK(dalloc(PhiF, (size_t)n * sF * sizeof(double)));
    CHK(dalloc(V, (size_t)n * sF * sizeof(double)));
    CHK(dalloc(StV, (size_t)n * nt * STENCIL * sizeof(double)));
    CHK(dalloc(StC, (size_t)n * nt * STENCIL * sizeof(int32_t)));
    return CB_OK;
  }
  void release() {
    for (DevBuf* b : {&K, &Linv, &Y, &PS, &YI, &PSI, &Pd64, &KSw, &G, &Sc, &PhiF, &V, &StV, &StC}) b->release();
  }
};

// Local factorisation of subdomains [w0, w0 + nc) (Sect. 3.3-3.4): assembly
// of the local matrix, Cholesky in type T, the Dirichlet inverse and the
// constrained interface operator stored in type TS, the FP64 coarse basis
// and the local coarse matrix.  Pivot failures go to info[w].
template <typename T, typename TS>
int factor_chunk(cb_ctx* c, FactorWork<T>& fw, int w0, int nc, double* AcLoc) {
  hipStream_t st = c->st;
  const int NIp = c->NIp, NGp = c->NGp, NCp = c->NCp, nt = c->nt;
  const GridDev g = c->grid();
  const int nbig = std::max(NIp, NGp);
  const int64_t sK = (int64_t)nt * nt;
  const int64_t sL = (int64_t)diag_blocks(nt, NIp) * DB * DB;
  const int64_t sY = (int64_t)nbig * nbig;
  const int64_t sG = (int64_t)NGp * NCp, sC = (int64_t)NCp * NCp, sF = (int64_t)nt * NCp;
  const int64_t sP = (int64_t)NIp * NIp, sKS = (int64_t)NGp * NGp;
  const int64_t pkI = packed_elems(NIp), pkG = packed_elems(NGp);
  const int ns = c->ns;
  DevBuf &K = fw.K, &Linv = fw.Linv, &Y = fw.Y, &PS = fw.PS, &YI = fw.YI, &PSI = fw.PSI, &Pd64 = fw.Pd64,
         &KSw = fw.KSw, &G = fw.G, &Sc = fw.Sc, &PhiF = fw.PhiF, &V = fw.V, &StV = fw.StV, &StC = fw.StC;
  const int64_t sI2 = (int64_t)NIp * NIp;
  {
    const SubDev sd = c->sub(w0);
    const double* Dsw = c->Ds.as<double>() + (int64_t)w0 * nt;
    double* Phiw = c->Phi.as<double>() + (int64_t)w0 * sG;
    double* KS = KSw.as<double>();
    // The identity right-hand sides of the two triangular inverses touch
    // neither K nor the factor: they are written on the second stream
    // beside the assembly and the Cholesky, which leave it idle (in line on
    // st while profiling).  That stream first waits for st, whose previous
    // chunk still read Y.
    const bool overlap = !c->prof;
    hipStream_t sti = overlap ? c->aux_st : st;
    if (overlap) {
      HIPCHK(hipEventRecord(c->fill_ev, st));
      HIPCHK(hipStreamWaitEvent(sti, c->fill_ev, 0));
    }
    fill_identity<T>(sti, YI.as<T>(), NIp, sI2, NIp, nc);
    fill_identity<T>(sti, Y.as<T>(), NGp, sY, NGp, nc);
    if (overlap) HIPCHK(hipEventRecord(c->fill_ev, sti));
    launch_assemble_local<T>(st, sd, g, nc, K.as<T>(), c->diagAG.as<double>() + (int64_t)w0 * NGp,
                             c->Ds.as<double>() + (int64_t)w0 * nt, StV.as<double>(), StC.as<int32_t>());
    HIPCHK(hipGetLastError());
    int chol_rc = 0;
    // rows [nI, NIp) and [NIp + nG, nt) of K are identity padding: the
    // dense products skip the tiles and k stages that only meet them
    GemmRows act;
    act.na = sd.nI;
    act.nb = sd.nG;
    act.split = NIp;
    timed(c, "local_cholesky", [&] {
      const AuxStreams ax{c->aux_st, c->aux_st3, c->aux_ev, c->aux_ev3};
      chol_rc = cholesky<T>(st, K.as<T>(), nt, sK, nt, NIp, nc, Linv.as<T>(), sL, c->info_d.as<int>() + w0, &ax,
                            &act);
    });
    if (chol_rc != 0) return fail(CB_ERR_DEVICE, "event record or wait failed in the local factorisation");
    HIPCHK(hipGetLastError());
    // The interior and interface inverses only read the factor: the
    // interior one runs on the second stream beside the interface one
    // (in line on st while profiling, so that the group timers see it).
    if (overlap) {
      HIPCHK(hipEventRecord(c->aux_ev, st));
      HIPCHK(hipStreamWaitEvent(sti, c->aux_ev, 0));
    }
    // P = A_II^{-1} = D_I (Y_I^T Y_I) D_I (zero on the padding, which no
    // later step reads)
    timed(c, "local_inverse", [&] {
      tri_inverse<T>(sti, K.as<T>(), nt, sK, 0, NIp, NIp, nc, Linv.as<T>(), sL, YI.as<T>(), NIp, sI2, &act,
                     false);
      gemm<T>(sti, 1, 0, NIp, NIp, NIp, T(1), YI.as<T>(), NIp, sI2, YI.as<T>(), NIp, sI2, T(0), PSI.as<T>(), NIp,
              sI2, nc, GEMM_LOWER | GEMM_KFROM_DIAG, act);
    });
    launch_pack_lower<T, TS>(sti, NIp, nc, PSI.as<T>(), NIp, sI2, Dsw, nt, c->P_.as<TS>() + (int64_t)w0 * pkI);
    // full FP64 copy of A_II^{-1} for the harmonic extension of the coarse basis
    symmetrize_scale<T, double>(sti, PSI.as<T>(), NIp, sI2, Pd64.as<double>(), NIp, sP, Dsw, nt, NIp, nc);
    if (overlap) HIPCHK(hipEventRecord(c->aux_ev, sti));
    const double* Pd = Pd64.as<double>();
    HIPCHK(hipGetLastError());
    // K_S^{-1} = D_G (Y_G^T Y_G) D_G, kept in FP64 for the coarse basis
    // (zero on the padding)
    if (overlap) HIPCHK(hipStreamWaitEvent(st, c->fill_ev, 0));
    timed(c, "local_inverse", [&] {
      tri_inverse<T>(st, K.as<T>(), nt, sK, NIp, NGp, NIp, nc, Linv.as<T>(), sL, Y.as<T>(), NGp, sY, &act, false);
      gemm<T>(st, 1, 0, NGp, NGp, NGp, T(1), Y.as<T>(), NGp, sY, Y.as<T>(), NGp, sY, T(0), PS.as<T>(), NGp, sY, nc,
              GEMM_LOWER | GEMM_KFROM_DIAG, act.at(NIp, NIp, NIp));
    });
    symmetrize_scale<T, double>(st, PS.as<T>(), NGp, sY, KS, NGp, sKS, Dsw + NIp, nt, NGp, nc);
    HIPCHK(hipGetLastError());
    // coarse basis on the interface: G = K_S^{-1} C^T, S_c = C G,
    // Phi_G = G S_c^{-1} (C Phi_G = I, energy-minimising for S_A)
    launch_constraint_cols(st, sd, nc, KS, G.as<double>());
    launch_constraint_rows(st, sd, nc, G.as<double>(), Sc.as<double>());
    launch_small_spd_inverse(st, sd, nc, Sc.as<double>(), c->info_d.as<int>() + ns);
    gemm<double>(st, 1, 0, NGp, NCp, NCp, 1.0, G.as<double>(), NGp, sG, Sc.as<double>(), NCp, sC, 0.0, Phiw, NCp,
                 sG, nc, 0);
    HIPCHK(hipGetLastError());
    // full coarse basis Phi = [Phi_I; Phi_G] with Phi_I = -A_II^{-1} A_IG Phi_G,
    // and the local coarse matrix as the FP64 Gram matrix Phi^T A_omega Phi.
    // A_omega Phi vanishes on the interior rows, so the Gram matrix is
    // Phi_G^T (A_omega Phi)_G; only the needed rows of A_omega X are formed.
    // The first product reads only the interface rows of PhiF (its interior
    // rows are zero in [0; Phi_G]); the interior rows are then written, all
    // of them, by the GEMM that forms Phi_I.
    HIPCHK(hipMemcpy2DAsync(PhiF.as<double>() + (int64_t)NIp * NCp, sF * sizeof(double), Phiw,
                            (size_t)sG * sizeof(double), (size_t)sG * sizeof(double), nc, hipMemcpyDeviceToDevice,
                            st));
    launch_local_apply(st, sd, nc, StV.as<double>(), StC.as<int32_t>(), PhiF.as<double>(), V.as<double>(), 0, NIp,
                       NIp);
    // A_II^{-1} (and P) from the second stream
    if (overlap) HIPCHK(hipStreamWaitEvent(st, c->aux_ev, 0));
    gemm<double>(st, 0, 0, NIp, NCp, NIp, -1.0, Pd, NIp, sP, V.as<double>(), NCp, sF, 0.0, PhiF.as<double>(), NCp,
                 sF, nc, 0);
    launch_local_apply(st, sd, nc, StV.as<double>(), StC.as<int32_t>(), PhiF.as<double>(), V.as<double>(), NIp,
                       NGp);
    gemm<double>(st, 1, 0, NCp, NCp, NGp, 1.0, PhiF.as<double>() + (int64_t)NIp * NCp, NCp, sF,
                 V.as<double>() + (int64_t)NIp * NCp, NCp, sF, 0.0, AcLoc + (int64_t)w0 * sC, NCp, sC, nc, 0);
    // Kt = K_S^{-1} - Phi G^T: the lower part in place in K_S^{-1} (MFMA),
    // then packed with its mirror
    gemm<double>(st, 0, 0, NGp, NGp, NCp, -1.0, Phiw, NCp, sG, G.as<double>(), NGp, sG, 1.0, KS, NGp, sKS, nc,
                 GEMM_LOWER);
    launch_pack_lower<double, TS>(st, NGp, nc, KS, NGp, sKS, nullptr, 0, c->Kt.as<TS>() + (int64_t)w0 * pkG);
    HIPCHK(hipGetLastError());
  }
  return CB_OK;
}

// Subdomains whose FP32 local Cholesky met a non-positive pivot are factored
// again in FP64; their operators are then stored in FP32 like the others.
// CUTBDDC_FORCE_FP32_BREAKDOWN=w (test hook) treats global subdomain w as
// such a failure.  Returns the number of refactored subdomains in *n_redo.
int fp64_refactor(cb_ctx* c, double* AcLoc, int* n_redo) {
  hipStream_t st = c->st;
  const int ns = c->ns;
  std::vector<int> info(ns);
  HIPCHK(hipMemcpyAsync(info.data(), c->info_d.p, ns * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (const char* e = std::getenv("CUTBDDC_FORCE_FP32_BREAKDOWN")) {
    const int w = std::atoi(e);
    if (w >= 0 && w < ns && info[w] == 0) info[w] = 1;
  }
  std::vector<int> redo;
  for (int w = 0; w < ns; ++w)
    if (info[w] != 0) redo.push_back(w);
  *n_redo = (int)redo.size();
  if (redo.empty()) return CB_OK;
  FactorWork<double> fw;
  CHK(fw.alloc(c, 1));
  for (int w : redo) {
    HIPCHK(hipMemsetAsync(c->info_d.as<int>() + w, 0, sizeof(int), st));
    CHK((factor_chunk<double, float>(c, fw, w, 1, AcLoc)));
  }
  return CB_OK;
}

// Nested dissection of the coarse problem (coarse_nd.h): chosen for a
// context of one problem with at least 4 subdomains per axis and at least
// ND_MIN_COARSE coarse DOFs.  CUTBDDC_COARSE=dense or =nd (read at every
// cb_factor) overrides the rule; nd still needs one problem, 2 subdomains
// per axis and a nonempty separator.
constexpr int ND_MIN_COARSE = 1024;
bool coarse_nd_wanted(const cb_ctx* c) {
  if (c->P != 1 || c->pb[0].m < 2 || c->pb[0].n_coarse == 0) return false;
  const char* e = std::getenv("CUTBDDC_COARSE");
  if (e && std::strcmp(e, "dense") == 0) return false;
  if (e && std::strcmp(e, "nd") == 0) return true;
  return c->pb[0].m >= 4 && c->pb[0].n_coarse >= ND_MIN_COARSE;
}

// Envelope end per DB-wide column block (the env of cholesky_inverse) from
// last[f] = the largest row whose first nonzero column is f (at least f).
std::vector<int> envelope_ends(const std::vector<int32_t>& last) {
  const int L = (int)last.size();
  std::vector<int> env(diag_blocks(L, 0));
  int32_t run = 0, col = 0;
  for (size_t kb = 0; kb < env.size(); ++kb) {
    const int cend = std::min(L, (int)(kb + 1) * DB);
    for (; col < cend; ++col) run = std::max(run, last[col]);
    env[kb] = run + 1;
  }
  return env;
}

struct NDPlan {
  int Lo = 0, Lso = 0, Ls = 0, n_s = 0, n_o_max = 0;
  std::vector<int32_t> oid, sid, sep, pos;
  std::vector<int> env;   // envelope of the octant blocks (over the batch of 8)
};

// Octant partition of the coarse DOFs of the single problem from the coarse
// ids of every subdomain (cids: NCp slots per subdomain, ncs[w] used) and
// the block of every subdomain.  Octant of block (bx, by, bz): bit 0 for
// bx >= m/2, bit 1 for by >= m/2, bit 2 for bz >= m/2.  Within an octant
// and within the separator the DOFs keep their coarse order.  Returns false
// when there is no separator.
bool plan_nd(const cb_ctx* c, const std::vector<int32_t>& cids, const std::vector<int32_t>& ncs,
             const std::vector<int32_t>& blk, NDPlan& pl) {
  const ProbHost& h = c->pb[0];
  const int m = h.m, half = m / 2, nc = h.n_coarse, NCp = c->NCp;
  auto octant = [&](int b) {
    const int bx = b % m, by = (b / m) % m, bz = b / (m * m);
    return (bx >= half ? 1 : 0) + (by >= half ? 2 : 0) + (bz >= half ? 4 : 0);
  };
  auto ids_of = [&](int w) { return &cids[(size_t)w * NCp]; };
  // -2: held by no subdomain yet; 0..7: interior to that octant; -1: separator
  std::vector<int> oct(nc, -2);
  for (int w = h.sub_off; w < h.sub_off + h.ns; ++w) {
    const int o = octant(blk[w]);
    for (int t = 0; t < ncs[w]; ++t) {
      int& x = oct[ids_of(w)[t] - h.coarse_off];
      x = (x == -2 || x == o) ? o : -1;
    }
  }
  std::vector<int> loc(nc, -1);
  std::vector<std::vector<int32_t>> inner(8);
  std::vector<int32_t> sid;
  for (int i = 0; i < nc; ++i) {
    if (oct[i] == -2) return false;
    if (oct[i] >= 0) {
      loc[i] = (int)inner[oct[i]].size();
      inner[oct[i]].push_back(i);
    } else {
      loc[i] = (int)sid.size();
      sid.push_back(i);
    }
  }
  const int n_s = (int)sid.size();
  if (n_s == 0) return false;
  // separator DOFs held by a subdomain of each octant (the only separator
  // columns of A_os that can be nonzero), and the first interior column of
  // every interior row (its subdomains' smallest interior DOF)
  std::vector<std::vector<char>> cpl(8, std::vector<char>(n_s, 0));
  std::vector<std::vector<int32_t>> firstl(8);
  for (int o = 0; o < 8; ++o) {
    firstl[o].resize(inner[o].size());
    for (size_t i = 0; i < inner[o].size(); ++i) firstl[o][i] = (int32_t)i;
  }
  for (int w = h.sub_off; w < h.sub_off + h.ns; ++w) {
    const int o = octant(blk[w]);
    int32_t lo = INT32_MAX;
    for (int t = 0; t < ncs[w]; ++t) {
      const int i = ids_of(w)[t] - h.coarse_off;
      if (oct[i] == -1) cpl[o][loc[i]] = 1;
      else lo = std::min(lo, (int32_t)loc[i]);
    }
    for (int t = 0; t < ncs[w]; ++t) {
      const int i = ids_of(w)[t] - h.coarse_off;
      if (oct[i] >= 0) firstl[o][loc[i]] = std::min(firstl[o][loc[i]], lo);
    }
  }
  std::vector<std::vector<int32_t>> sep(8);
  int n_o_max = 0, n_so_max = 0;
  for (int o = 0; o < 8; ++o) {
    for (int t = 0; t < n_s; ++t)
      if (cpl[o][t]) sep[o].push_back(t);
    n_o_max = std::max(n_o_max, (int)inner[o].size());
    n_so_max = std::max(n_so_max, (int)sep[o].size());
  }
  pl.n_s = n_s;
  pl.n_o_max = n_o_max;
  pl.Lo = round_up(std::max(1, n_o_max), CHOL_BLOCK);
  pl.Lso = round_up(std::max(1, n_so_max), 32);
  pl.Ls = round_up(n_s, CHOL_BLOCK);
  pl.oid.assign((size_t)8 * pl.Lo, -1);
  pl.sep.assign((size_t)8 * pl.Lso, -1);
  pl.pos.assign((size_t)8 * n_s, -1);
  std::vector<int32_t> last(pl.Lo);
  for (int i = 0; i < pl.Lo; ++i) last[i] = i;
  for (int o = 0; o < 8; ++o) {
    for (size_t i = 0; i < inner[o].size(); ++i) {
      pl.oid[(size_t)o * pl.Lo + i] = inner[o][i];
      last[firstl[o][i]] = std::max(last[firstl[o][i]], (int32_t)i);
    }
    for (size_t a = 0; a < sep[o].size(); ++a) {
      pl.sep[(size_t)o * pl.Lso + a] = sep[o][a];
      pl.pos[(size_t)o * n_s + sep[o][a]] = (int32_t)a;
    }
  }
  pl.sid = std::move(sid);
  pl.env = envelope_ends(last);
  return true;
}

// Nested-dissection factorisation of the coarse problem (coarse_nd.h) from
// its full ldc x ldc matrix Ac (problem-local coarse ids; the single
// problem's ids start at 0).
int factor_coarse_nd(cb_ctx* c, const double* Ac, int ldc, const NDPlan& pl) {
  hipStream_t st = c->st;
  auto& nd = c->nd;
  const int Lo = pl.Lo, Lso = pl.Lso, Ls = pl.Ls;
  nd.Lo = Lo;
  nd.Lso = Lso;
  nd.Ls = Ls;
  nd.n_s = pl.n_s;
  nd.n_o_max = pl.n_o_max;
  CHK(upload(nd.oid, pl.oid, st));
  CHK(upload(nd.sid, pl.sid, st));
  CHK(upload(nd.sep, pl.sep, st));
  CHK(upload(nd.pos, pl.pos, st));
  const int64_t sO = (int64_t)Lo * Lo, sW = (int64_t)Lo * Lso, sS = (int64_t)Lso * Lso, sY = (int64_t)Ls * Ls;
  const int64_t sLo = (int64_t)diag_blocks(Lo, 0) * DB * DB, sLs = (int64_t)diag_blocks(Ls, 0) * DB * DB;
  CHK(dalloc(nd.Yo, (size_t)(8 * sO) * sizeof(double)));
  CHK(dalloc(nd.W, (size_t)(8 * sW) * sizeof(double)));
  CHK(dalloc(nd.WT, (size_t)(8 * sW) * sizeof(double)));
  CHK(dalloc(nd.Ys, (size_t)sY * sizeof(double)));
  CHK(dalloc(nd.to, (size_t)8 * Lo * sizeof(double)));
  for (DevBuf* b : {&nd.rs, &nd.us, &nd.xs}) CHK(dalloc(*b, (size_t)Ls * sizeof(double)));
  CHK(dalloc(nd.info, 9 * sizeof(int)));
  HIPCHK(hipMemsetAsync(nd.info.p, 0, 9 * sizeof(int), st));
  DevBuf Aoo, Aos, So, S, Lc, ones;
  CHK(dalloc(Aoo, (size_t)(8 * sO) * sizeof(double)));
  CHK(dalloc(Aos, (size_t)(8 * sW) * sizeof(double)));
  CHK(dalloc(So, (size_t)(8 * sS) * sizeof(double)));
  CHK(dalloc(S, (size_t)sY * sizeof(double)));
  CHK(dalloc(Lc, (size_t)std::max(8 * sLo, sLs) * sizeof(double)));
  CHK(upload(ones, std::vector<double>(std::max(Lo, Ls), 1.0), st));
  const NDDev d = nd.dev();
  const AuxStreams ax{c->aux_st, c->aux_st3, c->aux_ev, c->aux_ev3};
  int* info = nd.info.as<int>();
  launch_nd_gather(st, d, Ac, ldc, Aoo.as<double>(), Aos.as<double>());
  // the 8 octant blocks as one batch, then W_o = Y_o A_os (Y_o lower
  // triangular: a row tile's k loop ends at its last row)
  if (cholesky_inverse<double>(st, ax, Aoo.as<double>(), Lo, sO, Lo, 8, Lc.as<double>(), sLo, info,
                               nd.Yo.as<double>(), sO, pl.env.data()) != 0)
    return fail(CB_ERR_DEVICE, "event record or wait failed in the coarse factorisation");
  gemm<double>(st, 0, 0, Lo, Lso, Lo, 1.0, nd.Yo.as<double>(), Lo, sO, Aos.as<double>(), Lso, sW, 0.0,
               nd.W.as<double>(), Lso, sW, 8, GEMM_KTO_DIAG);
  symmetrize_scale<double, double>(st, nd.Yo.as<double>(), Lo, sO, nd.Yo.as<double>(), Lo, sO,
                                   ones.as<double>(), 0, Lo, 8);
  launch_nd_transpose(st, d, nd.W.as<double>(), nd.WT.as<double>());
  // S = A_ss - sum_o W_o^T W_o, then its factor and inverse
  gemm<double>(st, 1, 0, Lso, Lso, Lo, 1.0, nd.W.as<double>(), Lso, sW, nd.W.as<double>(), Lso, sW, 0.0,
               So.as<double>(), Lso, sS, 8, GEMM_LOWER);
  launch_nd_schur(st, d, Ac, ldc, So.as<double>(), S.as<double>());
  if (cholesky_inverse<double>(st, ax, S.as<double>(), Ls, sY, Ls, 1, Lc.as<double>(), sLs, info + 8,
                               nd.Ys.as<double>(), sY, nullptr) != 0)
    return fail(CB_ERR_DEVICE, "event record or wait failed in the coarse factorisation");
  symmetrize_scale<double, double>(st, nd.Ys.as<double>(), Ls, sY, nd.Ys.as<double>(), Ls, sY, ones.as<double>(),
                                   0, Ls, 1);
  HIPCHK(hipGetLastError());
  nd.on = true;
  return CB_OK;
}

template <typename T>
int factor_impl(cb_ctx* c) {
  hipStream_t st = c->st;
  const int ns = c->ns, NIp = c->NIp, NGp = c->NGp, NCp = c->NCp, nt = c->nt;
  const int64_t sG = (int64_t)NGp * NCp, sC = (int64_t)NCp * NCp;

  // persistent results (A_II^{-1} and the interface operator in packed
  // symmetric storage)
  const int64_t pkI = packed_elems(NIp), pkG = packed_elems(NGp);
  CHK(dalloc(c->P_, (size_t)ns * pkI * sizeof(T)));
  CHK(dalloc(c->Kt, (size_t)ns * pkG * sizeof(T)));
  CHK(dalloc(c->Phi, (size_t)ns * sG * sizeof(double)));
  CHK(dalloc(c->diagAG, (size_t)ns * NGp * sizeof(double)));
  CHK(dalloc(c->Ds, (size_t)ns * nt * sizeof(double)));
  CHK(dalloc(c->Dw, (size_t)ns * NGp * sizeof(double)));
  if (!c->aux_st) HIPCHK(pooled_stream(&c->aux_st));
  if (!c->aux_st3) HIPCHK(pooled_stream(&c->aux_st3));
  if (!c->aux_ev) HIPCHK(pooled_sync_event(&c->aux_ev));
  if (!c->aux_ev3) HIPCHK(pooled_sync_event(&c->aux_ev3));
  if (!c->fill_ev) HIPCHK(pooled_sync_event(&c->fill_ev));
  const int n_info = ns + 1 + c->P;
  CHK(dalloc(c->info_d, (size_t)n_info * sizeof(int)));
  HIPCHK(hipMemsetAsync(c->info_d.p, 0, (size_t)n_info * sizeof(int), st));
  HIPCHK(hipMemsetAsync(c->Dw.p, 0, (size_t)ns * NGp * sizeof(double), st));
  // coarse ids and blocks of every subdomain (fixed since setup), for the
  // host side of the coarse factorisation; read now, while only the fills
  // above are queued, so that the coarse section needs no synchronisation
  std::vector<int32_t> cids, ncs, blk;
  if (c->ac_total > 0) {
    cids.resize((size_t)ns * NCp);
    ncs.resize(ns);
    blk.resize(ns);
    HIPCHK(hipMemcpyAsync(cids.data(), c->Cids.p, cids.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(ncs.data(), c->nC.p, (size_t)ns * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(blk.data(), c->sub_blk_d.p, (size_t)ns * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  DevBuf AcLoc;
  CHK(dalloc(AcLoc, (size_t)ns * sC * sizeof(double)));
  // object member lists, once for all subdomains (sub() hands them out below)
  c->optr_d.release();
  c->omem_d.release();
  CHK(dalloc(c->optr_d, (size_t)ns * (NCp + 1) * sizeof(int32_t)));
  CHK(dalloc(c->omem_d, (size_t)ns * NGp * sizeof(int32_t)));
  launch_object_lists(st, c->sub(0), ns, c->optr_d.as<int32_t>(), c->omem_d.as<int32_t>());
  HIPCHK(hipGetLastError());

  // work buffers for a chunk of subdomains
  const int chunk =
      (int)std::max<size_t>(1, std::min<size_t>((size_t)ns, factor_work_budget() / FactorWork<T>::per_sub(c)));
  FactorWork<T> fw;
  CHK(fw.alloc(c, chunk));
  // on every exit, st waits for the other streams before the buffers above
  // return to the cache (destroyed after this guard)
  struct AuxJoin {
    cb_ctx* c;
    ~AuxJoin() {
      if (hipEventRecord(c->aux_ev, c->aux_st) == hipSuccess) (void)hipStreamWaitEvent(c->st, c->aux_ev, 0);
      if (hipEventRecord(c->aux_ev3, c->aux_st3) == hipSuccess) (void)hipStreamWaitEvent(c->st, c->aux_ev3, 0);
    }
  } aux_join{c};

  for (int w0 = 0; w0 < ns; w0 += chunk) CHK((factor_chunk<T, T>(c, fw, w0, std::min(chunk, ns - w0),
                                                                    AcLoc.as<double>())));
  c->n_fallbacks = 0;
  if (std::is_same<T, float>::value) {
    fw.release();
    CHK(fp64_refactor(c, AcLoc.as<double>(), &c->n_fallbacks));
    // the coarse restriction and prolongation of the FP32-local path read
    // Phi in FP32 (both with the same rounded copy, so that the coarse
    // correction stays symmetric); the coarse matrix is formed from Phi in FP64
    CHK(dalloc(c->Phi32, (size_t)ns * sG * sizeof(float)));
    convert_to_float(st, (int64_t)ns * sG, c->Phi.as<double>(), c->Phi32.as<float>());
  } else {
    c->Phi32.release();
  }
  launch_weights(st, c->n_iface_tot, c->if_ptr.as<int64_t>(), c->if_sub.as<int32_t>(), c->if_slot.as<int32_t>(),
                 NGp, c->diagAG.as<double>(), c->weighting == CB_W_STIFFNESS, c->Dw.as<double>());
  HIPCHK(hipGetLastError());

  // coarse matrices (one block per problem) and their inverses, in FP64;
  // the blocks of a group share their order and are factored as a batch
  std::vector<int> coarse_slot(c->P, -1);   // index into info_d after ns + 1
  c->nd.on = false;
  if (c->ac_total > 0) {
    // (the coarse ids and blocks of every subdomain were read back before
    // the local factorisation: the host work below runs while it does)
    NDPlan plan;
    const bool use_nd = coarse_nd_wanted(c) && plan_nd(c, cids, ncs, blk, plan);
    DevBuf Ac;
    CHK(dalloc(Ac, (size_t)c->ac_total * sizeof(double)));
    if (use_nd) c->Acinv.release();
    else CHK(dalloc(c->Acinv, (size_t)c->ac_total * sizeof(double)));
    size_t maxL = 0, maxD = 0;
    for (const CoarseGroup& gr : c->groups) {
      maxL = std::max(maxL, (size_t)gr.ldc);
      maxD = std::max(maxD, gr.probs.size() * (size_t)diag_blocks(gr.ldc, 0) * DB * DB);
    }
    // a single problem keeps its coarse matrix for export
    // (up to 1 GiB: larger coarse problems are for solving, not inspection)
    const bool keep = c->P == 1 && c->ac_total <= ((int64_t)1 << 27);
    if (keep) CHK(dalloc(c->AcKeep, (size_t)c->ac_total * sizeof(double)));
    else c->AcKeep.release();
    launch_coarse_assemble(st, c->batch(false), c->prow_off_d.as<int64_t>(), c->n_prows, (int)maxL,
                           c->cs_ptr.as<int64_t>(), c->cs_sub.as<int32_t>(), c->cs_row.as<int32_t>(), c->sub(0),
                           AcLoc.as<double>(), Ac.as<double>(), keep ? c->AcKeep.as<double>() : nullptr);
    HIPCHK(hipGetLastError());
    // Envelope of each coarse matrix: A_c couples two coarse DOFs only
    // when a subdomain holds both, so row i's first nonzero column is the
    // smallest coarse id among the subdomains that hold i.
    std::vector<int32_t> first(c->nc_tot);   // problem-local
    for (int k = 0; k < c->P; ++k)
      for (int i = 0; i < c->pb[k].n_coarse; ++i) first[c->pb[k].coarse_off + i] = i;
    for (int k = 0; k < c->P; ++k) {
      const ProbHost& h = c->pb[k];
      for (int w = h.sub_off; w < h.sub_off + h.ns; ++w) {
        const int32_t* ids = &cids[(size_t)w * NCp];
        int32_t lo = INT32_MAX;
        for (int t = 0; t < ncs[w]; ++t) lo = std::min(lo, ids[t] - h.coarse_off);
        for (int t = 0; t < ncs[w]; ++t) first[ids[t]] = std::min(first[ids[t]], lo);
      }
    }
    DevBuf Lc, ones;
    const std::vector<double> onesv(maxL, 1.0);
    CHK(dalloc(Lc, maxD * sizeof(double)));
    CHK(upload(ones, onesv, st));
    ProfScope cps(c, "coarse_factor");
    if (use_nd) CHK(factor_coarse_nd(c, Ac.as<double>() + c->pb[0].ac_off, c->pb[0].ldc, plan));
    int slot = 0;
    for (const CoarseGroup& gr : c->groups) {
      if (use_nd) break;
      const int L = gr.ldc, nb = (int)gr.probs.size();
      const int64_t sA = (int64_t)L * L, sLc = (int64_t)diag_blocks(L, 0) * DB * DB;
      for (int q = 0; q < nb; ++q) coarse_slot[gr.probs[q]] = slot + q;
      double* A = Ac.as<double>() + gr.ac_off;
      // the triangular inverse and the far trailing updates run beside the
      // factorisation on two more streams
      const AuxStreams ax{c->aux_st, c->aux_st3, c->aux_ev, c->aux_ev3};
      // envelope end per column block, over the problems of the group
      // (padding rows carry only their diagonal)
      std::vector<int32_t> last(L);
      for (int i = 0; i < L; ++i) last[i] = i;
      for (int q = 0; q < nb; ++q) {
        const ProbHost& h = c->pb[gr.probs[q]];
        for (int i = 0; i < h.n_coarse; ++i) {
          const int f = first[h.coarse_off + i];
          last[f] = std::max(last[f], i);
        }
      }
      const std::vector<int> env = envelope_ends(last);
      double* Y = c->Acinv.as<double>() + gr.ac_off;
      if (cholesky_inverse<double>(st, ax, A, L, sA, L, nb, Lc.as<double>(), sLc,
                                   c->info_d.as<int>() + ns + 1 + slot, Y, sA, env.data()) != 0)
        return fail(CB_ERR_DEVICE, "event record or wait failed in the coarse factorisation");
      // the solve applies Y^T (Y x): keep Y in the lower triangle and its
      // transpose in the upper one (in place: every 32 x 32 lower tile is
      // read into LDS by the one workgroup that writes it and its mirror)
      symmetrize_scale<double, double>(st, Y, L, sA, Y, L, sA, ones.as<double>(), 0, L, nb);
      HIPCHK(hipGetLastError());
      slot += nb;
    }
  }
  if (!c->nd.on)
    for (DevBuf* b : {&c->nd.oid, &c->nd.sid, &c->nd.sep, &c->nd.pos, &c->nd.Yo, &c->nd.W, &c->nd.WT, &c->nd.Ys,
                      &c->nd.to, &c->nd.rs, &c->nd.us, &c->nd.xs, &c->nd.info})
      b->release();
  // join the second stream before the chunk buffers go back to the cache
  HIPCHK(hipEventRecord(c->aux_ev, c->aux_st));
  HIPCHK(hipStreamWaitEvent(st, c->aux_ev, 0));
  fw.release();
  std::vector<int> info(n_info), nd_info(9, 0);
  HIPCHK(hipMemcpyAsync(info.data(), c->info_d.p, n_info * sizeof(int), hipMemcpyDeviceToHost, st));
  if (c->nd.on) HIPCHK(hipMemcpyAsync(nd_info.data(), c->nd.info.p, 9 * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<int32_t> sub_prob(ns);
  for (int k = 0; k < c->P; ++k)
    for (int b = 0; b < c->pb[k].ns; ++b) sub_prob[c->pb[k].sub_off + b] = k;
  auto where = [&](int k) { return c->P > 1 ? " of problem " + std::to_string(k) : std::string(); };
  for (int w = 0; w < ns; ++w)
    if (info[w] != 0) {
      const int k = sub_prob[w];
      return fail(CB_ERR_NOT_SPD, "local Cholesky failed in subdomain " + std::to_string(w - c->pb[k].sub_off) +
                                      where(k) + " at row " + std::to_string(info[w] - 1));
    }
  if (info[ns] != 0) return fail(CB_ERR_NOT_SPD, "singular local coarse matrix");
  for (int k = 0; k < c->P; ++k)
    if (coarse_slot[k] >= 0 && info[ns + 1 + coarse_slot[k]] != 0)
      return fail(CB_ERR_NOT_SPD, "coarse Cholesky failed" + where(k));
  for (int o = 0; o < 9; ++o)
    if (nd_info[o] != 0)
      return fail(CB_ERR_NOT_SPD, o < 8 ? "coarse Cholesky failed in the block of octant " + std::to_string(o)
                                        : std::string("coarse Cholesky failed in the separator's Schur complement"));
  return CB_OK;
}

int need_single(const cb_ctx* c) {
  if (c->P != 1) return fail(CB_ERR_STATE, "entry point needs a single-problem context (use cb_solve_batch)");
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
  if (p->coarse_variant < 0 || p->coarse_variant > 1)
    return fail(CB_ERR_ARG, "host indexing supports the standard objects and variant 1 (variant 2 needs the "
                            "integrated cut cells of cb_setup)");
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
    const int64_t sL = (int64_t)diag_blocks(np, 0) * DB * DB;
    CHK(dalloc(dL, (size_t)batch * sL * sizeof(T)));
    CHK(dalloc(dY, (size_t)batch * nn * sizeof(T)));
    CHK(dalloc(dP, (size_t)batch * nn * sizeof(T)));
    CHK(dalloc(dOut, (size_t)batch * nn * sizeof(double)));
    CHK(upload(dOnes, std::vector<double>((size_t)batch * np, 1.0), nullptr));
    CHK(upload(dInfo, std::vector<int>(batch, 0), nullptr));
    // the factorisation with the overlapped triangular inverse, as for the
    // coarse matrices
    AuxStreams ax{nullptr, nullptr, nullptr, nullptr};
    auto release = [&ax] {
      (void)hipDeviceSynchronize();
      if (ax.ev2) (void)hipEventDestroy(ax.ev2);
      if (ax.ev3) (void)hipEventDestroy(ax.ev3);
      if (ax.st2) (void)hipStreamDestroy(ax.st2);
      if (ax.st3) (void)hipStreamDestroy(ax.st3);
    };
    if (hipStreamCreateWithFlags(&ax.st2, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&ax.st3, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ax.ev2, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ax.ev3, hipEventDisableTiming) != hipSuccess) {
      release();
      return fail(CB_ERR_DEVICE, "stream or event creation failed");
    }
    const int rc = cholesky_inverse<T>(nullptr, ax, dA.as<T>(), np, nn, np, batch, dL.as<T>(), sL, dInfo.as<int>(),
                                       dY.as<T>(), nn);
    release();
    if (rc != 0) return fail(CB_ERR_DEVICE, "event record or wait failed");
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

int cb_setup(const cb_problem* p, void* stream, cb_ctx** out) { return setup_impl(p, 1, stream, out); }

int cb_setup_batch(const cb_problem* problems, int32_t n, void* stream, cb_ctx** out) {
  if (n < 1) return fail(CB_ERR_ARG, "batch size must be >= 1");
  return setup_impl(problems, n, stream, out);
}

int cb_factor(cb_ctx* c) {
  if (!c) return fail(CB_ERR_ARG, "null context");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  EventPair ev01{&e0, &e1};
  HIPCHK(pooled_time_event(&e0));
  HIPCHK(pooled_time_event(&e1));
  HIPCHK(hipEventRecord(e0, c->st));
  c->factored = false;
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  c->graph_failed = false;
  g_alloc_stream = c->st;
  int rc = c->precision == CB_FP32_LOCAL ? factor_impl<float>(c) : factor_impl<double>(c);
  if (rc != CB_OK) return rc;
  HIPCHK(hipEventRecord(e1, c->st));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  c->info.t_factor_ms = ms;
  c->factored = true;
  c->info.factored = 1;
  return CB_OK;
}

}  // extern "C"

namespace {

// PCG on c->bgrid, then the DOF values of x: into u (concatenated DOF
// vector) or, per problem, into u_ptrs.
int solve_common(cb_ctx* c, double* u_dev, double* const* u_ptrs_dev, double rtol, int32_t max_iter) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  EventPair ev01{&e0, &e1};
  HIPCHK(pooled_time_event(&e0));
  HIPCHK(pooled_time_event(&e1));
  HIPCHK(hipEventRecord(e0, c->st));
  int sweeps = 0;
  CHK(pcg(c, rtol, max_iter, &sweeps));
  if (u_ptrs_dev)
    launch_gather_dofs_batch(c->st, c->P, c->n_dof_tot, c->dof_off_d.as<int64_t>(), c->dof_node.as<int64_t>(),
                             c->x.as<double>(), u_ptrs_dev);
  else
    launch_gather_dofs(c->st, c->n_dof_tot, c->dof_node.as<int64_t>(), c->x.as<double>(), u_dev);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(e1, c->st));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  c->info.t_solve_ms = ms;
  c->solved = true;
  return CB_OK;
}

// Extreme eigenvalues of the Lanczos tridiagonal matrix of n CG steps
// (diagonal 1/alpha_j + beta_{j-1}/alpha_{j-1}, off-diagonal
// sqrt(beta_j)/alpha_j): bisection on Sturm counts within the Gershgorin
// interval.  n = 0 gives (1, 1).
int lanczos_extremes_impl(int n, const double* alpha, const double* beta, double* lmin, double* lmax) {
  if (n <= 0) {
    *lmin = *lmax = 1.0;
    return CB_OK;
  }
  for (int j = 0; j < n; ++j)
    if (!(alpha[j] > 0.0) || !std::isfinite(alpha[j]) || (j + 1 < n && (!(beta[j] >= 0.0) || !std::isfinite(beta[j]))))
      return fail(CB_ERR_ARG, "CG coefficients must have alpha > 0 and beta >= 0, finite");
  std::vector<double> d(n), e2(n, 0.0);
  double lo = 0.0, hi = 0.0;
  for (int j = 0; j < n; ++j) {
    d[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
    if (j + 1 < n) {
      const double e = std::sqrt(beta[j]) / alpha[j];
      e2[j] = e * e;
    }
  }
  for (int j = 0; j < n; ++j) {
    const double r = (j > 0 ? std::sqrt(e2[j - 1]) : 0.0) + (j + 1 < n ? std::sqrt(e2[j]) : 0.0);
    lo = j ? std::min(lo, d[j] - r) : d[j] - r;
    hi = j ? std::max(hi, d[j] + r) : d[j] + r;
  }
  // number of eigenvalues below x (signs of the pivots of T - x I)
  auto below = [&](double x) {
    int cnt = 0;
    double q = 1.0;
    for (int j = 0; j < n; ++j) {
      q = d[j] - x - (j > 0 ? e2[j - 1] / q : 0.0);
      if (q == 0.0) q = -std::numeric_limits<double>::min();
      if (q < 0.0) ++cnt;
    }
    return cnt;
  };
  auto kth = [&](int k) {   // k-th smallest eigenvalue, 1-based
    double a = lo, b = hi;
    for (int it = 0; it < 200 && b - a > 1e-15 * std::max(std::fabs(a), std::fabs(b)); ++it) {
      const double m = 0.5 * (a + b);
      if (below(m) >= k)
        b = m;
      else
        a = m;
    }
    return 0.5 * (a + b);
  };
  *lmin = kth(1);
  *lmax = kth(n);
  return CB_OK;
}

// The last solve's recorded PCG coefficients of problem k (alpha, the
// betas between iterations, relative residuals), n = iterations kept.
int read_history(const cb_ctx* c, int k, std::vector<double>* alpha, std::vector<double>* beta,
                 std::vector<double>* relres) {
  if (!c->solved) return fail(CB_ERR_STATE, "no solve has run on this context");
  const int n = std::min<int32_t>(c->pin_it()[k], HIST_CAP);
  std::vector<double> h((size_t)std::max(n, 1) * 3);
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(h.data(), c->hist.as<double>() + (size_t)k * HIST_CAP * 3, (size_t)n * 3 * sizeof(double),
                          hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
  }
  alpha->resize(n);
  beta->resize(n > 0 ? n - 1 : 0);
  relres->resize(n);
  for (int j = 0; j < n; ++j) {
    (*alpha)[j] = h[3 * j];
    (*relres)[j] = h[3 * j + 2];
    if (j > 0) (*beta)[j - 1] = h[3 * j + 1];
  }
  return CB_OK;
}

// Lanczos estimates of the last solve of problem k, or zeros (no solve,
// no iteration, or coefficients that are not those of an SPD system).
void fill_lanczos(const cb_ctx* c, int k, cb_info* out) {
  out->lanczos_lmin = out->lanczos_lmax = 0.0;
  if (!c->solved) return;
  std::vector<double> a, b, r;
  if (read_history(c, k, &a, &b, &r) != CB_OK || a.empty()) return;
  double lo = 0.0, hi = 0.0;
  if (lanczos_extremes_impl((int)a.size(), a.data(), b.data(), &lo, &hi) != CB_OK) return;
  out->lanczos_lmin = lo;
  out->lanczos_lmax = hi;
}

int single_result(cb_ctx* c, int32_t* iters, double* relres) {
  if (iters) *iters = c->pin_it()[0];
  if (relres) *relres = c->pin_relres()[0];
  return pcg_status(c, 0);
}

}  // namespace

extern "C" {

int cb_solve(cb_ctx* c, const double* f_nodes_dev, double* u_dev, double rtol, int32_t max_iter,
             int32_t* iters, double* final_relres) {
  if (!c || !u_dev) return fail(CB_ERR_ARG, "null argument");
  CHK(need_single(c));
  if (!c->factored) return fail(CB_ERR_STATE, "cb_solve before cb_factor");
  if (!(rtol > 0.0) || max_iter < 0) return fail(CB_ERR_ARG, "rtol must be > 0 and max_iter >= 0");
  if (!f_nodes_dev) {
    // a null per-problem pointer means f = 1
    c->pin_fptrs()[0] = nullptr;
    HIPCHK(hipMemcpyAsync(c->fptrs.p, c->pin_fptrs(), sizeof(double*), hipMemcpyHostToDevice, c->st));
  }
  launch_load(c->st, c->batch(false), c->nn, c->cellinfo.as<int32_t>(), c->Mc.as<double>(), c->dofmask.as<uint8_t>(),
              f_nodes_dev, f_nodes_dev ? nullptr : c->fptrs.as<const double* const>(), c->bgrid.as<double>());
  HIPCHK(hipGetLastError());
  CHK(solve_common(c, u_dev, nullptr, rtol, max_iter));
  return single_result(c, iters, final_relres);
}

int cb_solve_rhs(cb_ctx* c, const double* b_dev, double* u_dev, double rtol, int32_t max_iter, int32_t* iters,
                 double* final_relres) {
  if (!c || !u_dev || !b_dev) return fail(CB_ERR_ARG, "null argument");
  CHK(need_single(c));
  if (!c->factored) return fail(CB_ERR_STATE, "cb_solve_rhs before cb_factor");
  if (!(rtol > 0.0) || max_iter < 0) return fail(CB_ERR_ARG, "rtol must be > 0 and max_iter >= 0");
  launch_fill(c->st, c->nn, 0.0, c->bgrid.as<double>());
  launch_scatter_dofs(c->st, c->n_dof_tot, c->dof_node.as<int64_t>(), b_dev, c->bgrid.as<double>());
  HIPCHK(hipGetLastError());
  CHK(solve_common(c, u_dev, nullptr, rtol, max_iter));
  return single_result(c, iters, final_relres);
}

int cb_solve_batch(cb_ctx* c, const double* const* f_nodes_dev, double* const* u_dev, double rtol,
                   int32_t max_iter, int32_t* iters, double* final_relres) {
  if (!c || !u_dev) return fail(CB_ERR_ARG, "null argument");
  if (!c->factored) return fail(CB_ERR_STATE, "cb_solve_batch before cb_factor");
  if (!(rtol > 0.0) || max_iter < 0) return fail(CB_ERR_ARG, "rtol must be > 0 and max_iter >= 0");
  for (int k = 0; k < c->P; ++k)
    if (!u_dev[k] && c->pb[k].info.n_dof > 0) return fail(CB_ERR_ARG, "null output of problem " + std::to_string(k));
  // the staging area may still be read by the previous call's copies
  HIPCHK(hipStreamSynchronize(c->st));
  for (int k = 0; k < c->P; ++k) {
    c->pin_fptrs()[k] = f_nodes_dev ? f_nodes_dev[k] : nullptr;
    c->pin_uptrs()[k] = u_dev[k];
  }
  HIPCHK(hipMemcpyAsync(c->fptrs.p, c->pin_fptrs(), c->P * sizeof(double*), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipMemcpyAsync(c->uptrs.p, c->pin_uptrs(), c->P * sizeof(double*), hipMemcpyHostToDevice, c->st));
  launch_load(c->st, c->batch(false), c->nn, c->cellinfo.as<int32_t>(), c->Mc.as<double>(), c->dofmask.as<uint8_t>(),
              nullptr, c->fptrs.as<const double* const>(), c->bgrid.as<double>());
  HIPCHK(hipGetLastError());
  CHK(solve_common(c, nullptr, c->uptrs.as<double* const>(), rtol, max_iter));
  int rc = CB_OK;
  for (int k = 0; k < c->P; ++k) {
    if (iters) iters[k] = c->pin_it()[k];
    if (final_relres) final_relres[k] = c->pin_relres()[k];
  }
  for (int k = 0; k < c->P && rc == CB_OK; ++k)
    if (c->pin_status()[k] == 3) rc = pcg_status(c, k);
  for (int k = 0; k < c->P && rc == CB_OK; ++k)
    if (c->pin_status()[k] != 1) rc = pcg_status(c, k);
  return rc;
}

int cb_apply_operator(cb_ctx* c, const double* x_dev, double* y_dev) {
  if (!c || !x_dev || !y_dev) return fail(CB_ERR_ARG, "null argument");
  CHK(need_single(c));
  launch_fill(c->st, c->nn, 0.0, c->x.as<double>());
  launch_scatter_dofs(c->st, c->n_dof_tot, c->dof_node.as<int64_t>(), x_dev, c->x.as<double>());
  CHK(apply_A_grid(c, c->x.as<double>(), c->q.as<double>(), false));
  launch_gather_dofs(c->st, c->n_dof_tot, c->dof_node.as<int64_t>(), c->q.as<double>(), y_dev);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->st));
  return CB_OK;
}

int cb_apply_preconditioner(cb_ctx* c, const double* r_dev, double* z_dev) {
  if (!c || !r_dev || !z_dev) return fail(CB_ERR_ARG, "null argument");
  CHK(need_single(c));
  if (!c->factored) return fail(CB_ERR_STATE, "preconditioner applied before cb_factor");
  launch_fill(c->st, c->nn, 0.0, c->r.as<double>());
  launch_scatter_dofs(c->st, c->n_dof_tot, c->dof_node.as<int64_t>(), r_dev, c->r.as<double>());
  CHK(apply_M_grid(c, c->r.as<double>(), c->z.as<double>(), false));
  launch_gather_dofs(c->st, c->n_dof_tot, c->dof_node.as<int64_t>(), c->z.as<double>(), z_dev);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->st));
  return CB_OK;
}

int cb_load(cb_ctx* c, const double* f_nodes_dev, double* b_dev) {
  if (!c || !b_dev) return fail(CB_ERR_ARG, "null argument");
  CHK(need_single(c));
  if (!f_nodes_dev) {
    c->pin_fptrs()[0] = nullptr;
    HIPCHK(hipMemcpyAsync(c->fptrs.p, c->pin_fptrs(), sizeof(double*), hipMemcpyHostToDevice, c->st));
  }
  launch_load(c->st, c->batch(false), c->nn, c->cellinfo.as<int32_t>(), c->Mc.as<double>(), c->dofmask.as<uint8_t>(),
              f_nodes_dev, f_nodes_dev ? nullptr : c->fptrs.as<const double* const>(), c->bgrid.as<double>());
  launch_gather_dofs(c->st, c->n_dof_tot, c->dof_node.as<int64_t>(), c->bgrid.as<double>(), b_dev);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->st));
  return CB_OK;
}

static int mms_check(cb_ctx* c, const double* x0, double k, MmsParams* m) {
  if (!c || !x0) return fail(CB_ERR_ARG, "null argument");
  CHK(need_single(c));
  if (!std::isfinite(x0[0]) || !std::isfinite(x0[1]) || !std::isfinite(x0[2]) || !std::isfinite(k))
    return fail(CB_ERR_ARG, "x0 and k must be finite");
  if (c->kappa_given) return fail(CB_ERR_ARG, "the manufactured solution solves -Lap u = f: kappa must be 1");
  *m = MmsParams{{x0[0], x0[1], x0[2]}, k};
  return CB_OK;
}

int cb_manufactured_load(cb_ctx* c, const double* x0, double k, double* b_dev) {
  MmsParams m;
  CHK(mms_check(c, x0, k, &m));
  if (!b_dev && c->n_dof_tot > 0) return fail(CB_ERR_ARG, "null argument");
  hipStream_t st = c->st;
  DevBuf be;
  CHK(dalloc(be, std::max<int64_t>(1, c->n_cells_tot) * 8 * sizeof(double)));
  launch_mms_volume(st, c->batch(false), m, c->xi_d.as<double>(), c->balls.as<double>(), c->cellinfo.as<int32_t>(),
                    c->n_cells_tot, be.as<double>());
  if (!c->full_elements) {
    CHK(build_sphere_rules(c));
    launch_surface_load(st, c->batch(false), c->sr, c->balls.as<double>(), c->n_cells_tot, c->cut_d.as<int64_t>(),
                        c->n_cut_tot, c->nitsche ? 1 : 0, c->beta_d.as<double>(), m, be.as<double>());
  }
  double* bg = c->bgrid.as<double>();
  double* ud = c->t1.as<double>();
  double* y = c->t2.as<double>();
  launch_mms_gather(st, c->batch(false), c->nn, m, c->cellinfo.as<int32_t>(), c->dofmask.as<uint8_t>(),
                    be.as<double>(), bg, ud);
  CHK(apply_A_grid(c, ud, y, false));
  launch_mms_finish(st, c->n_dof_tot, c->dof_node.as<int64_t>(), bg, y, b_dev);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));   // be is released on return
  return CB_OK;
}

int cb_manufactured_errors(cb_ctx* c, const double* x0, double k, const double* u_dev, double* l2, double* h1) {
  MmsParams m;
  CHK(mms_check(c, x0, k, &m));
  if ((!u_dev && c->n_dof_tot > 0) || !l2 || !h1) return fail(CB_ERR_ARG, "null argument");
  hipStream_t st = c->st;
  DevBuf err, out;
  CHK(dalloc(err, std::max<int64_t>(1, c->n_cells_tot) * 2 * sizeof(double)));
  CHK(dalloc(out, 2 * sizeof(double)));
  double* ug = c->t1.as<double>();
  // the lift at the cube-face nodes, then the DOF values
  launch_mms_gather(st, c->batch(false), c->nn, m, c->cellinfo.as<int32_t>(), c->dofmask.as<uint8_t>(), nullptr,
                    c->t2.as<double>(), ug);
  launch_scatter_dofs(st, c->n_dof_tot, c->dof_node.as<int64_t>(), u_dev, ug);
  launch_mms_errors(st, c->batch(false), m, c->xi_d.as<double>(), c->balls.as<double>(), c->cellinfo.as<int32_t>(),
                    c->n_cells_tot, ug, err.as<double>(), out.as<double>());
  HIPCHK(hipGetLastError());
  double e2[2] = {0.0, 0.0};
  HIPCHK(hipMemcpyAsync(e2, out.p, sizeof(e2), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *l2 = std::sqrt(e2[0]);
  *h1 = std::sqrt(e2[1]);
  return CB_OK;
}

int cb_grad(cb_ctx* c, const double* u_dev, const double* lam_dev, double* dJ_dtheta_dev, double* dJ_df_dev) {
  if (!c || !u_dev || !lam_dev) return fail(CB_ERR_ARG, "null argument");
  CHK(need_single(c));
  const ProbHost& h = c->pb[0];
  const int64_t nn1 = (int64_t)(h.N + 1) * (h.N + 1) * (h.N + 1);
  double* ug = c->t1.as<double>();
  double* lg = c->t2.as<double>();
  launch_fill(c->st, c->nn, 0.0, ug);
  launch_fill(c->st, c->nn, 0.0, lg);
  launch_scatter_dofs(c->st, c->n_dof_tot, c->dof_node.as<int64_t>(), u_dev, ug);
  launch_scatter_dofs(c->st, c->n_dof_tot, c->dof_node.as<int64_t>(), lam_dev, lg);
  GridDesc g{h.N, h.h};
  if (dJ_dtheta_dev)
    launch_grad_theta(c->st, g, c->cellinfo.as<int32_t>(), c->kappa.as<double>(), c->Kc.as<double>(), ug, lg,
                      dJ_dtheta_dev);
  if (dJ_df_dev)
    launch_load(c->st, c->batch(false), nn1, c->cellinfo.as<int32_t>(), c->Mc.as<double>(), nullptr, lg, nullptr,
                dJ_df_dev);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->st));
  return CB_OK;
}

int cb_query(const cb_ctx* c, cb_info* out) {
  if (!c || !out) return fail(CB_ERR_ARG, "null argument");
  *out = c->info;
  out->n_fp64_fallbacks = c->n_fallbacks;
  out->factored = c->factored ? 1 : 0;
  out->lanczos_lmin = out->lanczos_lmax = 0.0;
  if (c->P == 1) fill_lanczos(c, 0, out);
  out->coarse_separator = c->nd.on ? c->nd.n_s : 0;
  out->coarse_octant_max = c->nd.on ? c->nd.n_o_max : 0;
  return CB_OK;
}

int cb_query_problem(const cb_ctx* c, int32_t k, cb_info* out) {
  if (!c || !out) return fail(CB_ERR_ARG, "null argument");
  if (k < 0 || k >= c->P) return fail(CB_ERR_ARG, "problem index out of range");
  *out = c->pb[k].info;
  out->factored = c->factored ? 1 : 0;
  fill_lanczos(c, k, out);
  return CB_OK;
}

int cb_pcg_history(const cb_ctx* c, int32_t k, int32_t cap, double* alpha, double* beta, double* relres, int32_t* n,
                   double* lambda_min, double* lambda_max) {
  if (!c || !n) return fail(CB_ERR_ARG, "null argument");
  if (k < 0 || k >= c->P) return fail(CB_ERR_ARG, "problem index out of range");
  if (cap < 0) return fail(CB_ERR_ARG, "cap must be >= 0");
  std::vector<double> a, b, r;
  CHK(read_history(c, k, &a, &b, &r));
  *n = (int32_t)a.size();
  for (int j = 0; j < (int)a.size() && j < cap; ++j) {
    if (alpha) alpha[j] = a[j];
    if (relres) relres[j] = r[j];
    if (beta && j < (int)b.size()) beta[j] = b[j];
  }
  if (lambda_min || lambda_max) {
    double lo = std::numeric_limits<double>::quiet_NaN(), hi = lo;
    if (lanczos_extremes_impl((int)a.size(), a.data(), b.data(), &lo, &hi) != CB_OK)
      lo = hi = std::numeric_limits<double>::quiet_NaN();
    if (lambda_min) *lambda_min = lo;
    if (lambda_max) *lambda_max = hi;
  }
  return CB_OK;
}

int cb_lanczos_extremes(int32_t n, const double* alpha, const double* beta, double* lambda_min,
                        double* lambda_max) {
  if (n < 0 || !lambda_min || !lambda_max || (n > 0 && !alpha) || (n > 1 && !beta))
    return fail(CB_ERR_ARG, "null argument or n < 0");
  return lanczos_extremes_impl(n, alpha, beta, lambda_min, lambda_max);
}

}  // extern "C"

namespace {

// Host copies of the integer indexing of problem k (see cb_export_indexing).
int export_indexing_impl(const cb_ctx* c, int k, uint8_t* cell_status, int32_t* cell_count, int64_t* dof_node,
                         int32_t* card, int64_t* obj_ptr, int64_t* obj_dofs, int8_t* obj_type,
                         int32_t* coarse_of_obj) {
  const ProbHost& h = c->pb[k];
  const int64_t ncell = (int64_t)h.N * h.N * h.N;
  const int64_t N1 = h.N + 1, nnode = N1 * N1 * N1;
  HIPCHK(hipStreamSynchronize(c->st));
  auto down = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
  };
  if (cell_status || cell_count) {
    std::vector<int32_t> cnt(ncell);
    HIPCHK(down(cnt.data(), c->count_d.as<int32_t>() + h.cell_off, ncell * sizeof(int32_t)));
    if (cell_status)
      for (int64_t i = 0; i < ncell; ++i) cell_status[i] = cnt[i] == 0 ? 0 : (cnt[i] == 512 ? 2 : 1);
    if (cell_count) std::memcpy(cell_count, cnt.data(), ncell * sizeof(int32_t));
  }
  // node data of the problem
  const IndexWork& w = c->iw;
  std::vector<uint8_t> smask(nnode), face(nnode);
  std::vector<int32_t> par1(nnode), par2(nnode), size2(nnode), oidx(nnode), ocid(nnode);
  std::vector<int64_t> dn(std::max<int64_t>(1, h.n_dof));
  HIPCHK(down(smask.data(), w.smask + h.node_off, nnode));
  HIPCHK(down(face.data(), w.face + h.node_off, nnode));
  HIPCHK(down(par1.data(), w.par1 + h.node_off, nnode * sizeof(int32_t)));
  HIPCHK(down(par2.data(), w.par2 + h.node_off, nnode * sizeof(int32_t)));
  HIPCHK(down(size2.data(), w.size2 + h.node_off, nnode * sizeof(int32_t)));
  HIPCHK(down(oidx.data(), w.oidx + h.node_off, nnode * sizeof(int32_t)));
  HIPCHK(down(ocid.data(), w.ocid + h.node_off, nnode * sizeof(int32_t)));
  if (h.n_dof) HIPCHK(down(dn.data(), c->dof_node.as<int64_t>() + h.dof_off, h.n_dof * sizeof(int64_t)));
  for (int64_t d = 0; d < h.n_dof; ++d) dn[d] -= h.node_off;
  if (dof_node) std::memcpy(dof_node, dn.data(), h.n_dof * sizeof(int64_t));
  if (card)
    for (int64_t d = 0; d < h.n_dof; ++d) card[d] = __builtin_popcount(smask[dn[d]]);
  // objects: interface DOFs grouped by their root, ascending within each
  const int64_t nobj = h.n_obj;
  std::vector<int64_t> ptr(nobj + 1, 0);
  auto obj_of = [&](int64_t ln) -> int64_t {
    const int64_t r = (int64_t)par2[ln] - h.node_off;
    if (r < 0 || r >= nnode) return -1;
    const int64_t o = (int64_t)oidx[r] - h.obj_off;
    return (o >= 0 && o < nobj) ? o : -1;
  };
  int64_t n_if = 0;
  for (int64_t d = 0; d < h.n_dof; ++d) {
    if (dn[d] < 0 || dn[d] >= nnode) return fail(CB_ERR_STATE, "index export: DOF node out of range");
    if (__builtin_popcount(smask[dn[d]]) < 2) continue;
    const int64_t o = obj_of(dn[d]);
    if (o < 0)
      return fail(CB_ERR_STATE, "index export: DOF " + std::to_string(d) + " (node " + std::to_string(dn[d]) +
                                    ") has root " + std::to_string(par2[dn[d]]) + " without an object index (" +
                                    std::to_string(oidx[std::min<int64_t>(std::max<int64_t>(0, par2[dn[d]] - h.node_off), nnode - 1)]) +
                                    ", objects " + std::to_string(nobj) + ")");
    ptr[o + 1]++;
    ++n_if;
  }
  if (n_if != h.n_iface) return fail(CB_ERR_STATE, "index export: interface count mismatch");
  for (int64_t o = 0; o < nobj; ++o) ptr[o + 1] += ptr[o];
  if (obj_ptr) std::memcpy(obj_ptr, ptr.data(), (nobj + 1) * sizeof(int64_t));
  if (obj_dofs) {
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t d = 0; d < h.n_dof; ++d)
      if (__builtin_popcount(smask[dn[d]]) >= 2) obj_dofs[fill[obj_of(dn[d])]++] = d;
  }
  for (int64_t ln = 0; ln < nnode; ++ln) {
    if (__builtin_popcount(smask[ln]) < 2 || par2[ln] != ln + h.node_off) continue;
    const int64_t o = oidx[ln] - h.obj_off;
    if (o < 0 || o >= nobj) return fail(CB_ERR_STATE, "index export: object index out of range");
    if (par1[ln] - h.node_off < 0 || par1[ln] - h.node_off >= nnode)
      return fail(CB_ERR_STATE, "index export: pass-1 root out of range");
    if (obj_type)
      obj_type[o] = size2[ln] == 1 ? OBJ_CORNER : (face[par1[ln] - h.node_off] ? OBJ_FACE : OBJ_EDGE);
    if (coarse_of_obj) coarse_of_obj[o] = ocid[ln] >= 0 ? ocid[ln] - h.coarse_off : -1;
  }
  return CB_OK;
}

}  // namespace

extern "C" {

int cb_export_indexing(const cb_ctx* c, uint8_t* cell_status, int32_t* cell_count, int64_t* dof_node,
                       int32_t* card, int64_t* obj_ptr, int64_t* obj_dofs, int8_t* obj_type,
                       int32_t* coarse_of_obj) {
  if (!c) return fail(CB_ERR_ARG, "null context");
  CHK(need_single(c));
  return export_indexing_impl(c, 0, cell_status, cell_count, dof_node, card, obj_ptr, obj_dofs, obj_type,
                              coarse_of_obj);
}

int cb_export_problem_indexing(const cb_ctx* c, int32_t k, uint8_t* cell_status, int32_t* cell_count,
                               int64_t* dof_node, int32_t* card, int64_t* obj_ptr, int64_t* obj_dofs,
                               int8_t* obj_type, int32_t* coarse_of_obj) {
  if (!c) return fail(CB_ERR_ARG, "null context");
  if (k < 0 || k >= c->P) return fail(CB_ERR_ARG, "problem index out of range");
  return export_indexing_impl(c, k, cell_status, cell_count, dof_node, card, obj_ptr, obj_dofs, obj_type,
                              coarse_of_obj);
}

int cb_export_subdomains(const cb_ctx* c, int32_t k, int64_t* sub_ptr, int64_t* sub_dofs) {
  if (!c || !sub_ptr) return fail(CB_ERR_ARG, "null argument");
  if (k < 0 || k >= c->P) return fail(CB_ERR_ARG, "problem index out of range");
  const ProbHost& h = c->pb[k];
  HIPCHK(hipStreamSynchronize(c->st));
  const int NIp = c->NIp, NGp = c->NGp;
  std::vector<int64_t> I((size_t)h.ns * NIp), G((size_t)h.ns * NGp), dn(std::max<int64_t>(1, h.n_dof));
  if (h.ns) {
    HIPCHK(hipMemcpy(I.data(), c->Iidx.as<int64_t>() + (int64_t)h.sub_off * NIp, I.size() * sizeof(int64_t),
                     hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(G.data(), c->Gidx.as<int64_t>() + (int64_t)h.sub_off * NGp, G.size() * sizeof(int64_t),
                     hipMemcpyDeviceToHost));
  }
  if (h.n_dof)
    HIPCHK(hipMemcpy(dn.data(), c->dof_node.as<int64_t>() + h.dof_off, h.n_dof * sizeof(int64_t),
                     hipMemcpyDeviceToHost));
  // grid node -> DOF id (DOFs are in ascending node order)
  auto dof_of = [&](int64_t node) -> int64_t {
    const auto it = std::lower_bound(dn.begin(), dn.begin() + h.n_dof, node);
    return (it != dn.begin() + h.n_dof && *it == node) ? (int64_t)(it - dn.begin()) : -1;
  };
  sub_ptr[0] = 0;
  std::vector<int64_t> loc;
  for (int w = 0; w < h.ns; ++w) {
    loc.clear();
    for (int i = 0; i < NIp; ++i)
      if (I[(size_t)w * NIp + i] >= 0) loc.push_back(dof_of(I[(size_t)w * NIp + i]));
    for (int j = 0; j < NGp; ++j)
      if (G[(size_t)w * NGp + j] >= 0) loc.push_back(dof_of(G[(size_t)w * NGp + j]));
    for (int64_t d : loc)
      if (d < 0) return fail(CB_ERR_STATE, "subdomain export: a local node is not a DOF");
    std::sort(loc.begin(), loc.end());
    if (sub_dofs) std::copy(loc.begin(), loc.end(), sub_dofs + sub_ptr[w]);
    sub_ptr[w + 1] = sub_ptr[w] + (int64_t)loc.size();
  }
  return CB_OK;
}

int cb_export_cut_matrices(const cb_ctx* c, double* K, double* M, int64_t* cut_cells) {
  if (!c) return fail(CB_ERR_ARG, "null context");
  CHK(need_single(c));
  const ProbHost& h = c->pb[0];
  const int64_t n = h.n_cut_stored;
  HIPCHK(hipStreamSynchronize(c->st));
  if (K && n) HIPCHK(hipMemcpy(K, c->Kc.p, n * PACK36 * sizeof(double), hipMemcpyDeviceToHost));
  if (M && n) HIPCHK(hipMemcpy(M, c->Mc.p, n * PACK36 * sizeof(double), hipMemcpyDeviceToHost));
  if (cut_cells && n) {
    HIPCHK(hipMemcpy(cut_cells, c->cut_d.as<int64_t>() + h.cut_off, n * sizeof(int64_t), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i) cut_cells[i] -= h.cell_off;
  }
  return CB_OK;
}

int cb_export_coarse(const cb_ctx* c, double* Ac) {
  if (!c || !Ac) return fail(CB_ERR_ARG, "null argument");
  CHK(need_single(c));
  if (!c->factored) return fail(CB_ERR_STATE, "coarse matrix requested before cb_factor");
  const ProbHost& h = c->pb[0];
  const int nc = h.n_coarse, ldc = h.ldc;
  if (nc == 0) return CB_OK;
  if (!c->AcKeep.p) return fail(CB_ERR_STATE, "the coarse matrix is kept only up to 1 GiB");
  HIPCHK(hipMemcpy2D(Ac, nc * sizeof(double), c->AcKeep.as<double>() + h.ac_off, ldc * sizeof(double),
                     nc * sizeof(double), nc, hipMemcpyDeviceToHost));
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

int cb_profile_launches(cb_ctx* c, const char* name, double* ms, int64_t cap, int64_t* n) {
  if (!c || !name || (cap > 0 && !ms)) return fail(CB_ERR_ARG, "null argument");
  HIPCHK(hipStreamSynchronize(c->st));
  int64_t k = 0;
  auto it = c->prof_ev.find(name);
  if (it != c->prof_ev.end())
    for (auto& e : it->second.ev) {
      if (k < cap) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, e.first, e.second));
        ms[k] = t;
      }
      ++k;
    }
  if (n) *n = k;
  return CB_OK;
}

int cb_time_kernel(cb_ctx* c, int32_t which, int32_t reps, double* avg_ms) {
  if (!c || !avg_ms || reps < 1 || which < 0 || which > 1) return fail(CB_ERR_ARG, "invalid argument");
  if (!c->factored) return fail(CB_ERR_STATE, "kernel timing requested before cb_factor");
  hipStream_t st = c->st;
  const SubDev sd = c->sub(0, false);
  const bool f32 = c->precision == CB_FP32_LOCAL;
  auto launch = [&] {
    if (which == 0) {
      if (f32) launch_apply_interior<float>(st, sd, c->ns, c->P_.as<float>(), c->r.as<double>(), nullptr,
                                            c->t1.as<double>());
      else launch_apply_interior<double>(st, sd, c->ns, c->P_.as<double>(), c->r.as<double>(), nullptr,
                                         c->t1.as<double>());
    } else {
      if (f32) launch_apply_neumann<float, float>(st, sd, c->ns, c->Kt.as<float>(), c->Phi32.as<float>(),
                                           c->Dw.as<double>(), c->r.as<double>(), c->t2.as<double>(),
                                           c->zbuf.as<double>(), c->cloc.as<double>());
      else launch_apply_neumann<double, double>(st, sd, c->ns, c->Kt.as<double>(), c->Phi.as<double>(),
                                        c->Dw.as<double>(), c->r.as<double>(), c->t2.as<double>(),
                                        c->zbuf.as<double>(), c->cloc.as<double>());
    }
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  EventPair ev01{&e0, &e1};
  HIPCHK(pooled_time_event(&e0));
  HIPCHK(pooled_time_event(&e1));
  launch();   // warm
  HIPCHK(hipEventRecord(e0, st));
  for (int i = 0; i < reps; ++i) launch();
  HIPCHK(hipEventRecord(e1, st));
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  *avg_ms = (double)ms / reps;
  return CB_OK;
}

void cb_destroy(cb_ctx* c) {
  if (!c) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  else (void)hipDeviceSynchronize();
  delete c;
}

}  // extern "C"

namespace cutbddc {
int report_error(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace cutbddc
