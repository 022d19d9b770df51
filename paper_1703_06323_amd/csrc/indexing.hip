// Device indexing for cut-cell BDDC (see indexing.h).
//
// Readings of the paper (which gives no algorithm for these steps); the host
// indexing follows the same rules:
//  * DOFs: grid nodes (I,J,K), 1 <= I,J,K <= N-1, touched by an active cell,
//    numbered by ascending node id (strong Dirichlet on the cube faces,
//    Sect. 5.1).
//  * S(xi): ascending ids of the subdomains owning an active cell that
//    contains xi; interior DOF iff |S| = 1 (Sect. 3.2).
//  * Objects: connected components of links between axis-adjacent interface
//    DOFs a, b with S(a) = S(b) such that every subdomain of S(a) has an
//    active cell containing the FE edge (a, b).  Corner if one DOF; face if
//    it holds the 4 DOFs of a mesh face whose two cells are active and lie in
//    the two subdomains of S; edge otherwise.  Ordered by smallest DOF.
//  * Variant 1 (Sect. 4.4): every DOF of a cut FE edge of an edge object is a
//    corner; the other DOFs form sub-edges through non-cut FE edges; a
//    one-DOF sub-edge is a corner.  FE edges are classified exactly against
//    the balls (segment distance for "inside Omega", chord coverage for
//    "outside Omega"), without FMA contraction.
//  * An active component (cells joined through shared DOF nodes) without a
//    cell on the cube boundary makes the operator singular.
//
// Connected components use a lock-free union-find in which a root is only
// ever hooked below a smaller node (compare-and-swap on the root's parent),
// so every component ends rooted at its smallest node whatever the order of
// the hooks: the result is deterministic.
#include "indexing.h"

#pragma clang fp contract(off)

namespace cutbddc {
namespace {

constexpr int IT = 256;               // threads per workgroup of every kernel here
constexpr int IE = 4;                 // scan elements per thread
constexpr int IBS = IT * IE;          // scan elements per workgroup

__device__ inline Count4 c4add(Count4 a, Count4 b) { return {a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w}; }
__device__ inline Count4 c4sub(Count4 a, Count4 b) { return {a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w}; }
__device__ inline Count4 shfl_up4(Count4 v, int d) {
  return {__shfl_up(v.x, d, 64), __shfl_up(v.y, d, 64), __shfl_up(v.z, d, 64), __shfl_up(v.w, d, 64)};
}

// Exclusive prefix of v over the workgroup (thread order); *tot = the sum.
// Every thread of the workgroup must call it.
__device__ Count4 block_exclusive(Count4 v, Count4* tot) {
  __shared__ Count4 wsum[IT / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  Count4 inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const Count4 o = shfl_up4(inc, d);
    if (lane >= d) inc = c4add(inc, o);
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  Count4 off = {0, 0, 0, 0}, all = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < IT / 64; ++q) {
    if (q < wv) off = c4add(off, wsum[q]);
    all = c4add(all, wsum[q]);
  }
  __syncthreads();
  *tot = all;
  return c4add(off, c4sub(inc, v));
}

// ---- three-pass exclusive scan over [0, n) of the Count4 values of a functor
template <class F>
__global__ __launch_bounds__(IT) void scan_reduce_kernel(F f, int64_t n, Count4* bsum) {
  const int64_t i0 = (int64_t)blockIdx.x * IBS + threadIdx.x * IE;
  Count4 s = {0, 0, 0, 0};
#pragma unroll
  for (int e = 0; e < IE; ++e)
    if (i0 + e < n) s = c4add(s, f.value(i0 + e));
  Count4 tot;
  (void)block_exclusive(s, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

template <class F>
__global__ __launch_bounds__(IT) void scan_top_kernel(F f, Count4* bsum, int64_t nblk) {
  Count4 carry = {0, 0, 0, 0};
  for (int64_t b0 = 0; b0 < nblk; b0 += IT) {
    const int64_t b = b0 + threadIdx.x;
    const Count4 v = b < nblk ? bsum[b] : Count4{0, 0, 0, 0};
    Count4 tot;
    const Count4 ex = block_exclusive(v, &tot);
    if (b < nblk) bsum[b] = c4add(carry, ex);
    carry = c4add(carry, tot);
  }
  if (threadIdx.x == 0) f.finish(carry);
}

template <class F>
__global__ __launch_bounds__(IT) void scan_apply_kernel(F f, int64_t n, const Count4* bsum) {
  const int64_t i0 = (int64_t)blockIdx.x * IBS + threadIdx.x * IE;
  Count4 v[IE];
  Count4 s = {0, 0, 0, 0};
#pragma unroll
  for (int e = 0; e < IE; ++e) {
    v[e] = (i0 + e < n) ? f.value(i0 + e) : Count4{0, 0, 0, 0};
    s = c4add(s, v[e]);
  }
  Count4 tot;
  Count4 pre = c4add(bsum[blockIdx.x], block_exclusive(s, &tot));
#pragma unroll
  for (int e = 0; e < IE; ++e)
    if (i0 + e < n) {
      f.write(i0 + e, pre, v[e]);
      pre = c4add(pre, v[e]);
    }
}

template <class F>
void run_scan(hipStream_t st, const F& f, int64_t n, Count4* bsum) {
  if (n <= 0) return;
  const int64_t nblk = (n + IBS - 1) / IBS;
  hipLaunchKernelGGL(scan_reduce_kernel<F>, dim3((unsigned)nblk), dim3(IT), 0, st, f, n, bsum);
  hipLaunchKernelGGL(scan_top_kernel<F>, dim3(1), dim3(IT), 0, st, f, bsum, nblk);
  hipLaunchKernelGGL(scan_apply_kernel<F>, dim3((unsigned)nblk), dim3(IT), 0, st, f, n, bsum);
}

// Records the running prefix at the first entry of every problem segment
// (segment starts are multiples of SEG_ALIGN) and the totals at entry P.
__device__ inline void record_segment(const int64_t* off, int P, int64_t i, Count4 pre, Count4* seg) {
  if (i % SEG_ALIGN != 0) return;
  const int p = find_segment(off, P, i);
  if (off[p] == i) seg[p] = pre;
}

// ---- node geometry ------------------------------------------------------
struct NodePos {
  int p, N, s, m;
  int I, J, K;
};
// Problem and grid coordinates of concatenated node n; false for padding.
__device__ inline bool node_pos(const BatchDev& b, int64_t n, NodePos& q) {
  q.p = find_segment(b.node_off, b.P, n);
  const ProbDev& d = b.prob[q.p];
  const int64_t N1 = d.N + 1, ln = n - d.node_off;
  if (ln >= N1 * N1 * N1) return false;
  q.N = d.N;
  q.s = d.s;
  q.m = d.m;
  q.I = (int)(ln % N1);
  q.J = (int)((ln / N1) % N1);
  q.K = (int)(ln / (N1 * N1));
  return true;
}

// Subdomain ids of the S-mask of the node at (I,J,K), ascending; returns |S|.
// Bit dx + 2 dy + 4 dz stands for block (bx0 + dx, by0 + dy, bz0 + dz), with
// (bx0, by0, bz0) the block of cell (I-1, J-1, K-1); ascending bits are
// ascending subdomain ids.
__device__ inline int mask_ids(uint32_t mask, int I, int J, int K, int s, int m, int32_t ids[8]) {
  const int bx = (I - 1) / s, by = (J - 1) / s, bz = (K - 1) / s;
  int c = 0;
  for (int u = 0; u < 8; ++u)
    if (mask >> u & 1u) ids[c++] = (bx + (u & 1)) + m * ((by + (u >> 1 & 1)) + m * (bz + (u >> 2)));
  return c;
}

// Position of subdomain block (Bx,By,Bz) in the S-mask of node (I,J,K), or -1
// if the block is not in S; *rank = its index in ascending S.
__device__ inline int mask_rank(uint32_t mask, int I, int J, int K, int s, int Bx, int By, int Bz) {
  const int dx = Bx - (I - 1) / s, dy = By - (J - 1) / s, dz = Bz - (K - 1) / s;
  if (dx < 0 || dx > 1 || dy < 0 || dy > 1 || dz < 0 || dz > 1) return -1;
  const int u = dx + 2 * dy + 4 * dz;
  if (!(mask >> u & 1u)) return -1;
  return __popc(mask & ((1u << u) - 1u));
}

// ---- union-find ---------------------------------------------------------
// Walks read parents with cacheable loads (relaxed atomics of workgroup
// scope), which may return an out-of-date parent: every value ever stored
// in par[x] is an ancestor of x (smaller, same set), so a walk still ends at
// a node that is or was a root, and a hook on a node that is no longer a
// root fails its compare-and-swap (agent scope) and is retried from the
// parent the swap returns.  Stores (path halving, only ever on non-roots)
// are agent-scope, so no cached copy can overwrite a hook.  Agent-coherent
// loads would be correct too but pay a memory round trip per step.
__device__ inline int32_t uf_load(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline int32_t uf_find(int32_t* par, int32_t x) {
  int32_t cur = uf_load(&par[x]);
  if (cur == x) return x;
  int32_t prev = x, next;
  while (cur > (next = uf_load(&par[cur]))) {
    __hip_atomic_store(&par[prev], next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    prev = cur;
    cur = next;
  }
  return cur;
}
__device__ inline void uf_unite(int32_t* par, int32_t a, int32_t b) {
  int32_t ra = uf_find(par, a), rb = uf_find(par, b);
  while (ra != rb) {
    if (ra < rb) {
      const int32_t t = ra;
      ra = rb;
      rb = t;
    }
    // hook the larger root below the smaller node
    const int32_t old = atomicCAS(&par[ra], ra, rb);
    if (old == ra) break;
    ra = uf_find(par, old);
  }
}

__global__ __launch_bounds__(IT) void iota_kernel(int64_t n, int32_t* par) {
  const int64_t i = (int64_t)blockIdx.x * IT + threadIdx.x;
  if (i < n) par[i] = (int32_t)i;
}
__global__ __launch_bounds__(IT) void zero_u8_kernel(int64_t n, uint8_t* a, uint8_t* b, uint8_t* c) {
  const int64_t i = (int64_t)blockIdx.x * IT + threadIdx.x;
  if (i < n) {
    a[i] = 0;
    b[i] = 0;
    c[i] = 0;
  }
}
__global__ __launch_bounds__(IT) void zero_i32_kernel(int64_t n, int32_t* a, int32_t* b) {
  const int64_t i = (int64_t)blockIdx.x * IT + threadIdx.x;
  if (i < n) {
    a[i] = 0;
    if (b) b[i] = 0;
  }
}
// After all joins: par[i] = root of i.  The walk reads coherent values and
// writes nothing, so the only store to par[i] is this thread's (and it
// stores the root).
__global__ __launch_bounds__(IT) void compress_kernel(int64_t n, int32_t* par) {
  const int64_t i = (int64_t)blockIdx.x * IT + threadIdx.x;
  if (i >= n) return;
  int32_t r = (int32_t)i, q;
  while ((q = __hip_atomic_load(&par[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != r) r = q;
  par[i] = r;
}

// ---- cells ---------------------------------------------------------------
struct CellScan {
  BatchDev b;
  const int32_t* count;
  int store_cut;
  int32_t* cellinfo;
  int64_t* cut;
  Count4* seg;
  __device__ Count4 value(int64_t c) const {
    const int p = find_segment(b.cell_off, b.P, c);
    const ProbDev& d = b.prob[p];
    const int64_t N = d.N;
    if (c - d.cell_off >= N * N * N) return {0, 0, 0, 0};
    const int32_t k = count[c];
    const int cutg = (k > 0 && k < 512) ? 1 : 0;
    return {k > 0 ? 1 : 0, cutg, store_cut ? cutg : 0, 0};
  }
  __device__ void write(int64_t c, Count4 pre, Count4 v) const {
    record_segment(b.cell_off, b.P, c, pre, seg);
    cellinfo[c] = v.z ? pre.z : (v.x ? CELL_UNCUT : CELL_INACTIVE);
    if (v.z) cut[pre.z] = c;
  }
  __device__ void finish(Count4 tot) const { seg[b.P] = tot; }
};

// ---- S masks and DOFs ----------------------------------------------------
__global__ __launch_bounds__(IT) void smask_kernel(BatchDev b, int64_t nn, const int32_t* __restrict__ count,
                                                   uint8_t* __restrict__ smask, uint8_t* __restrict__ dofmask) {
  const int64_t n = (int64_t)blockIdx.x * IT + threadIdx.x;
  if (n >= nn) return;
  NodePos q;
  uint32_t mask = 0;
  if (node_pos(b, n, q) && q.I >= 1 && q.J >= 1 && q.K >= 1 && q.I < q.N && q.J < q.N && q.K < q.N) {
    const int32_t* cnt = count + b.prob[q.p].cell_off;
    const int bx = (q.I - 1) / q.s, by = (q.J - 1) / q.s, bz = (q.K - 1) / q.s;
    for (int u = 0; u < 8; ++u) {
      const int ci = q.I - 1 + (u & 1), cj = q.J - 1 + (u >> 1 & 1), ck = q.K - 1 + (u >> 2);
      if (cnt[ci + (int64_t)q.N * (cj + (int64_t)q.N * ck)] <= 0) continue;
      const int dx = ci / q.s - bx, dy = cj / q.s - by, dz = ck / q.s - bz;
      mask |= 1u << (dx + 2 * dy + 4 * dz);
    }
  }
  smask[n] = (uint8_t)mask;
  dofmask[n] = mask ? 1 : 0;
}

struct NodeScan {
  BatchDev b;
  const uint8_t* smask;
  int64_t* dof_node;
  int32_t* gif;
  int32_t* gifp;
  Count4* seg;
  __device__ Count4 value(int64_t n) const {
    const uint32_t m = smask[n];
    const int card = __popc(m);
    return {m ? 1 : 0, card >= 2 ? 1 : 0, card >= 2 ? card : 0, 0};
  }
  __device__ void write(int64_t n, Count4 pre, Count4 v) const {
    record_segment(b.node_off, b.P, n, pre, seg);
    if (v.x) dof_node[pre.x] = n;
    gif[n] = v.y ? pre.y : -1;
    gifp[n] = v.y ? pre.z : -1;
  }
  __device__ void finish(Count4 tot) const { seg[b.P] = tot; }
};

__device__ inline int64_t axis_step(int axis, int64_t N1) { return axis == 0 ? 1 : (axis == 1 ? N1 : N1 * N1); }

// ---- floating components ---------------------------------------------------
// After the joins (float_local_kernel, float_cross_kernel, compression): an
// active cell on the cube boundary marks the component of its DOF corners
// as grounded.
__global__ __launch_bounds__(IT) void float_ground_kernel(BatchDev b, int64_t nc, const int32_t* __restrict__ count,
                                                          const uint8_t* __restrict__ smask,
                                                          const int32_t* __restrict__ par, uint8_t* ground) {
  const int64_t c = (int64_t)blockIdx.x * IT + threadIdx.x;
  if (c >= nc) return;
  const int p = find_segment(b.cell_off, b.P, c);
  const ProbDev& d = b.prob[p];
  const int64_t N = d.N, N1 = N + 1, lc = c - d.cell_off;
  if (lc >= N * N * N || count[c] <= 0) return;
  const int64_t i = lc % N, j = (lc / N) % N, k = lc / (N * N);
  if (!(i == 0 || j == 0 || k == 0 || i == N - 1 || j == N - 1 || k == N - 1)) return;
  for (int u = 0; u < 8; ++u) {
    const int64_t n = d.node_off + (i + (u & 1)) + N1 * ((j + (u >> 1 & 1)) + N1 * (k + (u >> 2)));
    if (smask[n]) {
      ground[par[n]] = 1;
      return;
    }
  }
}

// Edge-based joins for the floating check.  The DOF corners of an active
// cell are the cell's corners off the cube faces: a sub-box of the cell,
// connected through its edges, so DOF nodes joined by active cells are the
// DOF nodes joined by FE edges that belong to an active cell.  Whether the
// edge from node (I, J, K) along axis a is such an edge:
__device__ inline bool active_edge(const int32_t* __restrict__ cnt, int N, int I, int J, int K, int axis) {
  const int o1 = axis == 0 ? 1 : 0, o2 = axis == 2 ? 1 : 2;   // the two other axes
  const int ijk[3] = {I, J, K};
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      int c3[3] = {ijk[0], ijk[1], ijk[2]};
      c3[o1] -= u;
      c3[o2] -= v;
      if (c3[0] < 0 || c3[1] < 0 || c3[2] < 0 || c3[0] >= N || c3[1] >= N || c3[2] >= N) continue;
      if (cnt[c3[0] + (int64_t)N * (c3[1] + (int64_t)N * c3[2])] > 0) return true;
    }
  return false;
}

// Pass 1: joins along the active FE edges whose two nodes lie in the same
// block of IT consecutive nodes, by union-find in LDS (larger root below the
// smaller node); every node then points to its block-local root.  Pass 2
// (float_cross_kernel) joins the edges that leave the block, by the global
// union-find.
__global__ __launch_bounds__(IT) void float_local_kernel(BatchDev b, int64_t nn, const int32_t* __restrict__ count,
                                                         const uint8_t* __restrict__ smask, int32_t* __restrict__ par) {
  __shared__ int32_t lp[IT];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * IT, n = base + tid;
  lp[tid] = tid;
  __syncthreads();
  NodePos q;
  if (n < nn && smask[n] && node_pos(b, n, q)) {
    const ProbDev& d = b.prob[q.p];
    const int64_t N1 = q.N + 1;
    const int32_t* cnt = count + d.cell_off;
    const int ijk[3] = {q.I, q.J, q.K};
    for (int axis = 0; axis < 3; ++axis) {
      const int64_t m = n + axis_step(axis, N1);
      if (ijk[axis] + 1 > q.N || m >= base + IT || !smask[m] || !active_edge(cnt, q.N, q.I, q.J, q.K, axis))
        continue;
      int ra = tid, rb = (int)(m - base);
      for (;;) {
        while (true) {
          const int t = __hip_atomic_load(&lp[ra], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (t == ra) break;
          ra = t;
        }
        while (true) {
          const int t = __hip_atomic_load(&lp[rb], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (t == rb) break;
          rb = t;
        }
        if (ra == rb) break;
        if (ra < rb) {
          const int t = ra;
          ra = rb;
          rb = t;
        }
        if (atomicCAS(&lp[ra], ra, rb) == ra) break;
      }
    }
  }
  __syncthreads();
  if (n < nn) {
    int r = tid;
    while (true) {
      const int t = lp[r];
      if (t == r) break;
      r = t;
    }
    par[n] = (int32_t)(base + r);
  }
}

__global__ __launch_bounds__(IT) void float_cross_kernel(BatchDev b, int64_t nn, const int32_t* __restrict__ count,
                                                         const uint8_t* __restrict__ smask, int32_t* par) {
  const int64_t n = (int64_t)blockIdx.x * IT + threadIdx.x;
  const int64_t end = ((int64_t)blockIdx.x + 1) * IT;
  NodePos q;
  if (n >= nn || !smask[n] || !node_pos(b, n, q)) return;
  const ProbDev& d = b.prob[q.p];
  const int64_t N1 = q.N + 1;
  const int32_t* cnt = count + d.cell_off;
  const int ijk[3] = {q.I, q.J, q.K};
  for (int axis = 0; axis < 3; ++axis) {
    const int64_t m = n + axis_step(axis, N1);
    if (ijk[axis] + 1 > q.N || m < end || !smask[m] || !active_edge(cnt, q.N, q.I, q.J, q.K, axis)) continue;
    uf_unite(par, (int32_t)n, (int32_t)m);
  }
}

__global__ __launch_bounds__(IT) void float_check_kernel(BatchDev b, int64_t nn, const uint8_t* __restrict__ smask,
                                                         const int32_t* __restrict__ par,
                                                         const uint8_t* __restrict__ ground, int32_t* floating) {
  const int64_t n = (int64_t)blockIdx.x * IT + threadIdx.x;
  if (n >= nn || !smask[n] || par[n] != n || ground[n]) return;
  floating[find_segment(b.node_off, b.P, n)] = 1;
}

// ---- links and objects -----------------------------------------------------

__global__ __launch_bounds__(IT) void link_kernel(BatchDev b, int64_t nn, const int32_t* __restrict__ count,
                                                  const uint8_t* __restrict__ smask, uint8_t* __restrict__ link) {
  const int64_t n = (int64_t)blockIdx.x * IT + threadIdx.x;
  if (n >= nn) return;
  const uint32_t ma = smask[n];
  uint8_t bits = 0;
  NodePos q;
  if (__popc(ma) >= 2 && node_pos(b, n, q)) {
    const ProbDev& d = b.prob[q.p];
    const int32_t* cnt = count + d.cell_off;
    const int64_t N1 = q.N + 1, N = q.N;
    int32_t Sa[8];
    const int ca = mask_ids(ma, q.I, q.J, q.K, q.s, q.m, Sa);
    const int ijk[3] = {q.I, q.J, q.K};
    for (int axis = 0; axis < 3; ++axis) {
      const uint32_t mb = smask[n + axis_step(axis, N1)];
      if (__popc(mb) != ca) continue;
      int nijk[3] = {q.I, q.J, q.K};
      nijk[axis] += 1;
      int32_t Sb[8];
      (void)mask_ids(mb, nijk[0], nijk[1], nijk[2], q.s, q.m, Sb);
      bool same = true;
      for (int t = 0; t < ca; ++t)
        if (Sa[t] != Sb[t]) same = false;
      if (!same) continue;
      // subdomains of the active cells around the FE edge
      const int o1 = axis == 0 ? 1 : 0, o2 = axis == 2 ? 1 : 2;
      int32_t St[4];
      int nst = 0;
      for (int u = -1; u <= 0; ++u)
        for (int v = -1; v <= 0; ++v) {
          int c3[3] = {ijk[0], ijk[1], ijk[2]};
          c3[o1] += u;
          c3[o2] += v;
          if (c3[0] < 0 || c3[1] < 0 || c3[2] < 0 || c3[0] >= N || c3[1] >= N || c3[2] >= N) continue;
          if (cnt[c3[0] + N * (c3[1] + N * (int64_t)c3[2])] <= 0) continue;
          St[nst++] = c3[0] / q.s + q.m * (c3[1] / q.s + q.m * (c3[2] / q.s));
        }
      bool full = true;
      for (int t = 0; t < ca; ++t) {
        bool present = false;
        for (int z = 0; z < nst; ++z)
          if (St[z] == Sa[t]) present = true;
        if (!present) full = false;
      }
      if (full) bits |= (uint8_t)(1u << axis);
    }
  }
  link[n] = bits;
}

// Joins every link (pass 1), or every link that is not cut and touches no
// cut DOF (pass 2).
__global__ __launch_bounds__(IT) void link_join_kernel(BatchDev b, int64_t nn, const uint8_t* __restrict__ link,
                                                       const uint8_t* cutdof, int32_t* par) {
  const int64_t n = (int64_t)blockIdx.x * IT + threadIdx.x;
  if (n >= nn) return;
  const uint32_t L = link[n];
  if (!(L & 7u)) return;
  if (cutdof && cutdof[n]) return;
  const int p = find_segment(b.node_off, b.P, n);
  const int64_t N1 = b.prob[p].N + 1;
  for (int axis = 0; axis < 3; ++axis) {
    if (!(L >> axis & 1u)) continue;
    const int64_t m = n + axis_step(axis, N1);
    if (cutdof && ((L >> (3 + axis) & 1u) || cutdof[m])) continue;
    uf_unite(par, (int32_t)n, (int32_t)m);
  }
}

// Pass-1 objects holding a subdomain face: cells c (last layer of a block
// along an axis) and h = c + e_axis (first layer of the next block), both
// active, whose 4 shared nodes are interface DOFs of one object with
// S = {sub(c), sub(h)}.
__global__ __launch_bounds__(IT) void face_kernel(BatchDev b, int64_t nc, const int32_t* __restrict__ count,
                                                  const uint8_t* __restrict__ smask, const int32_t* __restrict__ par1,
                                                  uint8_t* face) {
  const int64_t c = (int64_t)blockIdx.x * IT + threadIdx.x;
  if (c >= nc || count[c] <= 0) return;
  const int p = find_segment(b.cell_off, b.P, c);
  const ProbDev& d = b.prob[p];
  const int64_t N = d.N, N1 = N + 1, lc = c - d.cell_off;
  if (lc >= N * N * N) return;
  const int s = d.s, m = d.m;
  const int c3[3] = {(int)(lc % N), (int)((lc / N) % N), (int)(lc / (N * N))};
  for (int axis = 0; axis < 3; ++axis) {
    if (c3[axis] % s != s - 1 || c3[axis] + 1 >= N) continue;
    int h3[3] = {c3[0], c3[1], c3[2]};
    h3[axis] += 1;
    if (count[d.cell_off + h3[0] + N * (h3[1] + N * (int64_t)h3[2])] <= 0) continue;
    const int o1 = axis == 0 ? 1 : 0, o2 = axis == 2 ? 1 : 2;
    int32_t root = -1;
    bool ok = true;
    int64_t n0 = -1;
    for (int uu = 0; uu <= 1 && ok; ++uu)
      for (int vv = 0; vv <= 1 && ok; ++vv) {
        int n3[3] = {h3[0], h3[1], h3[2]};
        n3[o1] += uu;
        n3[o2] += vv;
        const int64_t n = d.node_off + n3[0] + N1 * (n3[1] + N1 * (int64_t)n3[2]);
        if (__popc((uint32_t)smask[n]) < 2) {
          ok = false;
          break;
        }
        if (n0 < 0) {
          n0 = n;
          root = par1[n];
        } else if (par1[n] != root) {
          ok = false;
        }
      }
    if (!ok) continue;
    const uint32_t m0 = smask[n0];
    if (__popc(m0) != 2) continue;
    const int64_t l0 = n0 - d.node_off;
    int32_t S0[8];
    (void)mask_ids(m0, (int)(l0 % N1), (int)((l0 / N1) % N1), (int)(l0 / (N1 * N1)), s, m, S0);
    const int32_t w1 = c3[0] / s + m * (c3[1] / s + m * (c3[2] / s));
    const int32_t w2 = h3[0] / s + m * (h3[1] / s + m * (h3[2] / s));
    if (min(w1, w2) == S0[0] && max(w1, w2) == S0[1]) face[root] = 1;
  }
}

__global__ __launch_bounds__(IT) void object_size_kernel(int64_t nn, const uint8_t* __restrict__ smask,
                                                         const int32_t* __restrict__ par, int32_t* size) {
  const int64_t n = (int64_t)blockIdx.x * IT + threadIdx.x;
  if (n >= nn || __popc((uint32_t)smask[n]) < 2) return;
  atomicAdd(&size[par[n]], 1);
}

// Exact class of the FE edge from node (I,J,K) to (I,J,K) + e_axis against
// the balls of the problem: 0 inside Omega (farther than r from every
// centre), 1 outside (covered by the chords of the balls), 2 cut.
__device__ int edge_class(const ProbDev& d, const double* __restrict__ balls, int I, int J, int K, int axis) {
  const double h = d.h;
  const int ijk[3] = {I, J, K};
  const double p[3] = {(double)I * h, (double)J * h, (double)K * h};
  const double a = p[axis];
  const double bnd = (double)(ijk[axis] + 1) * h;
  const int o1 = axis == 0 ? 1 : 0, o2 = axis == 2 ? 1 : 2;
  bool interior = true;
  for (int i = 0; i < d.nb; ++i) {
    const double* B = balls + 4 * (int64_t)(d.ball_off + i);
    const double r2 = B[3];
    const double dy = p[o1] - B[o1];
    const double dz = p[o2] - B[o2];
    const double dy2 = dy * dy;
    const double dz2 = dz * dz;
    const double p2 = dy2 + dz2;
    double t = B[axis] < a ? a : B[axis];
    t = bnd < t ? bnd : t;
    const double dd = t - B[axis];
    const double dd2 = dd * dd;
    const double dist2 = p2 + dd2;
    if (!(dist2 > r2)) interior = false;
  }
  if (interior) return 0;
  // reach of the union of chords starting at a: the smallest fixed point of
  // x -> max(x, max{hi : lo <= x}) at or above a
  double cur = a;
  for (int it = 0; it <= d.nb; ++it) {
    double best = cur;
    for (int i = 0; i < d.nb; ++i) {
      const double* B = balls + 4 * (int64_t)(d.ball_off + i);
      const double r2 = B[3];
      const double dy = p[o1] - B[o1];
      const double dz = p[o2] - B[o2];
      const double dy2 = dy * dy;
      const double dz2 = dz * dz;
      const double p2 = dy2 + dz2;
      if (!(p2 <= r2)) continue;
      const double half = sqrt(r2 - p2);
      const double lo = B[axis] - half, hi = B[axis] + half;
      if (!(lo > cur) && hi > best) best = hi;
    }
    if (best >= bnd) return 1;
    if (!(best > cur)) break;
    cur = best;
  }
  return 2;
}

// Variant 1: classifies the links of pass-1 edge objects; a cut link marks
// its two DOFs.
__global__ __launch_bounds__(IT) void v1_classify_kernel(BatchDev b, int64_t nn, const double* __restrict__ balls,
                                                         const int32_t* __restrict__ par1,
                                                         const int32_t* __restrict__ size1,
                                                         const uint8_t* __restrict__ face, uint8_t* link,
                                                         uint8_t* cutdof) {
  const int64_t n = (int64_t)blockIdx.x * IT + threadIdx.x;
  if (n >= nn) return;
  const uint32_t L = link[n];
  if (!(L & 7u)) return;
  const int32_t r = par1[n];
  if (size1[r] < 2 || face[r]) return;   // not an edge object
  NodePos q;
  if (!node_pos(b, n, q)) return;
  const ProbDev& d = b.prob[q.p];
  if (d.nb == 0) return;
  const int64_t N1 = q.N + 1;
  uint32_t add = 0;
  for (int axis = 0; axis < 3; ++axis) {
    if (!(L >> axis & 1u)) continue;
    if (edge_class(d, balls, q.I, q.J, q.K, axis) != 2) continue;
    add |= 8u << axis;
    cutdof[n] = 1;
    cutdof[n + axis_step(axis, N1)] = 1;
  }
  if (add) link[n] = (uint8_t)(L | add);
}

// ---- variant 2 (Sect. 4.5) -------------------------------------------------
// Weighting coefficients of the interface node (I, J, K) with S-mask mask:
// W[t] = A^w_xixi / sum_{w' in S} A^w'_xixi for the t-th subdomain w of S
// (eq. alge-weighting), A^w_xixi = sum of kappa_e h K_e[a, a] over the active
// cells e of w around the node in ascending cell order; returns |S|.
__device__ inline int v2_coefficients(const ProbDev& d, uint32_t mask, int I, int J, int K,
                                      const int32_t* __restrict__ cellinfo, const double* __restrict__ kappa,
                                      const double* __restrict__ Kc, const double* __restrict__ kdiag,
                                      double W[8]) {
  const int N = d.N, s = d.s;
  const int bx0 = (I - 1) / s, by0 = (J - 1) / s, bz0 = (K - 1) / s;
  const int card = __popc(mask);
  double D[8];
  for (int t = 0; t < 8; ++t) D[t] = 0.0;
  for (int w = 0; w < 2; ++w)
    for (int v = 0; v < 2; ++v)
      for (int u = 0; u < 2; ++u) {
        const int ci = I - 1 + u, cj = J - 1 + v, ck = K - 1 + w;
        if (ci < 0 || cj < 0 || ck < 0 || ci >= N || cj >= N || ck >= N) continue;
        const int64_t c = d.cell_off + ci + (int64_t)N * (cj + (int64_t)N * ck);
        const int32_t info = cellinfo[c];
        if (info == CELL_INACTIVE) continue;
        const int a = (1 - u) + 2 * (1 - v) + 4 * (1 - w);   // the node's corner in the cell
        const int bit = (ci / s - bx0) + 2 * (cj / s - by0) + 4 * (ck / s - bz0);
        const int t = __popc(mask & ((1u << bit) - 1u));
        const double kd = info == CELL_UNCUT ? kdiag[a] : Kc[(int64_t)info * PACK36 + pack_index(a, a)];
        D[t] += kappa[c] * d.h * kd;
      }
  double tot = 0.0;
  for (int t = 0; t < card; ++t) tot += D[t];
  for (int t = 0; t < card; ++t) W[t] = D[t] / tot;
  return card;
}

// Variant 2: a link of a pass-1 edge object whose two DOFs have different
// weighting coefficients (some component differs by more than V2_TOL) is
// marked cut, so that the second join aggregates only equal neighbours.
__global__ __launch_bounds__(IT) void v2_classify_kernel(BatchDev b, int64_t nn, const int32_t* __restrict__ cellinfo,
                                                         const double* __restrict__ kappa,
                                                         const double* __restrict__ Kc,
                                                         const double* __restrict__ kdiag,
                                                         const uint8_t* __restrict__ smask,
                                                         const int32_t* __restrict__ par1,
                                                         const int32_t* __restrict__ size1,
                                                         const uint8_t* __restrict__ face, uint8_t* link) {
  const int64_t n = (int64_t)blockIdx.x * IT + threadIdx.x;
  if (n >= nn) return;
  const uint32_t L = link[n];
  if (!(L & 7u)) return;
  const int32_t r = par1[n];
  if (size1[r] < 2 || face[r]) return;   // not an edge object
  NodePos q;
  if (!node_pos(b, n, q)) return;
  const ProbDev& d = b.prob[q.p];
  const int64_t N1 = q.N + 1;
  double Wa[8], Wb[8];
  const int card = v2_coefficients(d, smask[n], q.I, q.J, q.K, cellinfo, kappa, Kc, kdiag, Wa);
  uint32_t add = 0;
  for (int axis = 0; axis < 3; ++axis) {
    if (!(L >> axis & 1u)) continue;
    const int64_t m = n + axis_step(axis, N1);
    (void)v2_coefficients(d, smask[m], q.I + (axis == 0), q.J + (axis == 1), q.K + (axis == 2), cellinfo, kappa,
                          Kc, kdiag, Wb);
    bool same = true;
    for (int t = 0; t < card; ++t)
      if (!(fabs(Wa[t] - Wb[t]) <= V2_TOL)) same = false;
    if (!same) add |= 8u << axis;
  }
  if (add) link[n] = (uint8_t)(L | add);
}

// Object kind at a final root r (pass-1 root r1 = par1[r]).
__device__ inline int object_kind(int32_t r, const int32_t* size2, const int32_t* par1, const uint8_t* face) {
  if (size2[r] == 1) return KIND_CORNER;
  return face[par1[r]] ? KIND_FACE : KIND_EDGE;
}

struct ObjectScan {
  BatchDev b;
  const uint8_t* smask;
  const int32_t* par1;
  const int32_t* par2;
  const int32_t* size2;
  const uint8_t* face;
  int objects;
  int32_t* oidx;
  int32_t* ocid;
  int32_t* ocsp;
  Count4* seg;
  __device__ Count4 value(int64_t n) const {
    const int card = __popc((uint32_t)smask[n]);
    if (card < 2 || par2[n] != n) return {0, 0, 0, 0};
    const int sel = (objects == 0 || object_kind((int32_t)n, size2, par1, face) != KIND_FACE) ? 1 : 0;
    return {1, sel, sel ? card : 0, 0};
  }
  __device__ void write(int64_t n, Count4 pre, Count4 v) const {
    record_segment(b.node_off, b.P, n, pre, seg);
    if (!v.x) {
      oidx[n] = -1;
      ocid[n] = -1;
      ocsp[n] = -1;
      return;
    }
    oidx[n] = pre.x;
    ocid[n] = v.y ? pre.y : -1;
    ocsp[n] = v.y ? pre.z : -1;
  }
  __device__ void finish(Count4 tot) const { seg[b.P] = tot; }
};

// ---- per-subdomain passes ------------------------------------------------
struct SubPos {
  int p, N, s, m, Bx, By, Bz;
  int64_t node_off;
};
__device__ inline SubPos sub_pos(const BatchDev& b, const int32_t* sub_off, int w) {
  SubPos q;
  q.p = find_segment(sub_off, b.P, w);
  const ProbDev& d = b.prob[q.p];
  const int wl = w - sub_off[q.p];
  q.N = d.N;
  q.s = d.s;
  q.m = d.m;
  q.Bx = wl % d.m;
  q.By = (wl / d.m) % d.m;
  q.Bz = wl / (d.m * d.m);
  q.node_off = d.node_off;
  return q;
}

// Class of block node e (ascending node order) of subdomain q: 0 none,
// 1 interior DOF, 2 interface DOF of the subdomain; *k = rank of the
// subdomain in S, *n = the global node.
__device__ inline int block_node(const SubPos& q, int e, const uint8_t* __restrict__ smask, int* k, int64_t* n) {
  const int s1 = q.s + 1;
  const int lx = e % s1, ly = (e / s1) % s1, lz = e / (s1 * s1);
  const int I = q.Bx * q.s + lx, J = q.By * q.s + ly, K = q.Bz * q.s + lz;
  const int64_t N1 = q.N + 1;
  *n = q.node_off + I + N1 * (J + N1 * (int64_t)K);
  const uint32_t mask = smask[*n];
  if (!mask) return 0;
  const int r = mask_rank(mask, I, J, K, q.s, q.Bx, q.By, q.Bz);
  if (r < 0) return 0;
  *k = r;
  return __popc(mask) == 1 ? 1 : 2;
}

__global__ __launch_bounds__(IT) void sub_count_kernel(BatchDev b, const int32_t* __restrict__ sub_off,
                                                       const uint8_t* __restrict__ smask,
                                                       const int32_t* __restrict__ ocid, int32_t* nI, int32_t* nG,
                                                       int32_t* nC) {
  const int w = blockIdx.x;
  const SubPos q = sub_pos(b, sub_off, w);
  const int s1 = q.s + 1, nbn = s1 * s1 * s1;
  Count4 acc = {0, 0, 0, 0};
  for (int e = threadIdx.x; e < nbn; e += IT) {
    int k;
    int64_t n;
    const int cls = block_node(q, e, smask, &k, &n);
    if (cls == 1) acc.x++;
    else if (cls == 2) {
      acc.y++;
      if (ocid[n] >= 0) acc.z++;
    }
  }
  Count4 tot;
  (void)block_exclusive(acc, &tot);
  if (threadIdx.x == 0) {
    nI[w] = tot.x;
    nG[w] = tot.y;
    nC[w] = tot.z;
  }
}

// One workgroup per subdomain: ordered compaction of the block's nodes into
// its interior, interface and coarse lists (LDS: interface slot and coarse
// row per block node).
__global__ __launch_bounds__(IT) void sub_fill_kernel(BatchDev b, const int32_t* __restrict__ sub_off,
                                                      IndexWork wk, IndexMaps mp) {
  extern __shared__ int32_t sh[];
  const int w = blockIdx.x;
  const SubPos q = sub_pos(b, sub_off, w);
  const int s1 = q.s + 1, nbn = s1 * s1 * s1;
  int32_t* crow = sh;   // [nbn] local coarse row of a selected object root, else -1
  const int NIp = mp.NIp, NGp = mp.NGp, NCp = mp.NCp;
  Count4 carry = {0, 0, 0, 0};
  for (int e0 = 0; e0 < nbn; e0 += IT) {
    const int e = e0 + threadIdx.x;
    int cls = 0, k = 0;
    int64_t n = -1;
    int cid = -1;
    if (e < nbn) {
      cls = block_node(q, e, wk.smask, &k, &n);
      if (cls == 2) cid = wk.ocid[n];
    }
    const Count4 v = {cls == 1 ? 1 : 0, cls == 2 ? 1 : 0, cid >= 0 ? 1 : 0, 0};
    Count4 tot;
    const Count4 pre = c4add(carry, block_exclusive(v, &tot));
    carry = c4add(carry, tot);
    if (e >= nbn) continue;
    int32_t row = -1;
    if (cls == 1) {
      mp.I_idx[(int64_t)w * NIp + pre.x] = n;
      row = pre.x;
    } else if (cls == 2) {
      const int j = pre.y;
      mp.G_idx[(int64_t)w * NGp + j] = n;
      row = NIp + j;
      const int32_t qi = wk.gif[n];
      const int64_t at = (int64_t)wk.gifp[n] + k;
      mp.if_sub[at] = w;
      mp.if_slot[at] = j;
      if (k == 0) {
        mp.iface_node[qi] = n;
        mp.if_ptr[qi] = wk.gifp[n];
      }
    }
    mp.bloc[(int64_t)w * nbn + e] = row;
    crow[e] = -1;
    if (cid >= 0) {
      const int t = pre.z;
      crow[e] = t;
      mp.C_ids[(int64_t)w * NCp + t] = cid;
      const int64_t at = (int64_t)wk.ocsp[n] + k;
      mp.cs_sub[at] = w;
      mp.cs_row[at] = t;
      if (k == 0) {
        mp.cs_ptr[cid] = wk.ocsp[n];
        mp.coarse_prob[cid] = q.p;
      }
    }
  }
  __syncthreads();
  // local coarse row of each interface row's object (its root is a node of
  // this block: every DOF of an object has the same S)
  const int nI = carry.x, nG = carry.y, nC = carry.z;
  const int64_t N1 = q.N + 1;
  for (int j = threadIdx.x; j < NGp; j += IT) {
    int32_t r = -1;
    if (j < nG) {
      const int64_t n = mp.G_idx[(int64_t)w * NGp + j];
      const int64_t root = wk.par2[n];
      if (wk.ocid[root] >= 0) {
        const int64_t l = root - q.node_off;
        const int lx = (int)(l % N1) - q.Bx * q.s, ly = (int)((l / N1) % N1) - q.By * q.s,
                  lz = (int)(l / (N1 * N1)) - q.Bz * q.s;
        if (lx >= 0 && ly >= 0 && lz >= 0 && lx < s1 && ly < s1 && lz < s1) r = crow[lx + s1 * (ly + s1 * lz)];
      }
    } else {
      mp.G_idx[(int64_t)w * NGp + j] = -1;
    }
    mp.G_obj[(int64_t)w * NGp + j] = r;
  }
  for (int i = nI + threadIdx.x; i < NIp; i += IT) mp.I_idx[(int64_t)w * NIp + i] = -1;
  for (int t = nC + threadIdx.x; t < NCp; t += IT) mp.C_ids[(int64_t)w * NCp + t] = -1;
  if (threadIdx.x == 0) {
    mp.sub_prob[w] = q.p;
    mp.sub_blk[w] = w - sub_off[q.p];
    if (w == 0) {
      mp.if_ptr[wk.seg_nodes[b.P].y] = wk.seg_nodes[b.P].z;
      mp.cs_ptr[wk.seg_obj[b.P].y] = wk.seg_obj[b.P].z;
    }
  }
}

inline unsigned grid_of(int64_t n) { return (unsigned)((n + IT - 1) / IT); }

}  // namespace

int64_t index_scan_blocks(int64_t n) { return (n + IBS - 1) / IBS + 1; }

void launch_index_cells(hipStream_t st, const BatchDev& b, int64_t n_cells_total, const int32_t* count,
                        int store_cut, const IndexWork& w, int32_t* cellinfo, int64_t* cut_cells) {
  CellScan f{b, count, store_cut, cellinfo, cut_cells, w.seg_cells};
  run_scan(st, f, n_cells_total, w.bsum);
}

void launch_index_nodes(hipStream_t st, const BatchDev& b, int64_t n_cells_total, int64_t nn, int ns,
                        const int32_t* sub_off, const int32_t* count, const double* balls, int variant, int objects,
                        const V2Inputs& v2, const IndexWork& w, uint8_t* dofmask, int64_t* dof_node, int32_t* nI,
                        int32_t* nG, int32_t* nC) {
  const dim3 gn(grid_of(nn)), gc(grid_of(n_cells_total)), blk(IT);
  // DOFs and subdomain sets
  hipLaunchKernelGGL(smask_kernel, gn, blk, 0, st, b, nn, count, w.smask, dofmask);
  NodeScan nsf{b, w.smask, dof_node, w.gif, w.gifp, w.seg_nodes};
  run_scan(st, nsf, nn, w.bsum);
  hipLaunchKernelGGL(zero_u8_kernel, gn, blk, 0, st, nn, w.ground, w.face, w.cutdof);
  hipLaunchKernelGGL(zero_i32_kernel, gn, blk, 0, st, nn, w.size1, w.size2);
  hipLaunchKernelGGL(zero_i32_kernel, dim3(grid_of(b.P)), blk, 0, st, (int64_t)b.P, w.floating, (int32_t*)nullptr);
  // floating components: join, compress, mark grounded roots, check
  hipLaunchKernelGGL(float_local_kernel, gn, blk, 0, st, b, nn, count, w.smask, w.par0);
  hipLaunchKernelGGL(float_cross_kernel, gn, blk, 0, st, b, nn, count, w.smask, w.par0);
  hipLaunchKernelGGL(compress_kernel, gn, blk, 0, st, nn, w.par0);
  hipLaunchKernelGGL(float_ground_kernel, gc, blk, 0, st, b, n_cells_total, count, w.smask, w.par0, w.ground);
  hipLaunchKernelGGL(float_check_kernel, gn, blk, 0, st, b, nn, w.smask, w.par0, w.ground, w.floating);
  // objects before the variant-1 split
  hipLaunchKernelGGL(link_kernel, gn, blk, 0, st, b, nn, count, w.smask, w.link);
  hipLaunchKernelGGL(iota_kernel, gn, blk, 0, st, nn, w.par1);
  hipLaunchKernelGGL(link_join_kernel, gn, blk, 0, st, b, nn, w.link, (const uint8_t*)nullptr, w.par1);
  hipLaunchKernelGGL(compress_kernel, gn, blk, 0, st, nn, w.par1);
  hipLaunchKernelGGL(face_kernel, gc, blk, 0, st, b, n_cells_total, count, w.smask, w.par1, w.face);
  hipLaunchKernelGGL(object_size_kernel, gn, blk, 0, st, nn, w.smask, w.par1, w.size1);
  // variant 1: cut FE edges of edge objects; variant 2 (stiffness weights
  // only): links between DOFs of unequal weighting coefficients; then the
  // final objects (without a split, the same links join the same sets)
  if (variant == 1)
    hipLaunchKernelGGL(v1_classify_kernel, gn, blk, 0, st, b, nn, balls, w.par1, w.size1, w.face, w.link,
                       w.cutdof);
  if (variant == 2 && v2.stiffness)
    hipLaunchKernelGGL(v2_classify_kernel, gn, blk, 0, st, b, nn, v2.cellinfo, v2.kappa, v2.Kc, v2.kdiag, w.smask,
                       w.par1, w.size1, w.face, w.link);
  hipLaunchKernelGGL(iota_kernel, gn, blk, 0, st, nn, w.par2);
  hipLaunchKernelGGL(link_join_kernel, gn, blk, 0, st, b, nn, w.link, (const uint8_t*)w.cutdof, w.par2);
  hipLaunchKernelGGL(compress_kernel, gn, blk, 0, st, nn, w.par2);
  hipLaunchKernelGGL(object_size_kernel, gn, blk, 0, st, nn, w.smask, w.par2, w.size2);
  // object and coarse numbering
  ObjectScan osf{b, w.smask, w.par1, w.par2, w.size2, w.face, objects, w.oidx, w.ocid, w.ocsp, w.seg_obj};
  run_scan(st, osf, nn, w.bsum);
  if (ns > 0)
    hipLaunchKernelGGL(sub_count_kernel, dim3(ns), blk, 0, st, b, sub_off, w.smask, w.ocid, nI, nG, nC);
}

void launch_index_fill(hipStream_t st, const BatchDev& b, int ns, int s, const int32_t* sub_off,
                       const IndexWork& w, const IndexMaps& m) {
  if (ns <= 0) return;
  const size_t sh = (size_t)(s + 1) * (s + 1) * (s + 1) * sizeof(int32_t);
  hipLaunchKernelGGL(sub_fill_kernel, dim3(ns), dim3(IT), sh, st, b, sub_off, w, m);
}

}  // namespace cutbddc
