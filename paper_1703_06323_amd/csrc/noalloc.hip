// Allocation-free batched SPD inverse (cb_dense_spd_inverse_noalloc).
//
// The same computation as cb_dense_spd_inverse (blocked Cholesky on MFMA,
// triangular inverse Y = L^-1, A^-1 = Y^T Y; the building block of the local
// and coarse factorisations, Sect. 3.3-3.4), for callers that may not
// allocate device memory.  Every intermediate lives in one file-scope device
// array, `scratch`, of NOALLOC_SCRATCH_BYTES per GPU; the host addresses it
// only through the pointer that hipGetSymbolAddress returns for the current
// device (kept per device after the first call on it).  The GEMMs use tile
// shapes already chosen by the autotuner, or the default shape, but never
// tune here (tuning allocates its test operands).
//
// Calls on one GPU share its array, and each call leaves its contents
// behind: every region a call reads is written earlier in the same call.
// Calls that overlap in time on one GPU (several host threads) race on the
// array; the caller must serialise them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "common.h"
#include "cutbddc.h"
#include "dense.h"

namespace cutbddc {
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return report_error(CB_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return report_error(CB_ERR_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return report_error(CB_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CB_OK;
}

// out[b] (np x np, type T) = in[b] (n x n, FP64) padded with the identity.
template <typename T>
__global__ __launch_bounds__(256) void pad_convert_kernel(const double* __restrict__ in, int n, int np,
                                                          T* __restrict__ out) {
  const int64_t b = blockIdx.y, i = blockIdx.x;
  for (int j = threadIdx.x; j < np; j += 256) {
    const double v = (i < n && j < n) ? in[(b * n + i) * n + j] : (i == j ? 1.0 : 0.0);
    out[(b * np + i) * np + j] = (T)v;
  }
}

// out[b] (n x n) = the leading n x n block of in[b] (np x np).
__global__ __launch_bounds__(256) void compact_kernel(const double* __restrict__ in, int n, int np,
                                                      double* __restrict__ out) {
  const int64_t b = blockIdx.y, i = blockIdx.x;
  for (int j = threadIdx.x; j < n; j += 256) out[(b * n + i) * n + j] = in[(b * np + i) * np + j];
}

__global__ __launch_bounds__(256) void zero_int_kernel(int* __restrict__ a, int n) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) a[i] = 0;
}

// *first = smallest b with info[b] != 0, or -1 (one workgroup).
__global__ __launch_bounds__(256) void first_failure_kernel(const int* __restrict__ info, int batch,
                                                            int* __restrict__ first) {
  __shared__ int best;
  if (threadIdx.x == 0) best = batch;
  __syncthreads();
  for (int b = threadIdx.x; b < batch; b += 256)
    if (info[b] != 0) atomicMin(&best, b);
  __syncthreads();
  if (threadIdx.x == 0) *first = best < batch ? best : -1;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
inline int round_up_to(int x, int q) { return ((x + q - 1) / q) * q; }

// Scratch regions of one call, in bytes from the start of the array.
struct Layout {
  size_t stage, A, L, Y, P, out, ones, info, first, total;
};

Layout layout(int n, int np, int batch, size_t elem) {
  const size_t nn = (size_t)np * np;
  const size_t sL = (size_t)diag_blocks(np, 0) * DB * DB;
  Layout l{};
  size_t at = 0;
  l.stage = at, at += align256((size_t)batch * n * n * sizeof(double));
  l.A = at, at += align256((size_t)batch * nn * elem);
  l.L = at, at += align256((size_t)batch * sL * elem);
  l.Y = at, at += align256((size_t)batch * nn * elem);
  l.P = at, at += align256((size_t)batch * nn * elem);
  l.out = at, at += align256((size_t)batch * nn * sizeof(double));
  l.ones = at, at += align256((size_t)np * sizeof(double));
  l.info = at, at += align256((size_t)batch * sizeof(int));
  l.first = at, at += align256(sizeof(int));
  l.total = at;
  return l;
}

template <typename T>
int spd_inverse_in_scratch(unsigned char* base, const Layout& l, int n, int np, int batch, const double* A,
                           double* Ainv) {
  hipStream_t st = nullptr;   // the default stream, as the allocating entry point
  const int64_t nn = (int64_t)np * np;
  const int64_t sL = (int64_t)diag_blocks(np, 0) * DB * DB;
  double* stage = reinterpret_cast<double*>(base + l.stage);
  T* dA = reinterpret_cast<T*>(base + l.A);
  T* dL = reinterpret_cast<T*>(base + l.L);
  T* dY = reinterpret_cast<T*>(base + l.Y);
  T* dP = reinterpret_cast<T*>(base + l.P);
  double* dOut = reinterpret_cast<double*>(base + l.out);
  double* ones = reinterpret_cast<double*>(base + l.ones);
  int* info = reinterpret_cast<int*>(base + l.info);
  int* first = reinterpret_cast<int*>(base + l.first);
  auto dev_err = [](hipError_t e, const char* what) {
    return report_error(e == hipErrorOutOfMemory ? CB_ERR_OOM : CB_ERR_DEVICE,
                        std::string(what) + ": " + hipGetErrorString(e));
  };
  hipError_t e = hipMemcpy(stage, A, (size_t)batch * n * n * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return dev_err(e, "hipMemcpy of the input");
  hipLaunchKernelGGL(pad_convert_kernel<T>, dim3(np, batch), dim3(256), 0, st, stage, n, np, dA);
  launch_fill(st, np, 1.0, ones);
  hipLaunchKernelGGL(zero_int_kernel, dim3((batch + 255) / 256), dim3(256), 0, st, info, batch);
  gemm_set_thread_tuning(false);
  cholesky<T>(st, dA, np, nn, np, 0, batch, dL, sL, info);
  tri_inverse<T>(st, dA, np, nn, 0, np, 0, batch, dL, sL, dY, np, nn);
  gemm<T>(st, 1, 0, np, np, np, T(1), dY, np, nn, dY, np, nn, T(0), dP, np, nn, batch, GEMM_LOWER | GEMM_KFROM_DIAG);
  gemm_set_thread_tuning(true);
  symmetrize_scale<T, double>(st, dP, np, nn, dOut, np, nn, ones, 0, np, batch);
  hipLaunchKernelGGL(compact_kernel, dim3(n, batch), dim3(256), 0, st, dOut, n, np, stage);
  hipLaunchKernelGGL(first_failure_kernel, dim3(1), dim3(256), 0, st, info, batch, first);
  e = hipGetLastError();
  if (e != hipSuccess) return dev_err(e, "kernel launch");
  e = hipMemcpy(Ainv, stage, (size_t)batch * n * n * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return dev_err(e, "hipMemcpy of the result");
  int bad = -1;
  e = hipMemcpy(&bad, first, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return dev_err(e, "hipMemcpy of the status");
  if (bad >= 0) return report_error(CB_ERR_NOT_SPD, "Cholesky breakdown in matrix " + std::to_string(bad));
  return CB_OK;
}

}  // namespace
}  // namespace cutbddc

extern "C" int cb_dense_spd_inverse_noalloc(int32_t n, int32_t batch, int32_t precision, const double* A,
                                            double* Ainv) {
  using namespace cutbddc;
  if (n < 1 || batch < 1 || !A || !Ainv || precision < 0 || precision > 1)
    return report_error(CB_ERR_ARG, "invalid argument");
  const int np = round_up_to(n, CHOL_BLOCK);
  const Layout l = layout(n, np, batch, precision == CB_FP32_LOCAL ? sizeof(float) : sizeof(double));
  if (l.total > NOALLOC_SCRATCH_BYTES)
    return report_error(CB_ERR_ARG, "n = " + std::to_string(n) + ", batch = " + std::to_string(batch) + " needs " +
                                        std::to_string(l.total) + " bytes of scratch (limit " +
                                        std::to_string(NOALLOC_SCRATCH_BYTES) + ")");
  void* p = nullptr;
  const int rc = scratch_address(&p);
  if (rc != CB_OK) return rc;
  unsigned char* base = static_cast<unsigned char*>(p);
  return precision == CB_FP32_LOCAL ? spd_inverse_in_scratch<float>(base, l, n, np, batch, A, Ainv)
                                    : spd_inverse_in_scratch<double>(base, l, n, np, batch, A, Ainv);
}
