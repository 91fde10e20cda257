// Device kernels of the aggregation AMG cycle (Sec. 3, pMG-AMG): sparse
// operator products on the algebraic levels, aggregate restriction and
// prolongation, the coarsest level's dense inverse, and two vector updates.
#include <hip/hip_runtime.h>

#include "amg.hpp"

namespace ipdg {
namespace {

constexpr int kThreads = 256;

int blocks_for(size_t n) { return n == 0 ? 1 : int((n + kThreads - 1) / kThreads); }

// one row per lane; columns ascending, summed in order
template <typename T>
__global__ __launch_bounds__(kThreads) void k_spmv(const int* __restrict__ ptr, const int* __restrict__ col,
                                                   const T* __restrict__ val, const T* __restrict__ x,
                                                   T* __restrict__ y, int n, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  T s = T(0);
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) s += val[k] * x[col[k]];
  y[i] = s;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_restrict(const int* __restrict__ mptr, const int* __restrict__ mem,
                                                       const T* __restrict__ f, const T* __restrict__ t,
                                                       T* __restrict__ rc, int nc, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= nc) return;
  T s = T(0);
  for (int k = mptr[i]; k < mptr[i + 1]; ++k) {
    const int j = mem[k];
    s += t ? f[j] - t[j] : f[j];
  }
  rc[i] = s;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_prolong(const int* __restrict__ agg, const T* __restrict__ zc,
                                                      T* __restrict__ z, int n, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int j = blockIdx.x * kThreads + threadIdx.x;
  if (j < n) z[j] += zc[agg[j]];
}

// one wave per row: lanes stride the row, then a butterfly sum
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dense(const T* __restrict__ inv, const T* __restrict__ f,
                                                    T* __restrict__ z, int n, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (i >= n) return;
  const T* row = inv + (size_t)i * n;
  T s = T(0);
  for (int j = lane; j < n; j += 64) s += row[j] * f[j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) z[i] = s;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_sub(const T* __restrict__ f, const T* __restrict__ t,
                                                  T* __restrict__ r, size_t n, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x;
  if (i < n) r[i] = f[i] - t[i];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_add(T* __restrict__ x, const T* __restrict__ y, size_t n,
                                                  const int* __restrict__ skip) {
  if (skip && *skip) return;
  const size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x;
  if (i < n) x[i] += y[i];
}

}  // namespace

hipError_t amg_spmv(bool fp32, const int* ptr, const int* col, const void* val, const void* x, void* y, int n,
                    const int* skip, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_spmv<float>, dim3(blocks_for(n)), dim3(kThreads), 0, s, ptr, col,
                       static_cast<const float*>(val), static_cast<const float*>(x), static_cast<float*>(y), n, skip);
  else
    hipLaunchKernelGGL(k_spmv<double>, dim3(blocks_for(n)), dim3(kThreads), 0, s, ptr, col,
                       static_cast<const double*>(val), static_cast<const double*>(x), static_cast<double*>(y), n,
                       skip);
  return hipGetLastError();
}

hipError_t amg_restrict(bool fp32, const int* mptr, const int* mem, const void* f, const void* t, void* rc, int nc,
                        const int* skip, hipStream_t s) {
  if (nc <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_restrict<float>, dim3(blocks_for(nc)), dim3(kThreads), 0, s, mptr, mem,
                       static_cast<const float*>(f), static_cast<const float*>(t), static_cast<float*>(rc), nc, skip);
  else
    hipLaunchKernelGGL(k_restrict<double>, dim3(blocks_for(nc)), dim3(kThreads), 0, s, mptr, mem,
                       static_cast<const double*>(f), static_cast<const double*>(t), static_cast<double*>(rc), nc,
                       skip);
  return hipGetLastError();
}

hipError_t amg_prolong(bool fp32, const int* agg, const void* zc, void* z, int n, const int* skip, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_prolong<float>, dim3(blocks_for(n)), dim3(kThreads), 0, s, agg,
                       static_cast<const float*>(zc), static_cast<float*>(z), n, skip);
  else
    hipLaunchKernelGGL(k_prolong<double>, dim3(blocks_for(n)), dim3(kThreads), 0, s, agg,
                       static_cast<const double*>(zc), static_cast<double*>(z), n, skip);
  return hipGetLastError();
}

hipError_t amg_dense(bool fp32, const void* inv, const void* f, void* z, int n, const int* skip, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int rows_per_block = kThreads / 64;
  const dim3 g((n + rows_per_block - 1) / rows_per_block);
  if (fp32)
    hipLaunchKernelGGL(k_dense<float>, g, dim3(kThreads), 0, s, static_cast<const float*>(inv),
                       static_cast<const float*>(f), static_cast<float*>(z), n, skip);
  else
    hipLaunchKernelGGL(k_dense<double>, g, dim3(kThreads), 0, s, static_cast<const double*>(inv),
                       static_cast<const double*>(f), static_cast<double*>(z), n, skip);
  return hipGetLastError();
}

hipError_t amg_sub(bool fp32, const void* f, const void* t, void* r, size_t n, const int* skip, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_sub<float>, dim3(blocks_for(n)), dim3(kThreads), 0, s, static_cast<const float*>(f),
                       static_cast<const float*>(t), static_cast<float*>(r), n, skip);
  else
    hipLaunchKernelGGL(k_sub<double>, dim3(blocks_for(n)), dim3(kThreads), 0, s, static_cast<const double*>(f),
                       static_cast<const double*>(t), static_cast<double*>(r), n, skip);
  return hipGetLastError();
}

hipError_t amg_add(bool fp32, void* x, const void* y, size_t n, const int* skip, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_add<float>, dim3(blocks_for(n)), dim3(kThreads), 0, s, static_cast<float*>(x),
                       static_cast<const float*>(y), n, skip);
  else
    hipLaunchKernelGGL(k_add<double>, dim3(blocks_for(n)), dim3(kThreads), 0, s, static_cast<double*>(x),
                       static_cast<const double*>(y), n, skip);
  return hipGetLastError();
}

}  // namespace ipdg
