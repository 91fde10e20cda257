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

// ---- K-cycle: one block of kRed threads sums each dot product ----
constexpr int kRed = 1024;

template <int NV>
__device__ __forceinline__ void red_block(double (&v)[NV]) {
  __shared__ double red[kRed / 64][NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    v[k] = s;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[w][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = red[0][k];
      for (int ww = 1; ww < kRed / 64; ++ww) s += red[ww][k];
      v[k] = s;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kRed) void k_kdot1(const T* __restrict__ v1, const T* __restrict__ rc,
                                                const T* __restrict__ w1, int n, KScal* __restrict__ S,
                                                const int* __restrict__ skip) {
  if (skip && *skip) return;
  double a[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += kRed) {
    const double v = v1[i], r = rc[i];
    a[0] += v * r;
    a[1] += v * static_cast<double>(w1[i]);
    a[2] += r * r;
  }
  red_block<3>(a);
  if (threadIdx.x == 0) {
    S->rho1 = a[0];
    S->a1 = a[1];
    S->rr = a[2];
  }
}

template <typename T>
__global__ __launch_bounds__(kRed) void k_kres(const T* __restrict__ rc, const T* __restrict__ w1,
                                               T* __restrict__ r2, int n, KScal* __restrict__ S, double t2,
                                               const int* __restrict__ skip) {
  if (skip && *skip) {
    if (threadIdx.x == 0) S->flag = 1;
    return;
  }
  const double c = S->rho1 / S->a1;
  double a[1] = {0.0};
  for (int i = threadIdx.x; i < n; i += kRed) {
    const T r = static_cast<T>(static_cast<double>(rc[i]) - c * static_cast<double>(w1[i]));
    r2[i] = r;
    a[0] += static_cast<double>(r) * static_cast<double>(r);
  }
  red_block<1>(a);
  if (threadIdx.x == 0) S->flag = a[0] <= t2 * S->rr ? 1 : 0;
}

template <typename T>
__global__ __launch_bounds__(kRed) void k_kdot2(const T* __restrict__ v2, const T* __restrict__ w1,
                                                const T* __restrict__ w2, const T* __restrict__ r2, int n,
                                                KScal* __restrict__ S) {
  if (S->flag) return;
  double a[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += kRed) {
    const double v = v2[i];
    a[0] += v * static_cast<double>(w1[i]);
    a[1] += v * static_cast<double>(w2[i]);
    a[2] += v * static_cast<double>(r2[i]);
  }
  red_block<3>(a);
  if (threadIdx.x == 0) {
    S->g = a[0];
    S->b = a[1];
    S->rho2 = a[2];
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_kcomb(const T* __restrict__ v1, const T* __restrict__ v2,
                                                    T* __restrict__ ec, int n, const KScal* __restrict__ S,
                                                    const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  if (S->flag) {
    ec[i] = static_cast<T>((S->rho1 / S->a1) * static_cast<double>(v1[i]));
  } else {
    const double a2 = S->b - S->g * S->g / S->a1;
    const double c1 = S->rho1 / S->a1 - S->g * S->rho2 / (S->a1 * a2), c2 = S->rho2 / a2;
    ec[i] = static_cast<T>(c1 * static_cast<double>(v1[i]) + c2 * static_cast<double>(v2[i]));
  }
}

}  // namespace

hipError_t amg_kdot1(bool fp32, const void* v1, const void* rc, const void* w1, int n, KScal* S, const int* skip,
                     hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_kdot1<float>, dim3(1), dim3(kRed), 0, s, static_cast<const float*>(v1),
                       static_cast<const float*>(rc), static_cast<const float*>(w1), n, S, skip);
  else
    hipLaunchKernelGGL(k_kdot1<double>, dim3(1), dim3(kRed), 0, s, static_cast<const double*>(v1),
                       static_cast<const double*>(rc), static_cast<const double*>(w1), n, S, skip);
  return hipGetLastError();
}

hipError_t amg_kres(bool fp32, const void* rc, const void* w1, void* r2, int n, KScal* S, double t2, const int* skip,
                    hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_kres<float>, dim3(1), dim3(kRed), 0, s, static_cast<const float*>(rc),
                       static_cast<const float*>(w1), static_cast<float*>(r2), n, S, t2, skip);
  else
    hipLaunchKernelGGL(k_kres<double>, dim3(1), dim3(kRed), 0, s, static_cast<const double*>(rc),
                       static_cast<const double*>(w1), static_cast<double*>(r2), n, S, t2, skip);
  return hipGetLastError();
}

hipError_t amg_kdot2(bool fp32, const void* v2, const void* w1, const void* w2, const void* r2, int n, KScal* S,
                     hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_kdot2<float>, dim3(1), dim3(kRed), 0, s, static_cast<const float*>(v2),
                       static_cast<const float*>(w1), static_cast<const float*>(w2), static_cast<const float*>(r2),
                       n, S);
  else
    hipLaunchKernelGGL(k_kdot2<double>, dim3(1), dim3(kRed), 0, s, static_cast<const double*>(v2),
                       static_cast<const double*>(w1), static_cast<const double*>(w2),
                       static_cast<const double*>(r2), n, S);
  return hipGetLastError();
}

hipError_t amg_kcomb(bool fp32, const void* v1, const void* v2, void* ec, int n, const KScal* S, const int* skip,
                     hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_kcomb<float>, dim3(blocks_for(n)), dim3(kThreads), 0, s, static_cast<const float*>(v1),
                       static_cast<const float*>(v2), static_cast<float*>(ec), n, S, skip);
  else
    hipLaunchKernelGGL(k_kcomb<double>, dim3(blocks_for(n)), dim3(kThreads), 0, s, static_cast<const double*>(v1),
                       static_cast<const double*>(v2), static_cast<double*>(ec), n, S, skip);
  return hipGetLastError();
}

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
