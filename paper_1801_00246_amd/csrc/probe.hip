// Empirical roofs of the device (the paper's Sec. 5.1 bounds the kernels by a
// measured device-to-device copy rate rather than the vendor figure): a
// vectorised copy kernel and a multiply-add throughput kernel, timed with HIP
// events on the caller's stream.
#include <hip/hip_runtime.h>

#include <vector>

#include "handle.hpp"
#include "probe.hpp"

namespace ipdg {
namespace {

constexpr int kProbeBlock = 256;

// dst = src, 16 bytes per lane and access, grid-stride
__global__ __launch_bounds__(kProbeBlock) void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                        size_t n16) {
  for (size_t i = blockIdx.x * (size_t)kProbeBlock + threadIdx.x; i < n16; i += (size_t)gridDim.x * kProbeBlock)
    dst[i] = src[i];
}

// kAcc independent multiply-add chains per lane, `iters` rounds, with
// wave-uniform (scalar) multipliers as the operator kernels use them; the
// result is stored so that nothing is removed.
template <typename T, int kAcc>
__global__ __launch_bounds__(kProbeBlock) void k_fma(const T* __restrict__ coef, T* __restrict__ out, int iters) {
  T a[kAcc];
#pragma unroll
  for (int k = 0; k < kAcc; ++k) a[k] = T(threadIdx.x + k);
  const T c0 = coef[0], c1 = coef[1];
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kAcc; ++k) a[k] = a[k] * c0 + c1;
  }
  T s = T(0);
#pragma unroll
  for (int k = 0; k < kAcc; ++k) s += a[k];
  out[blockIdx.x * (size_t)kProbeBlock + threadIdx.x] = s;
}

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  Events() {
    IPDG_HIP(hipEventCreate(&a));
    IPDG_HIP(hipEventCreate(&b));
  }
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  double ms() const {
    float t = 0.0f;
    IPDG_HIP(hipEventElapsedTime(&t, a, b));
    return double(t);
  }
};

}  // namespace

double probe_copy_gbs(size_t bytes, int sets, int reps, hipStream_t s) {
  const size_t n16 = bytes / 16;
  if (n16 == 0 || sets < 1 || reps < 1) throw Error(IPDG_EINVAL, "copy probe: empty size, sets or reps");
  std::vector<DevBuf> src, dst;
  for (int k = 0; k < sets; ++k) {
    src.emplace_back(n16 * 16);
    dst.emplace_back(n16 * 16);
    IPDG_HIP(hipMemsetAsync(src.back().get(), 0, n16 * 16, s));
  }
  int dev = 0, cus = 0;
  IPDG_HIP(hipGetDevice(&dev));
  IPDG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const size_t want = (n16 + kProbeBlock - 1) / kProbeBlock;
  const int grid = (int)std::min<size_t>(want, (size_t)cus * 32);
  auto launch = [&](int k) {
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(kProbeBlock), 0, s, src[k].as<const uint4>(),
                       dst[k].as<uint4>(), n16);
  };
  for (int k = 0; k < sets; ++k) launch(k);
  IPDG_HIP(hipGetLastError());
  Events ev;
  IPDG_HIP(hipEventRecord(ev.a, s));
  for (int r = 0; r < reps; ++r) launch(r % sets);
  IPDG_HIP(hipEventRecord(ev.b, s));
  IPDG_HIP(hipEventSynchronize(ev.b));
  IPDG_HIP(hipGetLastError());
  return 2.0 * double(n16 * 16) * reps / (ev.ms() * 1e-3) / 1e9;
}

double probe_fma_tflops(bool fp32, int reps, hipStream_t s) {
  if (reps < 1) throw Error(IPDG_EINVAL, "fma probe: reps < 1");
  constexpr int kAcc = 16;
  const int iters = 4096;
  int dev = 0, cus = 0;
  IPDG_HIP(hipGetDevice(&dev));
  IPDG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int grid = cus * 32;   // 8 blocks of 4 waves per CU: every SIMD fully occupied
  const size_t w = fp32 ? 4 : 8;
  DevBuf coef(2 * w), out((size_t)grid * kProbeBlock * w);
  if (fp32) {
    const float c[2] = {0.999f, 1e-3f};
    IPDG_HIP(hipMemcpyAsync(coef.get(), c, sizeof(c), hipMemcpyHostToDevice, s));
  } else {
    const double c[2] = {0.999, 1e-3};
    IPDG_HIP(hipMemcpyAsync(coef.get(), c, sizeof(c), hipMemcpyHostToDevice, s));
  }
  auto launch = [&]() {
    if (fp32)
      hipLaunchKernelGGL((k_fma<float, kAcc>), dim3(grid), dim3(kProbeBlock), 0, s, coef.as<const float>(),
                         out.as<float>(), iters);
    else
      hipLaunchKernelGGL((k_fma<double, kAcc>), dim3(grid), dim3(kProbeBlock), 0, s, coef.as<const double>(),
                         out.as<double>(), iters);
  };
  launch();
  IPDG_HIP(hipGetLastError());
  Events ev;
  IPDG_HIP(hipEventRecord(ev.a, s));
  for (int r = 0; r < reps; ++r) launch();
  IPDG_HIP(hipEventRecord(ev.b, s));
  IPDG_HIP(hipEventSynchronize(ev.b));
  IPDG_HIP(hipGetLastError());
  const double flops = 2.0 * double(grid) * kProbeBlock * kAcc * iters * reps;
  return flops / (ev.ms() * 1e-3) / 1e12;
}

}  // namespace ipdg
