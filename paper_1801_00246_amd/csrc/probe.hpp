// Empirical roofs of the device: copy bandwidth and multiply-add throughput.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace ipdg {

// GB/s of read + write traffic of a 16-byte-per-lane copy kernel copying
// `bytes`, rotating over `sets` source/destination pairs for `reps` copies.
double probe_copy_gbs(size_t bytes, int sets, int reps, hipStream_t s);
// TFLOP/s (2 per multiply-add) of independent multiply-add chains with
// wave-uniform multipliers, every SIMD occupied.
double probe_fma_tflops(bool fp32, int reps, hipStream_t s);

}  // namespace ipdg
