// Runtime-degree dispatch to the per-degree kernel instantiations.
#include "kernels.hpp"

#include <atomic>
#include <cstdlib>
#include <mutex>

namespace ipdg {

namespace {
// Operator kernel variant per precision (FP64, FP32) and degree; bits:
// 1 = LDS-staged inputs/outputs, 2 = raised occupancy (degrees <= 5).
// Defaults from measured sweeps of the 524,288-element operator workload.
std::atomic<int> g_variant[2][9] = {{0, 0, 0, 4, 4, 4, 4, 4, 4}, {0, 2, 2, 4, 4, 4, 4, 4, 4}};
std::once_flag env_once;

// The environment override, applied once per process before any variant is
// read or set (thread-safe).
void read_env() {
  std::call_once(env_once, [] {
    if (const char* v = std::getenv("IPDG_AX_VARIANT")) {
      const int k = std::atoi(v);
      for (int n = 1; n <= 8; ++n) {
        const int kn = ax_variant_exists(n, k) ? k : (k & 1);
        g_variant[0][n] = kn;
        g_variant[1][n] = kn;
      }
    }
  });
}
}  // namespace

int ax_variant(int N, bool fp32) {
  read_env();
  if (N < 1 || N > 8) return 0;
  return g_variant[fp32 ? 1 : 0][N].load();
}

void set_ax_variant(int N, bool fp32, int v) {
  read_env();   // the environment override is read before any explicit choice
  if (ax_variant_exists(N, v)) g_variant[fp32 ? 1 : 0][N] = v;
}

bool ax_variant_exists(int N, int v) {
  if (N < 1 || N > 8) return false;
  if (v == kAxCoop) return true;
  return v >= 0 && v < (N <= 5 ? 4 : 2);
}

int ax_partials(int N, bool fp32, int K) {
  if (ax_variant(N, fp32) == kAxCoop) {
    int per;
    return xcd_grid((K + kCoopTileElems - 1) / kCoopTileElems, per);
  }
  return elem_grid(K);
}

#define IPDG_SWITCH(N_, CALL)      \
  switch (N_) {                    \
    case 1: return CALL(1);        \
    case 2: return CALL(2);        \
    case 3: return CALL(3);        \
    case 4: return CALL(4);        \
    case 5: return CALL(5);        \
    case 6: return CALL(6);        \
    case 7: return CALL(7);        \
    case 8: return CALL(8);        \
    default: return hipErrorInvalidValue; \
  }

hipError_t ax(int N, Kind kind, const ElemArgs& a, hipStream_t s) {
#define C(n) launch_ax<n>(kind, a, s)
  IPDG_SWITCH(N, C)
#undef C
}
bool ax_batch_variant(int v) { return v == 0 || v == 2 || v == kAxCoop; }
hipError_t ax_batch(int N, Kind kind, bool kap, int variant, const ElemArgs* tab, const BlockRef* map, int nblocks,
                    hipStream_t s) {
#define C(n) launch_ax_batch<n>(kind, kap, variant, tab, map, nblocks, s)
  IPDG_SWITCH(N, C)
#undef C
}
hipError_t minv_batch(int N, Kind kind, const ElemArgs* tab, const BlockRef* map, int nblocks, hipStream_t s) {
#define C(n) launch_minv_batch<n>(kind, tab, map, nblocks, s)
  IPDG_SWITCH(N, C)
#undef C
}
hipError_t transfer_batch(int Nf, int Nc, bool restrict_op, Kind kind, const TransferArgs* tab, const BlockRef* map,
                          int nblocks, hipStream_t s) {
#define C(n) launch_transfer_batch<n>(Nc, restrict_op, kind, tab, map, nblocks, s)
  IPDG_SWITCH(Nf, C)
#undef C
}
hipError_t diag(int N, Kind kind, const ElemArgs& a, hipStream_t s) {
#define C(n) launch_diag<n>(kind, a, s)
  IPDG_SWITCH(N, C)
#undef C
}
hipError_t mass(int N, Kind kind, const ElemArgs& a, hipStream_t s) {
#define C(n) launch_mass<n>(kind, a, s)
  IPDG_SWITCH(N, C)
#undef C
}
hipError_t minv(int N, Kind kind, const ElemArgs& a, hipStream_t s) {
#define C(n) launch_minv<n>(kind, a, s)
  IPDG_SWITCH(N, C)
#undef C
}
hipError_t kgrad(int N, const KgradArgs& a, hipStream_t s) {
#define C(n) launch_kgrad<n>(a, s)
  IPDG_SWITCH(N, C)
#undef C
}
hipError_t restrict_(int Nf, int Nc, Kind kind, const TransferArgs& a, hipStream_t s) {
#define C(n) launch_restrict<n>(Nc, kind, a, s)
  IPDG_SWITCH(Nf, C)
#undef C
}
hipError_t prolong(int Nf, int Nc, Kind kind, const TransferArgs& a, hipStream_t s) {
#define C(n) launch_prolong<n>(Nc, kind, a, s)
  IPDG_SWITCH(Nf, C)
#undef C
}

hipError_t coarse_step(int N, Kind kind, const CoarseStepArgs& a, hipStream_t s) {
#define C(n) launch_coarse_step<n>(kind, a, s)
  IPDG_SWITCH(N, C)
#undef C
}

hipError_t coarse_batch(int N, Kind kind, const CoarseBatchArgs& a, int it, hipStream_t s) {
#define C(n) launch_coarse_batch<n>(kind, a, it, s)
  IPDG_SWITCH(N, C)
#undef C
}

hipError_t coarse_pcg(int N, Kind kind, const CoarseArgs& a, int grid, hipStream_t s) {
#define C(n) launch_coarse_pcg<n>(kind, a, grid, s)
  IPDG_SWITCH(N, C)
#undef C
}
int coarse_pcg_grid(int N, Kind kind, int K) {
  switch (N) {
    case 1: return coarse_pcg_grid<1>(kind, K);
    case 2: return coarse_pcg_grid<2>(kind, K);
    case 3: return coarse_pcg_grid<3>(kind, K);
    case 4: return coarse_pcg_grid<4>(kind, K);
    case 5: return coarse_pcg_grid<5>(kind, K);
    case 6: return coarse_pcg_grid<6>(kind, K);
    case 7: return coarse_pcg_grid<7>(kind, K);
    case 8: return coarse_pcg_grid<8>(kind, K);
    default: return 0;
  }
}

}  // namespace ipdg
