// Launch interface between the host solver code and the per-degree kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace ipdg {

// Compute / storage precision combinations of the element kernels.
//   F64      : FP64 arithmetic, FP64 in, FP64 out
//   F32      : FP32 arithmetic, FP32 in, FP32 out
//   F32_IN64 : FP32 arithmetic, FP64 in, FP32 out (block inverse mass applied
//              to the FP64 residual in mixed precision; not an operator kind)
enum class Kind { F64 = 0, F32 = 1, F32_IN64 = 2 };

// Type-erased arguments; geo/kap/ops are in the arithmetic precision.
struct ElemArgs {
  const void* x = nullptr;
  void* y = nullptr;
  const void* geo = nullptr;
  const Conn* conn = nullptr;
  const void* kap = nullptr;     // non-null => kappa-weighted operator
  const void* ops = nullptr;
  double lambda = 0.0, ctau = 0.0;
  int K = 0;
  double* partials = nullptr;    // optional: per-block sums of x.y
  const int* skip = nullptr;     // optional: device flag, kernel is a no-op when set
};

inline int elem_tiles(int K) { return (K + kBlock - 1) / kBlock; }
inline int elem_grid(int K) {
  int per;
  return xcd_grid(elem_tiles(K), per);
}

// Operator kernel variant per (degree, precision), degrees <= 5: bit 1 =
// LDS-staged coalesced loads/stores instead of direct per-lane ones, bit 2 =
// register budget lowered for one more resident wave per SIMD.  Set by
// set_ax_variant or IPDG_AX_VARIANT; defaults in dispatch.cpp.
int ax_variant(int N, bool fp32);
void set_ax_variant(int N, bool fp32, int v);
// Variant kAxCoop, at every degree: the cooperative kernel (three waves per
// tile of 64 elements).  Degrees 1..5 also have variants 0..3, degrees 6..8
// variants 0 and 1.
constexpr int kAxCoop = 4;
constexpr int kCoopTileElems = 64;   // elements per block of the cooperative kernel
bool ax_variant_exists(int N, int v);
// Blocks of the operator launch at degree N in this precision with the
// current variant: the number of partial sums it writes.
int ax_partials(int N, bool fp32, int K);

// y = A x (SIPDG operator).  Per degree, defined in the per-degree units.
template <int N> hipError_t launch_ax(Kind kind, const ElemArgs& a, hipStream_t s);
// Batched launches over many solves of degree N: tab holds one argument
// record per solve, map one entry per block (device memory).  The operator
// runs variant 0, 2 (element per lane, raised occupancy) or 4 (cooperative);
// each gives every solve the result of its own launch of that variant.
bool ax_batch_variant(int v);
template <int N> hipError_t launch_ax_batch(Kind kind, bool kap, int variant, const ElemArgs* tab,
                                            const BlockRef* map, int nblocks, hipStream_t s);
hipError_t ax_batch(int N, Kind kind, bool kap, int variant, const ElemArgs* tab, const BlockRef* map, int nblocks,
                    hipStream_t s);
// y = diag(A) (x unused).
template <int N> hipError_t launch_diag(Kind kind, const ElemArgs& a, hipStream_t s);
// y = J M x  (block-diagonal mass)
template <int N> hipError_t launch_mass(Kind kind, const ElemArgs& a, hipStream_t s);
// y = (J M)^{-1} x  (block inverse mass)
template <int N> hipError_t launch_minv(Kind kind, const ElemArgs& a, hipStream_t s);
// dL/dkappa_e = -w^T dA/dkappa_e u  (x = u, y unused, partials unused)
struct KgradArgs {
  const double* u; const double* w; double* out;
  const double* geo; const Conn* conn; const double* kap; const double* ops;
  double ctau; int K;
};
template <int N> hipError_t launch_kgrad(const KgradArgs& a, hipStream_t s);

// Inter-degree transfer: restriction rc = P^T (f - Az) and prolongation
// z += P zc, P the degree-Nc -> degree-Nf interpolation (Nf x Nc per element).
struct TransferArgs {
  const void* f = nullptr;   // restriction: fine right-hand side
  const void* Az = nullptr;  // restriction: A z on the fine level
  void* coarse = nullptr;    // restriction out / prolongation in
  void* fine = nullptr;      // prolongation in/out (z)
  const void* P = nullptr;   // interpolation matrix in arithmetic precision
  int K = 0;
  const int* skip = nullptr;
};
template <int Nf> hipError_t launch_restrict(int Nc, Kind kind, const TransferArgs& a, hipStream_t s);
template <int Nf> hipError_t launch_transfer_batch(int Nc, bool restrict_op, Kind kind, const TransferArgs* tab,
                                                   const BlockRef* map, int nblocks, hipStream_t s);
hipError_t transfer_batch(int Nf, int Nc, bool restrict_op, Kind kind, const TransferArgs* tab, const BlockRef* map,
                          int nblocks, hipStream_t s);
// Batched block inverse mass (kind as for launch_minv).
template <int N> hipError_t launch_minv_batch(Kind kind, const ElemArgs* tab, const BlockRef* map, int nblocks,
                                              hipStream_t s);
hipError_t minv_batch(int N, Kind kind, const ElemArgs* tab, const BlockRef* map, int nblocks, hipStream_t s);
template <int Nf> hipError_t launch_prolong(int Nc, Kind kind, const TransferArgs& a, hipStream_t s);

// Whole Jacobi-PCG solve of one (coarse) level in a single persistent launch:
// x = A^{-1} f to a relative residual tol or max_iters iterations, from x = 0.
// Blocks synchronise through a grid barrier with a bounded wait; the grid is
// sized so that every block is resident.  Degrees 1..4 only.
struct CoarseArgs {
  const void* f = nullptr;
  void* x = nullptr;
  void* r = nullptr;
  void* z = nullptr;
  void* p = nullptr;
  void* Ap = nullptr;
  const void* dinv = nullptr;
  ElemArgs op;                 // operator of the level (x, y, partials unused)
  double tol = 0.0;
  int max_iters = 0;
  double* partials = nullptr;  // 3 x kMaxPartials
  unsigned* bar = nullptr;     // 2 counters, zero between solves
  int* status = nullptr;       // [0] iterations, [1] barrier timeout, [2] breakdown
  const int* skip = nullptr;   // outer done flag
};
template <int N> hipError_t launch_coarse_pcg(Kind kind, const CoarseArgs& a, int grid, hipStream_t s);
template <int N> int coarse_pcg_grid(Kind kind, int K);   // resident grid size, 0 if unsupported

// One launch of the coarse Jacobi-PCG in single-reduction form (iteration
// `it`): every block reduces the (r, r), (r, u), (w, u) partials of the
// previous launch (pin slots 0..2 with n_rr, n_g, n_d entries), records the
// stop in sc, else updates p, s, x, r, u of its elements, forms the new u of
// the neighbours on the fly, writes w = A u and the next partials to pout.
// r, w, s are double-buffered by the caller (old / new by parity).
struct CGScal;
struct CoarseStepArgs {
  void* x = nullptr;
  void* p = nullptr;
  void* u = nullptr;
  const void* dinv = nullptr;
  const void* r_old = nullptr;
  void* r_new = nullptr;
  const void* w_old = nullptr;
  void* w_new = nullptr;
  const void* s_old = nullptr;
  void* s_new = nullptr;
  ElemArgs op;                 // operator of the level (x, y, partials unused)
  const double* pin = nullptr;
  int n_rr = 0, n_g = 0, n_d = 0;
  double* pout = nullptr;
  CGScal* sc = nullptr;
  const int* outer = nullptr;  // outer solve's done flag (checked at it = 0)
  int it = 0;
};
template <int N> hipError_t launch_coarse_step(Kind kind, const CoarseStepArgs& a, hipStream_t s);

// The coarsest levels of a batch of solves (same degree and precision) as one
// concatenated level: solve i owns elements [off, off + K) (off a multiple of
// kBlock, so tiles never straddle two solves) and tiles [tile0, tile0 + ntiles).
// Connectivity is stored with global element ids.  Each solve keeps its own
// operator constants, coarse-CG scalars, partial-sum slots (its tile range)
// and outer done flag; f and z are its own coarse right-hand side and
// solution buffers.
struct CoarseBatchEntry {
  int off = 0, K = 0, tile0 = 0, ntiles = 0;
  double lambda = 0.0, ctau = 0.0;
  const int* outer = nullptr;
  const void* f = nullptr;
  void* z = nullptr;
};
struct CoarseBatchArgs {
  const CoarseBatchEntry* ent = nullptr;   // device, one per solve
  const int* tile_solve = nullptr;         // device, grid entries: solve of each tile, -1 past the end
  int grid = 0, per = 0;                   // launch: grid = per * kXcd blocks
  void* x = nullptr;                       // concatenated coarse work vectors (level precision)
  void* p = nullptr;
  void* u = nullptr;
  const void* dinv = nullptr;
  void* r[2] = {nullptr, nullptr};
  void* w[2] = {nullptr, nullptr};
  void* s[2] = {nullptr, nullptr};
  const void* geo = nullptr;
  const Conn* conn = nullptr;
  const void* kap = nullptr;               // null: no solve has a coefficient
  const void* ops = nullptr;
  double* partials = nullptr;              // 2 sets of 3 slots of kMaxPartials
  CGScal* sc = nullptr;                    // device, one per solve
};
template <int N> hipError_t launch_coarse_batch(Kind kind, const CoarseBatchArgs& a, int it, hipStream_t s);

// Runtime-degree dispatch (dispatch.cpp)
hipError_t ax(int N, Kind kind, const ElemArgs& a, hipStream_t s);
hipError_t diag(int N, Kind kind, const ElemArgs& a, hipStream_t s);
hipError_t mass(int N, Kind kind, const ElemArgs& a, hipStream_t s);
hipError_t minv(int N, Kind kind, const ElemArgs& a, hipStream_t s);
hipError_t kgrad(int N, const KgradArgs& a, hipStream_t s);
hipError_t restrict_(int Nf, int Nc, Kind kind, const TransferArgs& a, hipStream_t s);
hipError_t prolong(int Nf, int Nc, Kind kind, const TransferArgs& a, hipStream_t s);
hipError_t coarse_pcg(int N, Kind kind, const CoarseArgs& a, int grid, hipStream_t s);
hipError_t coarse_step(int N, Kind kind, const CoarseStepArgs& a, hipStream_t s);
// it = -1: initial state and partials; 0.. : one coarse-CG iteration; -2:
// copy each solve's solution to its z buffer
hipError_t coarse_batch(int N, Kind kind, const CoarseBatchArgs& a, int it, hipStream_t s);
int coarse_pcg_grid(int N, Kind kind, int K);

}  // namespace ipdg
