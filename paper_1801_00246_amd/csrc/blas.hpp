// Device-resident CG scalars and vector kernels (blas.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace ipdg {

// Scalars of one CG solve, kept in device memory.
struct CGScal {
  double rz = 0, pAp = 0, alpha = 0, beta = 0, rr = 0, bb = 0, tol = 0, tol2 = 0;
  int done = 0, breakdown = 0, iters = 0, max_iters = 0, flexible = 0, pad = 0;
  double rzb[2] = {0, 0};   // coarse solve: (r, u) by iteration parity
  double ab[2] = {0, 0};    // coarse solve: alpha by iteration parity
};

// Partial-sum slots per reduction (>= blocks of any element or vector launch).
constexpr int kMaxPartials = 65536;

enum FinOp { kFinResidual = 0, kFinInit = 1, kFinAlpha = 2, kFinBeta = 3 };

// One member's arguments of a batched vector operation (the parameters of the
// direct launch, by role):
//   update   x += alpha p, r -= alpha Ap (+ Jacobi z): x=x, y=r, a=p, b=Ap, c=dinv, z
//   dots_rz  a=r, b=z, c=Ap        pupdate  x=p, a=z      jacobi  a=r, b=dinv, z
//   finalize a=partials, scw, nparts, nslots, op
//   cheb     mode, a=f, b=t, c=dinv, z, x=d, y=r, c0..c2   convert  x=dst, a=src
struct VecArgs {
  const void* a = nullptr;
  const void* b = nullptr;
  const void* c = nullptr;
  void* x = nullptr;
  void* y = nullptr;
  void* z = nullptr;
  const CGScal* sc = nullptr;
  CGScal* scw = nullptr;
  double c0 = 0, c1 = 0, c2 = 0;
  size_t n = 0;
  double* partials = nullptr;
  const int* skip = nullptr;
  int nparts = 0, nslots = 0, op = 0, mode = 0;
};

enum class VecOp { kUpdate, kDotsRz, kPupdate, kJacobi, kFinalize, kCheb, kConvert };

// Batched vector operation: fp32 selects the FP32 form (z of update, dots_rz,
// pupdate and jacobi; T of cheb), flag the Jacobi update or, for convert, the
// direction FP64 -> FP32.
hipError_t vec_batch(VecOp op, bool fp32, bool flag, const VecArgs* tab, const BlockRef* map, int nblocks,
                     hipStream_t s);

int flat_grid(size_t n);

// dst[i] = *src[i] for i < n (src: device array of n device pointers).
hipError_t scal_gather(const CGScal* const* src, CGScal* dst, int n, hipStream_t s);

hipError_t residual(const double* b, const double* Ax, double* r, size_t n, double* partials, hipStream_t s);
hipError_t cg_update(bool fp32z, bool jacobi, double* x, double* r, const double* p, const double* Ap,
                     const double* dinv, void* z, const CGScal* sc, size_t n, double* partials,
                     hipStream_t s);
hipError_t dots_rz(bool fp32z, const double* r, const void* z, const double* Ap, const CGScal* sc, size_t n,
                   double* partials, hipStream_t s);
hipError_t pupdate(bool fp32z, double* p, const void* z, const CGScal* sc, size_t n, hipStream_t s);
hipError_t jacobi(bool fp32z, const double* r, const double* dinv, void* z, size_t n, hipStream_t s);
hipError_t finalize(const double* partials, int nparts, int nslots, CGScal* sc, int op, hipStream_t s);
hipError_t cheb(bool fp32, int mode, const void* f, const void* t, const void* dinv, void* z, void* d,
                void* r, double c0, double c1, double c2, size_t n, const int* skip, hipStream_t s);
hipError_t convert(bool to_fp32, void* dst, const void* src, size_t n, const int* skip, hipStream_t s);
hipError_t cg_start0(bool fp32, const void* f, const void* dinv, void* x, void* r, void* z, void* p,
                     size_t n, double* partials, const int* skip, hipStream_t s);
hipError_t cg_start_fin(const double* partials, int nparts, CGScal* sc, const int* skip, hipStream_t s);
hipError_t cg_update_state(bool fp32, void* x, void* r, const void* p, const void* Ap, const void* dinv,
                           void* z, const CGScal* sc, size_t n, double* partials, hipStream_t s);
hipError_t cg_pupdate_state(bool fp32, void* p, const void* z, const CGScal* sc, size_t n, hipStream_t s);
hipError_t recip(double* d, float* d32, size_t n, hipStream_t s);
hipError_t set_scal(CGScal* sc, const CGScal& v, hipStream_t s);
hipError_t zero_ints(void* p, int n, hipStream_t s);
hipError_t fill(double* p, double v, size_t n, hipStream_t s);

}  // namespace ipdg
