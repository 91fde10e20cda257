// Vector kernels of the device-resident preconditioned CG solvers (Sec. 3).
//
// All scalars of an iteration (alpha, beta, dot products, convergence and
// breakdown flags) live in device memory, so an iteration is a fixed
// sequence of launches with no host round trip; each kernel takes a `skip`
// flag (the solve's done flag) and returns at once when it is set.  Dot
// products are reduced per block into a partials array and summed by a
// one-block finalize kernel in a fixed order (bitwise reproducible).
#include "blas.hpp"

namespace ipdg {
namespace {

__device__ __forceinline__ double ldd(const double* p, size_t i) { return p[i]; }
__device__ __forceinline__ double ldd(const float* p, size_t i) { return static_cast<double>(p[i]); }

// Position of a block in its launch: block b of nb.  A direct launch uses
// blockIdx.x of gridDim.x; a batched launch the member-local block of its
// block map, so that every member sees the launch shape of its own direct
// launch (the same partial-sum slots and summation order).
struct Blk {
  int b, nb;
};
__device__ __forceinline__ Blk direct_blk() { return Blk{(int)blockIdx.x, (int)gridDim.x}; }

template <int NV>
__device__ __forceinline__ void commit(double (&v)[NV], double* partials, int b) {
  block_sum<NV>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) partials[k * kMaxPartials + b] = v[k];
}
template <int NV>
__device__ __forceinline__ void commit(double (&v)[NV], double* partials) {
  commit<NV>(v, partials, (int)blockIdx.x);
}

// r = b - Ax; partials: (r, r), (b, b)
__global__ __launch_bounds__(kBlock) void k_residual(const double* __restrict__ b,
                                                     const double* __restrict__ Ax,
                                                     double* __restrict__ r, size_t n,
                                                     double* __restrict__ partials) {
  double v[2] = {0.0, 0.0};
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    const double bi = b[i];
    const double ri = bi - Ax[i];
    r[i] = ri;
    v[0] += ri * ri;
    v[1] += bi * bi;
  }
  commit<2>(v, partials);
}

// x += alpha p; r -= alpha Ap; optionally z = dinv r (Jacobi, z in TZ).
// partials: (r, r), and with Jacobi (r, z), (z, Ap).
template <typename TZ, bool JAC>
__device__ __forceinline__ void update_body(double* __restrict__ x, double* __restrict__ r,
                                            const double* __restrict__ p, const double* __restrict__ Ap,
                                            const double* __restrict__ dinv, TZ* __restrict__ z,
                                            const CGScal* __restrict__ sc, size_t n,
                                            double* __restrict__ partials, Blk k) {
  if (sc->done) return;
  const double alpha = sc->alpha;
  double v[3] = {0.0, 0.0, 0.0};
  for (size_t i = k.b * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)k.nb * kBlock) {
    const double api = Ap[i];
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * api;
    r[i] = ri;
    v[0] += ri * ri;
    if constexpr (JAC) {
      const TZ zi = static_cast<TZ>(dinv[i] * ri);
      z[i] = zi;
      v[1] += ri * static_cast<double>(zi);
      v[2] += static_cast<double>(zi) * api;
    }
  }
  commit<3>(v, partials, k.b);
}
template <typename TZ, bool JAC>
__global__ __launch_bounds__(kBlock) void k_update(double* __restrict__ x, double* __restrict__ r,
                                                   const double* __restrict__ p,
                                                   const double* __restrict__ Ap,
                                                   const double* __restrict__ dinv,
                                                   TZ* __restrict__ z, const CGScal* __restrict__ sc,
                                                   size_t n, double* __restrict__ partials) {
  update_body<TZ, JAC>(x, r, p, Ap, dinv, z, sc, n, partials, direct_blk());
}

// partials slots 1, 2: (r, z), (z, Ap)
template <typename TZ>
__device__ __forceinline__ void dots_rz_body(const double* __restrict__ r, const TZ* __restrict__ z,
                                             const double* __restrict__ Ap, const CGScal* __restrict__ sc,
                                             size_t n, double* __restrict__ partials, Blk k) {
  if (sc->done) return;
  double v[2] = {0.0, 0.0};
  for (size_t i = k.b * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)k.nb * kBlock) {
    const double zi = ldd(z, i);
    v[0] += r[i] * zi;
    if (Ap) v[1] += zi * Ap[i];
  }
  block_sum<2>(v);
  if (threadIdx.x == 0) {
    partials[1 * kMaxPartials + k.b] = v[0];
    partials[2 * kMaxPartials + k.b] = v[1];
  }
}
template <typename TZ>
__global__ __launch_bounds__(kBlock) void k_dots_rz(const double* __restrict__ r,
                                                    const TZ* __restrict__ z,
                                                    const double* __restrict__ Ap,
                                                    const CGScal* __restrict__ sc, size_t n,
                                                    double* __restrict__ partials) {
  dots_rz_body<TZ>(r, z, Ap, sc, n, partials, direct_blk());
}

// p = z + beta p
template <typename TZ>
__device__ __forceinline__ void pupdate_body(double* __restrict__ p, const TZ* __restrict__ z,
                                             const CGScal* __restrict__ sc, size_t n, Blk k) {
  if (sc->done) return;
  const double beta = sc->beta;
  for (size_t i = k.b * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)k.nb * kBlock)
    p[i] = ldd(z, i) + beta * p[i];
}
template <typename TZ>
__global__ __launch_bounds__(kBlock) void k_pupdate(double* __restrict__ p, const TZ* __restrict__ z,
                                                    const CGScal* __restrict__ sc, size_t n) {
  pupdate_body<TZ>(p, z, sc, n, direct_blk());
}

// z = dinv r (TZ) ; partials (r, z) in slot 1
template <typename TZ>
__device__ __forceinline__ void jacobi_body(const double* __restrict__ r, const double* __restrict__ dinv,
                                            TZ* __restrict__ z, size_t n, Blk k) {
  for (size_t i = k.b * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)k.nb * kBlock)
    z[i] = static_cast<TZ>(dinv[i] * r[i]);
}
template <typename TZ>
__global__ __launch_bounds__(kBlock) void k_jacobi(const double* __restrict__ r,
                                                   const double* __restrict__ dinv,
                                                   TZ* __restrict__ z, size_t n) {
  jacobi_body<TZ>(r, dinv, z, n, direct_blk());
}

// Sum the partials of `nslots` slots over nparts blocks (fixed order) and
// apply one step of the CG scalar recurrence.
__device__ __forceinline__ void finalize_body(const double* __restrict__ partials, int nparts, int nslots,
                                              CGScal* __restrict__ sc, int op) {
  if ((op == kFinAlpha || op == kFinBeta) && sc->done) return;
  __shared__ double red[3][kBlock];
  for (int k = 0; k < nslots; ++k) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kBlock) s += partials[k * kMaxPartials + i];
    red[k][threadIdx.x] = s;
  }
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < nslots; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double s0 = red[0][0], s1 = nslots > 1 ? red[1][0] : 0.0, s2 = nslots > 2 ? red[2][0] : 0.0;
  switch (op) {
    case kFinResidual:   // (r, r), (b, b); the recurrence restarts from here
      sc->rr = s0;
      sc->bb = s1;
      sc->tol2 = sc->tol * sc->tol * s1;
      sc->done = 0;
      break;
    case kFinInit:       // (r, z) after z = B r, p = z
      sc->rz = s1;
      sc->done = (sc->rr <= sc->tol2) || (sc->bb == 0.0) || (sc->max_iters <= sc->iters);
      break;
    case kFinAlpha: {    // (p, Ap)
      const double pAp = s0;
      sc->pAp = pAp;
      if (!(pAp > 0.0) || !isfinite(pAp) || !isfinite(sc->rz)) {
        sc->breakdown = 1;
        sc->done = 1;
      } else {
        sc->alpha = sc->rz / pAp;
      }
      break;
    }
    case kFinBeta: {     // (r, r), (r, z), (z, Ap)
      sc->rr = s0;
      sc->iters += 1;
      const double beta = sc->flexible ? -s2 / sc->pAp : s1 / sc->rz;
      sc->beta = beta;
      sc->rz = s1;
      if (!isfinite(s0)) { sc->breakdown = 1; sc->done = 1; }
      if (s0 <= sc->tol2 || sc->iters >= sc->max_iters) sc->done = 1;
      break;
    }
  }
}
__global__ __launch_bounds__(kBlock) void k_finalize(const double* __restrict__ partials,
                                                     int nparts, int nslots, CGScal* __restrict__ sc,
                                                     int op) {
  finalize_body(partials, nparts, nslots, sc, op);
}

// Chebyshev smoothing on D^{-1} A (Saad Alg. 12.1):
//   start from zero:     r = f;     d = c0 dinv f;      z = d
//   start from z:        r = f - t; d = c0 dinv r;      z += d    (t = A z)
//   step:                r -= t;    d = c1 d + c2 dinv r; z += d  (t = A d)
template <typename T>
__device__ __forceinline__ void cheb_body(int mode, const T* __restrict__ f, const T* __restrict__ t,
                                          const T* __restrict__ dinv, T* __restrict__ z, T* __restrict__ d,
                                          T* __restrict__ r, T c0, T c1, T c2, size_t n,
                                          const int* __restrict__ skip, Blk k) {
  if (skip && *skip) return;
  for (size_t i = k.b * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)k.nb * kBlock) {
    if (mode == 0) {
      const T ri = f[i];
      r[i] = ri;
      const T di = c0 * dinv[i] * ri;
      d[i] = di;
      z[i] = di;
    } else if (mode == 1) {
      const T ri = f[i] - t[i];
      r[i] = ri;
      const T di = c0 * dinv[i] * ri;
      d[i] = di;
      z[i] += di;
    } else {
      const T ri = r[i] - t[i];
      r[i] = ri;
      const T di = c1 * d[i] + c2 * dinv[i] * ri;
      d[i] = di;
      z[i] += di;
    }
  }
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cheb(int mode, const T* __restrict__ f,
                                                 const T* __restrict__ t, const T* __restrict__ dinv,
                                                 T* __restrict__ z, T* __restrict__ d,
                                                 T* __restrict__ r, T c0, T c1, T c2, size_t n,
                                                 const int* __restrict__ skip) {
  cheb_body<T>(mode, f, t, dinv, z, d, r, c0, c1, c2, n, skip, direct_blk());
}

template <typename TD, typename TS>
__device__ __forceinline__ void convert_body(TD* __restrict__ dst, const TS* __restrict__ src, size_t n,
                                             const int* __restrict__ skip, Blk k) {
  if (skip && *skip) return;
  for (size_t i = k.b * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)k.nb * kBlock)
    dst[i] = static_cast<TD>(src[i]);
}
template <typename TD, typename TS>
__global__ __launch_bounds__(kBlock) void k_convert(TD* __restrict__ dst, const TS* __restrict__ src,
                                                    size_t n, const int* __restrict__ skip) {
  convert_body<TD, TS>(dst, src, n, skip, direct_blk());
}

// ---------------------------------------------------------------------------
// Batched forms: one launch runs the same operation for many solves, each
// block reading its member's arguments from a table and its member-local
// block from the block map.
// ---------------------------------------------------------------------------
template <typename TZ, bool JAC>
__global__ __launch_bounds__(kBlock) void kb_update(const VecArgs* __restrict__ tab, const BlockRef* __restrict__ map) {
  const BlockRef m = map[blockIdx.x];
  const VecArgs& a = tab[m.s];
  update_body<TZ, JAC>(in_global((double*)a.x), in_global((double*)a.y), in_global((const double*)a.a),
                       in_global((const double*)a.b), in_global((const double*)a.c), in_global((TZ*)a.z),
                       in_global(a.sc), a.n, in_global(a.partials), Blk{m.b, m.nb});
}
template <typename TZ>
__global__ __launch_bounds__(kBlock) void kb_dots_rz(const VecArgs* __restrict__ tab, const BlockRef* __restrict__ map) {
  const BlockRef m = map[blockIdx.x];
  const VecArgs& a = tab[m.s];
  dots_rz_body<TZ>(in_global((const double*)a.a), in_global((const TZ*)a.b), in_global((const double*)a.c),
                   in_global(a.sc), a.n, in_global(a.partials), Blk{m.b, m.nb});
}
template <typename TZ>
__global__ __launch_bounds__(kBlock) void kb_pupdate(const VecArgs* __restrict__ tab, const BlockRef* __restrict__ map) {
  const BlockRef m = map[blockIdx.x];
  const VecArgs& a = tab[m.s];
  pupdate_body<TZ>(in_global((double*)a.x), in_global((const TZ*)a.a), in_global(a.sc), a.n, Blk{m.b, m.nb});
}
template <typename TZ>
__global__ __launch_bounds__(kBlock) void kb_jacobi(const VecArgs* __restrict__ tab, const BlockRef* __restrict__ map) {
  const BlockRef m = map[blockIdx.x];
  const VecArgs& a = tab[m.s];
  jacobi_body<TZ>(in_global((const double*)a.a), in_global((const double*)a.b), in_global((TZ*)a.z), a.n,
                  Blk{m.b, m.nb});
}
__global__ __launch_bounds__(kBlock) void kb_finalize(const VecArgs* __restrict__ tab, const BlockRef* __restrict__ map) {
  const BlockRef m = map[blockIdx.x];
  const VecArgs& a = tab[m.s];
  finalize_body(in_global((const double*)a.a), a.nparts, a.nslots, in_global(a.scw), a.op);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void kb_cheb(const VecArgs* __restrict__ tab, const BlockRef* __restrict__ map) {
  const BlockRef m = map[blockIdx.x];
  const VecArgs& a = tab[m.s];
  cheb_body<T>(a.mode, in_global((const T*)a.a), in_global((const T*)a.b), in_global((const T*)a.c),
               in_global((T*)a.z), in_global((T*)a.x), in_global((T*)a.y), T(a.c0), T(a.c1), T(a.c2), a.n,
               in_global(a.skip), Blk{m.b, m.nb});
}
template <typename TD, typename TS>
__global__ __launch_bounds__(kBlock) void kb_convert(const VecArgs* __restrict__ tab, const BlockRef* __restrict__ map) {
  const BlockRef m = map[blockIdx.x];
  const VecArgs& a = tab[m.s];
  convert_body<TD, TS>(in_global((TD*)a.x), in_global((const TS*)a.a), a.n, in_global(a.skip), Blk{m.b, m.nb});
}

// dst[i] = *src[i]: the CG scalars of many solves into one array
__global__ __launch_bounds__(64) void k_scal_gather(const CGScal* const* __restrict__ src, CGScal* __restrict__ dst,
                                                    int n) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i < n) dst[i] = *src[i];
}

// coarse-solve initialisation: x = 0, r = f, z = dinv f, p = z; partials
// (r, r), (r, z)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_start0(const T* __restrict__ f, const T* __restrict__ dinv,
                                                      T* __restrict__ x, T* __restrict__ r,
                                                      T* __restrict__ z, T* __restrict__ p, size_t n,
                                                      double* __restrict__ partials,
                                                      const int* __restrict__ skip) {
  if (skip && *skip) return;
  double v[2] = {0.0, 0.0};
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    const T fi = f[i];
    const T zi = dinv[i] * fi;
    x[i] = T(0);
    r[i] = fi;
    z[i] = zi;
    p[i] = zi;
    v[0] += double(fi) * double(fi);
    v[1] += double(fi) * double(zi);
  }
  commit<2>(v, partials);
}

// coarse-solve scalar setup after k_cg_start0: rr0, tol2 = tol^2 rr0, rz
__global__ void k_cg_start_fin(const double* __restrict__ partials, int nparts, CGScal* sc,
                               const int* __restrict__ skip) {
  __shared__ double red[2][kBlock];
  for (int k = 0; k < 2; ++k) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kBlock) s += partials[k * kMaxPartials + i];
    red[k][threadIdx.x] = s;
  }
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 2; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (skip && *skip) {     // outer solve finished: keep the last solve's record
    sc->done = 1;
    return;
  }
  sc->rr = red[0][0];
  sc->bb = red[0][0];
  sc->rz = red[1][0];
  sc->rzb[0] = red[1][0];
  sc->tol2 = sc->tol * sc->tol * sc->rr;
  sc->iters = 0;
  sc->breakdown = 0;
  sc->done = sc->rr == 0.0 || sc->max_iters <= 0;
}

// single-precision-state coarse CG update: x += a p; r -= a Ap; z = dinv r;
// partials (r,r), (r,z), (z,Ap)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_update(T* __restrict__ x, T* __restrict__ r,
                                                      const T* __restrict__ p, const T* __restrict__ Ap,
                                                      const T* __restrict__ dinv, T* __restrict__ z,
                                                      const CGScal* __restrict__ sc, size_t n,
                                                      double* __restrict__ partials) {
  if (sc->done) return;
  const T alpha = static_cast<T>(sc->alpha);
  double v[3] = {0.0, 0.0, 0.0};
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    x[i] += alpha * p[i];
    const T ri = r[i] - alpha * Ap[i];
    r[i] = ri;
    const T zi = dinv[i] * ri;
    z[i] = zi;
    v[0] += double(ri) * double(ri);
    v[1] += double(ri) * double(zi);
    v[2] += double(zi) * double(Ap[i]);
  }
  commit<3>(v, partials);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_pupdate(T* __restrict__ p, const T* __restrict__ z,
                                                       const CGScal* __restrict__ sc, size_t n) {
  if (sc->done) return;
  const T beta = static_cast<T>(sc->beta);
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    p[i] = z[i] + beta * p[i];
}

// reciprocal of the diagonal (in place) and an optional FP32 copy
__global__ __launch_bounds__(kBlock) void k_recip(double* __restrict__ d, float* __restrict__ d32, size_t n) {
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    const double v = 1.0 / d[i];
    d[i] = v;
    if (d32) d32[i] = static_cast<float>(v);
  }
}

__global__ void k_set_scal(CGScal* sc, CGScal v) { *sc = v; }

__global__ __launch_bounds__(kBlock) void k_fill(double* __restrict__ p, double v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) p[i] = v;
}

__global__ void k_zero_ints(int* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

}  // namespace

int flat_grid(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > (size_t)kMaxPartials) b = kMaxPartials;
  return b < 1 ? 1 : int(b);
}

#define LAUNCH(kern, n, s, ...) \
  hipLaunchKernelGGL(kern, dim3(flat_grid(n)), dim3(kBlock), 0, s, __VA_ARGS__)

hipError_t residual(const double* b, const double* Ax, double* r, size_t n, double* partials, hipStream_t s) {
  LAUNCH(k_residual, n, s, b, Ax, r, n, partials);
  return hipGetLastError();
}

hipError_t cg_update(bool fp32z, bool jacobi, double* x, double* r, const double* p, const double* Ap,
                     const double* dinv, void* z, const CGScal* sc, size_t n, double* partials,
                     hipStream_t s) {
  if (fp32z) {
    if (jacobi) LAUNCH((k_update<float, true>), n, s, x, r, p, Ap, dinv, (float*)z, sc, n, partials);
    else LAUNCH((k_update<float, false>), n, s, x, r, p, Ap, dinv, (float*)z, sc, n, partials);
  } else {
    if (jacobi) LAUNCH((k_update<double, true>), n, s, x, r, p, Ap, dinv, (double*)z, sc, n, partials);
    else LAUNCH((k_update<double, false>), n, s, x, r, p, Ap, dinv, (double*)z, sc, n, partials);
  }
  return hipGetLastError();
}

hipError_t dots_rz(bool fp32z, const double* r, const void* z, const double* Ap, const CGScal* sc, size_t n,
                   double* partials, hipStream_t s) {
  if (fp32z) LAUNCH(k_dots_rz<float>, n, s, r, (const float*)z, Ap, sc, n, partials);
  else LAUNCH(k_dots_rz<double>, n, s, r, (const double*)z, Ap, sc, n, partials);
  return hipGetLastError();
}

hipError_t pupdate(bool fp32z, double* p, const void* z, const CGScal* sc, size_t n, hipStream_t s) {
  if (fp32z) LAUNCH(k_pupdate<float>, n, s, p, (const float*)z, sc, n);
  else LAUNCH(k_pupdate<double>, n, s, p, (const double*)z, sc, n);
  return hipGetLastError();
}

hipError_t jacobi(bool fp32z, const double* r, const double* dinv, void* z, size_t n, hipStream_t s) {
  if (fp32z) LAUNCH(k_jacobi<float>, n, s, r, dinv, (float*)z, n);
  else LAUNCH(k_jacobi<double>, n, s, r, dinv, (double*)z, n);
  return hipGetLastError();
}

hipError_t finalize(const double* partials, int nparts, int nslots, CGScal* sc, int op, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, partials, nparts, nslots, sc, op);
  return hipGetLastError();
}

hipError_t cheb(bool fp32, int mode, const void* f, const void* t, const void* dinv, void* z, void* d,
                void* r, double c0, double c1, double c2, size_t n, const int* skip, hipStream_t s) {
  if (fp32)
    LAUNCH(k_cheb<float>, n, s, mode, (const float*)f, (const float*)t, (const float*)dinv, (float*)z,
           (float*)d, (float*)r, float(c0), float(c1), float(c2), n, skip);
  else
    LAUNCH(k_cheb<double>, n, s, mode, (const double*)f, (const double*)t, (const double*)dinv,
           (double*)z, (double*)d, (double*)r, c0, c1, c2, n, skip);
  return hipGetLastError();
}

hipError_t convert(bool to_fp32, void* dst, const void* src, size_t n, const int* skip, hipStream_t s) {
  if (to_fp32) LAUNCH((k_convert<float, double>), n, s, (float*)dst, (const double*)src, n, skip);
  else LAUNCH((k_convert<double, float>), n, s, (double*)dst, (const float*)src, n, skip);
  return hipGetLastError();
}

hipError_t cg_start0(bool fp32, const void* f, const void* dinv, void* x, void* r, void* z, void* p,
                     size_t n, double* partials, const int* skip, hipStream_t s) {
  if (fp32)
    LAUNCH(k_cg_start0<float>, n, s, (const float*)f, (const float*)dinv, (float*)x, (float*)r, (float*)z,
           (float*)p, n, partials, skip);
  else
    LAUNCH(k_cg_start0<double>, n, s, (const double*)f, (const double*)dinv, (double*)x, (double*)r,
           (double*)z, (double*)p, n, partials, skip);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipSuccess;
}

hipError_t cg_start_fin(const double* partials, int nparts, CGScal* sc, const int* skip, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_start_fin, dim3(1), dim3(kBlock), 0, s, partials, nparts, sc, skip);
  return hipGetLastError();
}

hipError_t cg_update_state(bool fp32, void* x, void* r, const void* p, const void* Ap, const void* dinv,
                           void* z, const CGScal* sc, size_t n, double* partials, hipStream_t s) {
  if (fp32)
    LAUNCH(k_cg_update<float>, n, s, (float*)x, (float*)r, (const float*)p, (const float*)Ap,
           (const float*)dinv, (float*)z, sc, n, partials);
  else
    LAUNCH(k_cg_update<double>, n, s, (double*)x, (double*)r, (const double*)p, (const double*)Ap,
           (const double*)dinv, (double*)z, sc, n, partials);
  return hipGetLastError();
}

hipError_t cg_pupdate_state(bool fp32, void* p, const void* z, const CGScal* sc, size_t n, hipStream_t s) {
  if (fp32) LAUNCH(k_cg_pupdate<float>, n, s, (float*)p, (const float*)z, sc, n);
  else LAUNCH(k_cg_pupdate<double>, n, s, (double*)p, (const double*)z, sc, n);
  return hipGetLastError();
}

hipError_t recip(double* d, float* d32, size_t n, hipStream_t s) {
  LAUNCH(k_recip, n, s, d, d32, n);
  return hipGetLastError();
}

hipError_t zero_ints(void* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, s, static_cast<int*>(p), n);
  return hipGetLastError();
}

hipError_t fill(double* p, double v, size_t n, hipStream_t s) {
  LAUNCH(k_fill, n, s, p, v, n);
  return hipGetLastError();
}

hipError_t vec_batch(VecOp op, bool fp32, bool flag, const VecArgs* tab, const BlockRef* map, int nblocks,
                     hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  const dim3 g(nblocks), b(kBlock);
  switch (op) {
    case VecOp::kUpdate:
      if (fp32) {
        if (flag) hipLaunchKernelGGL((kb_update<float, true>), g, b, 0, s, tab, map);
        else hipLaunchKernelGGL((kb_update<float, false>), g, b, 0, s, tab, map);
      } else {
        if (flag) hipLaunchKernelGGL((kb_update<double, true>), g, b, 0, s, tab, map);
        else hipLaunchKernelGGL((kb_update<double, false>), g, b, 0, s, tab, map);
      }
      break;
    case VecOp::kDotsRz:
      if (fp32) hipLaunchKernelGGL(kb_dots_rz<float>, g, b, 0, s, tab, map);
      else hipLaunchKernelGGL(kb_dots_rz<double>, g, b, 0, s, tab, map);
      break;
    case VecOp::kPupdate:
      if (fp32) hipLaunchKernelGGL(kb_pupdate<float>, g, b, 0, s, tab, map);
      else hipLaunchKernelGGL(kb_pupdate<double>, g, b, 0, s, tab, map);
      break;
    case VecOp::kJacobi:
      if (fp32) hipLaunchKernelGGL(kb_jacobi<float>, g, b, 0, s, tab, map);
      else hipLaunchKernelGGL(kb_jacobi<double>, g, b, 0, s, tab, map);
      break;
    case VecOp::kFinalize:
      hipLaunchKernelGGL(kb_finalize, g, b, 0, s, tab, map);
      break;
    case VecOp::kCheb:
      if (fp32) hipLaunchKernelGGL(kb_cheb<float>, g, b, 0, s, tab, map);
      else hipLaunchKernelGGL(kb_cheb<double>, g, b, 0, s, tab, map);
      break;
    case VecOp::kConvert:
      if (flag) hipLaunchKernelGGL((kb_convert<float, double>), g, b, 0, s, tab, map);
      else hipLaunchKernelGGL((kb_convert<double, float>), g, b, 0, s, tab, map);
      break;
  }
  return hipGetLastError();
}

hipError_t scal_gather(const CGScal* const* src, CGScal* dst, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scal_gather, dim3((n + 63) / 64), dim3(64), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t set_scal(CGScal* sc, const CGScal& v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_scal, dim3(1), dim3(1), 0, s, sc, v);
  return hipGetLastError();
}

}  // namespace ipdg
