// Element kernels of one polynomial degree (compiled once per degree with
// -DIPDG_N=<N>).  One lane owns one element; a block owns kBlock consecutive
// elements; blocks are mapped to tiles so that neighbouring tiles run on the
// same die (shared L2 for the neighbour gathers).
#include "kernels.hpp"
#include "sipdg_core.hpp"
#include "sipdg_coop.hpp"
#include "blas.hpp"

#include <algorithm>

#ifndef IPDG_N
#error "IPDG_N must be defined"
#endif

namespace ipdg {
namespace {

constexpr int N = IPDG_N;
constexpr int kMaxPartialsCoarse = 4096;
constexpr int Np = Tri<N>::Np;

// Occupancy-raised variant: waves per SIMD the register allocator must leave
// room for (one more than the unconstrained allocation gives; 0 = none).
// The operator kernel holds one element per lane, so its footprint grows
// with Np; FP32 halves it.
template <typename TC>
constexpr int ax_boost_waves() {
  if constexpr (sizeof(TC) == 8) return N <= 2 ? 5 : (N <= 4 ? 4 : 3);
  else return N <= 1 ? 0 : (N <= 2 ? 8 : (N <= 3 ? 7 : (N <= 4 ? 6 : 5)));
}

// LDS pitch (elements) of the staging buffer: odd in 8-byte words, so that
// both the cooperative copy and the per-lane accesses avoid bank conflicts.
constexpr int kPitch = kBlock + 1;

// STAGE: the block's own inputs and outputs go through LDS, so that global
// loads and stores are fully coalesced (lane t touches word t of the block's
// contiguous chunk) instead of Np-strided per lane.
// blk: the block's position in its (member-local) launch grid, per: that
// grid's die-mapping stride.
template <typename TC, typename TX, typename TY, bool KAP, bool STAGE>
__device__ __forceinline__ void ax_body(const TX* __restrict__ x, TY* __restrict__ y, const TC* __restrict__ geo,
                                        const Conn* __restrict__ conn, const TC* __restrict__ kap,
                                        const TC* __restrict__ ops, TC lambda, TC ctau, int K, int per,
                                        double* __restrict__ partials, const int* __restrict__ skip, int blk) {
  if (skip && *skip) return;
  const int e0 = xcd_tile(blk, per) * kBlock;
  const int e = e0 + threadIdx.x;
  const bool want_dot = partials != nullptr;
  double dot = 0.0;
  if constexpr (STAGE) {
    __shared__ TC buf[Np * kPitch];
    const int ne = K - e0 < kBlock ? K - e0 : kBlock;
    if (ne > 0) {
      const TX* src = x + (size_t)e0 * Np;
      for (int t = threadIdx.x; t < ne * Np; t += kBlock) {
        const int le = t / Np, j = t - le * Np;
        buf[j * kPitch + le] = static_cast<TC>(src[t]);
      }
    }
    __syncthreads();
    if (e < K) {
      TC u[Np];
      const TX* xe = x + (size_t)e * Np;
      sipdg_element_own<N, TC, TX, KAP, false>(
          e, x, geo, conn, kap, ops, lambda, ctau, 0, u,
          [&](int i, TC v) {
            buf[i * kPitch + threadIdx.x] = v;
            if (want_dot) dot += static_cast<double>(xe[i]) * static_cast<double>(v);
          },
          [&](int j) { return buf[j * kPitch + threadIdx.x]; });
    }
    __syncthreads();
    if (ne > 0) {
      TY* dst = y + (size_t)e0 * Np;
      for (int t = threadIdx.x; t < ne * Np; t += kBlock) {
        const int le = t / Np, j = t - le * Np;
        dst[t] = static_cast<TY>(buf[j * kPitch + le]);
      }
    }
  } else {
    if (e < K) {
      TC u[Np];
      TY* ye = y + (size_t)e * Np;
      const TX* xe = x + (size_t)e * Np;
      sipdg_element<N, TC, TX, KAP, false>(e, x, geo, conn, kap, ops, lambda, ctau, 0, u,
                                           [&](int i, TC v) {
                                             ye[i] = static_cast<TY>(v);
                                             if (want_dot)
                                               dot += static_cast<double>(xe[i]) * static_cast<double>(v);
                                           });
    }
  }
  if (partials) {
    double v[1] = {dot};
    block_sum<1>(v);
    if (threadIdx.x == 0) partials[blk] = v[0];
  }
}

template <typename TC, typename TX, typename TY, bool KAP, bool STAGE, int WAVES>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WAVES > 0 ? WAVES : 1)))
void k_ax(const TX* __restrict__ x, TY* __restrict__ y, const TC* __restrict__ geo, const Conn* __restrict__ conn,
          const TC* __restrict__ kap, const TC* __restrict__ ops, TC lambda, TC ctau, int K, int per,
          double* __restrict__ partials, const int* __restrict__ skip) {
  ax_body<TC, TX, TY, KAP, STAGE>(x, y, geo, conn, kap, ops, lambda, ctau, K, per, partials, skip, blockIdx.x);
}

// Batched form (many solves of this degree in one launch; variants 0 and 2).
template <typename TC, typename TX, typename TY, bool KAP, int WAVES>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WAVES > 0 ? WAVES : 1)))
void kb_ax(const ElemArgs* __restrict__ tab, const BlockRef* __restrict__ map) {
  const BlockRef m = map[blockIdx.x];
  const ElemArgs& a = tab[m.s];
  ax_body<TC, TX, TY, KAP, false>(in_global(static_cast<const TX*>(a.x)), in_global(static_cast<TY*>(a.y)),
                                  in_global(static_cast<const TC*>(a.geo)), in_global(a.conn),
                                  in_global(static_cast<const TC*>(a.kap)), in_constant(static_cast<const TC*>(a.ops)),
                                  TC(a.lambda), TC(a.ctau), a.K, m.per, in_global(a.partials), in_global(a.skip), m.b);
}

// Waves per SIMD the cooperative kernel's register allocation must leave
// room for (1: no constraint).  FP64 at degrees <= 3 fits five without
// spilling.
template <typename TC>
constexpr int coop_waves() {
  return (sizeof(TC) == 8 && N <= 3) ? 5 : 1;
}

// Cooperative operator (sipdg_coop.hpp): a block of three waves per tile of
// 64 elements; the partial sum of x . y (optional) is one per block.
template <typename TC, typename TX, typename TY, bool KAP>
__device__ __forceinline__ void axc_body(const TX* __restrict__ x, TY* __restrict__ y, const TC* __restrict__ geo,
                                         const Conn* __restrict__ conn, const TC* __restrict__ kap,
                                         const TC* __restrict__ ops, TC lambda, TC ctau, int K, int per,
                                         double* __restrict__ partials, const int* __restrict__ skip, int blk) {
  if (skip && *skip) return;
  using CL = CoopLayout<N>;
  constexpr int Nfp = Tri<N>::Nfp, P = kCoopPitch;
  // degrees >= 5: the row phase on the matrix cores
  constexpr bool kMf = N >= 5;
  __shared__ TC U[Np * P];          // the tile's own values, then its outputs
  __shared__ TC JM[3 * Nfp * P];    // jumps [u]_f at the face nodes
  __shared__ TC TS[3 * Nfp * P];    // J |F|/|E| s_f at the face nodes
  __shared__ TC SC[kMf ? sc_slot::kCount * P : 1];   // per-element row-phase factors
  __shared__ double red[3];
  const int e0 = xcd_tile(blk, per) * kCoopTile;
  const int ne = K - e0 < kCoopTile ? K - e0 : kCoopTile;
  if (ne <= 0) {                    // a block past the last tile (the grid is rounded up)
    if (partials && threadIdx.x == 0) partials[blk] = 0.0;
    return;
  }
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool live = lane < ne;
  // lanes past the mesh's end work on the tile's first element; their
  // results are never stored
  const int e = e0 + (live ? lane : 0);
  CoopElem<TC> el;
  el.rx = geo[4 * e + 0];
  el.sx = geo[4 * e + 1];
  el.ry = geo[4 * e + 2];
  el.sy = geo[4 * e + 3];
  el.ke = KAP ? kap[e] : TC(1);
  el.c = conn[e];
  // wave w's neighbour (across face w), in flight during the staging below
  CoopNbr<N, TC> nb;
  if (w == 0) coop_gather<N, 0, TC, TX, KAP>(el, x, geo, kap, nb);
  else if (w == 1) coop_gather<N, 1, TC, TX, KAP>(el, x, geo, kap, nb);
  else coop_gather<N, 2, TC, TX, KAP>(el, x, geo, kap, nb);
  {
    const TX* __restrict__ src = x + (size_t)e0 * Np;
    for (int t = threadIdx.x; t < ne * Np; t += kCoopThreads) {
      const int le = t / Np, j = t - le * Np;
      U[j * P + le] = static_cast<TC>(src[t]);
    }
  }
  el.J = rcp_pos(el.rx * el.sy - el.sx * el.ry);
  if constexpr (kMf) {
    if (w == 0) coop_factors(el, lambda, SC, lane);
  }
  __syncthreads();
  TC dnj[Nfp], tau, Fs, iFs;
  if (w == 0) coop_face<N, 0, TC, TX>(el, nb, ops, ctau, U, JM, lane, dnj, tau, Fs, iFs);
  else if (w == 1) coop_face<N, 1, TC, TX>(el, nb, ops, ctau, U, JM, lane, dnj, tau, Fs, iFs);
  else coop_face<N, 2, TC, TX>(el, nb, ops, ctau, U, JM, lane, dnj, tau, Fs, iFs);
  // the volume rows after the face phase: the neighbour's values are no
  // longer live
  TC acc[CL::kMaxRows];
  if constexpr (!kMf) {
    phase_fence();
    auto vol = [&](auto lam) {
      constexpr bool LAM = decltype(lam)::value;
      if (w == 0) coop_rows_vol<N, 0, LAM>(el, ops, U, lane, lambda, acc);
      else if (w == 1) coop_rows_vol<N, 1, LAM>(el, ops, U, lane, lambda, acc);
      else coop_rows_vol<N, 2, LAM>(el, ops, U, lane, lambda, acc);
    };
    if (lambda != TC(0)) vol(std::true_type{});
    else vol(std::false_type{});
  }
  __syncthreads();
  const bool want_dot = partials != nullptr;
  double dot = 0.0;
  if constexpr (kMf) {
    typename Mfma<TC>::v4 macc[4];
    auto rows = [&](auto lam) {
      constexpr bool LAM = decltype(lam)::value;
      if (w == 0) {
        coop_lift<N, 0>(el, ops, JM, TS, lane, dnj, tau, Fs, iFs);
        phase_fence();   // keeps the lift's registers apart from the row phase's
        coop_rows_mfma<N, 0, LAM>(ops, U, JM, SC, lane, macc);
      } else if (w == 1) {
        coop_lift<N, 1>(el, ops, JM, TS, lane, dnj, tau, Fs, iFs);
        phase_fence();   // keeps the lift's registers apart from the row phase's
        coop_rows_mfma<N, 1, LAM>(ops, U, JM, SC, lane, macc);
      } else {
        coop_lift<N, 2>(el, ops, JM, TS, lane, dnj, tau, Fs, iFs);
        phase_fence();   // keeps the lift's registers apart from the row phase's
        coop_rows_mfma<N, 2, LAM>(ops, U, JM, SC, lane, macc);
      }
    };
    if (lambda != TC(0)) rows(std::true_type{});
    else rows(std::false_type{});
    __syncthreads();
    if (w == 0) coop_rows_mfma_face<N, 0>(ops, U, TS, lane, ne, macc, want_dot, dot);
    else if (w == 1) coop_rows_mfma_face<N, 1>(ops, U, TS, lane, ne, macc, want_dot, dot);
    else coop_rows_mfma_face<N, 2>(ops, U, TS, lane, ne, macc, want_dot, dot);
    __syncthreads();
    if (w == 0) coop_rows_mfma_store<N, 0>(U, lane, macc);
    else if (w == 1) coop_rows_mfma_store<N, 1>(U, lane, macc);
    else coop_rows_mfma_store<N, 2>(U, lane, macc);
  } else {
    if (w == 0) {
      coop_lift<N, 0>(el, ops, JM, TS, lane, dnj, tau, Fs, iFs);
      coop_rows_jump<N, 0>(el, ops, JM, lane, acc);
    } else if (w == 1) {
      coop_lift<N, 1>(el, ops, JM, TS, lane, dnj, tau, Fs, iFs);
      coop_rows_jump<N, 1>(el, ops, JM, lane, acc);
    } else {
      coop_lift<N, 2>(el, ops, JM, TS, lane, dnj, tau, Fs, iFs);
      coop_rows_jump<N, 2>(el, ops, JM, lane, acc);
    }
    __syncthreads();
    if (w == 0) coop_rows_out<N, 0>(ops, U, TS, lane, acc, want_dot, dot);
    else if (w == 1) coop_rows_out<N, 1>(ops, U, TS, lane, acc, want_dot, dot);
    else coop_rows_out<N, 2>(ops, U, TS, lane, acc, want_dot, dot);
    dot = live ? dot : 0.0;
  }
  if (want_dot) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dot += __shfl_down(dot, off, 64);
    if (lane == 0) red[w] = dot;
  }
  __syncthreads();
  {
    TY* __restrict__ dst = y + (size_t)e0 * Np;
    for (int t = threadIdx.x; t < ne * Np; t += kCoopThreads) {
      const int le = t / Np, j = t - le * Np;
      dst[t] = static_cast<TY>(U[j * P + le]);
    }
  }
  if (want_dot && threadIdx.x == 0) partials[blk] = (red[0] + red[1]) + red[2];
}

template <typename TC, typename TX, typename TY, bool KAP>
__global__ __launch_bounds__(kCoopThreads) __attribute__((amdgpu_waves_per_eu(coop_waves<TC>())))
void k_axc(const TX* __restrict__ x, TY* __restrict__ y, const TC* __restrict__ geo, const Conn* __restrict__ conn,
           const TC* __restrict__ kap, const TC* __restrict__ ops, TC lambda, TC ctau, int K, int per,
           double* __restrict__ partials, const int* __restrict__ skip) {
  axc_body<TC, TX, TY, KAP>(x, y, geo, conn, kap, ops, lambda, ctau, K, per, partials, skip, blockIdx.x);
}

// Batched form (many solves of this degree in one launch).
template <typename TC, typename TX, typename TY, bool KAP>
__global__ __launch_bounds__(kCoopThreads) __attribute__((amdgpu_waves_per_eu(coop_waves<TC>())))
void kb_axc(const ElemArgs* __restrict__ tab, const BlockRef* __restrict__ map) {
  const BlockRef m = map[blockIdx.x];
  const ElemArgs& a = tab[m.s];
  axc_body<TC, TX, TY, KAP>(in_global(static_cast<const TX*>(a.x)), in_global(static_cast<TY*>(a.y)),
                            in_global(static_cast<const TC*>(a.geo)), in_global(a.conn),
                            in_global(static_cast<const TC*>(a.kap)), in_constant(static_cast<const TC*>(a.ops)),
                            TC(a.lambda), TC(a.ctau), a.K, m.per, in_global(a.partials), in_global(a.skip), m.b);
}

template <typename TC, bool KAP>
__global__ __launch_bounds__(kBlock) void k_diag(TC* __restrict__ d, const TC* __restrict__ geo,
                                                 const Conn* __restrict__ conn,
                                                 const TC* __restrict__ kap,
                                                 const TC* __restrict__ ops, TC lambda, TC ctau,
                                                 int K, int per) {
  const int e = xcd_tile(blockIdx.x, per) * kBlock + threadIdx.x;
  if (e >= K) return;
  for (int i = 0; i < Np; ++i) {
    TC u[Np];
    TC di = TC(0);
    sipdg_element<N, TC, TC, KAP, true>(e, static_cast<const TC*>(nullptr), geo, conn, kap, ops,
                                        lambda, ctau, i, u,
                                        [&](int j, TC v) { di = (j == i) ? v : di; });
    d[(size_t)e * Np + i] = di;
  }
}

// y = J M x (INV = false) or y = (J M)^{-1} x (INV = true)
template <typename TC, typename TX, typename TY, bool INV>
__device__ __forceinline__ void mass_body(const TX* __restrict__ x, TY* __restrict__ y, const TC* __restrict__ geo,
                                          const TC* __restrict__ ops, int K, int per, const int* __restrict__ skip,
                                          int blk) {
  if (skip && *skip) return;
  using L = OpsLayout<N>;
  const int e = xcd_tile(blk, per) * kBlock + threadIdx.x;
  if (e >= K) return;
  const TC rx = geo[4 * e + 0], sx = geo[4 * e + 1], ry = geo[4 * e + 2], sy = geo[4 * e + 3];
  const TC det = rx * sy - sx * ry;  // 1 / J
  TC u[Np];
#pragma unroll
  for (int j = 0; j < Np; ++j) u[j] = static_cast<TC>(x[(size_t)e * Np + j]);
#pragma unroll
  for (int i = 0; i < Np; ++i) {
    TC acc = TC(0);
#pragma unroll
    for (int j = 0; j < Np; ++j) acc += ops[(INV ? L::Minv : L::M) + i * Np + j] * u[j];
    y[(size_t)e * Np + i] = static_cast<TY>(INV ? acc * det : acc / det);
  }
}
template <typename TC, typename TX, typename TY, bool INV>
__global__ __launch_bounds__(kBlock) void k_mass(const TX* __restrict__ x, TY* __restrict__ y,
                                                 const TC* __restrict__ geo,
                                                 const TC* __restrict__ ops, int K, int per,
                                                 const int* __restrict__ skip) {
  mass_body<TC, TX, TY, INV>(x, y, geo, ops, K, per, skip, blockIdx.x);
}
template <typename TC, typename TX, typename TY, bool INV>
__global__ __launch_bounds__(kBlock) void kb_mass(const ElemArgs* __restrict__ tab, const BlockRef* __restrict__ map) {
  const BlockRef m = map[blockIdx.x];
  const ElemArgs& a = tab[m.s];
  mass_body<TC, TX, TY, INV>(in_global(static_cast<const TX*>(a.x)), in_global(static_cast<TY*>(a.y)),
                             in_global(static_cast<const TC*>(a.geo)), in_constant(static_cast<const TC*>(a.ops)), a.K,
                             m.per, in_global(a.skip), m.b);
}

// Restriction rc = P^T (f - Az) and prolongation z += P zc per element.
template <int NC, typename T>
__device__ __forceinline__ void restrict_body(const T* __restrict__ f, const T* __restrict__ Az, T* __restrict__ rc,
                                              const T* __restrict__ P, int K, int per, const int* __restrict__ skip,
                                              int blk) {
  if (skip && *skip) return;
  constexpr int Npc = Tri<NC>::Np;
  const int e = xcd_tile(blk, per) * kBlock + threadIdx.x;
  if (e >= K) return;
  T r[Np];
#pragma unroll
  for (int j = 0; j < Np; ++j) r[j] = f[(size_t)e * Np + j] - Az[(size_t)e * Np + j];
#pragma unroll
  for (int c = 0; c < Npc; ++c) {
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < Np; ++j) acc += P[j * Npc + c] * r[j];
    rc[(size_t)e * Npc + c] = acc;
  }
}
template <int NC, typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(const T* __restrict__ f, const T* __restrict__ Az,
                                                     T* __restrict__ rc, const T* __restrict__ P,
                                                     int K, int per, const int* __restrict__ skip) {
  restrict_body<NC, T>(f, Az, rc, P, K, per, skip, blockIdx.x);
}
template <int NC, typename T>
__global__ __launch_bounds__(kBlock) void kb_restrict(const TransferArgs* __restrict__ tab,
                                                      const BlockRef* __restrict__ map) {
  const BlockRef m = map[blockIdx.x];
  const TransferArgs& a = tab[m.s];
  restrict_body<NC, T>(in_global(static_cast<const T*>(a.f)), in_global(static_cast<const T*>(a.Az)),
                       in_global(static_cast<T*>(a.coarse)), in_constant(static_cast<const T*>(a.P)), a.K, m.per,
                       in_global(a.skip), m.b);
}

template <int NC, typename T>
__device__ __forceinline__ void prolong_body(const T* __restrict__ zc, T* __restrict__ z, const T* __restrict__ P,
                                             int K, int per, const int* __restrict__ skip, int blk) {
  if (skip && *skip) return;
  constexpr int Npc = Tri<NC>::Np;
  const int e = xcd_tile(blk, per) * kBlock + threadIdx.x;
  if (e >= K) return;
  T c[Npc];
#pragma unroll
  for (int j = 0; j < Npc; ++j) c[j] = zc[(size_t)e * Npc + j];
#pragma unroll
  for (int i = 0; i < Np; ++i) {
    T acc = z[(size_t)e * Np + i];
#pragma unroll
    for (int j = 0; j < Npc; ++j) acc += P[i * Npc + j] * c[j];
    z[(size_t)e * Np + i] = acc;
  }
}
template <int NC, typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(const T* __restrict__ zc, T* __restrict__ z,
                                                    const T* __restrict__ P, int K, int per,
                                                    const int* __restrict__ skip) {
  prolong_body<NC, T>(zc, z, P, K, per, skip, blockIdx.x);
}
template <int NC, typename T>
__global__ __launch_bounds__(kBlock) void kb_prolong(const TransferArgs* __restrict__ tab,
                                                     const BlockRef* __restrict__ map) {
  const BlockRef m = map[blockIdx.x];
  const TransferArgs& a = tab[m.s];
  prolong_body<NC, T>(in_global(static_cast<const T*>(a.coarse)), in_global(static_cast<T*>(a.fine)),
                      in_constant(static_cast<const T*>(a.P)), a.K, m.per, in_global(a.skip), m.b);
}


// dL/dkappa_e = -w^T (dA/dkappa_e) u for the kappa-weighted form
//   a(u,v) = sum_e k_e (grad u, grad v)_E
//          - sum_F ({k d_n u}, <v>)_F + ({k d_n v}, <u>)_F - tau_F (<u>, <v>)_F
// with <u> = u- - u+ and tau_F = c_tau max(k- Fs-, k+ Fs+); the Dirichlet
// ghost takes k+ = k-.  Per element e:
//   d/dk_e = (grad u, grad w)_E
//          + sum_{interior f} [ -1/2 (d_n u-, <w>)_f - 1/2 (d_n w-, <u>)_f
//                               + dtau_f (<u>, <w>)_f ]
//          + sum_{Dirichlet f} [ -(d_n u, w)_f - (d_n w, u)_f
//                                + 2 c_tau Fs_f (u, w)_f ]
// where dtau_f = c_tau Fs_f when e's side attains the max (ties go to the
// lower element id), else 0.  Face integrals use sJ_f M1D on face nodes.
__global__ __launch_bounds__(kBlock) void k_kgrad(const double* __restrict__ u,
                                                  const double* __restrict__ w,
                                                  double* __restrict__ out,
                                                  const double* __restrict__ geo,
                                                  const Conn* __restrict__ conn,
                                                  const double* __restrict__ kap,
                                                  const double* __restrict__ ops, double ctau,
                                                  int K, int per) {
  using G = Tri<N>;
  using L = OpsLayout<N>;
  constexpr int Nfp = G::Nfp;
  const int e = xcd_tile(blockIdx.x, per) * kBlock + threadIdx.x;
  if (e >= K) return;
  const double rx = geo[4 * e + 0], sx = geo[4 * e + 1], ry = geo[4 * e + 2], sy = geo[4 * e + 3];
  const double J = 1.0 / (rx * sy - sx * ry);
  const double ke = kap[e];
  double ue[Np], we[Np];
#pragma unroll
  for (int j = 0; j < Np; ++j) {
    ue[j] = u[(size_t)e * Np + j];
    we[j] = w[(size_t)e * Np + j];
  }
  double ur[Np], us[Np], wr[Np], ws[Np];
#pragma unroll
  for (int i = 0; i < Np; ++i) {
    double a = 0, b = 0, c = 0, d = 0;
#pragma unroll
    for (int j = 0; j < Np; ++j) {
      a += ops[L::Dr + i * Np + j] * ue[j];
      b += ops[L::Ds + i * Np + j] * ue[j];
      c += ops[L::Dr + i * Np + j] * we[j];
      d += ops[L::Ds + i * Np + j] * we[j];
    }
    ur[i] = a; us[i] = b; wr[i] = c; ws[i] = d;
  }
  const double grr = rx * rx + ry * ry, grs = rx * sx + ry * sy, gss = sx * sx + sy * sy;
  double vol = 0.0;
#pragma unroll
  for (int i = 0; i < Np; ++i) {
    double mwr = 0, mws = 0;
#pragma unroll
    for (int j = 0; j < Np; ++j) {
      mwr += ops[L::M + i * Np + j] * wr[j];
      mws += ops[L::M + i * Np + j] * ws[j];
    }
    vol += grr * ur[i] * mwr + grs * (ur[i] * mws + us[i] * mwr) + gss * us[i] * mws;
  }
  double tot = J * vol;
  const Conn c = conn[e];
  const double gx[3] = {-sx, rx + sx, -rx};
  const double gy[3] = {-sy, ry + sy, -ry};
  static_for<0, 3>([&](auto fc) {
    constexpr int f = decltype(fc)::value;
    const int bc = conn_bc(c.info, f);
    if (bc == 2) return;
    const double Fs = sqrt(gx[f] * gx[f] + gy[f] * gy[f]);
    const double nx = gx[f] / Fs, ny = gy[f] / Fs;
    const double nr = nx * rx + ny * ry, ns = nx * sx + ny * sy;
    const double sJ = Fs * J;
    const int nb = c.nb[f];
    const int fp = conn_fp(c.info, f);
    double du[Nfp], dw[Nfp], ju[Nfp], jw[Nfp];
    static_for<0, Nfp>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      constexpr int vm = G::fm(f, k);
      constexpr int m = Nfp - 1 - k;
      constexpr int o1 = G::rot(1, m), o2 = G::rot(2, m);
      const int o = fp == 0 ? m : (fp == 1 ? o1 : o2);
      du[k] = nr * ur[vm] + ns * us[vm];
      dw[k] = nr * wr[vm] + ns * ws[vm];
      const double up = (bc == 0) ? u[(size_t)nb * Np + o] : -ue[vm];
      const double wp = (bc == 0) ? w[(size_t)nb * Np + o] : -we[vm];
      ju[k] = ue[vm] - up;
      jw[k] = we[vm] - wp;
    });
    double t1 = 0, t2 = 0, t3 = 0;
#pragma unroll
    for (int p = 0; p < Nfp; ++p) {
      double a = 0, b = 0;
#pragma unroll
      for (int k = 0; k < Nfp; ++k) {
        a += ops[L::M1D + p * Nfp + k] * jw[k];
        b += ops[L::M1D + p * Nfp + k] * ju[k];
      }
      t1 += du[p] * a;      // (d_n u, <w>)
      t2 += dw[p] * b;      // (d_n w, <u>)
      t3 += ju[p] * a;      // (<u>, <w>)
    }
    if (bc == 0) {
      // neighbour face scale: grad s' of the neighbour's rotated frame
      const double prx = geo[4 * nb + 0], psx = geo[4 * nb + 1], pry = geo[4 * nb + 2], psy = geo[4 * nb + 3];
      const double qx = -(prx + psx), qy = -(pry + psy);
      const double Sx = fp == 0 ? psx : (fp == 1 ? qx : prx);
      const double Sy = fp == 0 ? psy : (fp == 1 ? qy : pry);
      const double Fsp = sqrt(Sx * Sx + Sy * Sy);
      const double mine = ke * Fs, other = kap[nb] * Fsp;
      const bool owns = mine > other || (mine == other && e < nb);
      const double dtau = owns ? ctau * Fs : 0.0;
      tot += sJ * (-0.5 * t1 - 0.5 * t2 + dtau * t3);
    } else {
      // Dirichlet: <u> = 2u, <w> = 2w on the mirror ghost
      tot += sJ * (-0.5 * t1 - 0.5 * t2 + 0.5 * ctau * Fs * t3);
    }
  });
  out[e] = -tot;
}


// ---------------------------------------------------------------------------
// Persistent Jacobi-PCG of one level (the coarsest level of the p-multigrid
// cycle): textbook PCG from x = 0, all iterations in one launch.
// ---------------------------------------------------------------------------
constexpr unsigned kSpinLimit = 1u << 22;

// Grid-wide barrier: one arrival counter and one generation counter, both
// agent-scope atomics.  The wait is bounded: on timeout the block records the
// failure in status[1] and reports false, so that the kernel still ends.
__device__ bool grid_barrier(unsigned* bar, unsigned nblocks, int* status) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    ok = 1;
    // one agent-scope release fence for this block's writes, relaxed polling,
    // one acquire fence after the wait (an acquire on every poll would
    // invalidate the caches on each turn of the spin)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned prev = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == nblocks - 1) {
      // the last arrival takes in every other block's writes before it
      // releases the waiters
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (++spins > kSpinLimit) {
          ok = 0;
          __hip_atomic_store(&status[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return ok != 0;
}

// Sum slot `slot` of the partials over nblocks entries; every block computes
// the same value in the same order.
__device__ double grid_total(const double* partials, int slot, int nblocks) {
  __shared__ double tot;
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < nblocks; i += kBlock)
    v[0] += __hip_atomic_load(&partials[slot * kMaxPartials + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  block_sum<1>(v);
  if (threadIdx.x == 0) tot = v[0];
  __syncthreads();
  const double t = tot;
  __syncthreads();
  return t;
}

template <int NV>
__device__ void put_partials(double (&v)[NV], double* partials, const int* slots) {
  block_sum<NV>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k)
      __hip_atomic_store(&partials[slots[k] * kMaxPartials + blockIdx.x], v[k], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

template <int NN, typename T, bool KAP>
__global__ __launch_bounds__(kBlock) void k_coarse_pcg(const T* __restrict__ f, T* __restrict__ x,
                                                       T* __restrict__ r, T* __restrict__ z,
                                                       T* __restrict__ p, T* __restrict__ Ap,
                                                       const T* __restrict__ dinv,
                                                       const T* __restrict__ geo,
                                                       const Conn* __restrict__ conn,
                                                       const T* __restrict__ kap,
                                                       const T* __restrict__ ops, T lambda, T ctau,
                                                       int K, double tol, int max_iters,
                                                       double* __restrict__ partials,
                                                       unsigned* __restrict__ bar,
                                                       int* __restrict__ status,
                                                       const int* __restrict__ skip) {
  if (skip && *skip) return;          // the same flag value for every block
  if (blockIdx.x == 0 && threadIdx.x == 0) status[2] = 0;
  constexpr int Np = Tri<NN>::Np;
  const int G = gridDim.x;
  const size_t n = (size_t)K * Np;
  const int ntiles = (K + kBlock - 1) / kBlock;
  const size_t stride = (size_t)G * kBlock;
  // x = 0, r = f, z = D^-1 f, p = z
  {
    double v[2] = {0.0, 0.0};
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += stride) {
      const T fi = f[i];
      const T zi = dinv[i] * fi;
      x[i] = T(0);
      r[i] = fi;
      z[i] = zi;
      p[i] = zi;
      v[0] += double(fi) * double(fi);
      v[1] += double(fi) * double(zi);
    }
    // slots 1, 2: slot 0 is rewritten by the first operator phase, which a
    // fast block may reach while a slow one still reads these totals
    const int sl[2] = {1, 2};
    put_partials<2>(v, partials, sl);
  }
  if (!grid_barrier(bar, G, status)) return;
  const double rr0 = grid_total(partials, 1, G);
  double rz = grid_total(partials, 2, G);
  const double tol2 = tol * tol * rr0;
  int it = 0;
  bool done = !(rr0 > 0.0);
  while (!done && it < max_iters) {
    // Ap = A p, (p, Ap)
    double dot = 0.0;
    for (int t = blockIdx.x; t < ntiles; t += G) {
      const int e = t * kBlock + threadIdx.x;
      if (e < K) {
        T u[Np];
        T* ye = Ap + (size_t)e * Np;
        sipdg_element<NN, T, T, KAP, false>(e, p, geo, conn, kap, ops, lambda, ctau, 0, u,
                                           [&](int i, T vv) {
                                             ye[i] = vv;
                                             dot += double(p[(size_t)e * Np + i]) * double(vv);
                                           });
      }
    }
    {
      double v[1] = {dot};
      const int sl[1] = {0};
      put_partials<1>(v, partials, sl);
    }
    if (!grid_barrier(bar, G, status)) return;
    const double pAp = grid_total(partials, 0, G);
    if (!(pAp > 0.0)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) status[2] = 1;
      break;
    }
    const double alpha = rz / pAp;
    double v[2] = {0.0, 0.0};
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += stride) {
      x[i] += T(alpha) * p[i];
      const T ri = r[i] - T(alpha) * Ap[i];
      r[i] = ri;
      const T zi = dinv[i] * ri;
      z[i] = zi;
      v[0] += double(ri) * double(ri);
      v[1] += double(ri) * double(zi);
    }
    {
      const int sl[2] = {1, 2};
      put_partials<2>(v, partials, sl);
    }
    if (!grid_barrier(bar, G, status)) return;
    const double rr = grid_total(partials, 1, G);
    const double rz_new = grid_total(partials, 2, G);
    ++it;
    if (rr <= tol2) break;
    const double beta = rz_new / rz;
    rz = rz_new;
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += stride)
      p[i] = z[i] + T(beta) * p[i];
    if (!grid_barrier(bar, G, status)) return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) status[0] = it;
}

// Slots 0, 1, 2 of the partials summed over n0, n1, n2 entries (each at most
// kMaxPartials), returned to every thread (the same values and order in every
// block).  Every entry below the largest count is read unconditionally (the
// slots are kMaxPartials long) and masked by a select, two strides per trip,
// so that a thread's loads are all in flight before the first is waited on.
__device__ void slot_totals3(const double* __restrict__ partials, int n0, int n1, int n2, double (&t)[3]) {
  __shared__ double tot[3];
  double v[3] = {0.0, 0.0, 0.0};
  const int nm = n0 > n1 ? (n0 > n2 ? n0 : n2) : (n1 > n2 ? n1 : n2);
  for (int i = threadIdx.x; i < nm; i += 2 * kBlock) {
    const int j = i + kBlock < nm ? i + kBlock : i;
    const double a0 = partials[i], a1 = partials[kMaxPartials + i], a2 = partials[2 * kMaxPartials + i];
    const double b0 = partials[j], b1 = partials[kMaxPartials + j], b2 = partials[2 * kMaxPartials + j];
    const bool two = j != i;
    v[0] += (i < n0 ? a0 : 0.0) + (two && j < n0 ? b0 : 0.0);
    v[1] += (i < n1 ? a1 : 0.0) + (two && j < n1 ? b1 : 0.0);
    v[2] += (i < n2 ? a2 : 0.0) + (two && j < n2 ? b2 : 0.0);
  }
  block_sum<3>(v);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) tot[k] = v[k];
  __syncthreads();
  for (int k = 0; k < 3; ++k) t[k] = tot[k];
  __syncthreads();
}

// Coarse Jacobi-PCG in the single-reduction form of Chronopoulos and Gear
// (1989): with u = D^-1 r and w = A u, the recurrences
//   p = u + beta p,  s = w + beta s (= A p),  x += alpha p,  r -= alpha s,
//   u = D^-1 r,  w = A u,  gamma = (r, u),  delta = (w, u),
//   beta = gamma / gamma_prev,  alpha = gamma / (delta - beta gamma / alpha_prev)
// are textbook PCG rearranged so that one iteration needs one global
// reduction: one launch per iteration.  The launch reads the reductions of
// the previous one, updates its own elements and applies the operator to
// the new u; the new u of a neighbour is formed on the fly from that
// neighbour's previous r, w and s, which are double-buffered by iteration
// parity (the launch writes the other copy).

// u_new = D^-1 (r - alpha (w + beta s)) of any node, from the previous state
template <typename T>
struct NextUSrc {
  const T* __restrict__ dinv;
  const T* __restrict__ r;
  const T* __restrict__ w;
  const T* __restrict__ s;
  T alpha, beta;
  bool first;   // s = w
  __device__ __forceinline__ T operator()(size_t i) const {
    const T si = first ? w[i] : w[i] + beta * s[i];
    return dinv[i] * (r[i] - alpha * si);
  }
};

// The same values for the three neighbours, face by face in the element
// template's rotated order, formed from raw values loaded in advance.
template <typename T>
struct NextUFaces {
  static constexpr bool kPerFace = true;
  T v[3][Np];
  T m[4][5];   // metric (r_x, s_x, r_y, s_y) and coefficient: the element's, then
               // face 0, 1, 2's neighbour's
  template <int f, int j>
  __device__ __forceinline__ T at() const { return v[f][j]; }
  __device__ __forceinline__ T own_metric(int k) const { return m[0][k]; }
  template <int f>
  __device__ __forceinline__ T nbr_metric(int k) const { return m[1 + f][k]; }
};

// Low degrees load the neighbours' raw r, w, s, D^-1 before the reduction too
// (4 x 3 Np values per lane); higher degrees read them after it.
constexpr bool kCoarsePrefetch = N <= 2;

// BATCH: the concatenated coarsest levels of a batch of solves; each block
// belongs to one solve (tile_solve), whose constants, scalars, partial-sum
// range and done flag it uses.  Otherwise K, lambda, ctau, sc, outer and the
// partial counts describe the one level.
template <typename T, bool KAP, bool BATCH>
__global__ __launch_bounds__(kBlock) void k_coarse_cgcg(
    T* __restrict__ x, T* __restrict__ p, T* __restrict__ u, const T* __restrict__ dinv,
    const T* __restrict__ r_old, T* __restrict__ r_new, const T* __restrict__ w_old, T* __restrict__ w_new,
    const T* __restrict__ s_old, T* __restrict__ s_new, const T* __restrict__ geo,
    const Conn* __restrict__ conn, const T* __restrict__ kap, const T* __restrict__ ops, T lambda, T ctau,
    int K, int per, const double* __restrict__ pin, int n_rr, int n_g, int n_d, double* __restrict__ pout,
    CGScal* __restrict__ sc, const int* __restrict__ outer, int it,
    const CoarseBatchEntry* __restrict__ ent, const int* __restrict__ tile_solve) {
  const bool first = it == 0;
  const int par = it & 1;
  const int tile = xcd_tile(blockIdx.x, per);
  int base = 0, ltile = tile, slot = blockIdx.x;
  bool lead = blockIdx.x == 0;
  if constexpr (BATCH) {
    const int si = tile_solve[tile];
    if (si < 0) return;
    const CoarseBatchEntry& d = ent[si];
    base = d.off;
    K = d.K;
    ltile = tile - d.tile0;
    lead = ltile == 0;
    slot = tile;
    lambda = T(d.lambda);
    ctau = T(d.ctau);
    outer = d.outer;
    sc += si;
    pin += d.tile0;
    n_rr = n_g = n_d = d.ntiles;
  }
  const bool b0 = lead && threadIdx.x == 0;
  // true: this launch has nothing to do (the outer solve, or this coarse
  // solve, is finished)
  auto finished = [&]() -> bool {
    if (first) {
      if (outer && *outer) {             // outer solve finished: keep the last record
        if (b0) sc->done = 1;
        return true;
      }
      return false;
    }
    return sc->done != 0;
  };
  // In a batch many members finish their coarse solve early: test first.
  if constexpr (BATCH) {
    if (finished()) return;
  }
  // The element's own state does not depend on alpha and beta: its loads
  // are issued before the reduction (and, for one solve, before the done
  // test) so that the latencies overlap.
  const bool live = ltile * kBlock + (int)threadIdx.x < K;
  const int e = base + ltile * kBlock + threadIdx.x;   // element (global id in a batch)
  const size_t o = (size_t)(live ? e : 0) * Np;
  T r0[Np], w0[Np], s0[Np], d0[Np], p0[Np], x0[Np], u0[Np];
  if (live) {
#pragma unroll
    for (int j = 0; j < Np; ++j) {
      r0[j] = r_old[o + j];
      w0[j] = w_old[o + j];
      d0[j] = dinv[o + j];
      x0[j] = x[o + j];
      u0[j] = u[o + j];
      s0[j] = s_old[o + j];   // unused (and possibly unset) at it = 0
      p0[j] = p[o + j];
    }
  }
  T nd[3][Np], nr[3][Np], nw[3][Np], ns[3][Np];
  NextUFaces<T> pre;
  if constexpr (kCoarsePrefetch) {
    if (live) {
      // (the connectivity is read again by the element computation: this
      // load leaves it in cache)
      const Conn c = conn[e];
      auto metric = [&](int el, T (&mm)[5]) {
        for (int k = 0; k < 4; ++k) mm[k] = geo[4 * el + k];
        mm[4] = KAP ? kap[el] : T(1);
      };
      metric(e, pre.m[0]);
      for (int f = 0; f < 3; ++f) metric(c.nb[f], pre.m[1 + f]);
      static_for<0, 3>([&](auto fc) {
        constexpr int f = decltype(fc)::value;
        const int fp = conn_fp(c.info, f);
        const size_t xn = (size_t)c.nb[f] * Np;
        static_for<0, Np>([&](auto jc) {
          constexpr int j = decltype(jc)::value;
          constexpr int o1 = Tri<N>::rot(1, j), o2 = Tri<N>::rot(2, j);
          const size_t i = xn + (fp == 0 ? j : (fp == 1 ? o1 : o2));
          nd[f][j] = dinv[i];
          nr[f][j] = r_old[i];
          nw[f][j] = w_old[i];
          ns[f][j] = s_old[i];
        });
      });
    }
  }
  if constexpr (!BATCH) {
    if (finished()) return;
  }
  double tot[3];
  slot_totals3(pin, n_rr, n_g, n_d, tot);
  const double rr = tot[0], gam = tot[1], del = tot[2];
  double alpha, beta = 0.0;
  if (first) {
    const bool stop = !(rr > 0.0) || sc->max_iters <= 0;
    alpha = gam / del;
    const bool bad = !stop && !(del > 0.0 && isfinite(alpha));
    if (b0) {
      sc->tol2 = sc->tol * sc->tol * rr;
      sc->rr = rr;
      sc->iters = 0;
      sc->breakdown = bad ? 1 : 0;
      sc->done = (stop || bad) ? 1 : 0;
      sc->rzb[par] = gam;
      sc->ab[par] = alpha;
    }
    if (stop || bad) return;
  } else {
    const bool stop = rr <= sc->tol2 || !isfinite(rr);
    beta = gam / sc->rzb[1 - par];
    const double den = del - beta * gam / sc->ab[1 - par];
    alpha = gam / den;
    const bool bad = !stop && !(den > 0.0 && isfinite(alpha));
    if (b0) {
      sc->rr = rr;
      sc->rzb[par] = gam;
      sc->ab[par] = alpha;
      if (bad) sc->breakdown = 1;
      if (stop || bad) sc->done = 1;
    }
    if (stop || bad) return;
  }
  if (b0) sc->iters = it + 1;
  const T a = static_cast<T>(alpha), b = static_cast<T>(beta);
  double v[3] = {0.0, 0.0, 0.0};
  if (live) {
    T ue[Np], rn[Np];
    auto run = [&](const auto& src) {
      sipdg_element_src<N, T, KAP, false>(
        e, src, geo, conn, kap, ops, lambda, ctau, 0, ue,
        [&](int i, T wi) {
          w_new[o + i] = wi;
          const double ri = double(rn[i]), ui = double(ue[i]);
          v[0] += ri * ri;
          v[1] += ri * ui;
          v[2] += double(wi) * ui;
        },
        [&](int j) {
          const size_t k = o + j;
          const T pj = first ? u0[j] : u0[j] + b * p0[j];
          const T sj = first ? w0[j] : w0[j] + b * s0[j];
          p[k] = pj;
          s_new[k] = sj;
          x[k] = x0[j] + a * pj;
          const T rj = r0[j] - a * sj;
          r_new[k] = rj;
          rn[j] = rj;
          const T uj = d0[j] * rj;
          u[k] = uj;
          return uj;
        });
    };
    if constexpr (kCoarsePrefetch) {
#pragma unroll
      for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int j = 0; j < Np; ++j) {
          const T sj = first ? nw[f][j] : nw[f][j] + b * ns[f][j];
          pre.v[f][j] = nd[f][j] * (nr[f][j] - a * sj);
        }
      run(pre);
    } else {
      run(NextUSrc<T>{dinv, r_old, w_old, s_old, a, b, first});
    }
  }
  block_sum<3>(v);
  if (threadIdx.x == 0) {
    pout[0 * kMaxPartials + slot] = v[0];
    pout[1 * kMaxPartials + slot] = v[1];
    pout[2 * kMaxPartials + slot] = v[2];
  }
}

// u = D^-1 f of any node of a batch solve's level, read from that solve's own
// right-hand side (element ids are global, f is indexed from the solve's first)
template <typename T>
struct DinvRhsSrc {
  const T* __restrict__ dinv;
  const T* __restrict__ f;
  size_t base;   // first node of the solve
  __device__ __forceinline__ T operator()(size_t i) const { return dinv[i] * f[i - base]; }
};

// Start of the batched coarse solves: x = 0, r = f, u = D^-1 r, w = A u and
// the block partials of (r, r), (r, u), (u, w) in the solve's tile slots.
template <typename T, bool KAP>
__global__ __launch_bounds__(kBlock) void k_coarse_binit(
    T* __restrict__ x, T* __restrict__ u, const T* __restrict__ dinv, T* __restrict__ r, T* __restrict__ w,
    const T* __restrict__ geo, const Conn* __restrict__ conn, const T* __restrict__ kap,
    const T* __restrict__ ops, int per, double* __restrict__ pout, const CoarseBatchEntry* __restrict__ ent,
    const int* __restrict__ tile_solve) {
  const int tile = xcd_tile(blockIdx.x, per);
  const int si = tile_solve[tile];
  if (si < 0) return;
  const CoarseBatchEntry& d = ent[si];
  if (d.outer && *d.outer) return;   // the first iteration then marks the solve done
  const int ltile = tile - d.tile0;
  const bool live = ltile * kBlock + (int)threadIdx.x < d.K;
  const int e = d.off + ltile * kBlock + threadIdx.x;
  const size_t o = (size_t)e * Np, base = (size_t)d.off * Np;
  const T* __restrict__ f = static_cast<const T*>(d.f);
  double v[3] = {0.0, 0.0, 0.0};
  if (live) {
    T ue[Np], fe[Np];
#pragma unroll
    for (int j = 0; j < Np; ++j) fe[j] = f[o - base + j];
    sipdg_element_src<N, T, KAP, false>(
        e, DinvRhsSrc<T>{dinv, f, base}, geo, conn, kap, ops, T(d.lambda), T(d.ctau), 0, ue,
        [&](int i, T wi) {
          w[o + i] = wi;
          v[0] += double(fe[i]) * double(fe[i]);
          v[1] += double(fe[i]) * double(ue[i]);
          v[2] += double(wi) * double(ue[i]);
        },
        [&](int j) {
          const T uj = dinv[o + j] * fe[j];
          x[o + j] = T(0);
          r[o + j] = fe[j];
          u[o + j] = uj;
          return uj;
        });
  }
  block_sum<3>(v);
  if (threadIdx.x == 0) {
    pout[0 * kMaxPartials + tile] = v[0];
    pout[1 * kMaxPartials + tile] = v[1];
    pout[2 * kMaxPartials + tile] = v[2];
  }
}

// End of the batched coarse solves: each unfinished solve's x to its own z.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_bscatter(const T* __restrict__ x, int per,
                                                            const CoarseBatchEntry* __restrict__ ent,
                                                            const int* __restrict__ tile_solve) {
  const int tile = xcd_tile(blockIdx.x, per);
  const int si = tile_solve[tile];
  if (si < 0) return;
  const CoarseBatchEntry& d = ent[si];
  if (d.outer && *d.outer) return;
  const int le = (tile - d.tile0) * kBlock + threadIdx.x;
  if (le >= d.K) return;
  T* __restrict__ z = static_cast<T*>(d.z);
  const size_t o = (size_t)(d.off + le) * Np;
#pragma unroll
  for (int j = 0; j < Np; ++j) z[(size_t)le * Np + j] = x[o + j];
}

template <typename T>
hipError_t run_coarse_batch(const CoarseBatchArgs& a, int it, hipStream_t s) {
  if (a.grid == 0) return hipSuccess;
  if (it == -2) {
    hipLaunchKernelGGL(k_coarse_bscatter<T>, dim3(a.grid), dim3(kBlock), 0, s, (const T*)a.x, a.per, a.ent,
                       a.tile_solve);
    return hipGetLastError();
  }
  double* set0 = a.partials;
  double* set1 = a.partials + 3 * (size_t)kMaxPartials;
  if (it == -1) {
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(a.grid), dim3(kBlock), 0, s, (T*)a.x, (T*)a.u, (const T*)a.dinv, (T*)a.r[0],
                         (T*)a.w[0], (const T*)a.geo, a.conn, (const T*)a.kap, (const T*)a.ops, a.per, set0, a.ent,
                         a.tile_solve);
    };
    if (a.kap) go(k_coarse_binit<T, true>);
    else go(k_coarse_binit<T, false>);
    return hipGetLastError();
  }
  const int o = it & 1, nw = 1 - o;
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(a.grid), dim3(kBlock), 0, s, (T*)a.x, (T*)a.p, (T*)a.u, (const T*)a.dinv,
                       (const T*)a.r[o], (T*)a.r[nw], (const T*)a.w[o], (T*)a.w[nw], (const T*)a.s[o],
                       (T*)a.s[nw], (const T*)a.geo, a.conn, (const T*)a.kap, (const T*)a.ops, T(0), T(0), 0,
                       a.per, o ? set1 : set0, 0, 0, 0, o ? set0 : set1, a.sc, nullptr, it, a.ent, a.tile_solve);
  };
  if (a.kap) go(k_coarse_cgcg<T, true, true>);
  else go(k_coarse_cgcg<T, false, true>);
  return hipGetLastError();
}

template <typename T>
hipError_t run_coarse_step(const CoarseStepArgs& a, hipStream_t s) {
  const ElemArgs& o = a.op;
  int per;
  const int grid = xcd_grid(elem_tiles(o.K), per);
  if (o.K == 0) return hipSuccess;
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, (T*)a.x, (T*)a.p, (T*)a.u, (const T*)a.dinv,
                       (const T*)a.r_old, (T*)a.r_new, (const T*)a.w_old, (T*)a.w_new, (const T*)a.s_old,
                       (T*)a.s_new, (const T*)o.geo, o.conn, (const T*)o.kap, (const T*)o.ops, T(o.lambda),
                       T(o.ctau), o.K, per, a.pin, a.n_rr, a.n_g, a.n_d, a.pout, a.sc, a.outer, a.it, nullptr,
                       nullptr);
  };
  if (o.kap) go(k_coarse_cgcg<T, true, false>);
  else go(k_coarse_cgcg<T, false, false>);
  return hipGetLastError();
}

template <int NN, typename T>
hipError_t run_coarse(const CoarseArgs& a, int grid, hipStream_t s) {
  const ElemArgs& o = a.op;
  if (o.kap)
    hipLaunchKernelGGL((k_coarse_pcg<NN, T, true>), dim3(grid), dim3(kBlock), 0, s,
                       (const T*)a.f, (T*)a.x, (T*)a.r, (T*)a.z, (T*)a.p, (T*)a.Ap, (const T*)a.dinv,
                       (const T*)o.geo, o.conn, (const T*)o.kap, (const T*)o.ops, T(o.lambda), T(o.ctau),
                       o.K, a.tol, a.max_iters, a.partials, a.bar, a.status, a.skip);
  else
    hipLaunchKernelGGL((k_coarse_pcg<NN, T, false>), dim3(grid), dim3(kBlock), 0, s,
                       (const T*)a.f, (T*)a.x, (T*)a.r, (T*)a.z, (T*)a.p, (T*)a.Ap, (const T*)a.dinv,
                       (const T*)o.geo, o.conn, (const T*)o.kap, (const T*)o.ops, T(o.lambda), T(o.ctau),
                       o.K, a.tol, a.max_iters, a.partials, a.bar, a.status, a.skip);
  return hipGetLastError();
}

template <int NN, typename T>
int resident_grid(int K) {
  int dev = 0, cus = 0, per_cu = 0, per_cu_k = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_coarse_pcg<NN, T, false>, kBlock, 0) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_k, (const void*)k_coarse_pcg<NN, T, true>, kBlock, 0) != hipSuccess)
    return 0;
  const int resident = cus * std::min(per_cu, per_cu_k);
  const int tiles = (K + kBlock - 1) / kBlock;
  const int g = std::min(resident, tiles);
  return g > kMaxPartialsCoarse ? kMaxPartialsCoarse : g;
}

// the LDS-staged variant exists at every degree (at N = 8, FP64, its buffer
// is 92 KB: one block per CU, the occupancy the register use allows anyway);
// the raised-occupancy variants at degrees <= 5
constexpr bool kHasBoost = N <= 5;

template <typename TC, typename TX, typename TY, bool KAP, bool STAGE, int WAVES>
void launch_ax_variant(const ElemArgs& a, int grid, int per, hipStream_t s) {
  hipLaunchKernelGGL((k_ax<TC, TX, TY, KAP, STAGE, WAVES>), dim3(grid), dim3(kBlock), 0, s,
                     static_cast<const TX*>(a.x), static_cast<TY*>(a.y),
                     static_cast<const TC*>(a.geo), a.conn, static_cast<const TC*>(a.kap),
                     static_cast<const TC*>(a.ops), TC(a.lambda), TC(a.ctau), a.K, per, a.partials,
                     a.skip);
}

template <typename TC, typename TX, typename TY>
hipError_t run_ax(const ElemArgs& a, hipStream_t s) {
  if (a.K == 0) return hipSuccess;
  // variant 4: the cooperative kernel; bits of variants 0..3: 1 = LDS-staged
  // inputs/outputs, 2 = raised occupancy
  const int v = ax_variant(N, sizeof(TC) == 4);
  if (v == kAxCoop) {
    int per;
    const int grid = xcd_grid((a.K + kCoopTile - 1) / kCoopTile, per);
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(grid), dim3(kCoopThreads), 0, s, static_cast<const TX*>(a.x),
                         static_cast<TY*>(a.y), static_cast<const TC*>(a.geo), a.conn,
                         static_cast<const TC*>(a.kap), static_cast<const TC*>(a.ops), TC(a.lambda),
                         TC(a.ctau), a.K, per, a.partials, a.skip);
    };
    if (a.kap) go(k_axc<TC, TX, TY, true>);
    else go(k_axc<TC, TX, TY, false>);
    return hipGetLastError();
  }
  int per;
  const int grid = xcd_grid(elem_tiles(a.K), per);
  constexpr int W = ax_boost_waves<TC>();
  if ((v & 3) == 1) {
    if (a.kap) launch_ax_variant<TC, TX, TY, true, true, 0>(a, grid, per, s);
    else launch_ax_variant<TC, TX, TY, false, true, 0>(a, grid, per, s);
    return hipGetLastError();
  }
  if constexpr (kHasBoost) {
    switch (v & 3) {
      case 2:
        if (a.kap) launch_ax_variant<TC, TX, TY, true, false, W>(a, grid, per, s);
        else launch_ax_variant<TC, TX, TY, false, false, W>(a, grid, per, s);
        return hipGetLastError();
      case 3:
        if (a.kap) launch_ax_variant<TC, TX, TY, true, true, W>(a, grid, per, s);
        else launch_ax_variant<TC, TX, TY, false, true, W>(a, grid, per, s);
        return hipGetLastError();
      default:
        break;
    }
  }
  if (a.kap) launch_ax_variant<TC, TX, TY, true, false, 0>(a, grid, per, s);
  else launch_ax_variant<TC, TX, TY, false, false, 0>(a, grid, per, s);
  return hipGetLastError();
}

template <typename TC>
hipError_t run_diag(const ElemArgs& a, hipStream_t s) {
  int per;
  const int grid = xcd_grid(elem_tiles(a.K), per);
  if (a.K == 0) return hipSuccess;
  if (a.kap)
    hipLaunchKernelGGL((k_diag<TC, true>), dim3(grid), dim3(kBlock), 0, s, static_cast<TC*>(a.y),
                       static_cast<const TC*>(a.geo), a.conn, static_cast<const TC*>(a.kap),
                       static_cast<const TC*>(a.ops), TC(a.lambda), TC(a.ctau), a.K, per);
  else
    hipLaunchKernelGGL((k_diag<TC, false>), dim3(grid), dim3(kBlock), 0, s, static_cast<TC*>(a.y),
                       static_cast<const TC*>(a.geo), a.conn, static_cast<const TC*>(a.kap),
                       static_cast<const TC*>(a.ops), TC(a.lambda), TC(a.ctau), a.K, per);
  return hipGetLastError();
}

template <typename TC, typename TX, typename TY, bool INV>
hipError_t run_mass(const ElemArgs& a, hipStream_t s) {
  int per;
  const int grid = xcd_grid(elem_tiles(a.K), per);
  if (a.K == 0) return hipSuccess;
  hipLaunchKernelGGL((k_mass<TC, TX, TY, INV>), dim3(grid), dim3(kBlock), 0, s,
                     static_cast<const TX*>(a.x), static_cast<TY*>(a.y),
                     static_cast<const TC*>(a.geo), static_cast<const TC*>(a.ops), a.K, per, a.skip);
  return hipGetLastError();
}

template <int NC, typename T>
hipError_t run_restrict(const TransferArgs& a, hipStream_t s) {
  int per;
  const int grid = xcd_grid(elem_tiles(a.K), per);
  if (a.K == 0) return hipSuccess;
  hipLaunchKernelGGL((k_restrict<NC, T>), dim3(grid), dim3(kBlock), 0, s,
                     static_cast<const T*>(a.f), static_cast<const T*>(a.Az),
                     static_cast<T*>(a.coarse), static_cast<const T*>(a.P), a.K, per, a.skip);
  return hipGetLastError();
}

template <int NC, typename T>
hipError_t run_prolong(const TransferArgs& a, hipStream_t s) {
  int per;
  const int grid = xcd_grid(elem_tiles(a.K), per);
  if (a.K == 0) return hipSuccess;
  hipLaunchKernelGGL((k_prolong<NC, T>), dim3(grid), dim3(kBlock), 0, s,
                     static_cast<const T*>(a.coarse), static_cast<T*>(a.fine),
                     static_cast<const T*>(a.P), a.K, per, a.skip);
  return hipGetLastError();
}

template <int NC>
hipError_t transfer_dispatch(bool restrict_op, Kind kind, const TransferArgs& a, hipStream_t s) {
  if (kind == Kind::F64)
    return restrict_op ? run_restrict<NC, double>(a, s) : run_prolong<NC, double>(a, s);
  return restrict_op ? run_restrict<NC, float>(a, s) : run_prolong<NC, float>(a, s);
}

hipError_t transfer(int Nc, bool restrict_op, Kind kind, const TransferArgs& a, hipStream_t s) {
  if (Nc >= N || Nc < 1) return hipErrorInvalidValue;
  switch (Nc) {
#define IPDG_TCASE(c) \
  case c:             \
    if constexpr (c < N) return transfer_dispatch<c>(restrict_op, kind, a, s); \
    break;
    IPDG_TCASE(1) IPDG_TCASE(2) IPDG_TCASE(3) IPDG_TCASE(4) IPDG_TCASE(5) IPDG_TCASE(6) IPDG_TCASE(7)
#undef IPDG_TCASE
  }
  return hipErrorInvalidValue;
}

}  // namespace

template <>
hipError_t launch_ax<N>(Kind kind, const ElemArgs& a, hipStream_t s) {
  switch (kind) {
    case Kind::F64: return run_ax<double, double, double>(a, s);
    case Kind::F32: return run_ax<float, float, float>(a, s);
    case Kind::F32_IN64: break;   // not used: operators read their own precision
  }
  return hipErrorInvalidValue;
}

template <>
hipError_t launch_coarse_step<N>(Kind kind, const CoarseStepArgs& a, hipStream_t s) {
  return kind == Kind::F64 ? run_coarse_step<double>(a, s) : run_coarse_step<float>(a, s);
}

template <>
hipError_t launch_coarse_batch<N>(Kind kind, const CoarseBatchArgs& a, int it, hipStream_t s) {
  return kind == Kind::F64 ? run_coarse_batch<double>(a, it, s) : run_coarse_batch<float>(a, it, s);
}

template <>
hipError_t launch_diag<N>(Kind kind, const ElemArgs& a, hipStream_t s) {
  return kind == Kind::F64 ? run_diag<double>(a, s) : run_diag<float>(a, s);
}

template <>
hipError_t launch_mass<N>(Kind kind, const ElemArgs& a, hipStream_t s) {
  switch (kind) {
    case Kind::F64: return run_mass<double, double, double, false>(a, s);
    case Kind::F32: return run_mass<float, float, float, false>(a, s);
    case Kind::F32_IN64: return run_mass<float, double, float, false>(a, s);
  }
  return hipErrorInvalidValue;
}

template <>
hipError_t launch_minv<N>(Kind kind, const ElemArgs& a, hipStream_t s) {
  switch (kind) {
    case Kind::F64: return run_mass<double, double, double, true>(a, s);
    case Kind::F32: return run_mass<float, float, float, true>(a, s);
    case Kind::F32_IN64: return run_mass<float, double, float, true>(a, s);
  }
  return hipErrorInvalidValue;
}

template <>
hipError_t launch_kgrad<N>(const KgradArgs& a, hipStream_t s) {
  int per;
  const int grid = xcd_grid(elem_tiles(a.K), per);
  if (a.K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_kgrad, dim3(grid), dim3(kBlock), 0, s, a.u, a.w, a.out, a.geo, a.conn, a.kap,
                     a.ops, a.ctau, a.K, per);
  return hipGetLastError();
}

template <int NN>
hipError_t coarse_impl(Kind kind, const CoarseArgs& a, int grid, hipStream_t s) {
  if constexpr (NN <= 4) {
    if (grid < 1) return hipErrorInvalidValue;
    return kind == Kind::F64 ? run_coarse<NN, double>(a, grid, s) : run_coarse<NN, float>(a, grid, s);
  } else {
    return hipErrorNotSupported;
  }
}

template <int NN>
int coarse_grid_impl(Kind kind, int K) {
  if constexpr (NN <= 4) {
    return kind == Kind::F64 ? resident_grid<NN, double>(K) : resident_grid<NN, float>(K);
  } else {
    return 0;
  }
}

template <>
hipError_t launch_coarse_pcg<N>(Kind kind, const CoarseArgs& a, int grid, hipStream_t s) {
  return coarse_impl<N>(kind, a, grid, s);
}

template <>
int coarse_pcg_grid<N>(Kind kind, int K) {
  return coarse_grid_impl<N>(kind, K);
}

template <>
hipError_t launch_restrict<N>(int Nc, Kind kind, const TransferArgs& a, hipStream_t s) {
  return transfer(Nc, true, kind, a, s);
}

template <>
hipError_t launch_prolong<N>(int Nc, Kind kind, const TransferArgs& a, hipStream_t s) {
  return transfer(Nc, false, kind, a, s);
}

template <>
hipError_t launch_ax_batch<N>(Kind kind, bool kap, int variant, const ElemArgs* tab, const BlockRef* map, int nblocks,
                              hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (!ax_batch_variant(variant) || !ax_variant_exists(N, variant)) return hipErrorInvalidValue;
  auto go = [&](auto kern, int threads) {
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(threads), 0, s, tab, map);
    return hipGetLastError();
  };
  // the element-per-lane kernel at the variant's occupancy (variant 2 =
  // raised occupancy, where the degree has it)
  auto lane = [&](auto tc, auto kp) {
    using TC = decltype(tc);
    constexpr bool KP = decltype(kp)::value;
    if constexpr (kHasBoost && ax_boost_waves<TC>() > 0) {
      if (variant == 2) return go(kb_ax<TC, TC, TC, KP, ax_boost_waves<TC>()>, kBlock);
    }
    return go(kb_ax<TC, TC, TC, KP, 0>, kBlock);
  };
  auto one = [&](auto tc) {
    using TC = decltype(tc);
    if (variant == kAxCoop) {
      if (kap) return go(kb_axc<TC, TC, TC, true>, kCoopThreads);
      return go(kb_axc<TC, TC, TC, false>, kCoopThreads);
    }
    if (kap) return lane(tc, std::true_type{});
    return lane(tc, std::false_type{});
  };
  if (kind == Kind::F64) return one(double{});
  if (kind == Kind::F32) return one(float{});
  return hipErrorInvalidValue;
}

template <>
hipError_t launch_minv_batch<N>(Kind kind, const ElemArgs* tab, const BlockRef* map, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  switch (kind) {
    case Kind::F64:
      hipLaunchKernelGGL((kb_mass<double, double, double, true>), dim3(nblocks), dim3(kBlock), 0, s, tab, map);
      break;
    case Kind::F32:
      hipLaunchKernelGGL((kb_mass<float, float, float, true>), dim3(nblocks), dim3(kBlock), 0, s, tab, map);
      break;
    case Kind::F32_IN64:
      hipLaunchKernelGGL((kb_mass<float, double, float, true>), dim3(nblocks), dim3(kBlock), 0, s, tab, map);
      break;
  }
  return hipGetLastError();
}

template <>
hipError_t launch_transfer_batch<N>(int Nc, bool restrict_op, Kind kind, const TransferArgs* tab, const BlockRef* map,
                                    int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (Nc >= N || Nc < 1) return hipErrorInvalidValue;
  auto go = [&](auto nc) -> hipError_t {
    constexpr int NCC = decltype(nc)::value;
    if constexpr (NCC < N) {
      if (kind == Kind::F64) {
        if (restrict_op) hipLaunchKernelGGL((kb_restrict<NCC, double>), dim3(nblocks), dim3(kBlock), 0, s, tab, map);
        else hipLaunchKernelGGL((kb_prolong<NCC, double>), dim3(nblocks), dim3(kBlock), 0, s, tab, map);
      } else {
        if (restrict_op) hipLaunchKernelGGL((kb_restrict<NCC, float>), dim3(nblocks), dim3(kBlock), 0, s, tab, map);
        else hipLaunchKernelGGL((kb_prolong<NCC, float>), dim3(nblocks), dim3(kBlock), 0, s, tab, map);
      }
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  };
  switch (Nc) {
    case 1: return go(std::integral_constant<int, 1>{});
    case 2: return go(std::integral_constant<int, 2>{});
    case 3: return go(std::integral_constant<int, 3>{});
    case 4: return go(std::integral_constant<int, 4>{});
    case 5: return go(std::integral_constant<int, 5>{});
    case 6: return go(std::integral_constant<int, 6>{});
    case 7: return go(std::integral_constant<int, 7>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ipdg
