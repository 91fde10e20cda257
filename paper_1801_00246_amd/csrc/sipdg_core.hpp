// One-element evaluation of the SIPDG screened-Poisson operator.
//
// For element e (Sec. 5.2, Eq. ellipticOp3, with the reference-element
// factorisation of Eq. elementOps; the jump is [u] = u+ - u-):
//
//   y_e = -J k_e (S_r a + S_s b) + lambda J M u - sum_f sJ_f M1D s_f
//   a = grad r . q,  b = grad s . q,   q = grad u + l,
//   l   = 1/2 sum_f n_f Fs_f L^f [u]_f          (lifted jump, vector field)
//   s_f = 1/2 [k d_n u]_f + tau_f [u]_f - k_e n_f . l   (at face-f nodes)
//
// with S_r = M D_r, S_s = M D_s, L^f the lift of face f, Fs_f = |F|/|E| and
// sJ_f = Fs_f J.  The paper's kernel pseudo-code takes the same steps (local
// gradient, lifted jumps, volume term, surface term, lift, mass) in two
// kernels; here they are fused into one pass over the element and its three
// neighbours.  Because the metric is constant per element, S_r a + S_s b
// expands into products of fixed reference matrices and the element's nodal
// values:
//   S_r a + S_s b = (g_rr K_rr + g_rs K_rs + g_ss K_ss) u
//                 + sum_f (c^r_f Q^r_f + c^s_f Q^s_f) [u]_f
// with K_rr = M D_r D_r, K_rs = M (D_r D_s + D_s D_r), K_ss = M D_s D_s,
// Q^r_f = M D_r L^f, Q^s_f = M D_s L^f, g_.. = grad . . grad ., and
// c^r_f = 1/2 grad r . g_f, c^s_f = 1/2 grad s . g_f.  Only u and O(N) face
// values are then live at once, which keeps the one-element-per-lane mapping
// in registers up to N = 8.
//
// Every geometric quantity is derived in-register from the four metric
// terms (r_x, s_x, r_y, s_y): outward face directions g_0 = -grad s,
// g_1 = grad r + grad s, g_2 = -grad r, Fs_f = |g_f|, n_f = g_f / Fs_f,
// J = 1 / (r_x s_y - s_x r_y).
//
// The neighbour's normal derivative on the shared face is evaluated in the
// frame whose vertex 0 is the neighbour's vertex fp (its face fp becomes face
// 0), so the derivative rows used are always those of face 0 and all operator
// entries are wave-uniform compile-time offsets (scalar loads), while the
// neighbour's nodal values are gathered in rotated order.
#pragma once
#include <cmath>

#include "device_common.hpp"
#include "tri.hpp"

namespace ipdg {

template <typename TX, typename TC>
__host__ __device__ __forceinline__ TC ld(const TX* p) { return static_cast<TC>(*p); }

// Entry k of the element's metric (r_x, s_x, r_y, s_y), or with k = -1 its
// coefficient, from a per-face source (own_metric(k), k = 4 for the
// coefficient) or from memory (g = metric or coefficient array).
template <bool PF, typename TC, typename Src>
__host__ __device__ __forceinline__ TC own_metric(const Src& src, const TC* __restrict__ g, int e, int k) {
  if constexpr (PF) return src.own_metric(k < 0 ? 4 : k);
  else return k < 0 ? g[e] : g[4 * e + k];
}

// A source that already holds the neighbours' values, face by face in the
// rotated order below, declares kPerFace and serves them through at<f, j>()
// instead of a node index, the element's metric and coefficient through
// own_metric(k) and each neighbour's through nbr_metric<f>(k), so that those
// loads can be issued ahead of the element computation.
template <typename S, typename = void>
struct PerFaceSrc { static constexpr bool value = false; };
template <typename S>
struct PerFaceSrc<S, decltype(void(S::kPerFace))> { static constexpr bool value = S::kPerFace; };

// 1/sqrt(x) and 1/x for a positive normal x (lengths and Jacobians of
// non-degenerate elements).  On the device: the hardware estimate and one
// Newton-Raphson step, y <- y (3 - x y^2)/2 and y <- y (2 - x y), which
// squares the estimate's relative error (a few units in the last place
// remain); the IEEE-rounded sqrt and division sequences cost several times
// more instructions.  FP32 takes the estimate alone (about one unit).
template <typename TC>
__host__ __device__ __forceinline__ TC rsqrt_pos(TC x) {
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (sizeof(TC) == 8) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = __builtin_fma(-x * y, y, 1.0);   // 1 - x y^2
    return __builtin_fma(0.5 * y, e, y);
  } else {
    return __builtin_amdgcn_rsqf(x);
  }
#else
  return TC(1) / std::sqrt(x);
#endif
}
template <typename TC>
__host__ __device__ __forceinline__ TC rcp_pos(TC x) {
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (sizeof(TC) == 8) {
    const double y = __builtin_amdgcn_rcp(x);
    const double e = __builtin_fma(-x, y, 1.0);        // 1 - x y
    return __builtin_fma(y, e, y);
  } else {
    return __builtin_amdgcn_rcpf(x);
  }
#else
  return TC(1) / x;
#endif
}

// A zero the optimiser cannot see through.  Added to the operator offsets of
// one phase (a face, a face node, an output row), it keeps that phase's
// scalar operator loads from being hoisted to the top of the kernel, where
// hundreds of them would be live at once and spill.  One s_mov per phase.
__host__ __device__ __forceinline__ int opaque_zero() {
#if defined(__HIP_DEVICE_COMPILE__)
  int z;
  asm volatile("s_mov_b32 %0, 0" : "=s"(z));
  return z;
#else
  return 0;
#endif
}

// Keeps the scheduler from hoisting the next phase's neighbour gathers above
// the current one (which would hold three neighbours' values in registers).
__host__ __device__ __forceinline__ void phase_fence() {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_sched_barrier(0);
#endif
}

// Nodal values of the operand: x[i] from a vector in TX, converted to TC.
template <typename TX, typename TC>
struct VecSrc {
  const TX* __restrict__ x;
  __host__ __device__ __forceinline__ TC operator()(size_t i) const { return ld<TX, TC>(x + i); }
};

// Computes y_e and hands each output row to out(i, y_i) as soon as it is
// formed (so no output array stays live).  The element's own nodal values
// come from own(j) (e.g. a block-wide staging buffer), the neighbours' from
// src(i), i = e Np + j (a vector, or one formed on the fly from two others).
// DIAG: u = unit vector e_unit on this element and zero neighbours (Jacobi
// diagonal).  u holds the element's values throughout.
template <int N, typename TC, bool KAP, bool DIAG, typename Src, typename Out, typename Own>
__host__ __device__ __forceinline__ void sipdg_element_src(int e, const Src& src,
                                                           const TC* __restrict__ geo,
                                                           const Conn* __restrict__ conn,
                                                           const TC* __restrict__ kap,
                                                           const TC* __restrict__ ops, TC lambda,
                                                           TC ctau, int unit, TC (&u)[Tri<N>::Np],
                                                           Out&& out, Own&& own) {
  using G = Tri<N>;
  using L = OpsLayout<N>;
  constexpr int Np = G::Np, Nfp = G::Nfp;
  constexpr bool PF = PerFaceSrc<Src>::value;
  const TC rx = own_metric<PF>(src, geo, e, 0), sx = own_metric<PF>(src, geo, e, 1);
  const TC ry = own_metric<PF>(src, geo, e, 2), sy = own_metric<PF>(src, geo, e, 3);
  // LEAN (degrees <= 5, where the per-face work is a large share): reciprocal
  // square roots and reciprocals from the refined estimates, boundary types
  // as coefficients; higher degrees keep IEEE sqrt/division and selects
  // (their register allocation is at an occupancy boundary)
  constexpr bool LEAN = N <= 5;
  const TC J = LEAN ? rcp_pos(rx * sy - sx * ry) : TC(1) / (rx * sy - sx * ry);
  const TC ke = KAP ? own_metric<PF>(src, kap, e, -1) : TC(1);
  const Conn c = conn[e];

#pragma unroll
  for (int j = 0; j < Np; ++j) {
    if constexpr (DIAG) u[j] = (j == unit) ? TC(1) : TC(0);
    else u[j] = own(j);
  }

  const TC gx[3] = {-sx, rx + sx, -rx};
  const TC gy[3] = {-sy, ry + sy, -ry};
  TC Fs[3], iFs[3], tau[3];
  TC jmp[3][Nfp], dnj[3][Nfp];

  // EARLY: all loads of a neighbour are issued before the element's own face
  // derivative, which then covers their latency (costs Np live values; used
  // where that keeps the occupancy); otherwise they stream into the
  // neighbour's derivative sums.
  constexpr bool EARLY = N <= 5;
  static_for<0, 3>([&](auto fc) {
    constexpr int f = decltype(fc)::value;
    phase_fence();
    const TC* __restrict__ opf = ops + opaque_zero();
    const int bc = conn_bc(c.info, f);
    const int nb = c.nb[f];
    const int fp = conn_fp(c.info, f);
    const size_t xn = (size_t)nb * Np;
    // the neighbour's nodal values in the rotated order that puts its face
    // fp at face 0
    auto nbr_value = [&](auto jc) -> TC {
      constexpr int j = decltype(jc)::value;
      if constexpr (PF) {
        return src.template at<f, j>();
      } else {
        constexpr int o1 = G::rot(1, j), o2 = G::rot(2, j);
        const int o = fp == 0 ? j : (fp == 1 ? o1 : o2);
        return src(xn + o);
      }
    };
    TC xv[Np];
    if constexpr (EARLY && !DIAG) static_for<0, Np>([&](auto jc) { xv[decltype(jc)::value] = nbr_value(jc); });
    auto nmetric = [&](int k) -> TC {
      if constexpr (PF) return src.template nbr_metric<f>(k);
      else return k < 4 ? geo[4 * nb + k] : (KAP ? kap[nb] : TC(1));
    };
    const TC prx = nmetric(0), psx = nmetric(1), pry = nmetric(2), psy = nmetric(3);
    const TC kp = nmetric(4);
    if constexpr (EARLY) phase_fence();
    if constexpr (LEAN) {
      const TC g2 = gx[f] * gx[f] + gy[f] * gy[f];
      iFs[f] = rsqrt_pos(g2);
      Fs[f] = g2 * iFs[f];
    } else {
      Fs[f] = sqrt(gx[f] * gx[f] + gy[f] * gy[f]);
      iFs[f] = TC(1) / Fs[f];
    }
    const TC nx = gx[f] * iFs[f], ny = gy[f] * iFs[f];
    const TC nr = nx * rx + ny * ry, ns = nx * sx + ny * sy;
    // own normal derivative at face node k
    auto own_at = [&](auto kc) -> TC {
      constexpr int k = decltype(kc)::value;
      constexpr int vm = G::fm(f, k);
      TC dr = TC(0), ds = TC(0);
#pragma unroll
      for (int j = 0; j < Np; ++j) {
        dr += opf[L::Dr + vm * Np + j] * u[j];
        ds += opf[L::Ds + vm * Np + j] * u[j];
      }
      return nr * dr + ns * ds;
    };
    TC own[Nfp];
    if constexpr (EARLY) static_for<0, Nfp>([&](auto kc) { own[decltype(kc)::value] = own_at(kc); });
    // neighbour metric in its rotated frame; reference derivatives at its
    // face-0 nodes
    const TC qx = -(prx + psx), qy = -(pry + psy);
    const TC Rx = fp == 0 ? prx : (fp == 1 ? psx : qx);
    const TC Ry = fp == 0 ? pry : (fp == 1 ? psy : qy);
    const TC Sx = fp == 0 ? psx : (fp == 1 ? qx : prx);
    const TC Sy = fp == 0 ? psy : (fp == 1 ? qy : pry);
    const TC S2 = Sx * Sx + Sy * Sy;
    const TC Fsp = LEAN ? S2 * rsqrt_pos(S2) : sqrt(S2);
    const TC nrp = nx * Rx + ny * Ry, nsp = nx * Sx + ny * Sy;
    const bool inner = (bc == 0);
    const bool dir = (bc == 1);
    // boundary type as coefficients (no selects): [u] = cu_p u+ + cu_m u-,
    // [k d_n u] = cd_p d_n u+ + cd_m d_n u- with the mirror ghost states
    // (Dirichlet: [u] = -2 u-, jump of the flux 0; Neumann: [u] = 0, jump of
    // the flux -2 k d_n u-)
    const TC c_in = inner ? TC(1) : TC(0);
    const TC cu_m = -(c_in + (dir ? TC(2) : TC(0)));
    const TC cd_p = c_in * kp;
    const TC cd_m = -(c_in + ((!inner && !dir) ? TC(2) : TC(0))) * ke;
    TC pr[Nfp], ps[Nfp];
#pragma unroll
    for (int m = 0; m < Nfp; ++m) pr[m] = ps[m] = TC(0);
    if constexpr (!DIAG) {
      static_for<0, Np>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        TC v;
        if constexpr (EARLY) v = xv[j];
        else {
          v = nbr_value(jc);
          if constexpr (j < Nfp) xv[j] = v;
        }
#pragma unroll
        for (int m = 0; m < Nfp; ++m) {
          pr[m] += opf[L::NBR + (j * 2 + 0) * Nfp + m] * v;
          ps[m] += opf[L::NBR + (j * 2 + 1) * Nfp + m] * v;
        }
      });
    }
    // 4. jumps of the value and of the normal flux (face-0 nodes of the
    //    neighbour are ids 0..N, in reverse order along the shared face)
    static_for<0, Nfp>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      constexpr int m = Nfp - 1 - k;
      constexpr int vm = G::fm(f, k);
      TC ownk;
      if constexpr (EARLY) ownk = own[k];
      else ownk = own_at(kc);
      const TC dnp = nrp * pr[m] + nsp * ps[m];
      const TC um = u[vm];
      const TC pv = DIAG ? TC(0) : xv[m];
      if constexpr (LEAN) {
        jmp[f][k] = c_in * pv + cu_m * um;
        dnj[f][k] = cd_p * dnp + cd_m * ownk;
      } else {
        const TC ji = pv - um;
        const TC di = kp * dnp - ke * ownk;
        jmp[f][k] = inner ? ji : (dir ? TC(-2) * um : TC(0));
        dnj[f][k] = inner ? di : (dir ? TC(0) : TC(-2) * ke * ownk);
      }
    });
    // branch-free: a boundary face takes the element's own side only
    tau[f] = ctau * fmax(ke * Fs[f], (LEAN ? c_in : TC(inner ? 1 : 0)) * (kp * Fsp));
  });

  phase_fence();
  // s_f at the nodes of face f2, including n_f2 . l there
  TC sf[3][Nfp];
  static_for<0, 3>([&](auto f2c) {
    constexpr int f2 = decltype(f2c)::value;
    TC cn[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) cn[f] = TC(0.5) * (gx[f2] * gx[f] + gy[f2] * gy[f]) * iFs[f2];
    const TC* __restrict__ opp = ops + opaque_zero();
    static_for<0, Nfp>([&](auto pc) {
      constexpr int p = decltype(pc)::value;
      constexpr int i = G::fm(f2, p);
      TC nl = TC(0);
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        TC w = TC(0);
#pragma unroll
        for (int k = 0; k < Nfp; ++k) w += opp[L::LIFT + i * 3 * Nfp + f * Nfp + k] * jmp[f][k];
        nl += cn[f] * w;
      }
      sf[f2][p] = TC(0.5) * dnj[f2][p] + tau[f2] * jmp[f2][p] - ke * nl;
    });
  });

  const TC grr = rx * rx + ry * ry, grs = rx * sx + ry * sy, gss = sx * sx + sy * sy;
  TC ca[3], cb[3], ts[3][Nfp];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    ca[f] = TC(0.5) * (rx * gx[f] + ry * gy[f]);
    cb[f] = TC(0.5) * (sx * gx[f] + sy * gy[f]);
#pragma unroll
    for (int k = 0; k < Nfp; ++k) ts[f][k] = Fs[f] * J * sf[f][k];
  }
  phase_fence();
  // Output rows: a runtime loop over the packed per-row operator stream, so
  // the scalar loads of one row are contiguous and only one row is in flight.
  const bool has_lambda = (lambda != TC(0));
  const TC* __restrict__ rowp = ops + L::ROW;
#pragma unroll 1
  for (int i = 0; i < Np; ++i, rowp += L::RowLen) {
    TC trr = TC(0), trs = TC(0), tss = TC(0);
#pragma unroll
    for (int j = 0; j < Np; ++j) {
      trr += rowp[j] * u[j];
      trs += rowp[Np + j] * u[j];
      tss += rowp[2 * Np + j] * u[j];
    }
    TC acc = grr * trr + grs * trs + gss * tss;
    TC fa = TC(0);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      TC qa = TC(0), qb = TC(0);
#pragma unroll
      for (int k = 0; k < Nfp; ++k) {
        qa += rowp[3 * Np + f * Nfp + k] * jmp[f][k];
        qb += rowp[3 * Np + 3 * Nfp + f * Nfp + k] * jmp[f][k];
        fa += rowp[3 * Np + 6 * Nfp + f * Nfp + k] * ts[f][k];
      }
      acc += ca[f] * qa + cb[f] * qb;
    }
    acc = -ke * acc;
    if (has_lambda) {
      TC m = TC(0);
#pragma unroll
      for (int j = 0; j < Np; ++j) m += rowp[3 * Np + 9 * Nfp + j] * u[j];
      acc += lambda * m;
    }
    out(i, acc * J - fa);
  }
}

template <int N, typename TC, typename TX, bool KAP, bool DIAG, typename Out, typename Own>
__host__ __device__ __forceinline__ void sipdg_element_own(int e, const TX* __restrict__ x,
                                                           const TC* __restrict__ geo,
                                                           const Conn* __restrict__ conn,
                                                           const TC* __restrict__ kap,
                                                           const TC* __restrict__ ops, TC lambda,
                                                           TC ctau, int unit, TC (&u)[Tri<N>::Np],
                                                           Out&& out, Own&& own) {
  sipdg_element_src<N, TC, KAP, DIAG>(e, VecSrc<TX, TC>{x}, geo, conn, kap, ops, lambda, ctau, unit, u, out,
                                      own);
}

template <int N, typename TC, typename TX, bool KAP, bool DIAG, typename Out>
__host__ __device__ __forceinline__ void sipdg_element(int e, const TX* __restrict__ x,
                                                       const TC* __restrict__ geo,
                                                       const Conn* __restrict__ conn,
                                                       const TC* __restrict__ kap,
                                                       const TC* __restrict__ ops, TC lambda,
                                                       TC ctau, int unit, TC (&u)[Tri<N>::Np],
                                                       Out&& out) {
  sipdg_element_own<N, TC, TX, KAP, DIAG>(e, x, geo, conn, kap, ops, lambda, ctau, unit, u, out,
                                          [&](int j) { return ld<TX, TC>(x + (size_t)e * Tri<N>::Np + j); });
}


}  // namespace ipdg
