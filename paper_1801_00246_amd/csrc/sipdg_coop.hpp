// Cooperative form of the SIPDG screened-Poisson operator: one tile of 64
// elements (one per lane) is shared by three waves, so that each wave holds a
// third of an element's work and state instead of all of it.
//
// The arithmetic is that of sipdg_element_src (Sec. 5.2, Eq. ellipticOp3
// with the lifted jump as a vector field; the local gradient and the SIPDG
// kernel of Alg. AxG and Alg. AxKernel fused), split into phases that
// exchange per-element values through LDS (lane l of every wave owns element
// e0 + l, so each wave reads and writes its own LDS column):
//   1. face phase, wave f handles face f: the element's normal derivative at
//      the face nodes (own values streamed from LDS), the neighbour's values
//      gathered in the rotated order that puts the shared face at reference
//      face 0, the neighbour's normal derivative, the jumps [u]_f (to LDS)
//      and [k d_n u]_f, the penalty tau_f;
//   2. lift phase, wave f2: s_f2 = 1/2 [k d_n u] + tau [u] - k n_f2 . l at the
//      nodes of face f2 (l from all three faces' jumps), scaled by
//      |F|/|E| J (to LDS);
//   3. row phase, wave w: its third of the output rows, streaming the
//      element's values and jumps column by column:
//        y_i = -k J (g_rr K_rr + g_rs K_rs + g_ss K_ss)_i u + lambda J M_i u
//              - k J sum_f (c^r_f Q^r_f + c^s_f Q^s_f)_i [u]_f
//              - sum_f (M1D s_f J |F|/|E|) at the face-f rows;
//   4. the tile's outputs leave through LDS as one contiguous, coalesced
//      block (and the optional partial sum of x . y).
// Every operator entry a wave reads is wave-uniform (a scalar operand), in
// streams laid out by CoopLayout<N> in the order they are read.
#pragma once
#include "kernels.hpp"
#include "sipdg_core.hpp"

namespace ipdg {

constexpr int kCoopTile = kCoopTileElems;     // elements per tile, one per lane
constexpr int kCoopThreads = 3 * kCoopTile;   // three waves per tile
constexpr int kCoopPitch = kCoopTile + 1;     // LDS row pitch (values)

// Per-lane element data used by every phase.
template <typename TC>
struct CoopElem {
  TC rx, sx, ry, sy, J, ke;
  Conn c;
};

// Outward face direction g_f = n_f |F|/|E| from the metric terms:
// g_0 = -grad s, g_1 = grad r + grad s, g_2 = -grad r.
template <int F, typename TC>
__device__ __forceinline__ void coop_g(const CoopElem<TC>& el, TC& gx, TC& gy) {
  gx = F == 0 ? -el.sx : (F == 1 ? el.rx + el.sx : -el.rx);
  gy = F == 0 ? -el.sy : (F == 1 ? el.ry + el.sy : -el.ry);
}

// The neighbour across face F: its values in the rotated order that puts its
// shared face fp at face 0 of the frame, its metric and coefficient.  The
// loads are issued before the tile's first barrier so that their latency is
// covered by the staging and the volume rows.
template <int N, typename TC>
struct CoopNbr {
  // degrees <= 5 load the neighbour's values ahead (their registers are
  // affordable there); higher degrees stream them into the derivative sums
  static constexpr bool kAhead = N <= 5;
  TC v[kAhead ? Tri<N>::Np : 1];
  const void* xn;
  int fp;
  TC prx, psx, pry, psy, kp;
};

template <int N, int F, typename TC, typename TX, bool KAP>
__device__ __forceinline__ void coop_gather(const CoopElem<TC>& el, const TX* __restrict__ x,
                                            const TC* __restrict__ geo, const TC* __restrict__ kap,
                                            CoopNbr<N, TC>& nb) {
  using G = Tri<N>;
  constexpr int Np = G::Np;
  const int e = el.c.nb[F];
  const int fp = conn_fp(el.c.info, F);
  const TX* __restrict__ xn = x + (size_t)e * Np;
  nb.xn = xn;
  nb.fp = fp;
  if constexpr (CoopNbr<N, TC>::kAhead) {
    static_for<0, Np>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      constexpr int o1 = G::rot(1, j), o2 = G::rot(2, j);
      const int o = fp == 0 ? j : (fp == 1 ? o1 : o2);
      nb.v[j] = static_cast<TC>(xn[o]);
    });
  }
  nb.prx = geo[4 * e + 0];
  nb.psx = geo[4 * e + 1];
  nb.pry = geo[4 * e + 2];
  nb.psy = geo[4 * e + 3];
  nb.kp = KAP ? kap[e] : TC(1);
}

// Phase 1, face F: jumps to JM (LDS), [k d_n u] at the face nodes, tau_F,
// |F|/|E| and its reciprocal in registers.
template <int N, int F, typename TC, typename TX>
__device__ __forceinline__ void coop_face(const CoopElem<TC>& el, const CoopNbr<N, TC>& nb,
                                          const TC* __restrict__ ops, TC ctau, const TC* U, TC* JM,
                                          int lane, TC (&dnj)[Tri<N>::Nfp], TC& tau, TC& Fs, TC& iFs) {
  using G = Tri<N>;
  using L = OpsLayout<N>;
  using CL = CoopLayout<N>;
  constexpr int Np = G::Np, Nfp = G::Nfp, P = kCoopPitch;
  const int fp = conn_fp(el.c.info, F);
  const int bc = conn_bc(el.c.info, F);
  TC gx, gy;
  coop_g<F>(el, gx, gy);
  const TC g2 = gx * gx + gy * gy;
  iFs = rsqrt_pos(g2);
  Fs = g2 * iFs;
  const TC nx = gx * iFs, ny = gy * iFs;
  const TC nr = nx * el.rx + ny * el.ry, ns = nx * el.sx + ny * el.sy;

  // the neighbour's normal derivative at its face-0 nodes first (its values,
  // already loaded, die as they are consumed), in its rotated frame
  const TC qx = -(nb.prx + nb.psx), qy = -(nb.pry + nb.psy);
  const TC Rx = fp == 0 ? nb.prx : (fp == 1 ? nb.psx : qx);
  const TC Ry = fp == 0 ? nb.pry : (fp == 1 ? nb.psy : qy);
  const TC Sx = fp == 0 ? nb.psx : (fp == 1 ? qx : nb.prx);
  const TC Sy = fp == 0 ? nb.psy : (fp == 1 ? qy : nb.pry);
  const TC S2 = Sx * Sx + Sy * Sy;
  const TC Fsp = S2 * rsqrt_pos(S2);
  const TC nrp = nx * Rx + ny * Ry, nsp = nx * Sx + ny * Sy;
  TC dnp[Nfp], vface[Nfp];
  {
    TC pr[Nfp], ps[Nfp];
#pragma unroll
    for (int m = 0; m < Nfp; ++m) pr[m] = ps[m] = TC(0);
    const TC* __restrict__ nbr = ops + L::NBR + opaque_zero();
    const TX* __restrict__ xn = static_cast<const TX*>(nb.xn);
    static_for<0, Np>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      TC vj;
      if constexpr (CoopNbr<N, TC>::kAhead) {
        vj = nb.v[j];
      } else {
        constexpr int o1 = G::rot(1, j), o2 = G::rot(2, j);
        const int o = nb.fp == 0 ? j : (nb.fp == 1 ? o1 : o2);
        vj = static_cast<TC>(xn[o]);
        if constexpr (j < Nfp) vface[j] = vj;
      }
#pragma unroll
      for (int m = 0; m < Nfp; ++m) {
        pr[m] += nbr[(j * 2 + 0) * Nfp + m] * vj;
        ps[m] += nbr[(j * 2 + 1) * Nfp + m] * vj;
      }
    });
#pragma unroll
    for (int m = 0; m < Nfp; ++m) dnp[m] = nrp * pr[m] + nsp * ps[m];
  }
  // own normal derivative at the face nodes, the element's values streamed
  // from LDS
  TC dn[Nfp], uf[Nfp];
  {
    TC dr[Nfp], ds[Nfp];
#pragma unroll
    for (int k = 0; k < Nfp; ++k) dr[k] = ds[k] = TC(0);
    const TC* __restrict__ fd = ops + CL::FD + F * Np * Nfp * 2 + opaque_zero();
    static_for<0, Np>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      const TC uj = U[j * P + lane];
      if constexpr (G::fpos(F, j) >= 0) uf[G::fpos(F, j)] = uj;
#pragma unroll
      for (int k = 0; k < Nfp; ++k) {
        dr[k] += fd[(j * Nfp + k) * 2 + 0] * uj;
        ds[k] += fd[(j * Nfp + k) * 2 + 1] * uj;
      }
    });
#pragma unroll
    for (int k = 0; k < Nfp; ++k) dn[k] = nr * dr[k] + ns * ds[k];
  }
  // boundary type as coefficients (mirror ghost states): interior [u] =
  // u+ - u-, [k d_n u] = k+ d_n u+ - k- d_n u-; Dirichlet [u] = -2 u-,
  // flux jump 0; Neumann [u] = 0, flux jump -2 k- d_n u-
  const bool inner = bc == 0, dir = bc == 1;
  const TC c_in = inner ? TC(1) : TC(0);
  const TC cu_m = -(c_in + (dir ? TC(2) : TC(0)));
  const TC cd_p = c_in * nb.kp;
  const TC cd_m = -(c_in + ((!inner && !dir) ? TC(2) : TC(0))) * el.ke;
#pragma unroll
  for (int k = 0; k < Nfp; ++k) {
    const int m = Nfp - 1 - k;   // the shared face runs the other way in the neighbour
    TC vm;
    if constexpr (CoopNbr<N, TC>::kAhead) vm = nb.v[m];
    else vm = vface[m];
    JM[(F * Nfp + k) * P + lane] = c_in * vm + cu_m * uf[k];
    dnj[k] = cd_p * dnp[m] + cd_m * dn[k];
  }
  tau = ctau * fmax(el.ke * Fs, c_in * (nb.kp * Fsp));
}

// Phase 2, face F2: J |F2|/|E| s_F2 at the face nodes, to TS (LDS).
template <int N, int F2, typename TC>
__device__ __forceinline__ void coop_lift(const CoopElem<TC>& el, const TC* __restrict__ ops, const TC* JM, TC* TS,
                                          int lane, const TC (&dnj)[Tri<N>::Nfp], TC tau, TC Fs, TC iFs) {
  using CL = CoopLayout<N>;
  constexpr int Nfp = Tri<N>::Nfp, P = kCoopPitch;
  TC gx[3], gy[3];
  coop_g<0>(el, gx[0], gy[0]);
  coop_g<1>(el, gx[1], gy[1]);
  coop_g<2>(el, gx[2], gy[2]);
  TC cn[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) cn[f] = TC(0.5) * (gx[F2] * gx[f] + gy[F2] * gy[f]) * iFs;
  // n_F2 . l at the face nodes, the jumps streamed from LDS once
  TC nl[Nfp];
#pragma unroll
  for (int p = 0; p < Nfp; ++p) nl[p] = TC(0);
  TC jown[Nfp];
  const TC* __restrict__ lf = ops + CL::LF + F2 * Nfp * 3 * Nfp + opaque_zero();
#pragma unroll
  for (int f = 0; f < 3; ++f)
#pragma unroll
    for (int k = 0; k < Nfp; ++k) {
      const TC jk = JM[(f * Nfp + k) * P + lane];
      if (f == F2) jown[k] = jk;
      const TC c = cn[f] * jk;
#pragma unroll
      for (int p = 0; p < Nfp; ++p) nl[p] += lf[p * 3 * Nfp + f * Nfp + k] * c;
    }
  const TC sc = Fs * el.J;
#pragma unroll
  for (int p = 0; p < Nfp; ++p) {
    const TC sf = TC(0.5) * dnj[p] + tau * jown[p] - el.ke * nl[p];
    TS[(F2 * Nfp + p) * P + lane] = sc * sf;
  }
}

// Volume terms of wave W's rows (the element's values streamed from LDS
// once): acc_i = -k J (g_rr K_rr + g_rs K_rs + g_ss K_ss)_i u
// [+ lambda J M_i u].
template <int N, int W, bool LAM, typename TC>
__device__ __forceinline__ void coop_rows_vol(const CoopElem<TC>& el, const TC* __restrict__ ops, const TC* U,
                                              int lane, TC lambda, TC (&acc)[CoopLayout<N>::kMaxRows]) {
  using CL = CoopLayout<N>;
  constexpr int Np = Tri<N>::Np, P = kCoopPitch;
  constexpr int nr = CL::nrows(W);
  const TC sc = -el.ke * el.J;
  const TC srr = sc * (el.rx * el.rx + el.ry * el.ry);
  const TC srs = sc * (el.rx * el.sx + el.ry * el.sy);
  const TC sss = sc * (el.sx * el.sx + el.sy * el.sy);
  const TC sl = lambda * el.J;
#pragma unroll
  for (int i = 0; i < nr; ++i) acc[i] = TC(0);
  const TC* __restrict__ cv = ops + CL::CV(W) + opaque_zero();
  const TC* __restrict__ cm = ops + CL::CM(W) + opaque_zero();
#pragma unroll
  for (int j = 0; j < Np; ++j) {
    const TC uj = U[j * P + lane];
    const TC c1 = srr * uj, c2 = srs * uj, c3 = sss * uj;
    // one multiply-add per entry (a sum of products would cost a multiply and
    // an add more per row)
#pragma unroll
    for (int i = 0; i < nr; ++i) {
      acc[i] += cv[(j * nr + i) * 3 + 0] * c1;
      acc[i] += cv[(j * nr + i) * 3 + 1] * c2;
      acc[i] += cv[(j * nr + i) * 3 + 2] * c3;
    }
    if constexpr (LAM) {
      const TC c4 = sl * uj;
#pragma unroll
      for (int i = 0; i < nr; ++i) acc[i] += cm[j * nr + i] * c4;
    }
  }
}

// Lifted-jump terms of wave W's rows: acc_i -= k J sum_f (c^r_f Q^r_f +
// c^s_f Q^s_f)_i [u]_f, the jumps read from JM.
template <int N, int W, typename TC>
__device__ __forceinline__ void coop_rows_jump(const CoopElem<TC>& el, const TC* __restrict__ ops, const TC* JM,
                                               int lane, TC (&acc)[CoopLayout<N>::kMaxRows]) {
  using CL = CoopLayout<N>;
  constexpr int Nfp = Tri<N>::Nfp, P = kCoopPitch;
  constexpr int nr = CL::nrows(W);
  const TC sc = -el.ke * el.J;
  const TC* __restrict__ cq = ops + CL::CQ(W) + opaque_zero();
  static_for<0, 3>([&](auto fc) {
    constexpr int f = decltype(fc)::value;
    TC gx, gy;
    coop_g<f>(el, gx, gy);
    const TC sa = sc * TC(0.5) * (el.rx * gx + el.ry * gy);
    const TC sb = sc * TC(0.5) * (el.sx * gx + el.sy * gy);
#pragma unroll
    for (int k = 0; k < Nfp; ++k) {
      const TC jk = JM[(f * Nfp + k) * P + lane];
      const TC a = sa * jk, b = sb * jk;
#pragma unroll
      for (int i = 0; i < nr; ++i) {
        acc[i] += cq[((f * Nfp + k) * nr + i) * 2 + 0] * a;
        acc[i] += cq[((f * Nfp + k) * nr + i) * 2 + 1] * b;
      }
    }
  });
}

// Phase 3b, wave W: the face-mass term of the rows on a face, the partial
// x . y, and the finished rows written over the element's values in U (this
// wave's rows only; every wave has finished reading U).
template <int N, int W, typename TC>
__device__ __forceinline__ void coop_rows_out(const TC* __restrict__ ops, TC* U, const TC* TS, int lane,
                                              TC (&acc)[CoopLayout<N>::kMaxRows], bool want_dot, double& dot) {
  using G = Tri<N>;
  using L = OpsLayout<N>;
  using CL = CoopLayout<N>;
  constexpr int Nfp = G::Nfp, P = kCoopPitch;
  constexpr int b = CL::row_begin(W), nr = CL::nrows(W);
  const TC* __restrict__ m1 = ops + L::M1D + opaque_zero();
  static_for<0, nr>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    static_for<0, 3>([&](auto fc) {
      constexpr int f = decltype(fc)::value;
      constexpr int p = G::fpos(f, b + i);
      if constexpr (p >= 0) {
#pragma unroll
        for (int k = 0; k < Nfp; ++k) acc[i] -= m1[p * Nfp + k] * TS[(f * Nfp + k) * P + lane];
      }
    });
    if (want_dot) dot += static_cast<double>(U[(b + i) * P + lane]) * static_cast<double>(acc[i]);
    U[(b + i) * P + lane] = acc[i];
  });
}


// ---------------------------------------------------------------------------
// Matrix-core row phase (degrees >= 5).  The tile's output (Np rows x 64
// elements) is cut into 16 x 16 blocks (row block rb, column block cb of 16
// elements); each block accumulates
//   sum_t K_t (s_t o U) + Q^r (s^r o [u]) + Q^s (s^s o [u]) - E TS
// with 16 x 16 x 4 matrix multiply-accumulates: the operators are the A
// operands (MfmaLayout, read from memory in lane order), the element data the
// B operands (LDS, column cb of the tile, scaled per element), so each
// operator entry serves 16 elements per instruction.  s_t, s^r, s^s are the
// per-element factors of the row phase (-k J g_rr, ..., lambda J, -k J c^r_f,
// -k J c^s_f), kept in LDS.
// ---------------------------------------------------------------------------
namespace sc_slot {
constexpr int kRR = 0, kRS = 1, kSS = 2, kLam = 3, kFace = 4;   // kFace + 2 f: c^r_f, + 1: c^s_f
constexpr int kCount = 10;
}  // namespace sc_slot

template <typename TC>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row within the 16 x 16 block held by lane l in accumulator entry r
  static __device__ __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};

// Blocks of wave w: with three row blocks, row block w and all four column
// blocks; with two, row block w and column blocks 0..2 for waves 0 and 1,
// column block 3 of both row blocks for wave 2; with one, column blocks
// {0, 3}, {1}, {2}.
__host__ __device__ constexpr int mf_ntiles(int RB, int w) {
  return RB >= 3 ? 4 : (RB == 2 ? (w < 2 ? 3 : 2) : (w == 0 ? 2 : 1));
}
__host__ __device__ constexpr int mf_rb(int RB, int w, int i) { return RB >= 3 ? w : (RB == 2 ? (w < 2 ? w : i) : 0); }
__host__ __device__ constexpr int mf_cb(int RB, int w, int i) {
  return RB >= 3 ? i : (RB == 2 ? (w < 2 ? i : 3) : (w == 0 ? (i == 0 ? 0 : 3) : w));
}

// Per-element factors of the row phase into SC (LDS), lane's own element.
template <typename TC>
__device__ __forceinline__ void coop_factors(const CoopElem<TC>& el, TC lambda, TC* SC, int lane) {
  constexpr int P = kCoopPitch;
  const TC sc = -el.ke * el.J;
  SC[sc_slot::kRR * P + lane] = sc * (el.rx * el.rx + el.ry * el.ry);
  SC[sc_slot::kRS * P + lane] = sc * (el.rx * el.sx + el.ry * el.sy);
  SC[sc_slot::kSS * P + lane] = sc * (el.sx * el.sx + el.sy * el.sy);
  SC[sc_slot::kLam * P + lane] = lambda * el.J;
  static_for<0, 3>([&](auto fc) {
    constexpr int f = decltype(fc)::value;
    TC gx, gy;
    coop_g<f>(el, gx, gy);
    SC[(sc_slot::kFace + 2 * f) * P + lane] = sc * TC(0.5) * (el.rx * gx + el.ry * gy);
    SC[(sc_slot::kFace + 2 * f + 1) * P + lane] = sc * TC(0.5) * (el.sx * gx + el.sy * gy);
  });
}

// Volume and lifted-jump blocks of wave W (before the face-mass term).
template <int N, int W, bool LAM, typename TC>
__device__ __forceinline__ void coop_rows_mfma(const TC* __restrict__ ops, const TC* U, const TC* JM, const TC* SC,
                                               int lane, typename Mfma<TC>::v4 (&acc)[4]) {
  using ML = MfmaLayout<N>;
  using M = Mfma<TC>;
  constexpr int Np = Tri<N>::Np, Nfp = Tri<N>::Nfp, P = kCoopPitch;
  constexpr int RB = ML::RB, NT = mf_ntiles(RB, W);
  const int kk = lane >> 4, nn = lane & 15;
#pragma unroll
  for (int i = 0; i < NT; ++i) acc[i] = typename M::v4{TC(0), TC(0), TC(0), TC(0)};
  // volume operators; entries past the operator's columns are zero in A, the
  // matching B rows read a valid row
  static_for<0, LAM ? 4 : 3>([&](auto tc) {
    constexpr int t = decltype(tc)::value;
    TC s[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) s[i] = SC[t * P + mf_cb(RB, W, i) * 16 + nn];
#pragma unroll
    for (int kb = 0; kb < ML::KBV; ++kb) {
      const int j = 4 * kb + kk < Np ? 4 * kb + kk : Np - 1;
      TC a[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) a[rb] = ops[ML::vol(t, rb, kb) + lane];
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        const TC b = U[j * P + mf_cb(RB, W, i) * 16 + nn] * s[i];
        acc[i] = M::mma(a[mf_rb(RB, W, i)], b, acc[i]);
      }
    }
  });
  // lifted-jump operators: column fk = 4 kb + kk of the jumps belongs to
  // face fk / Nfp
#pragma unroll
  for (int kb = 0; kb < ML::KBF; ++kb) {
    const int fk0 = 4 * kb + kk;
    const int fk = fk0 < 3 * Nfp ? fk0 : 3 * Nfp - 1;
    const int f = fk / Nfp;
    TC ar[RB], as[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      ar[rb] = ops[ML::face(0, rb, kb) + lane];
      as[rb] = ops[ML::face(1, rb, kb) + lane];
    }
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const int col = mf_cb(RB, W, i) * 16 + nn;
      const TC jk = JM[fk * P + col];
      const TC br = jk * SC[(sc_slot::kFace + 2 * f) * P + col];
      const TC bs = jk * SC[(sc_slot::kFace + 2 * f + 1) * P + col];
      acc[i] = M::mma(ar[mf_rb(RB, W, i)], br, acc[i]);
      acc[i] = M::mma(as[mf_rb(RB, W, i)], bs, acc[i]);
    }
  }
}

// Face-mass blocks of wave W (TS complete) and the partial x . y over the
// wave's blocks (x read from U before any wave overwrites it).
template <int N, int W, typename TC>
__device__ __forceinline__ void coop_rows_mfma_face(const TC* __restrict__ ops, const TC* U, const TC* TS, int lane,
                                                    int ne, typename Mfma<TC>::v4 (&acc)[4], bool want_dot,
                                                    double& dot) {
  using ML = MfmaLayout<N>;
  using M = Mfma<TC>;
  constexpr int Np = Tri<N>::Np, Nfp = Tri<N>::Nfp, P = kCoopPitch;
  constexpr int RB = ML::RB, NT = mf_ntiles(RB, W);
  const int kk = lane >> 4, nn = lane & 15;
#pragma unroll
  for (int kb = 0; kb < ML::KBF; ++kb) {
    const int fk0 = 4 * kb + kk;
    const int fk = fk0 < 3 * Nfp ? fk0 : 3 * Nfp - 1;
    TC a[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) a[rb] = ops[ML::face(2, rb, kb) + lane];
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = M::mma(a[mf_rb(RB, W, i)], TS[fk * P + mf_cb(RB, W, i) * 16 + nn], acc[i]);
  }
  if (want_dot) {
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const int col = mf_cb(RB, W, i) * 16 + nn;
      if (col >= ne) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = mf_rb(RB, W, i) * 16 + M::row(lane, r);
        if (row < Np) dot += static_cast<double>(U[row * P + col]) * static_cast<double>(acc[i][r]);
      }
    }
  }
}

// Finished blocks of wave W written over U (every wave has read U).
template <int N, int W, typename TC>
__device__ __forceinline__ void coop_rows_mfma_store(TC* U, int lane, const typename Mfma<TC>::v4 (&acc)[4]) {
  using ML = MfmaLayout<N>;
  using M = Mfma<TC>;
  constexpr int Np = Tri<N>::Np, P = kCoopPitch;
  constexpr int RB = ML::RB, NT = mf_ntiles(RB, W);
  const int nn = lane & 15;
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = mf_rb(RB, W, i) * 16 + M::row(lane, r);
      if (row < Np) U[row * P + mf_cb(RB, W, i) * 16 + nn] = acc[i][r];
    }
}

}  // namespace ipdg
