// DG gradient G and divergence D with central fluxes (Sec. 2.1, Eq.
// INS_SD_4_1 and INS_SD_4_2), in strong nodal form per element:
//   G p = grad p + LIFT (|F|/|E|) n (p* - p-),
//   D u = div u  + LIFT (|F|/|E|) n . (u* - u-),
// p* = {p}, u* = {u} on interior faces; on Dirichlet (velocity) faces
// u* = g_D and p* = p-, on Neumann faces u* = u- and p* = 0.  The divergence,
// and the gradient and the advection term from degree 2, run on the matrix
// cores, 16 elements per wave (the form below `Matrix-core form`); at degree
// 1 those two and the Dirichlet-data terms run one element per lane, the
// reference operators read from the degree's FP64 table through wave-uniform
// loads.  Normals and face scales |F|/|E| come from the element's metric
// terms (face 0: -grad s, face 1: grad r + grad s, face 2: -grad r; each
// vector's length is |F|/|E|).
#include <hip/hip_runtime.h>

#include <cmath>

#include "gradiv.hpp"
#include "tri.hpp"

namespace ipdg {
namespace {

// Elements per block: a block stages its elements' contiguous fields through
// one LDS buffer of kElems x pitch values, so that global loads and stores
// are coalesced while each lane works on one element from registers.
template <int N>
constexpr int kElems() {
  return Tri<N>::Np <= 15 ? 256 : 128;
}
// LDS row pitch in doubles: odd, so that the lanes' rows start in different
// banks
template <int N>
constexpr int kPitchGD() {
  constexpr int Np = Tri<N>::Np;
  return (Np % 2) ? Np : Np + 1;
}

// the block's n elements' values of src, row by row, into the lanes'
// registers r[] through the LDS buffer (coalesced global reads)
template <int N>
__device__ __forceinline__ void load_rows(const double* __restrict__ src, double* lds, int e0, int n,
                                          double (&r)[Tri<N>::Np]) {
  constexpr int Np = Tri<N>::Np, P = kPitchGD<N>(), B = kElems<N>();
  const int total = n * Np;
  for (int i = threadIdx.x; i < total; i += B) lds[(i / Np) * P + i % Np] = src[(size_t)e0 * Np + i];
  __syncthreads();
  if ((int)threadIdx.x < n)
#pragma unroll
    for (int j = 0; j < Np; ++j) r[j] = lds[threadIdx.x * P + j];
  __syncthreads();
}
// the rows the lanes wrote into the LDS buffer, out to dst (coalesced)
template <int N>
__device__ __forceinline__ void store_rows(const double* lds, double* __restrict__ dst, int e0, int n) {
  constexpr int Np = Tri<N>::Np, P = kPitchGD<N>(), B = kElems<N>();
  __syncthreads();
  const int total = n * Np;
  for (int i = threadIdx.x; i < total; i += B) dst[(size_t)e0 * Np + i] = lds[(i / Np) * P + i % Np];
  __syncthreads();
}

// J M x for one element's values (registers)
template <int N>
__device__ __forceinline__ void mass_rows(const double* __restrict__ ops, double J, double (&x)[Tri<N>::Np]) {
  using L = OpsLayout<N>;
  constexpr int Np = Tri<N>::Np;
  double y[Np];
  for (int i = 0; i < Np; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < Np; ++j) s += ops[L::M + i * Np + j] * x[j];
    y[i] = J * s;
  }
#pragma unroll
  for (int i = 0; i < Np; ++i) x[i] = y[i];
}

template <int N, bool MASS>
__global__ __launch_bounds__(kElems<N>()) void k_grad(GradArgs a) {
  using T = Tri<N>;
  using L = OpsLayout<N>;
  constexpr int Np = T::Np, Nfp = T::Nfp, B = kElems<N>(), P = kPitchGD<N>();
  __shared__ double buf[B * P];
  const int e0 = blockIdx.x * B;
  const int n = min(B, a.K - e0);
  const double* __restrict__ ops = a.ops;
  const double* __restrict__ p = a.p;
  double pe[Np];
  load_rows<N>(p, buf, e0, n, pe);
  const int t = threadIdx.x, e = e0 + t;
  double gx[Np], gy[Np];
  if (t < n) {
    const double rx = a.geo[4 * (size_t)e], sx = a.geo[4 * (size_t)e + 1];
    const double ry = a.geo[4 * (size_t)e + 2], sy = a.geo[4 * (size_t)e + 3];
    // face terms (p* - p-) per face node
    double fl[3][Nfp];
    double fax[3], fay[3];
    const Conn c = a.conn[e];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const int bc = conn_bc(c.info, f);
      const int fp = conn_fp(c.info, f), nb = c.nb[f];
      face_vec(f, rx, sx, ry, sy, fax[f], fay[f]);
#pragma unroll
      for (int k = 0; k < Nfp; ++k) {
        const double pm = pe[T::fm(f, k)];
        // Dirichlet: p* = p-; Neumann: p* = 0; interior: p* = {p}
        fl[f][k] = bc == 1 ? 0.0 : (bc == 0 ? 0.5 * (p[(size_t)nb * Np + T::fm(fp, N - k)] - pm) : -pm);
      }
    }
    for (int i = 0; i < Np; ++i) {
      double dr = 0.0, ds = 0.0;
#pragma unroll
      for (int j = 0; j < Np; ++j) {
        dr += ops[L::Dr + i * Np + j] * pe[j];
        ds += ops[L::Ds + i * Np + j] * pe[j];
      }
      double vx = rx * dr + sx * ds, vy = ry * dr + sy * ds;
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < Nfp; ++k) s += ops[L::LIFT + i * 3 * Nfp + f * Nfp + k] * fl[f][k];
        vx += fax[f] * s;
        vy += fay[f] * s;
      }
      gx[i] = a.a_grad * vx;
      gy[i] = a.a_grad * vy;
    }
    if (a.base_x) {
#pragma unroll
      for (int i = 0; i < Np; ++i) {
        gx[i] += a.a_base * a.base_x[(size_t)e * Np + i];
        gy[i] += a.a_base * a.base_y[(size_t)e * Np + i];
      }
    }
    if constexpr (MASS) {
      const double J = 1.0 / (rx * sy - ry * sx);
      mass_rows<N>(ops, J, gx);
      mass_rows<N>(ops, J, gy);
    }
#pragma unroll
    for (int i = 0; i < Np; ++i) buf[t * P + i] = gx[i];
  }
  store_rows<N>(buf, a.out_x, e0, n);
  if (t < n)
#pragma unroll
    for (int i = 0; i < Np; ++i) buf[t * P + i] = gy[i];
  store_rows<N>(buf, a.out_y, e0, n);
  if (a.p_out) {
    if (t < n)
#pragma unroll
      for (int i = 0; i < Np; ++i) buf[t * P + i] = pe[i];
    __syncthreads();
    const int total = n * Np;
    for (int i = threadIdx.x; i < total; i += B)
      a.p_out[(size_t)e0 * Np + i] = buf[(i / Np) * P + i % Np] + a.add_p[(size_t)e0 * Np + i];
  }
}

// ---------------------------------------------------------------------------
// Matrix-core form (layout GdDims in gradiv.hpp; the divergence at every
// degree, the gradient and the advection term from degree 2).  A wave
// computes 16 elements as the columns of 16 x 16 blocks of
// v_mfma_f64_16x16x4f64: D_r and D_s times the elements' nodal values (B
// operands in registers), the face terms as LIFT_f times the face-node fluxes
// (B operands formed per lane from the gathered traces), the metric terms
// applied lane by lane on the accumulators.  With the mass option the
// accumulators are fed back as B operands of J M: accumulator entry r of lane
// l is row l/16 + 4 r of its block, the B operand of k-step r.  Outputs leave
// through LDS as one contiguous block per wave.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kGdWaves = 2;   // waves per block, 16 elements each

// J M g for the wave's 16 columns (g in accumulator layout, RB blocks)
template <int N>
__device__ __forceinline__ void mf_mass(const double* __restrict__ tab, int lane, double J,
                                        v4d (&g)[gd_dims(N).RB]) {
  constexpr GdDims D = gd_dims(N);
  v4d m[D.RB];
#pragma unroll
  for (int R = 0; R < D.RB; ++R) m[R] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int R2 = 0; R2 < D.RB; ++R2)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int R = 0; R < D.RB; ++R) m[R] = mma(tab[D.oM + ((R * D.RB + R2) * 4 + t) * 64 + lane], g[R2][t], m[R]);
#pragma unroll
  for (int R = 0; R < D.RB; ++R) g[R] = J * m[R];
}

// the wave's 16 columns (accumulator layout) into its LDS block, element-major
template <int N>
__device__ __forceinline__ void mf_stage(double* st, int nn, int kk, const v4d (&g)[gd_dims(N).RB]) {
  constexpr GdDims D = gd_dims(N);
#pragma unroll
  for (int R = 0; R < D.RB; ++R)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = 16 * R + kk + 4 * r;
      if (n < D.Np) st[nn * D.Np + n] = g[R][r];
    }
}

// One wave's tile of 16 elements from e0 (tab: the operator table in global
// memory or LDS; st0, st1: the wave's two LDS staging rows of 16 Np values).
// Contains a block barrier: every wave of the block calls it equally often.
template <int N, bool MASS>
__device__ __forceinline__ void grad_tile(const GradArgs& a, const double* __restrict__ tab, int e0, double* st0,
                                          double* st1) {
  using T = Tri<N>;
  constexpr GdDims D = gd_dims(N);
  constexpr int Np = D.Np, Nfp = D.Nfp;
  const int lane = threadIdx.x & 63;
  const int nn = lane & 15, kk = lane >> 4;
  const int ec = e0 + nn < a.K ? e0 + nn : a.K - 1;   // lanes past the end read a valid element
  const double* __restrict__ p = a.p;
  const double rx = a.geo[4 * (size_t)ec], sx = a.geo[4 * (size_t)ec + 1];
  const double ry = a.geo[4 * (size_t)ec + 2], sy = a.geo[4 * (size_t)ec + 3];
  v4d gr[D.RB], gs[D.RB], fx[D.RB], fy[D.RB];
#pragma unroll
  for (int R = 0; R < D.RB; ++R) gr[R] = gs[R] = fx[R] = fy[R] = v4d{0.0, 0.0, 0.0, 0.0};
  {
    double pb[D.KB];
#pragma unroll
    for (int kb = 0; kb < D.KB; ++kb) pb[kb] = p[(size_t)ec * Np + (4 * kb + kk < Np ? 4 * kb + kk : Np - 1)];
#pragma unroll
    for (int kb = 0; kb < D.KB; ++kb)
#pragma unroll
      for (int R = 0; R < D.RB; ++R) {
        gr[R] = mma(tab[D.oDr + (R * D.KB + kb) * 64 + lane], pb[kb], gr[R]);
        gs[R] = mma(tab[D.oDs + (R * D.KB + kb) * 64 + lane], pb[kb], gs[R]);
      }
  }
  // face terms: LIFT_f ((|F|/|E|) n (p* - p-)) at the face nodes
  const Conn c = a.conn[ec];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int bc = conn_bc(c.info, f), fp = conn_fp(c.info, f), nb = c.nb[f];
    double ax, ay;
    face_vec(f, rx, sx, ry, sy, ax, ay);
#pragma unroll
    for (int kb = 0; kb < D.KF; ++kb) {
      const int k = 4 * kb + kk < Nfp ? 4 * kb + kk : Nfp - 1;
      const double pm = p[(size_t)ec * Np + T::fm(f, k)];
      // Dirichlet: p* = p-; Neumann: p* = 0; interior: p* = {p}
      const double fl = bc == 1 ? 0.0 : (bc == 0 ? 0.5 * (p[(size_t)nb * Np + T::fm(fp, N - k)] - pm) : -pm);
#pragma unroll
      for (int R = 0; R < D.RB; ++R) {
        const double L = tab[D.oL + ((f * D.RB + R) * D.KF + kb) * 64 + lane];
        fx[R] = mma(L, ax * fl, fx[R]);
        fy[R] = mma(L, ay * fl, fy[R]);
      }
    }
  }
  // metric terms, scaling and the optional base fields (rows 16 R + l/16 + 4 r)
#pragma unroll
  for (int R = 0; R < D.RB; ++R)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double vx = a.a_grad * (rx * gr[R][r] + sx * gs[R][r] + fx[R][r]);
      double vy = a.a_grad * (ry * gr[R][r] + sy * gs[R][r] + fy[R][r]);
      if (a.base_x) {
        const int n = 16 * R + kk + 4 * r;
        const size_t i = (size_t)ec * Np + (n < Np ? n : Np - 1);
        vx += a.a_base * a.base_x[i];
        vy += a.a_base * a.base_y[i];
      }
      gr[R][r] = vx;
      gs[R][r] = vy;
    }
  if constexpr (MASS) {
    const double J = 1.0 / (rx * sy - ry * sx);
    mf_mass<N>(tab, lane, J, gr);
    mf_mass<N>(tab, lane, J, gs);
  }
  mf_stage<N>(st0, nn, kk, gr);
  mf_stage<N>(st1, nn, kk, gs);
  __syncthreads();
  const int ne = a.K - e0 < 16 ? a.K - e0 : 16;
  const size_t g0 = (size_t)e0 * Np;
  for (int idx = lane; idx < ne * Np; idx += 64) {
    a.out_x[g0 + idx] = st0[idx];
    a.out_y[g0 + idx] = st1[idx];
    if (a.p_out) a.p_out[g0 + idx] = p[g0 + idx] + a.add_p[g0 + idx];
  }
}

template <int N, bool MASS>
__device__ __forceinline__ void div_tile(const DivArgs& a, const double* __restrict__ tab, int e0, double* st0,
                                         double*) {
  using T = Tri<N>;
  constexpr GdDims D = gd_dims(N);
  constexpr int Np = D.Np, Nfp = D.Nfp;
  const int lane = threadIdx.x & 63;
  const int nn = lane & 15, kk = lane >> 4;
  const int ec = e0 + nn < a.K ? e0 + nn : a.K - 1;
  const double* __restrict__ u = a.u;
  const double* __restrict__ v = a.v;
  const double rx = a.geo[4 * (size_t)ec], sx = a.geo[4 * (size_t)ec + 1];
  const double ry = a.geo[4 * (size_t)ec + 2], sy = a.geo[4 * (size_t)ec + 3];
  v4d ur[D.RB], us[D.RB], vr[D.RB], vs[D.RB], fl[D.RB];
#pragma unroll
  for (int R = 0; R < D.RB; ++R) ur[R] = us[R] = vr[R] = vs[R] = fl[R] = v4d{0.0, 0.0, 0.0, 0.0};
  {
    double ub[D.KB], vb[D.KB];
#pragma unroll
    for (int kb = 0; kb < D.KB; ++kb) {
      const size_t i = (size_t)ec * Np + (4 * kb + kk < Np ? 4 * kb + kk : Np - 1);
      ub[kb] = u[i];
      vb[kb] = v[i];
    }
#pragma unroll
    for (int kb = 0; kb < D.KB; ++kb)
#pragma unroll
      for (int R = 0; R < D.RB; ++R) {
        const double Ar = tab[D.oDr + (R * D.KB + kb) * 64 + lane], As = tab[D.oDs + (R * D.KB + kb) * 64 + lane];
        ur[R] = mma(Ar, ub[kb], ur[R]);
        us[R] = mma(As, ub[kb], us[R]);
        vr[R] = mma(Ar, vb[kb], vr[R]);
        vs[R] = mma(As, vb[kb], vs[R]);
      }
  }
  // face terms: LIFT_f ((|F|/|E|) n . (u* - u-)) at the face nodes
  const Conn c = a.conn[ec];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int bc = conn_bc(c.info, f), fp = conn_fp(c.info, f), nb = c.nb[f];
    double ax, ay;
    face_vec(f, rx, sx, ry, sy, ax, ay);
#pragma unroll
    for (int kb = 0; kb < D.KF; ++kb) {
      const int k = 4 * kb + kk < Nfp ? 4 * kb + kk : Nfp - 1;
      const size_t im = (size_t)ec * Np + T::fm(f, k);
      const double um = u[im], vm = v[im];
      double ju = 0.0, jv = 0.0;   // Neumann: u* = u-
      if (bc == 0) {
        const size_t ip = (size_t)nb * Np + T::fm(fp, N - k);
        ju = 0.5 * (u[ip] - um);
        jv = 0.5 * (v[ip] - vm);
      } else if (bc == 1) {
        ju = (a.gu ? a.gu[im] : 0.0) - um;
        jv = (a.gv ? a.gv[im] : 0.0) - vm;
      }
      const double b = ax * ju + ay * jv;
#pragma unroll
      for (int R = 0; R < D.RB; ++R) fl[R] = mma(tab[D.oL + ((f * D.RB + R) * D.KF + kb) * 64 + lane], b, fl[R]);
    }
  }
#pragma unroll
  for (int R = 0; R < D.RB; ++R)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      ur[R][r] = (rx * ur[R][r] + sx * us[R][r]) + (ry * vr[R][r] + sy * vs[R][r]) + fl[R][r];
  if constexpr (MASS) mf_mass<N>(tab, lane, 1.0 / (rx * sy - ry * sx), ur);
  mf_stage<N>(st0, nn, kk, ur);
  __syncthreads();
  const int ne = a.K - e0 < 16 ? a.K - e0 : 16;
  const size_t g0 = (size_t)e0 * Np;
  for (int idx = lane; idx < ne * Np; idx += 64) a.out[g0 + idx] = a.scale * st0[idx];
}

// Nodal Lax-Friedrichs advection term on the matrix cores (same shape as
// k_div_mf): the metric terms are folded into the nodal products first,
//   N_u = D_r (r_x uu + r_y uv) + D_s (s_x uu + s_y uv) + sum_f LIFT_f (|F|/|E|) flux_u,
// and likewise for N_v with (uv, vv); out = a_base base + a_adv N.
template <int N, bool MASS_UNUSED>
__device__ __forceinline__ void advect_tile(const AdvectArgs& a, const double* __restrict__ tab, int e0, double* st0,
                                            double* st1) {
  using T = Tri<N>;
  constexpr GdDims D = gd_dims(N);
  constexpr int Np = D.Np, Nfp = D.Nfp;
  const int lane = threadIdx.x & 63;
  const int nn = lane & 15, kk = lane >> 4;
  const int ec = e0 + nn < a.K ? e0 + nn : a.K - 1;   // lanes past the end read a valid element
  const double* __restrict__ u = a.u;
  const double* __restrict__ v = a.v;
  const double rx = a.geo[4 * (size_t)ec], sx = a.geo[4 * (size_t)ec + 1];
  const double ry = a.geo[4 * (size_t)ec + 2], sy = a.geo[4 * (size_t)ec + 3];
  v4d nu[D.RB], nv[D.RB];
#pragma unroll
  for (int R = 0; R < D.RB; ++R) nu[R] = nv[R] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kb = 0; kb < D.KB; ++kb) {
    const size_t i = (size_t)ec * Np + (4 * kb + kk < Np ? 4 * kb + kk : Np - 1);
    const double uj = u[i], vj = v[i];
    const double uu = uj * uj, uv = uj * vj, vv = vj * vj;
    const double bru = rx * uu + ry * uv, bsu = sx * uu + sy * uv;
    const double brv = rx * uv + ry * vv, bsv = sx * uv + sy * vv;
#pragma unroll
    for (int R = 0; R < D.RB; ++R) {
      const double Ar = tab[D.oDr + (R * D.KB + kb) * 64 + lane], As = tab[D.oDs + (R * D.KB + kb) * 64 + lane];
      nu[R] = mma(Ar, bru, nu[R]);
      nu[R] = mma(As, bsu, nu[R]);
      nv[R] = mma(Ar, brv, nv[R]);
      nv[R] = mma(As, bsv, nv[R]);
    }
  }
  const Conn c = a.conn[ec];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int bc = conn_bc(c.info, f), fp = conn_fp(c.info, f), nb = c.nb[f];
    double ax, ay;
    face_vec(f, rx, sx, ry, sy, ax, ay);
    const double fs = sqrt(ax * ax + ay * ay);
    const double nx = ax / fs, ny = ay / fs;
#pragma unroll
    for (int kb = 0; kb < D.KF; ++kb) {
      const int k = 4 * kb + kk < Nfp ? 4 * kb + kk : Nfp - 1;
      const size_t im = (size_t)ec * Np + T::fm(f, k);
      const double um = u[im], vm = v[im];
      double up = um, vp = vm;                       // Neumann: u+ = u-
      if (bc == 0) {
        const size_t ip = (size_t)nb * Np + T::fm(fp, N - k);
        up = u[ip];
        vp = v[ip];
      } else if (bc == 1) {
        up = a.gu ? a.gu[im] : 0.0;
        vp = a.gv ? a.gv[im] : 0.0;
      }
      const double unm = nx * um + ny * vm, unp = nx * up + ny * vp;
      const double lam = 2.0 * fmax(fabs(unm), fabs(unp));
      const double fu = fs * (0.5 * (um * unm + up * unp) + 0.5 * lam * (um - up) - um * unm);
      const double fv = fs * (0.5 * (vm * unm + vp * unp) + 0.5 * lam * (vm - vp) - vm * unm);
#pragma unroll
      for (int R = 0; R < D.RB; ++R) {
        const double L = tab[D.oL + ((f * D.RB + R) * D.KF + kb) * 64 + lane];
        nu[R] = mma(L, fu, nu[R]);
        nv[R] = mma(L, fv, nv[R]);
      }
    }
  }
  mf_stage<N>(st0, nn, kk, nu);
  mf_stage<N>(st1, nn, kk, nv);
  __syncthreads();
  const int ne = a.K - e0 < 16 ? a.K - e0 : 16;
  const size_t g0 = (size_t)e0 * Np;
  for (int idx = lane; idx < ne * Np; idx += 64) {
    double ou = a.a_adv * st0[idx], ov = a.a_adv * st1[idx];
    if (a.base_u) {
      ou += a.a_base * a.base_u[g0 + idx];
      ov += a.a_base * a.base_v[g0 + idx];
    }
    a.out_u[g0 + idx] = ou;
    a.out_v[g0 + idx] = ov;
  }
}

// The two launch forms of a tile function: one tile per wave with the table
// read from global memory, or persistent blocks of gd_pwaves waves that keep
// the table in LDS and walk over the tiles (all waves of a block take the
// same number of steps, so the tile's barrier is reached by all).
// waves per persistent block with ROWS staging rows per wave: 8 if the table
// and eight waves' rows fit the 160 KiB of LDS, else 4
template <int N, int ROWS>
constexpr int gd_pwaves() {
  return (gd_dims(N).total + 8 * ROWS * 16 * gd_dims(N).Np) * 8 <= 160 * 1024 ? 8 : 4;
}

#define IPDG_GD_KERNELS(NAME, TILE, ARGS, ROWS)                                                                    \
  template <int N, bool MASS>                                                                                \
  __global__ __launch_bounds__(64 * kGdWaves) void NAME(ARGS a, const double* __restrict__ tab) {            \
    __shared__ double stage[kGdWaves][ROWS][16 * gd_dims(N).Np];                                             \
    const int w = threadIdx.x >> 6;                                                                          \
    TILE<N, MASS>(a, tab, (blockIdx.x * kGdWaves + w) * 16, stage[w][0], stage[w][ROWS - 1]);                \
  }                                                                                                          \
  template <int N, bool MASS>                                                                                \
  __global__ __launch_bounds__((64 * gd_pwaves<N, ROWS>())) void NAME##p(ARGS a, const double* __restrict__ gtab) { \
    constexpr GdDims D = gd_dims(N);                                                                         \
    constexpr int W = gd_pwaves<N, ROWS>();                                                                  \
    __shared__ double tab[D.total];                                                                          \
    __shared__ double stage[W][ROWS][16 * D.Np];                                                             \
    for (int i = threadIdx.x; i < D.total; i += 64 * W) tab[i] = gtab[i];                                    \
    __syncthreads();                                                                                         \
    const int w = threadIdx.x >> 6;                                                                          \
    const int ntiles = (a.K + 16 * W - 1) / (16 * W);                                                        \
    for (int bt = blockIdx.x; bt < ntiles; bt += gridDim.x) {                                                \
      TILE<N, MASS>(a, tab, (bt * W + w) * 16, stage[w][0], stage[w][ROWS - 1]);                             \
      __syncthreads();                                                                                       \
    }                                                                                                        \
  }

IPDG_GD_KERNELS(k_grad_mf, grad_tile, GradArgs, 2)
IPDG_GD_KERNELS(k_div_mf, div_tile, DivArgs, 1)
IPDG_GD_KERNELS(k_advect_mf, advect_tile, AdvectArgs, 2)
#undef IPDG_GD_KERNELS

// One element per lane; only elements with Dirichlet faces add anything.
// Face integrals from the face-node values: with h = (|F| / 2) M1D g (the
// face mass on [-1, 1] times the half face length), (g, l_i)_F = h at the
// face nodes, and (g, d_n l_i)_F = sum_k h_k (d_n l_i)(x_k), d_n l_i at a
// face node read off the derivative matrices (exact: both traces are
// polynomials the face nodes represent).
template <int N>
__global__ __launch_bounds__(256) void k_dirichlet_rhs(DirichletArgs a) {
  using T = Tri<N>;
  using L = OpsLayout<N>;
  constexpr int Np = T::Np, Nfp = T::Nfp;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= a.K) return;
  const Conn c = a.conn[e];
  if (conn_bc(c.info, 0) != 1 && conn_bc(c.info, 1) != 1 && conn_bc(c.info, 2) != 1) return;
  const double* __restrict__ ops = a.ops;
  const double rx = a.geo[4 * (size_t)e], sx = a.geo[4 * (size_t)e + 1];
  const double ry = a.geo[4 * (size_t)e + 2], sy = a.geo[4 * (size_t)e + 3];
  const double J = 1.0 / (rx * sy - ry * sx);
  const double kap = a.kap ? a.kap[e] : 1.0;
  double* b = a.b + (size_t)e * Np;
  for (int f = 0; f < 3; ++f) {
    if (conn_bc(c.info, f) != 1) continue;
    double ax, ay;
    face_vec(f, rx, sx, ry, sy, ax, ay);
    const double fs = sqrt(ax * ax + ay * ay);          // |F| / |E|
    const double nx = ax / fs, ny = ay / fs;
    const double half_len = fs * J;                     // |F| / 2 (|E| = 2 J)
    const double tau = a.ctau * kap * fs;
    double gk[Nfp], h[Nfp];
#pragma unroll
    for (int k = 0; k < Nfp; ++k) gk[k] = a.g[(size_t)e * Np + T::fm(f, k)];
#pragma unroll
    for (int k = 0; k < Nfp; ++k) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < Nfp; ++m) s += ops[L::M1D + k * Nfp + m] * gk[m];
      h[k] = half_len * s;
    }
    // -kappa (g, d_n l_i)_F for every row i
    for (int i = 0; i < Np; ++i) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < Nfp; ++k) {
        const int q = T::fm(f, k);
        const double dx = rx * ops[L::Dr + q * Np + i] + sx * ops[L::Ds + q * Np + i];
        const double dy = ry * ops[L::Dr + q * Np + i] + sy * ops[L::Ds + q * Np + i];
        s += h[k] * (nx * dx + ny * dy);
      }
      b[i] -= kap * s;
    }
    // 2 tau_F (g, l_i)_F on the face nodes
#pragma unroll
    for (int k = 0; k < Nfp; ++k) b[T::fm(f, k)] += 2.0 * tau * h[k];
  }
}

template <int N>
__global__ __launch_bounds__(kElems<N>()) void k_advect(AdvectArgs a) {
  using T = Tri<N>;
  using L = OpsLayout<N>;
  constexpr int Np = T::Np, Nfp = T::Nfp, B = kElems<N>(), P = kPitchGD<N>();
  __shared__ double buf[B * P];
  const int e0 = blockIdx.x * B;
  const int n = min(B, a.K - e0);
  const double* __restrict__ ops = a.ops;
  const double* __restrict__ u = a.u;
  const double* __restrict__ v = a.v;
  double ue[Np], ve[Np];
  load_rows<N>(u, buf, e0, n, ue);
  load_rows<N>(v, buf, e0, n, ve);
  const int t = threadIdx.x, e = e0 + t;
  double nu[Np], nv[Np];
  if (t < n) {
    const double rx = a.geo[4 * (size_t)e], sx = a.geo[4 * (size_t)e + 1];
    const double ry = a.geo[4 * (size_t)e + 2], sy = a.geo[4 * (size_t)e + 3];
    // div (u_c u) from the nodal products
    for (int i = 0; i < Np; ++i) {
      double uur = 0.0, uus = 0.0, uvr = 0.0, uvs = 0.0, vvr = 0.0, vvs = 0.0;
#pragma unroll
      for (int j = 0; j < Np; ++j) {
        const double dr = ops[L::Dr + i * Np + j], ds = ops[L::Ds + i * Np + j];
        const double uu = ue[j] * ue[j], uv = ue[j] * ve[j], vv = ve[j] * ve[j];
        uur += dr * uu;
        uus += ds * uu;
        uvr += dr * uv;
        uvs += ds * uv;
        vvr += dr * vv;
        vvs += ds * vv;
      }
      nu[i] = (rx * uur + sx * uus) + (ry * uvr + sy * uvs);
      nv[i] = (rx * uvr + sx * uvs) + (ry * vvr + sy * vvs);
    }
    const Conn c = a.conn[e];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const int bc = conn_bc(c.info, f);
      const int fp = conn_fp(c.info, f), nb = c.nb[f];
      double ax, ay;
      face_vec(f, rx, sx, ry, sy, ax, ay);
      const double fs = sqrt(ax * ax + ay * ay);
      const double nx = ax / fs, ny = ay / fs;
      double fu[Nfp], fv[Nfp];
#pragma unroll
      for (int k = 0; k < Nfp; ++k) {
        const int m = T::fm(f, k);
        const double um = ue[m], vm = ve[m];
        double up = um, vp = vm;                       // Neumann: u+ = u-
        if (bc == 0) {
          const size_t ip = (size_t)nb * Np + T::fm(fp, N - k);
          up = u[ip];
          vp = v[ip];
        } else if (bc == 1) {
          const size_t im = (size_t)e * Np + m;
          up = a.gu ? a.gu[im] : 0.0;
          vp = a.gv ? a.gv[im] : 0.0;
        }
        const double unm = nx * um + ny * vm, unp = nx * up + ny * vp;
        const double lam = 2.0 * fmax(fabs(unm), fabs(unp));
        fu[k] = fs * (0.5 * (um * unm + up * unp) + 0.5 * lam * (um - up) - um * unm);
        fv[k] = fs * (0.5 * (vm * unm + vp * unp) + 0.5 * lam * (vm - vp) - vm * unm);
      }
      for (int i = 0; i < Np; ++i) {
        double su = 0.0, sv = 0.0;
#pragma unroll
        for (int k = 0; k < Nfp; ++k) {
          const double l = ops[L::LIFT + i * 3 * Nfp + f * Nfp + k];
          su += l * fu[k];
          sv += l * fv[k];
        }
        nu[i] += su;
        nv[i] += sv;
      }
    }
    for (int i = 0; i < Np; ++i) {
      nu[i] *= a.a_adv;
      nv[i] *= a.a_adv;
    }
    if (a.base_u)
      for (int i = 0; i < Np; ++i) {
        nu[i] += a.a_base * a.base_u[(size_t)e * Np + i];
        nv[i] += a.a_base * a.base_v[(size_t)e * Np + i];
      }
#pragma unroll
    for (int i = 0; i < Np; ++i) buf[t * P + i] = nu[i];
  }
  store_rows<N>(buf, a.out_u, e0, n);
  if (t < n)
#pragma unroll
    for (int i = 0; i < Np; ++i) buf[t * P + i] = nv[i];
  store_rows<N>(buf, a.out_v, e0, n);
}

__global__ __launch_bounds__(256) void k_axpby(double a, const double* __restrict__ x, double b,
                                               const double* __restrict__ y, double* __restrict__ z, size_t n) {
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) z[i] = a * x[i] + b * y[i];
}

// one block: work[0] = sum b (fixed order)
__global__ __launch_bounds__(1024) void k_sum(const double* __restrict__ b, size_t n, double* __restrict__ work) {
  __shared__ double red[16];
  double s = 0.0;
  for (size_t i = threadIdx.x; i < n; i += 1024) s += b[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w];
    work[0] = t;
  }
}

// b_i -= (work[0] / area) J_e sum_j M_ij
template <int N>
__global__ __launch_bounds__(256) void k_sub_mean(double* __restrict__ b, double area, const double* __restrict__ geo,
                                                  const double* __restrict__ ops, int K,
                                                  const double* __restrict__ work) {
  using L = OpsLayout<N>;
  constexpr int Np = Tri<N>::Np;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= K) return;
  const double c = work[0] / area;
  const double J = 1.0 / (geo[4 * (size_t)e] * geo[4 * (size_t)e + 3] - geo[4 * (size_t)e + 2] * geo[4 * (size_t)e + 1]);
  for (int i = 0; i < Np; ++i) {
    double s = 0.0;
    for (int j = 0; j < Np; ++j) s += ops[L::M + i * Np + j];
    b[(size_t)e * Np + i] -= c * J * s;
  }
}


template <int N>
int blocks(int K) { return (K + kElems<N>() - 1) / kElems<N>(); }

}  // namespace

hipError_t dirichlet_rhs(int N, const DirichletArgs& a, hipStream_t s) {
  if (a.K == 0) return hipSuccess;
  const dim3 g((a.K + 255) / 256);
  switch (N) {
#define IPDG_R(n) \
  case n: hipLaunchKernelGGL(k_dirichlet_rhs<n>, g, dim3(256), 0, s, a); break;
    IPDG_R(1) IPDG_R(2) IPDG_R(3) IPDG_R(4) IPDG_R(5) IPDG_R(6) IPDG_R(7) IPDG_R(8)
#undef IPDG_R
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

namespace {

// degrees from which the persistent form (table in LDS) runs: measured on
// 524,288 triangles it is 10-28 % faster from degree 3 (the plain form reads
// the whole table from L2 for every 16 elements, three to four times the
// kernel's HBM bytes at degree 7), and even at degree 2
template <int N>
constexpr bool gd_persistent() {
  return N >= 3;
}

// The persistent form needs enough tiles to fill the device with blocks that
// each pay for one table load: below 256 block tiles (32,768 elements at
// eight waves) the plain form is faster (8,192 triangles at N = 5: 10-12
// against 14-15 us).
constexpr int kGdPersistentMinK = 32768;

template <int N, int ROWS, typename Args, typename K1, typename K2>
void launch_gd(const Args& a, hipStream_t s, K1 plain, K2 persistent) {
  if constexpr (gd_persistent<N>()) {
    if (a.K >= kGdPersistentMinK) {
      constexpr int W = gd_pwaves<N, ROWS>();
      const int ntiles = (a.K + 16 * W - 1) / (16 * W);
      hipLaunchKernelGGL(persistent, dim3(ntiles < 512 ? ntiles : 512), dim3(64 * W), 0, s, a, device_gd_tab(N));
      return;
    }
  }
  hipLaunchKernelGGL(plain, dim3((a.K + 16 * kGdWaves - 1) / (16 * kGdWaves)), dim3(64 * kGdWaves), 0, s, a,
                     device_gd_tab(N));
}

template <int N>
void launch_grad_mf(const GradArgs& a, hipStream_t s) {
  if (a.mass) launch_gd<N, 2>(a, s, k_grad_mf<N, true>, k_grad_mfp<N, true>);
  else launch_gd<N, 2>(a, s, k_grad_mf<N, false>, k_grad_mfp<N, false>);
}

template <int N>
void launch_div_mf(const DivArgs& a, hipStream_t s) {
  if (a.mass) launch_gd<N, 1>(a, s, k_div_mf<N, true>, k_div_mfp<N, true>);
  else launch_gd<N, 1>(a, s, k_div_mf<N, false>, k_div_mfp<N, false>);
}

template <int N>
void launch_advect_mf(const AdvectArgs& a, hipStream_t s) {
  launch_gd<N, 2>(a, s, k_advect_mf<N, false>, k_advect_mfp<N, false>);
}

}  // namespace

hipError_t advect_apply(int N, const AdvectArgs& a, hipStream_t s) {
  if (a.K == 0) return hipSuccess;
  switch (N) {
    // one element per lane is faster only at degree 1
    case 1: hipLaunchKernelGGL(k_advect<1>, dim3(blocks<1>(a.K)), dim3(kElems<1>()), 0, s, a); break;
    case 2: launch_advect_mf<2>(a, s); break;
    case 3: launch_advect_mf<3>(a, s); break;
    case 4: launch_advect_mf<4>(a, s); break;
    case 5: launch_advect_mf<5>(a, s); break;
    case 6: launch_advect_mf<6>(a, s); break;
    case 7: launch_advect_mf<7>(a, s); break;
    case 8: launch_advect_mf<8>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t axpby(double a, const double* x, double b, const double* y, double* z, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)g), dim3(256), 0, s, a, x, b, y, z, n);
  return hipGetLastError();
}

hipError_t remove_mean(int N, double* b, double area, const double* geo, const double* ops, int K, double* work,
                       hipStream_t s) {
  if (K == 0) return hipSuccess;
  const size_t n = (size_t)K * ((N + 1) * (N + 2) / 2);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, s, b, n, work);
  const dim3 g((K + 255) / 256);
  switch (N) {
#define IPDG_M(nn) \
  case nn: hipLaunchKernelGGL(k_sub_mean<nn>, g, dim3(256), 0, s, b, area, geo, ops, K, work); break;
    IPDG_M(1) IPDG_M(2) IPDG_M(3) IPDG_M(4) IPDG_M(5) IPDG_M(6) IPDG_M(7) IPDG_M(8)
#undef IPDG_M
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}


hipError_t grad_apply(int N, const GradArgs& a, hipStream_t s) {
  if (a.K == 0) return hipSuccess;
  switch (N) {
    // one element per lane is faster only at degree 1
    case 1:
      if (a.mass) hipLaunchKernelGGL((k_grad<1, true>), dim3(blocks<1>(a.K)), dim3(kElems<1>()), 0, s, a);
      else hipLaunchKernelGGL((k_grad<1, false>), dim3(blocks<1>(a.K)), dim3(kElems<1>()), 0, s, a);
      break;
    case 2: launch_grad_mf<2>(a, s); break;
    case 3: launch_grad_mf<3>(a, s); break;
    case 4: launch_grad_mf<4>(a, s); break;
    case 5: launch_grad_mf<5>(a, s); break;
    case 6: launch_grad_mf<6>(a, s); break;
    case 7: launch_grad_mf<7>(a, s); break;
    case 8: launch_grad_mf<8>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t div_apply(int N, const DivArgs& a, hipStream_t s) {
  if (a.K == 0) return hipSuccess;
  switch (N) {
    case 1: launch_div_mf<1>(a, s); break;
    case 2: launch_div_mf<2>(a, s); break;
    case 3: launch_div_mf<3>(a, s); break;
    case 4: launch_div_mf<4>(a, s); break;
    case 5: launch_div_mf<5>(a, s); break;
    case 6: launch_div_mf<6>(a, s); break;
    case 7: launch_div_mf<7>(a, s); break;
    case 8: launch_div_mf<8>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ipdg
