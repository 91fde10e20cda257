// DG gradient G and divergence D with central fluxes (Sec. 2.1, Eq.
// INS_SD_4_1 and INS_SD_4_2), in strong nodal form per element:
//   G p = grad p + LIFT (|F|/|E|) n (p* - p-),
//   D u = div u  + LIFT (|F|/|E|) n . (u* - u-),
// p* = {p}, u* = {u} on interior faces; on Dirichlet (velocity) faces
// u* = g_D and p* = p-, on Neumann faces u* = u- and p* = 0.  One element per
// lane; the reference operators D_r, D_s, LIFT and M come from the degree's
// FP64 table through wave-uniform loads, the normals and face scales
// |F|/|E| from the element's metric terms (face 0: -grad s, face 1:
// grad r + grad s, face 2: -grad r; each vector's length is |F|/|E|).
#include <hip/hip_runtime.h>

#include <cmath>

#include "gradiv.hpp"
#include "tri.hpp"

namespace ipdg {
namespace {

constexpr int kThreads = 256;

// outward face vector of face f: its direction is the unit normal and its
// length the face scale |F| / |E|
__device__ __forceinline__ void face_vec(int f, double rx, double sx, double ry, double sy, double& ax, double& ay) {
  if (f == 0) {
    ax = -sx;
    ay = -sy;
  } else if (f == 1) {
    ax = rx + sx;
    ay = ry + sy;
  } else {
    ax = -rx;
    ay = -ry;
  }
}

template <int N>
__global__ __launch_bounds__(kThreads) void k_grad(GradArgs a) {
  using T = Tri<N>;
  using L = OpsLayout<N>;
  constexpr int Np = T::Np, Nfp = T::Nfp;
  const int e = blockIdx.x * kThreads + threadIdx.x;
  if (e >= a.K) return;
  const double* __restrict__ ops = a.ops;
  const double* __restrict__ p = a.p;
  double pe[Np];
#pragma unroll
  for (int i = 0; i < Np; ++i) pe[i] = p[(size_t)e * Np + i];
  const double rx = a.geo[4 * (size_t)e], sx = a.geo[4 * (size_t)e + 1];
  const double ry = a.geo[4 * (size_t)e + 2], sy = a.geo[4 * (size_t)e + 3];
  double gx[Np], gy[Np];
  for (int i = 0; i < Np; ++i) {
    double dr = 0.0, ds = 0.0;
#pragma unroll
    for (int j = 0; j < Np; ++j) {
      dr += ops[L::Dr + i * Np + j] * pe[j];
      ds += ops[L::Ds + i * Np + j] * pe[j];
    }
    gx[i] = rx * dr + sx * ds;
    gy[i] = ry * dr + sy * ds;
  }
  const Conn c = a.conn[e];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int bc = conn_bc(c.info, f);
    if (bc == 1) continue;                        // Dirichlet: p* = p-
    const int fp = conn_fp(c.info, f), nb = c.nb[f];
    double ax, ay;
    face_vec(f, rx, sx, ry, sy, ax, ay);
    double fl[Nfp];
#pragma unroll
    for (int k = 0; k < Nfp; ++k) {
      const double pm = pe[T::fm(f, k)];
      fl[k] = bc == 0 ? 0.5 * (p[(size_t)nb * Np + T::fm(fp, N - k)] - pm) : -pm;
    }
    for (int i = 0; i < Np; ++i) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < Nfp; ++k) s += ops[L::LIFT + i * 3 * Nfp + f * Nfp + k] * fl[k];
      gx[i] += ax * s;
      gy[i] += ay * s;
    }
  }
  double ox[Np], oy[Np];
  for (int i = 0; i < Np; ++i) {
    ox[i] = a.a_grad * gx[i];
    oy[i] = a.a_grad * gy[i];
    if (a.base_x) {
      ox[i] += a.a_base * a.base_x[(size_t)e * Np + i];
      oy[i] += a.a_base * a.base_y[(size_t)e * Np + i];
    }
  }
  if (a.mass) {
    const double J = 1.0 / (rx * sy - ry * sx);
    for (int i = 0; i < Np; ++i) {
      double sxm = 0.0, sym = 0.0;
#pragma unroll
      for (int j = 0; j < Np; ++j) {
        sxm += ops[L::M + i * Np + j] * ox[j];
        sym += ops[L::M + i * Np + j] * oy[j];
      }
      a.out_x[(size_t)e * Np + i] = J * sxm;
      a.out_y[(size_t)e * Np + i] = J * sym;
    }
  } else {
#pragma unroll
    for (int i = 0; i < Np; ++i) {
      a.out_x[(size_t)e * Np + i] = ox[i];
      a.out_y[(size_t)e * Np + i] = oy[i];
    }
  }
  if (a.p_out) {
#pragma unroll
    for (int i = 0; i < Np; ++i) a.p_out[(size_t)e * Np + i] = pe[i] + a.add_p[(size_t)e * Np + i];
  }
}

template <int N>
__global__ __launch_bounds__(kThreads) void k_div(DivArgs a) {
  using T = Tri<N>;
  using L = OpsLayout<N>;
  constexpr int Np = T::Np, Nfp = T::Nfp;
  const int e = blockIdx.x * kThreads + threadIdx.x;
  if (e >= a.K) return;
  const double* __restrict__ ops = a.ops;
  const double* __restrict__ u = a.u;
  const double* __restrict__ v = a.v;
  const double rx = a.geo[4 * (size_t)e], sx = a.geo[4 * (size_t)e + 1];
  const double ry = a.geo[4 * (size_t)e + 2], sy = a.geo[4 * (size_t)e + 3];
  double d[Np];
  {
    double ue[Np], ve[Np];
#pragma unroll
    for (int i = 0; i < Np; ++i) {
      ue[i] = u[(size_t)e * Np + i];
      ve[i] = v[(size_t)e * Np + i];
    }
    for (int i = 0; i < Np; ++i) {
      double ur = 0.0, us = 0.0, vr = 0.0, vs = 0.0;
#pragma unroll
      for (int j = 0; j < Np; ++j) {
        const double dr = ops[L::Dr + i * Np + j], ds = ops[L::Ds + i * Np + j];
        ur += dr * ue[j];
        us += ds * ue[j];
        vr += dr * ve[j];
        vs += ds * ve[j];
      }
      d[i] = (rx * ur + sx * us) + (ry * vr + sy * vs);
    }
  }
  const Conn c = a.conn[e];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int bc = conn_bc(c.info, f);
    if (bc == 2) continue;                        // Neumann: u* = u-
    const int fp = conn_fp(c.info, f), nb = c.nb[f];
    double ax, ay;
    face_vec(f, rx, sx, ry, sy, ax, ay);
    double fl[Nfp];
#pragma unroll
    for (int k = 0; k < Nfp; ++k) {
      const size_t im = (size_t)e * Np + T::fm(f, k);
      const double um = u[im], vm = v[im];
      double ju, jv;
      if (bc == 0) {
        const size_t ip = (size_t)nb * Np + T::fm(fp, N - k);
        ju = 0.5 * (u[ip] - um);
        jv = 0.5 * (v[ip] - vm);
      } else {
        ju = (a.gu ? a.gu[im] : 0.0) - um;
        jv = (a.gv ? a.gv[im] : 0.0) - vm;
      }
      fl[k] = ax * ju + ay * jv;
    }
    for (int i = 0; i < Np; ++i) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < Nfp; ++k) s += ops[L::LIFT + i * 3 * Nfp + f * Nfp + k] * fl[k];
      d[i] += s;
    }
  }
  if (a.mass) {
    const double J = 1.0 / (rx * sy - ry * sx);
    for (int i = 0; i < Np; ++i) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < Np; ++j) s += ops[L::M + i * Np + j] * d[j];
      a.out[(size_t)e * Np + i] = a.scale * (J * s);
    }
  } else {
#pragma unroll
    for (int i = 0; i < Np; ++i) a.out[(size_t)e * Np + i] = a.scale * d[i];
  }
}

int blocks(int K) { return (K + kThreads - 1) / kThreads; }

}  // namespace

hipError_t grad_apply(int N, const GradArgs& a, hipStream_t s) {
  if (a.K == 0) return hipSuccess;
  switch (N) {
#define IPDG_G(n) \
  case n: hipLaunchKernelGGL(k_grad<n>, dim3(blocks(a.K)), dim3(kThreads), 0, s, a); break;
    IPDG_G(1) IPDG_G(2) IPDG_G(3) IPDG_G(4) IPDG_G(5) IPDG_G(6) IPDG_G(7) IPDG_G(8)
#undef IPDG_G
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t div_apply(int N, const DivArgs& a, hipStream_t s) {
  if (a.K == 0) return hipSuccess;
  switch (N) {
#define IPDG_D(n) \
  case n: hipLaunchKernelGGL(k_div<n>, dim3(blocks(a.K)), dim3(kThreads), 0, s, a); break;
    IPDG_D(1) IPDG_D(2) IPDG_D(3) IPDG_D(4) IPDG_D(5) IPDG_D(6) IPDG_D(7) IPDG_D(8)
#undef IPDG_D
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ipdg
