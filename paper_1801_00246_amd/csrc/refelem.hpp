// Nodal reference triangle of degree N (1..8) for the device operators.
//
// Sec. 2.1: Lagrange basis of P_N at Warp & Blend nodes.  Sec. 5.2
// (Eq. elMass, elStiff, elLift, elementOps): reference mass M, derivative
// matrices D_r, D_s and lift L = M^{-1} E on the bi-unit triangle
// (-1,-1), (1,-1), (-1,1).  Built here from the orthonormal (Dubiner) basis
// and its Vandermonde matrix V: D_r = V_r V^{-1}, M = (V V^T)^{-1}.
#pragma once
#include <vector>

namespace ipdg {

constexpr int kMaxN = 8;

struct RefOps {
  int N = 0, Np = 0, Nfp = 0;
  std::vector<double> r, s;         // nodes
  std::vector<int> fmask;           // 3 x Nfp node ids, each face counter-clockwise
  std::vector<double> Dr, Ds;       // Np x Np, row-major
  std::vector<double> M, Minv;      // Np x Np
  std::vector<double> Sr, Ss;       // M Dr, M Ds
  std::vector<double> LIFT;         // Np x (3 Nfp)
  std::vector<double> M1D;          // Nfp x Nfp face mass on [-1, 1]
  std::vector<int> rot[3];          // rot[k][n]: node of the unrotated triangle
                                    // sitting at node n of the frame whose
                                    // vertex 0 is vertex k
};

// Cached per degree; throws std::runtime_error on internal inconsistency.
const RefOps& ref_ops(int N);

// Np(Nf) x Np(Nc): degree-Nc Lagrange basis evaluated at degree-Nf nodes.
std::vector<double> interp_matrix(int Nc, int Nf);

inline int np_of(int N) { return (N + 1) * (N + 2) / 2; }

// Cubature operators of the subcycling advection term (Sec. 5.3, Eq. KSS_3).
// Volume: the collapsed-coordinate product of two q-point Gauss-Legendre
// rules, q = floor(3N/2) + 1, exact for the degree-(3N-1) volume integrand on
// an affine triangle.  Faces: the q-point Gauss-Legendre rule (exact to degree
// 3N), points running counter-clockwise like the face nodes.
struct CubOps {
  int N = 0, Np = 0, Nfp = 0, q = 0, Nc = 0, Nfc = 0;
  std::vector<double> I;       // Nc x Np: interpolation to the volume nodes
  std::vector<double> Pr, Ps;  // Np x Nc: M^{-1} (I dl/dr)^T W, M^{-1} (I dl/ds)^T W
  std::vector<double> If[3];   // Nfc x Nfp: face f's nodes to its Gauss points
  std::vector<double> Lc[3];   // Np x Nfc: cubature lift M^{-1} (I^f)^T W^f
};
inline int cub_points(int N) { return 3 * N / 2 + 1; }
// Cached per degree (1..8).
const CubOps& cub_ops(int N);

}  // namespace ipdg
