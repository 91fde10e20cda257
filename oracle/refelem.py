"""Reference triangle for the oracle (TEST INFRASTRUCTURE ONLY).

Follows Sec. 2.1 (nodal Lagrange basis of P_N at Warp & Blend nodes) and the
reference-element mapping of Sec. 5.2 (bi-unit triangle -1 <= r, s, r+s <= 1
with vertices (-1,-1), (1,-1), (-1,1)).

Everything here is built independently of the GPU library's host setup:
  * the Lagrange basis is evaluated as psi(r,s)^T V^{-1} with psi the
    orthonormal Dubiner basis written through scipy's Jacobi polynomials;
  * integrals (mass, stiffness, face mass) are taken with collapsed-coordinate
    (Duffy) Gauss-Legendre quadrature, never from Vandermonde identities.

Node order: row by row, j = 0..N (distance from face 0), i = 0..N-j along face
0.  Faces: 0 = v0v1 (s = -1), 1 = v1v2 (r + s = 0), 2 = v2v0 (r = -1).
"""
from __future__ import annotations

import functools
import math

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.special import eval_jacobi, gammaln

# Optimised blending parameters alpha of the Warp & Blend construction, for
# N = 1..15, from Warburton's explicit construction of interpolation nodes on
# the simplex (the node family the paper cites in Sec. 2.1).  They only move
# interior nodes (N >= 4 here); the discrete operator, as a map on P_N, does
# not depend on them.
_WB_ALPHA = (0.0000, 0.0000, 1.4152, 0.1001, 0.2751, 0.9800, 1.0999, 1.2832,
             1.3648, 1.4773, 1.4959, 1.5743, 1.5770, 1.6223, 1.6258)


def np_of(N: int) -> int:
    return (N + 1) * (N + 2) // 2


# ---------------------------------------------------------------------------
# 1-D building blocks
# ---------------------------------------------------------------------------

def jacobi_normalized(x, a: float, b: float, n: int):
    """Jacobi polynomial P_n^{(a,b)} normalised to unit L2 norm under the
    weight (1-x)^a (1+x)^b on [-1, 1]."""
    logh = ((a + b + 1) * math.log(2.0) - math.log(2 * n + a + b + 1)
            + gammaln(n + a + 1) + gammaln(n + b + 1)
            - gammaln(n + a + b + 1) - gammaln(n + 1))
    return eval_jacobi(n, a, b, x) / math.exp(0.5 * logh)


def jacobi_normalized_deriv(x, a: float, b: float, n: int):
    """d/dx of ``jacobi_normalized`` (uses dP_n^{(a,b)}/dx =
    (n+a+b+1)/2 P_{n-1}^{(a+1,b+1)})."""
    if n == 0:
        return np.zeros_like(np.asarray(x, dtype=np.float64))
    logh = ((a + b + 1) * math.log(2.0) - math.log(2 * n + a + b + 1)
            + gammaln(n + a + 1) + gammaln(n + b + 1)
            - gammaln(n + a + b + 1) - gammaln(n + 1))
    d = 0.5 * (n + a + b + 1) * eval_jacobi(n - 1, a + 1, b + 1, x)
    return d / math.exp(0.5 * logh)


def gauss_legendre(q: int):
    """q-point Gauss-Legendre rule on [-1, 1] (exact to degree 2q-1)."""
    return npleg.leggauss(q)


def gll_points(N: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre points: -1, 1 and the roots of P_N'."""
    if N == 1:
        return np.array([-1.0, 1.0])
    inner = npleg.Legendre.basis(N).deriv().roots()
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


# ---------------------------------------------------------------------------
# Warp & Blend nodes
# ---------------------------------------------------------------------------

def _warp(N: int, rout: np.ndarray) -> np.ndarray:
    """1-D warp: displacement from equispaced to GLL points, interpolated at
    ``rout`` by the degree-N polynomial through the equispaced points and
    divided by the edge bubble 1 - r^2 (zero at the end points)."""
    req = np.linspace(-1.0, 1.0, N + 1)
    disp = gll_points(N) - req
    # Lagrange interpolation through equispaced points (plain products).
    w = np.zeros_like(rout)
    for i in range(N + 1):
        li = np.ones_like(rout)
        for j in range(N + 1):
            if j != i:
                li = li * (rout - req[j]) / (req[i] - req[j])
        w = w + disp[i] * li
    inner = np.abs(rout) < 1.0 - 1e-10
    out = np.zeros_like(rout)
    out[inner] = w[inner] / (1.0 - rout[inner] ** 2)
    return out


@functools.lru_cache(maxsize=None)
def wb_nodes(N: int):
    """Warp & Blend nodes (r, s) on the bi-unit triangle, in node order."""
    alpha = _WB_ALPHA[N - 1] if N <= len(_WB_ALPHA) else 5.0 / 3.0
    L1l, L3l = [], []
    for j in range(N + 1):
        for i in range(N + 1 - j):
            L1l.append(j / N)
            L3l.append(i / N)
    L1 = np.array(L1l)
    L3 = np.array(L3l)
    L2 = 1.0 - L1 - L3
    # equilateral triangle with vertices (-1,-1/sqrt3), (1,-1/sqrt3), (0,2/sqrt3)
    x = -L2 + L3
    y = (-L2 - L3 + 2.0 * L1) / math.sqrt(3.0)
    b1 = 4.0 * L2 * L3
    b2 = 4.0 * L1 * L3
    b3 = 4.0 * L1 * L2
    w1 = b1 * _warp(N, L3 - L2) * (1.0 + (alpha * L1) ** 2)
    w2 = b2 * _warp(N, L1 - L3) * (1.0 + (alpha * L2) ** 2)
    w3 = b3 * _warp(N, L2 - L1) * (1.0 + (alpha * L3) ** 2)
    x = x + w1 + math.cos(2 * math.pi / 3) * w2 + math.cos(4 * math.pi / 3) * w3
    y = y + math.sin(2 * math.pi / 3) * w2 + math.sin(4 * math.pi / 3) * w3
    # equilateral -> barycentric -> bi-unit (r, s)
    l1 = (math.sqrt(3.0) * y + 1.0) / 3.0
    l2 = (-3.0 * x - math.sqrt(3.0) * y + 2.0) / 6.0
    l3 = (3.0 * x - math.sqrt(3.0) * y + 2.0) / 6.0
    r = -l2 + l3 - l1
    s = -l2 - l3 + l1
    return r, s


def face_node_ids(N: int):
    """Volume-node ids on faces 0, 1, 2, each ordered counter-clockwise along
    the element boundary."""
    ids = {}
    k = 0
    for j in range(N + 1):
        for i in range(N + 1 - j):
            ids[(i, j)] = k
            k += 1
    f0 = [ids[(i, 0)] for i in range(N + 1)]
    f1 = [ids[(N - j, j)] for j in range(N + 1)]
    f2 = [ids[(0, N - j)] for j in range(N + 1)]
    return np.array([f0, f1, f2], dtype=np.int64)


# ---------------------------------------------------------------------------
# Orthonormal (Dubiner) basis on the triangle and the nodal Lagrange basis
# ---------------------------------------------------------------------------

def _collapse(r, s):
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    a = np.full_like(r, -1.0)
    ok = np.abs(1.0 - s) > 1e-14
    a[ok] = 2.0 * (1.0 + r[ok]) / (1.0 - s[ok]) - 1.0
    return a, s


def dubiner(N: int, r, s):
    """Values and (r, s)-gradients of the orthonormal basis psi_{ij}, i+j <= N,
    at points (r, s).  Returns three arrays of shape (npts, Np).
    psi_ij = sqrt2 P_i(a) P_j^{(2i+1,0)}(b) (1-b)^i, a, b collapsed coords."""
    a, b = _collapse(r, s)
    cols, dr, ds = [], [], []
    for i in range(N + 1):
        for j in range(N + 1 - i):
            fa = jacobi_normalized(a, 0.0, 0.0, i)
            dfa = jacobi_normalized_deriv(a, 0.0, 0.0, i)
            gb = jacobi_normalized(b, 2.0 * i + 1.0, 0.0, j)
            dgb = jacobi_normalized_deriv(b, 2.0 * i + 1.0, 0.0, j)
            omb = 1.0 - b
            cols.append(math.sqrt(2.0) * fa * gb * omb ** i)
            if i == 0:
                d_r = np.zeros_like(a)
                d_s = math.sqrt(2.0) * fa * dgb
            else:
                d_r = math.sqrt(2.0) * dfa * gb * 2.0 * omb ** (i - 1)
                d_s = math.sqrt(2.0) * (dfa * gb * omb ** (i - 1) * (1.0 + a)
                                        + fa * (dgb * omb ** i - i * gb * omb ** (i - 1)))
            dr.append(d_r)
            ds.append(d_s)
    return np.stack(cols, 1), np.stack(dr, 1), np.stack(ds, 1)


class RefTriangle:
    """Nodal degree-N reference triangle of the oracle."""

    def __init__(self, N: int):
        self.N = N
        self.Np = np_of(N)
        self.Nfp = N + 1
        self.r, self.s = wb_nodes(N)
        self.Fmask = face_node_ids(N)
        V, _, _ = dubiner(N, self.r, self.s)
        self.V = V
        self.Vinv = np.linalg.inv(V)
        # volume quadrature (Duffy), exact to degree 2N+3 in each collapsed
        # direction
        q = N + 3
        ga, wa = gauss_legendre(q)
        A, B = np.meshgrid(ga, ga, indexing="ij")
        WA, WB = np.meshgrid(wa, wa, indexing="ij")
        self.qr = ((1.0 + A) * (1.0 - B) / 2.0 - 1.0).ravel()
        self.qs = B.ravel()
        self.qw = (WA * WB * (1.0 - B) / 2.0).ravel()
        self.qL, self.qLr, self.qLs = self.lagrange(self.qr, self.qs)
        # 1-D rule for faces
        self.g1, self.w1 = gauss_legendre(N + 3)

    def lagrange(self, r, s):
        """Nodal Lagrange basis (values, d/dr, d/ds) at points (r, s)."""
        P, Pr, Ps = dubiner(self.N, r, s)
        return P @ self.Vinv, Pr @ self.Vinv, Ps @ self.Vinv

    # -- reference operators, computed by quadrature (for pins and for the
    #    p-multigrid reference), never used to build the GPU operators --
    def mass(self):
        L = self.qL
        return (L * self.qw[:, None]).T @ L

    def face_points(self, f, t):
        """Reference coordinates of face f at the 1-D parameter t in [-1, 1],
        running counter-clockwise from vertex f to vertex (f+1) % 3."""
        t = np.asarray(t, dtype=np.float64)
        if f == 0:
            return t, -np.ones_like(t)
        if f == 1:
            return -t, t
        return -np.ones_like(t), -t

    def lift(self):
        """LIFT = M^{-1} E (Np x 3 Nfp, Eq. elLift on the reference element):
        column f Nfp + k holds face f's mass against face node k,
        E_ij = int_{-1}^{1} l_i l_j dt along the face parameter of length 2
        (the physical length enters through the surface factor), by 1-D
        Gauss quadrature."""
        g, w = self.g1, self.w1
        E = np.zeros((self.Np, 3 * self.Nfp))
        for f in range(3):
            Lf, _, _ = self.lagrange(*self.face_points(f, g))
            Ef = (Lf * w[:, None]).T @ Lf
            E[:, f * self.Nfp:(f + 1) * self.Nfp] = Ef[:, self.Fmask[f]]
        return np.linalg.solve(self.mass(), E)

    def deriv_matrices(self):
        """D_r, D_s with (D_r u)_i = d/dr of the interpolant at node i,
        obtained from the L2 projection M^{-1} (l_i, d l_j/dr)."""
        M = self.mass()
        Sr = (self.qL * self.qw[:, None]).T @ self.qLr
        Ss = (self.qL * self.qw[:, None]).T @ self.qLs
        return np.linalg.solve(M, Sr), np.linalg.solve(M, Ss)
