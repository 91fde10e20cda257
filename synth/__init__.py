"""Seeded synthetic workloads for the IPDG elliptic solver.

This module only draws inputs: meshes (vertex coordinates, element-to-vertex
lists, boundary flags), random nodal fields and the per-solve parameter draws
of the batched and differentiable workloads.  It holds none of the method's
arithmetic (no basis, no quadrature, no operator), so that the CPU oracle and
the GPU path can both consume the same arrays without sharing any code.

Mesh convention (shared data format, both sides implement it on their own):
  * EToV is int32 (K, 3), counter-clockwise, 0-based vertex ids;
  * face f of an element joins local vertices (f, (f+1) % 3);
  * EToB is int8 (K, 3): 0 = interior face, 1 = Dirichlet, 2 = Neumann.

The structured mesh splits each square of an n x n grid on the unit square by
its (i,j)-(i+1,j+1) diagonal into two counter-clockwise triangles.
"""
from __future__ import annotations

import numpy as np

BC_INTERIOR = 0
BC_DIRICHLET = 1
BC_NEUMANN = 2


class Mesh:
    """Plain container of mesh arrays (host, numpy)."""

    def __init__(self, VX, VY, EToV, EToB, n=None):
        self.VX = np.ascontiguousarray(VX, dtype=np.float64)
        self.VY = np.ascontiguousarray(VY, dtype=np.float64)
        self.EToV = np.ascontiguousarray(EToV, dtype=np.int32)
        self.EToB = np.ascontiguousarray(EToB, dtype=np.int8)
        self.n = n

    @property
    def K(self):
        return self.EToV.shape[0]

    @property
    def Nv(self):
        return self.VX.shape[0]


def square_mesh(n: int, jitter: float = 0.0, seed: int = 0, bc: str = "dirichlet",
                x0: float = 0.0, y0: float = 0.0, L: float = 1.0) -> Mesh:
    """n x n squares on [x0, x0+L] x [y0, y0+L], each split into 2 triangles.

    Vertex (i, j) has id j*(n+1) + i.  Square (i, j) yields element
    2*(j*n + i) (lower-right triangle) and 2*(j*n + i) + 1 (upper-left).
    ``jitter`` moves interior vertices by U(-jitter*h, jitter*h) in x and y
    (PCG64 stream of ``seed``).  ``bc`` is 'dirichlet', 'neumann' or 'mixed'
    (mixed: Dirichlet on x = x0 and y = y0, Neumann on the other two sides).
    """
    h = L / n
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    VX = (x0 + ii * h).astype(np.float64).ravel()
    VY = (y0 + jj * h).astype(np.float64).ravel()
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        interior = ((ii > 0) & (ii < n) & (jj > 0) & (jj < n)).ravel()
        d = rng.uniform(-jitter * h, jitter * h, size=(VX.size, 2))
        VX = VX + np.where(interior, d[:, 0], 0.0)
        VY = VY + np.where(interior, d[:, 1], 0.0)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    v00 = j * (n + 1) + i
    v10 = v00 + 1
    v01 = v00 + (n + 1)
    v11 = v01 + 1
    EToV = np.empty((2 * n * n, 3), dtype=np.int32)
    EToV[0::2] = np.stack([v00, v10, v11], axis=1)   # lower-right, CCW
    EToV[1::2] = np.stack([v00, v11, v01], axis=1)   # upper-left, CCW
    EToB = boundary_flags(VX, VY, EToV, bc, x0, y0, L)
    return Mesh(VX, VY, EToV, EToB, n=n)


def boundary_flags(VX, VY, EToV, bc: str, x0=0.0, y0=0.0, L=1.0):
    """Flag faces lying on the boundary of the square [x0,x0+L]^2."""
    K = EToV.shape[0]
    EToB = np.zeros((K, 3), dtype=np.int8)
    tol = 1e-12 * max(L, 1.0)
    for f in range(3):
        a = EToV[:, f]
        b = EToV[:, (f + 1) % 3]
        xa, ya, xb, yb = VX[a], VY[a], VX[b], VY[b]
        left = (np.abs(xa - x0) < tol) & (np.abs(xb - x0) < tol)
        right = (np.abs(xa - x0 - L) < tol) & (np.abs(xb - x0 - L) < tol)
        bottom = (np.abs(ya - y0) < tol) & (np.abs(yb - y0) < tol)
        top = (np.abs(ya - y0 - L) < tol) & (np.abs(yb - y0 - L) < tol)
        onb = left | right | bottom | top
        if bc == "dirichlet":
            EToB[onb, f] = BC_DIRICHLET
        elif bc == "neumann":
            EToB[onb, f] = BC_NEUMANN
        elif bc == "mixed":
            EToB[left | bottom, f] = BC_DIRICHLET
            EToB[right | top, f] = BC_NEUMANN
        else:
            raise ValueError(f"unknown bc {bc!r}")
    return EToB


def permuted(mesh: Mesh, seed: int) -> Mesh:
    """Same triangulation with elements shuffled and each element's vertex list
    rotated by a random amount (orientation kept CCW).  Exercises unstructured
    neighbour patterns and all face-pair orientations."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(mesh.K)
    rot = rng.integers(0, 3, size=mesh.K)
    EToV = mesh.EToV[perm]
    EToB = mesh.EToB[perm]
    idx = (np.arange(3)[None, :] + rot[:, None]) % 3
    EToV = np.take_along_axis(EToV, idx, axis=1)
    EToB = np.take_along_axis(EToB, idx, axis=1)
    return Mesh(mesh.VX, mesh.VY, EToV, EToB, n=mesh.n)


def nodal_normal(K: int, Np: int, seed: int) -> np.ndarray:
    """x ~ N(0,1) per node, element-major (K*Np,), PCG64 stream of ``seed``."""
    return np.random.default_rng(seed).standard_normal(K * Np)


def np_of(N: int) -> int:
    """Number of nodes of a degree-N triangle (a counting fact, no arithmetic
    of the method)."""
    return (N + 1) * (N + 2) // 2


# -- workload recipes ---------------------------------------------------------

def ax_sweep_mesh(n: int = 512, seed: int = 0) -> Mesh:
    """Ax throughput workload: n x n squares (2 n^2 triangles), interior
    vertices jittered by +-0.2 h, all faces Dirichlet."""
    return square_mesh(n, jitter=0.2, seed=seed, bc="dirichlet")


def batch_draws(nb: int = 64, seed: int = 4, nmin: int = 32, nmax: int = 128,
                Nmin: int = 4, Nmax: int = 8):
    """Per-solve draws of the batched Helmholtz workload: mesh size n_i ~
    U{nmin..nmax}, order N_i ~ U{Nmin..Nmax}, lambda_i = 10^U(0,3)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=nb)
    Ns = rng.integers(Nmin, Nmax + 1, size=nb)
    lams = 10.0 ** rng.uniform(0.0, 3.0, size=nb)
    fseeds = rng.integers(0, 2**31 - 1, size=nb)
    return ns, Ns, lams, fseeds


def kappa_draw(K: int, seed: int = 2, sigma: float = 0.5) -> np.ndarray:
    """Per-element coefficient kappa_e = exp(sigma * N(0,1))."""
    return np.exp(sigma * np.random.default_rng(seed).standard_normal(K))


def smooth_coeffs(seed: int = 3, kmax: int = 4) -> np.ndarray:
    """Coefficients a_kl ~ N(0,1)/(k^2+l^2), k,l = 1..kmax, of a smooth target
    u_t = sum a_kl sin(k pi x) sin(l pi y)."""
    rng = np.random.default_rng(seed)
    k = np.arange(1, kmax + 1)
    return rng.standard_normal((kmax, kmax)) / (k[:, None] ** 2 + k[None, :] ** 2)


def smooth_field(x: np.ndarray, y: np.ndarray, coeffs: np.ndarray) -> np.ndarray:
    """Evaluate sum a_kl sin(k pi x) sin(l pi y) at given points."""
    out = np.zeros_like(x)
    kmax = coeffs.shape[0]
    for k in range(1, kmax + 1):
        sx = np.sin(k * np.pi * x)
        for l in range(1, kmax + 1):
            out += coeffs[k - 1, l - 1] * sx * np.sin(l * np.pi * y)
    return out
