"""DG gradient and divergence of the oracle, and the projection half of the
algebraic splitting step (TEST INFRASTRUCTURE ONLY: imported by tests/).

Sec. 2.1, Eq. INS_SD_4_1 and INS_SD_4_2: multiplying by a test function and
integrating by parts twice with the central fluxes p* = {p}, u* = {u} gives,
per element and in strong nodal form,

    G p = grad p + LIFT (|F|/|E|) n (p* - p-),
    D u = div u  + LIFT (|F|/|E|) n . (u* - u-),

with the boundary rules of the same section: on Dirichlet (velocity) faces
u* = g_D and p* = p-, on Neumann faces u* = u- and p* = 0.  The face terms use
the reference lift (the inverse mass matrix times the face mass), so the
matrices below are exactly M^-1 times the integrals of the variational forms.

Sec. 2.2, Eq. INS_TD_3_3 and INS_TD_3_4 (the steps after the velocity
Helmholtz solve): the pressure increment solves -L dP = -(gamma / dt) D U^^,
and the velocity is corrected as U = U^^ - (dt / gamma) G dP, the pressure as
P = dP + sigma P.  With the mass-weighted SIPDG stiffness S = -M L of
``assemble`` (lambda = 0) the increment solves S dP = -(gamma / dt) M D U^^.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .assemble import BC_DIRICHLET, BC_INTERIOR, BC_NEUMANN, OracleMesh, mass_matrix
from .matfree import MatFree


def grad_div_matrices(m: OracleMesh):
    """(Gx, Gy, Dx, Dy, Bx, By): G p = (Gx p, Gy p); D (u, v) = Dx u + Dy v +
    Bx gu + By gv, with gu, gv nodal fields whose values on Dirichlet face
    nodes are the boundary data g_D (elsewhere unused)."""
    mf = MatFree(m)
    K, Np, Nfp = m.K, mf.Np, mf.Nfp
    n = K * Np
    rows, cols = [], []
    val = {k: [] for k in ("gx", "gy", "dx", "dy", "bx", "by")}

    def add(r, c, gx, gy, dx, dy, bx, by):
        rows.append(r)
        cols.append(c)
        val["gx"].append(gx)
        val["gy"].append(gy)
        val["dx"].append(dx)
        val["dy"].append(dy)
        val["bx"].append(bx)
        val["by"].append(by)

    for e in range(K):
        base = e * Np
        rx, sx, ry, sy = m.rx[e], m.sx[e], m.ry[e], m.sy[e]
        # volume: grad = (rx Dr + sx Ds, ry Dr + sy Ds)
        Vx = rx * mf.Dr + sx * mf.Ds
        Vy = ry * mf.Dr + sy * mf.Ds
        for i in range(Np):
            for j in range(Np):
                add(base + i, base + j, Vx[i, j], Vy[i, j], Vx[i, j], Vy[i, j], 0.0, 0.0)
        for f in range(3):
            bc = m.EToB[e, f]
            L = mf.LIFT[:, f * Nfp:(f + 1) * Nfp]               # (Np, Nfp)
            sc = mf.fscale[e, f]
            nx, ny = mf.nx[e, f], mf.ny[e, f]
            for k in range(Nfp):
                jm = mf.vmapM[e, f, k]
                jp = mf.vmapP[e, f, k]
                for i in range(Np):
                    w = L[i, k] * sc
                    if bc == BC_INTERIOR:
                        # p* - p- = (p+ - p-) / 2, the same for u
                        add(base + i, jp, 0.5 * w * nx, 0.5 * w * ny, 0.5 * w * nx, 0.5 * w * ny, 0, 0)
                        add(base + i, jm, -0.5 * w * nx, -0.5 * w * ny, -0.5 * w * nx, -0.5 * w * ny, 0, 0)
                    elif bc == BC_DIRICHLET:
                        # p* = p-: no pressure term; u* = g_D: -u- plus the data
                        add(base + i, jm, 0.0, 0.0, -w * nx, -w * ny, w * nx, w * ny)
                    elif bc == BC_NEUMANN:
                        # p* = 0: -p-; u* = u-: no velocity term
                        add(base + i, jm, -w * nx, -w * ny, 0.0, 0.0, 0.0, 0.0)
    out = []
    for k in ("gx", "gy", "dx", "dy", "bx", "by"):
        out.append(sp.csr_matrix((val[k], (rows, cols)), shape=(n, n)))
    return tuple(out)


class GradDiv:
    """The gradient and divergence of one mesh, with the projection step."""

    def __init__(self, m: OracleMesh):
        self.m = m
        self.Gx, self.Gy, self.Dx, self.Dy, self.Bx, self.By = grad_div_matrices(m)
        self.M = mass_matrix(m)

    def grad(self, p):
        return self.Gx @ p, self.Gy @ p

    def div(self, u, v, gu=None, gv=None):
        d = self.Dx @ u + self.Dy @ v
        if gu is not None:
            d = d + self.Bx @ gu
        if gv is not None:
            d = d + self.By @ gv
        return d

    def pressure_rhs(self, gamma, dt, u, v, gu=None, gv=None):
        """-(gamma / dt) M D U^^: the right-hand side of S dP (Eq. INS_TD_3_3)."""
        return -(gamma / dt) * (self.M @ self.div(u, v, gu, gv))

    def correct(self, gamma, dt, u, v, dp, sigma_p):
        """Eq. INS_TD_3_4: U = U^^ - (dt / gamma) G dP, P = dP + sigma P."""
        gx, gy = self.grad(dp)
        return u - (dt / gamma) * gx, v - (dt / gamma) * gy, dp + sigma_p


def swapped_bc(EToB):
    """Pressure boundary flags of a velocity mesh: Dirichlet velocity faces
    are Neumann for the pressure, Neumann (outflow) faces Dirichlet."""
    B = np.array(EToB, copy=True)
    d = B == BC_DIRICHLET
    nm = B == BC_NEUMANN
    B[d] = BC_NEUMANN
    B[nm] = BC_DIRICHLET
    return B
