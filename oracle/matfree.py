"""Matrix-free SIPDG operator of the oracle (TEST INFRASTRUCTURE ONLY).

The steps of the paper's two GPU kernels, written out plainly over all
elements at once (Sec. 5.2):

  * Alg. AxG (local gradient): u_r = D_r u, u_s = D_s u per element, then
    u_x = r_x u_r + s_x u_s, u_y = r_y u_r + s_y u_s with the geometric
    factors G = (r_x, s_x, r_y, s_y) of Eq. operators2;
  * Alg. AxKernel (SIPDG kernel), i.e. Eq. ellipticOp3 mapped to the reference
    element with Eq. elementOps: lifted jumps L = 1/2 sum_f n_f (J^ef/J^e)
    L^f [u]_f, the volume term -D . (grad u + L), the surface term
    s = (J^ef/J^e) (1/2 n . [grad u] + tau [u] - n . L^-) lifted with the
    reference lift, then the mass matrix J^e M.

Traces are taken through index maps vmapM / vmapP (the paper's idM / idP)
built here by matching physical node coordinates, so no face-orientation
convention enters.  Readings where the paper's listing is garbled or silent
(each stated in the design notes):

  * the L_y line of Alg. AxKernel uses n_y (the listing repeats n_x);
  * the face factors n, J^ef inside the sum belong to each face f;
  * the volume term sums D_ij (.)_j with the index inside the sum;
  * the trace term of Eq. ellipticOp3 is the normal component of the vector
    lift, n . L^-, as Alg. AxKernel computes it;
  * lambda J^e M u is added (absent from Eq. ellipticOp3 and the listing);
  * boundary faces take the mirror ghost state (Dirichlet u+ = -u-,
    grad u+ = grad u-; Neumann u+ = u-, n . grad u+ = -n . grad u-), and
    tau_F = c_tau max(kappa- J^ef/J^e, kappa+ ...) (one-sided on the boundary);
  * with a per-element coefficient kappa: the volume and lift terms carry
    kappa_e and the flux jump is [kappa grad u] (the kappa-weighted form of
    the assembled operator).

The result is the same operator as ``assemble.assemble`` (an algebraic
identity, because every integral involved is exact); the tests pin the two
together at round-off.
"""
from __future__ import annotations

import numpy as np

from .assemble import BC_DIRICHLET, BC_INTERIOR, BC_NEUMANN, OracleMesh


class MatFree:
    """Reference operators, geometric factors and trace maps of one mesh."""

    def __init__(self, m: OracleMesh):
        self.m = m
        ref = m.ref
        self.Np, self.Nfp = ref.Np, ref.Nfp
        self.Dr, self.Ds = ref.deriv_matrices()
        self.M = ref.mass()
        self.LIFT = ref.lift()
        K, Nfp = m.K, self.Nfp
        # surface factors per (element, face): outward unit normal and
        # J^ef / J^e = |F| / |E|
        self.nx = np.zeros((K, 3))
        self.ny = np.zeros((K, 3))
        self.fscale = np.zeros((K, 3))
        e = np.arange(K)
        for f in range(3):
            _, _, _, _, length, nx, ny = m.face_geometry(e, f)
            self.nx[:, f], self.ny[:, f] = nx, ny
            self.fscale[:, f] = length / m.area
        # vmapM: volume index of each face node; vmapP: the index of the node
        # at the same physical position in the neighbour (self on boundaries)
        Fm = ref.Fmask                                    # (3, Nfp)
        self.vmapM = (e[:, None, None] * self.Np + Fm[None]).astype(np.int64)
        x, y = m.node_coords()
        X, Y = x.ravel(), y.ravel()
        self.vmapP = self.vmapM.copy()
        for f in range(3):
            nb = m.EToE[:, f]
            inner = np.flatnonzero(nb >= 0)
            if inner.size == 0:
                continue
            fp = m.EToF[inner, f]
            cand = nb[inner, None] * self.Np + Fm[fp]          # (n, Nfp)
            own = self.vmapM[inner, f]                        # (n, Nfp)
            d = (np.abs(X[own][:, :, None] - X[cand][:, None, :])
                 + np.abs(Y[own][:, :, None] - Y[cand][:, None, :]))
            k = np.argmin(d, axis=2)
            self.vmapP[inner, f] = np.take_along_axis(cand, k, axis=1)
        self.bc = m.EToB.copy()

    # -- Alg. AxG -----------------------------------------------------------
    def local_gradient(self, u):
        """(u_x, u_y), each K x Np."""
        m = self.m
        U = np.asarray(u, dtype=np.float64).reshape(m.K, self.Np)
        ur = U @ self.Dr.T
        us = U @ self.Ds.T
        ux = m.rx[:, None] * ur + m.sx[:, None] * us
        uy = m.ry[:, None] * ur + m.sy[:, None] * us
        return ux, uy

    # -- Alg. AxKernel ------------------------------------------------------
    def apply(self, lam: float, ctau: float, u, kappa=None, elems=None):
        """y = A u for the elements ``elems`` (default: all), shape
        (len(elems) * Np,) -- the rows of those elements."""
        m = self.m
        Np, Nfp = self.Np, self.Nfp
        K = m.K
        U = np.asarray(u, dtype=np.float64).reshape(K, Np)
        kap = np.ones(K) if kappa is None else np.asarray(kappa, dtype=np.float64)
        E = np.arange(K) if elems is None else np.asarray(elems, dtype=np.int64)
        # the gradient is needed on the elements and their neighbours
        need = np.unique(np.r_[E, m.EToE[E][m.EToE[E] >= 0]])
        ux = np.zeros((K, Np))
        uy = np.zeros((K, Np))
        sub_x, sub_y = self.local_gradient_rows(U, need)
        ux[need], uy[need] = sub_x, sub_y
        uf, uxf, uyf = U.ravel(), ux.ravel(), uy.ravel()

        vM, vP = self.vmapM[E], self.vmapP[E]                 # (n, 3, Nfp)
        bc = self.bc[E][:, :, None]
        nx, ny = self.nx[E][:, :, None], self.ny[E][:, :, None]
        fs = self.fscale[E]                                   # (n, 3)
        km = kap[E]
        nbr = np.where(m.EToE[E] >= 0, m.EToE[E], E[:, None])
        kp = np.where(self.bc[E] == BC_INTERIOR, kap[nbr], km[:, None])

        # traces and the mirror ghost states; jump [u] = u+ - u-
        uM, uP = uf[vM], uf[vP]
        uP = np.where(bc == BC_DIRICHLET, -uM, uP)
        du = uP - uM
        gxM, gyM = uxf[vM], uyf[vM]
        gxP, gyP = uxf[vP], uyf[vP]
        dnM = nx * gxM + ny * gyM
        # Neumann: reflect the normal component of the ghost gradient
        gxP = np.where(bc == BC_NEUMANN, gxM - 2 * nx * dnM, gxP)
        gyP = np.where(bc == BC_NEUMANN, gyM - 2 * ny * dnM, gyP)
        gxP = np.where(bc == BC_DIRICHLET, gxM, gxP)
        gyP = np.where(bc == BC_DIRICHLET, gyM, gyP)

        # lifted jumps L = 1/2 sum_f n_f (J^ef/J^e) L^f [u]_f (a vector field)
        Lx = np.zeros((E.size, Np))
        Ly = np.zeros((E.size, Np))
        for f in range(3):
            lf = du[:, f, :] @ self.LIFT[:, f * Nfp:(f + 1) * Nfp].T   # (n, Np)
            Lx += 0.5 * (self.nx[E, f] * fs[:, f])[:, None] * lf
            Ly += 0.5 * (self.ny[E, f] * fs[:, f])[:, None] * lf

        # volume contribution -D . (grad u + L), weighted by kappa_e
        rx, sx, ry, sy = m.rx[E][:, None], m.sx[E][:, None], m.ry[E][:, None], m.sy[E][:, None]
        qx = ux[E] + Lx
        qy = uy[E] + Ly
        Au = -((rx * qx + ry * qy) @ self.Dr.T) - ((sx * qx + sy * qy) @ self.Ds.T)
        Au *= km[:, None]

        # surface contribution s at the face nodes, then its lift
        Fm = m.ref.Fmask
        LxM = np.stack([Lx[:, Fm[f]] for f in range(3)], 1)           # (n, 3, Nfp)
        LyM = np.stack([Ly[:, Fm[f]] for f in range(3)], 1)
        hM = fs
        nbr_fs = np.where(self.bc[E] == BC_INTERIOR, self._fscale_across(E), hM)
        tau = ctau * np.maximum(km[:, None] * hM,
                                np.where(self.bc[E] == BC_INTERIOR, kp * nbr_fs, 0.0))
        flux = (nx * (kp[:, :, None] * gxP - km[:, None, None] * gxM)
                + ny * (kp[:, :, None] * gyP - km[:, None, None] * gyM))
        s = fs[:, :, None] * (0.5 * flux + tau[:, :, None] * du
                              - km[:, None, None] * (nx * LxM + ny * LyM))
        Au -= s.reshape(E.size, 3 * Nfp) @ self.LIFT.T

        # mass matrix J^e M, and the screening term lambda J^e M u
        y = m.J[E][:, None] * ((Au + lam * U[E]) @ self.M.T)
        return y.ravel()

    def local_gradient_rows(self, U, rows):
        m = self.m
        Ur = U[rows]
        ur = Ur @ self.Dr.T
        us = Ur @ self.Ds.T
        ux = m.rx[rows, None] * ur + m.sx[rows, None] * us
        uy = m.ry[rows, None] * ur + m.sy[rows, None] * us
        return ux, uy

    def _fscale_across(self, E):
        """|F| / |E+| of the neighbour across each face of the elements E
        (the element's own value on boundary faces)."""
        m = self.m
        nb = m.EToE[E]
        nbs = np.where(nb >= 0, nb, E[:, None])
        f2 = np.where(nb >= 0, m.EToF[E], 0)
        return np.where(nb >= 0, self.fscale[nbs, f2], self.fscale[E])


def apply(m: OracleMesh, lam: float, ctau: float, u, kappa=None) -> np.ndarray:
    """y = A u over the whole mesh, matrix-free."""
    return MatFree(m).apply(lam, ctau, u, kappa=kappa)
