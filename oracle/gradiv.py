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


def dirichlet_rhs(m: OracleMesh, ctau: float, g, kappa=None):
    """Right-hand-side contribution of inhomogeneous Dirichlet data g to the
    SIPDG system of ``assemble`` (Sec. 2.1, Eq. INS_SD_5 with the boundary
    rules stated after it): the operator's Dirichlet faces take the mirror
    ghost u+ = 2 g - u-, so that u* = {u} = g; the terms that carry g move to
    the right-hand side,

        b_i = sum over Dirichlet faces of
              -kappa (g, d_n l_i)_F + 2 tau_F (g, l_i)_F,

    with tau_F = c_tau kappa |F| / |E| as in ``block_rows``.  g is a nodal
    field whose trace on each Dirichlet face (its face-node values) is the
    data.  A = b_f + b_g then reproduces any global polynomial of degree <= N
    exactly when g is its trace."""
    from .assemble import _physical_grad
    ref = m.ref
    Np = ref.Np
    kap = np.ones(m.K) if kappa is None else np.asarray(kappa, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64).reshape(m.K, Np)
    b = np.zeros((m.K, Np))
    gq, wq = ref.g1, ref.w1
    for f in range(3):
        ef = np.flatnonzero(m.EToB[:, f] == BC_DIRICHLET)
        if ef.size == 0:
            continue
        xa, ya, xb, yb, length, nx, ny = m.face_geometry(ef, f)
        t = gq[None, :]
        qx = 0.5 * (1 - t) * xa[:, None] + 0.5 * (1 + t) * xb[:, None]
        qy = 0.5 * (1 - t) * ya[:, None] + 0.5 * (1 + t) * yb[:, None]
        Wq = (0.5 * length)[:, None] * wq[None, :]
        rm, sm = m.to_ref(ef[:, None], qx, qy)
        V, Lr, Ls = ref.lagrange(rm.ravel(), sm.ravel())
        nF, q = qx.shape
        V = V.reshape(nF, q, Np)
        gx, gy = _physical_grad(m, ef, Lr.reshape(nF, q, Np), Ls.reshape(nF, q, Np))
        Dn = nx[:, None, None] * gx + ny[:, None, None] * gy        # d_n l_i at the points
        gval = np.einsum("fqj,fj->fq", V, g[ef])                     # trace of g
        tau = ctau * kap[ef] * length / m.area[ef]
        b[ef] += (-kap[ef][:, None] * np.einsum("fq,fqi->fi", Wq * gval, Dn)
                  + (2.0 * tau)[:, None] * np.einsum("fq,fqi->fi", Wq * gval, V))
    return b.ravel()


def advection(m: OracleMesh, u, v, gu=None, gv=None, lax=1.0):
    """Nonlinear term N(u) of Sec. 2.1 (Eq. INS_SD_2, INS_SD_3) for the
    velocity (u, v), component by component, in strong nodal form:

        N_c = div F_c(u) + LIFT (|F|/|E|) (n . F_c* - n . F_c(u-)),
        F_c(u) = u_c u,   n . F_c* = {n . F_c} + (Lambda / 2) (u_c- - u_c+),
        Lambda = 2 max(|n . u-|, |n . u+|),

    the flux products taken at the nodes (no cubature).  Readings: Lambda is
    the largest |eigenvalue| of n . dF/du = (n . u) I + u n^T over the segment
    [u-, u+] (eigenvalues n . u and 2 n . u; linear along the segment, so the
    maximum sits at an end); the jump term carries the dissipative sign
    (u- - u+), the paper's [u] = u+ - u- with its printed sign would remove
    energy from the wrong side.  Dirichlet faces take u+ = g_D (gu, gv nodal
    fields read on the face nodes; None = 0), Neumann faces u+ = u-.  ``lax``
    scales Lambda (1: the paper's flux; 0: the central flux, for tests)."""
    mf = MatFree(m)
    K, Np, Nfp = m.K, mf.Np, mf.Nfp
    U = np.asarray(u, dtype=np.float64).reshape(K, Np)
    V = np.asarray(v, dtype=np.float64).reshape(K, Np)
    GU = np.zeros((K, Np)) if gu is None else np.asarray(gu, dtype=np.float64).reshape(K, Np)
    GV = np.zeros((K, Np)) if gv is None else np.asarray(gv, dtype=np.float64).reshape(K, Np)
    rx, sx, ry, sy = (a[:, None] for a in (m.rx, m.sx, m.ry, m.sy))
    dx = lambda w: rx * (w @ mf.Dr.T) + sx * (w @ mf.Ds.T)
    dy = lambda w: ry * (w @ mf.Dr.T) + sy * (w @ mf.Ds.T)
    Nu = dx(U * U) + dy(U * V)
    Nv = dx(U * V) + dy(V * V)
    uf, vf = U.ravel(), V.ravel()
    for f in range(3):
        jm = mf.vmapM[:, f, :]                                 # (K, Nfp)
        jp = mf.vmapP[:, f, :]
        um, vm = uf[jm], vf[jm]
        up, vp = uf[jp], vf[jp]
        bc = m.EToB[:, f][:, None]
        dirich = np.broadcast_to(bc == BC_DIRICHLET, um.shape)
        neum = np.broadcast_to(bc == BC_NEUMANN, um.shape)
        up = np.where(dirich, GU.ravel()[jm], np.where(neum, um, up))
        vp = np.where(dirich, GV.ravel()[jm], np.where(neum, vm, vp))
        nx, ny = mf.nx[:, f][:, None], mf.ny[:, f][:, None]
        unm, unp = nx * um + ny * vm, nx * up + ny * vp        # n . u-, n . u+
        lam = lax * 2.0 * np.maximum(np.abs(unm), np.abs(unp))
        fu = 0.5 * (um * unm + up * unp) + 0.5 * lam * (um - up) - um * unm
        fv = 0.5 * (vm * unm + vp * unp) + 0.5 * lam * (vm - vp) - vm * unm
        L = mf.LIFT[:, f * Nfp:(f + 1) * Nfp]
        sc = mf.fscale[:, f][:, None]
        Nu += (sc * fu) @ L.T
        Nv += (sc * fv) @ L.T
    return Nu.ravel(), Nv.ravel()


def ins_step(m: OracleMesh, mp: OracleMesh, nu, dt, ctau, un, vn, pn, pnm1, gun=None, gvn=None, gu1=None,
             gv1=None, subcycles=0):
    """One first-order step of the algebraic splitting scheme (Sec. 2.2, Eq.
    INS_TD_3_1 to INS_TD_3_4 with gamma = beta_0 = alpha_0 = 1 and the
    pressure increment over sigma P = 2 P^n - P^{n-1}), with direct solves:
    m carries the velocity boundary flags, mp the swapped ones.  A pressure
    level without Dirichlet faces is solved with the constraint (M 1, dP) = 0
    after the constant component of its right-hand side is removed; the
    velocity is independent of that constant (G 1 = 0 there).

    ``subcycles`` > 0: the advection stage is the Lagrangian form of Sec. 2.3
    at first order (S = 0): U^ = U~(t^{n+1}) with dU~/dt = -N~(U^n, U~) from
    U~(t^n) = U^n, advanced by that many substeps of ``subcycle.subcycle``,
    the Dirichlet data linear in time from g^n to g^{n+1}."""
    import scipy.sparse.linalg as spla
    from .assemble import assemble
    gd = GradDiv(m)
    M = gd.M
    if subcycles:
        from .subcycle import subcycle
        z = np.zeros_like(np.asarray(un, dtype=np.float64))
        g0u = z if gun is None else np.asarray(gun, dtype=np.float64)
        g0v = z if gvn is None else np.asarray(gvn, dtype=np.float64)
        g1u = ((z if gu1 is None else np.asarray(gu1, dtype=np.float64)) - g0u) / dt
        g1v = ((z if gv1 is None else np.asarray(gv1, dtype=np.float64)) - g0v) / dt
        uh, vh = subcycle(m, un, vn, un, vn, dt, subcycles, gu0=g0u, gv0=g0v, gu1=g1u, gv1=g1v)
    else:
        Nu, Nv = advection(m, un, vn, gun, gvn)
        uh, vh = un - dt * Nu, vn - dt * Nv                   # Eq. INS_TD_3_1
    sp_ = 2.0 * pn - pnm1
    gx, gy = gd.grad(sp_)
    A = assemble(m, 1.0 / (nu * dt), ctau)
    bu = M @ (uh / (nu * dt) - gx / nu)                        # Eq. INS_TD_3_2
    bv = M @ (vh / (nu * dt) - gy / nu)
    if gu1 is not None:
        bu = bu + dirichlet_rhs(m, ctau, gu1)
    if gv1 is not None:
        bv = bv + dirichlet_rhs(m, ctau, gv1)
    uhh = spla.spsolve(A.tocsc(), bu)
    vhh = spla.spsolve(A.tocsc(), bv)
    bp = -(1.0 / dt) * (M @ gd.div(uhh, vhh, gu1, gv1))       # Eq. INS_TD_3_3
    S = assemble(mp, 0.0, ctau)
    if np.any(mp.EToB == BC_DIRICHLET):
        dp = spla.spsolve(S.tocsc(), bp)
    else:
        m1 = M @ np.ones(S.shape[0])
        bp = bp - (bp.sum() / m1.sum()) * m1
        n = S.shape[0]
        Sb = sp.bmat([[S, sp.csr_matrix(m1[:, None])], [sp.csr_matrix(m1[None, :]), None]], format="csc")
        dp = spla.spsolve(Sb, np.concatenate([bp, [0.0]]))[:n]
    gx, gy = gd.grad(dp)                                       # Eq. INS_TD_3_4
    return uhh - dt * gx, vhh - dt * gy, dp + sp_
