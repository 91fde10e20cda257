"""Assembled SIPDG operator of the oracle (TEST INFRASTRUCTURE ONLY).

The operator is the plain definition: A_ij = a_h(l_j, l_i) + lambda (l_j, l_i)
in the nodal basis, where a_h is the bilinear form obtained by summing the
element-wise SIPDG form (Eq. INS_SD_5, rewritten for A = -L + lambda in
Eq. ellipticOp1) over all elements.  With the jump [u] = u+ - u- of Sec. 2.1
and n the outward normal of the element that owns the face, that sum is

  a_h(u, v) = sum_E (grad u, grad v)_E
            - sum_{interior F} ({d_n u}, <v>)_F + ({d_n v}, <u>)_F - tau_F (<u>, <v>)_F
            - sum_{Dirichlet F} (d_n u, v)_F + (d_n v, u)_F - 2 tau_F (u, v)_F

with <u> = u- - u+.  Boundary faces use the mirror ghost (Dirichlet
u+ = -u-, grad u+ = grad u-; Neumann u+ = u-, n.grad u+ = -n.grad u-), which
keeps the form symmetric; homogeneous data only.  The penalty follows
Eq. Ch2.PenaltyParameter with its constant made a parameter c_tau:
tau_F = c_tau max(|F|/|E-|, |F|/|E+|) (one-sided on boundary faces).

Every integral is a Gauss quadrature exact for the polynomial integrand:
volume integrals on the reference triangle (affine map, constant metric),
face integrals along the physical edge, with each element's basis evaluated at
the physical quadrature points through the inverse of its own affine map.  No
face-node ordering convention enters the oracle.

Unknowns are element-major: global index e*Np + i.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .refelem import RefTriangle

BC_INTERIOR, BC_DIRICHLET, BC_NEUMANN = 0, 1, 2


class MeshError(ValueError):
    pass


class OracleMesh:
    """Geometry and connectivity of a triangle mesh, plus the degree-N
    reference element (Sec. 5.2, Eq. operators1/operators2/elementOps)."""

    def __init__(self, VX, VY, EToV, EToB, N: int):
        self.N = N
        self.ref = RefTriangle(N)
        self.Np = self.ref.Np
        self.VX = np.asarray(VX, dtype=np.float64)
        self.VY = np.asarray(VY, dtype=np.float64)
        self.EToV = np.asarray(EToV, dtype=np.int64)
        self.EToB = np.asarray(EToB, dtype=np.int64)
        self.K = self.EToV.shape[0]
        v = self.EToV
        self.x0, self.x1, self.x2 = self.VX[v[:, 0]], self.VX[v[:, 1]], self.VX[v[:, 2]]
        self.y0, self.y1, self.y2 = self.VY[v[:, 0]], self.VY[v[:, 1]], self.VY[v[:, 2]]
        # affine map x = -(r+s)/2 x0 + (1+r)/2 x1 + (1+s)/2 x2
        self.xr = 0.5 * (self.x1 - self.x0)
        self.xs = 0.5 * (self.x2 - self.x0)
        self.yr = 0.5 * (self.y1 - self.y0)
        self.ys = 0.5 * (self.y2 - self.y0)
        self.J = self.xr * self.ys - self.xs * self.yr
        if np.any(self.J <= 0.0):
            raise MeshError("element with non-positive Jacobian")
        self.rx = self.ys / self.J
        self.ry = -self.xs / self.J
        self.sx = -self.yr / self.J
        self.sy = self.xr / self.J
        self.area = 2.0 * self.J
        self._connect()

    # -- connectivity by exact vertex-id matching ---------------------------
    def _connect(self):
        K = self.K
        a = self.EToV
        b = np.roll(self.EToV, -1, axis=1)          # face f = (v_f, v_{f+1})
        lo = np.minimum(a, b).ravel()
        hi = np.maximum(a, b).ravel()
        nv = int(max(self.VX.size, 1))
        key = lo * nv + hi
        order = np.argsort(key, kind="stable")
        ks = key[order]
        self.EToE = np.full((K, 3), -1, dtype=np.int64)
        self.EToF = np.full((K, 3), -1, dtype=np.int64)
        start = np.flatnonzero(np.r_[True, ks[1:] != ks[:-1]])
        count = np.diff(np.r_[start, ks.size])
        if np.any(count > 2):
            raise MeshError("face shared by more than two elements")
        two = start[count == 2]
        g0 = order[two]
        g1 = order[two + 1]
        e0, f0 = g0 // 3, g0 % 3
        e1, f1 = g1 // 3, g1 % 3
        self.EToE[e0, f0] = e1
        self.EToF[e0, f0] = f1
        self.EToE[e1, f1] = e0
        self.EToF[e1, f1] = f0
        matched = self.EToE >= 0
        if np.any(matched & (self.EToB != BC_INTERIOR)):
            raise MeshError("matched face flagged as boundary")
        if np.any(~matched & (self.EToB == BC_INTERIOR)):
            raise MeshError("unmatched face flagged interior")
        if np.any(~np.isin(self.EToB, (BC_INTERIOR, BC_DIRICHLET, BC_NEUMANN))):
            raise MeshError("unknown boundary flag")

    # -- helpers -------------------------------------------------------------
    def node_coords(self):
        """Physical coordinates of all nodes, shape (K, Np) each."""
        r, s = self.ref.r, self.ref.s
        x = (-(r + s)[None, :] * self.x0[:, None] + (1 + r)[None, :] * self.x1[:, None]
             + (1 + s)[None, :] * self.x2[:, None]) / 2.0
        y = (-(r + s)[None, :] * self.y0[:, None] + (1 + r)[None, :] * self.y1[:, None]
             + (1 + s)[None, :] * self.y2[:, None]) / 2.0
        return x, y

    def to_ref(self, e, x, y):
        """Reference coordinates of physical points (x, y) in elements e
        (arrays broadcast together)."""
        dx = x - self.x0[e]
        dy = y - self.y0[e]
        r = self.rx[e] * dx + self.ry[e] * dy - 1.0
        s = self.sx[e] * dx + self.sy[e] * dy - 1.0
        return r, s

    def face_geometry(self, e, f):
        """End points, length and outward unit normal of face f of element e."""
        v = self.EToV
        pa = v[e, f]
        pb = v[e, (f + 1) % 3]
        xa, ya, xb, yb = self.VX[pa], self.VY[pa], self.VX[pb], self.VY[pb]
        dx, dy = xb - xa, yb - ya
        length = np.hypot(dx, dy)
        # counter-clockwise element: outward normal = edge direction turned
        # clockwise
        return xa, ya, xb, yb, length, dy / length, -dx / length


def _physical_grad(m, e, Lr, Ls):
    gx = m.rx[e][:, None, None] * Lr + m.sx[e][:, None, None] * Ls
    gy = m.ry[e][:, None, None] * Lr + m.sy[e][:, None, None] * Ls
    return gx, gy


def block_rows(m: OracleMesh, lam: float, ctau: float, elems=None, kappa=None):
    """Block rows of A for the elements ``elems`` (default: all).

    Returns (rows, cols, blocks): block (Np x Np) ``blocks[k]`` sits at block
    row ``rows[k]``, block column ``cols[k]``; repeated (row, col) pairs are
    to be summed.  ``kappa`` (per-element coefficient) scales the volume term
    by kappa_e, the consistency terms by the face average of kappa d_n, and
    the penalty by tau_F = c_tau max(kappa- |F|/|E-|, kappa+ |F|/|E+|)
    (Dirichlet ghost: kappa+ = kappa-).
    """
    ref = m.ref
    Np = ref.Np
    if elems is None:
        elems = np.arange(m.K)
    elems = np.asarray(elems, dtype=np.int64)
    kap = np.ones(m.K) if kappa is None else np.asarray(kappa, dtype=np.float64)
    rows, cols, blks = [], [], []

    # volume: (grad l_j, grad l_i)_E + lambda (l_j, l_i)_E with constant metric
    W = ref.qw
    Srr = (ref.qLr * W[:, None]).T @ ref.qLr
    Srs = (ref.qLr * W[:, None]).T @ ref.qLs
    Sss = (ref.qLs * W[:, None]).T @ ref.qLs
    Mref = (ref.qL * W[:, None]).T @ ref.qL
    e = elems
    crr = m.rx[e] ** 2 + m.ry[e] ** 2
    crs = m.rx[e] * m.sx[e] + m.ry[e] * m.sy[e]
    css = m.sx[e] ** 2 + m.sy[e] ** 2
    vol = (kap[e] * crr)[:, None, None] * Srr[None] \
        + (kap[e] * crs)[:, None, None] * (Srs + Srs.T)[None] \
        + (kap[e] * css)[:, None, None] * Sss[None] \
        + lam * Mref[None]
    vol = vol * m.J[e][:, None, None]
    rows.append(e)
    cols.append(e)
    blks.append(vol)

    # faces, each seen from the test element's side
    g, w = ref.g1, ref.w1
    for f in range(3):
        ef = e
        bc = m.EToB[ef, f]
        nb = m.EToE[ef, f]
        sel = bc != BC_NEUMANN
        ef, nb, bc = ef[sel], nb[sel], bc[sel]
        if ef.size == 0:
            continue
        xa, ya, xb, yb, length, nx, ny = m.face_geometry(ef, f)
        # physical quadrature points along the edge
        t = g[None, :]
        qx = 0.5 * (1 - t) * xa[:, None] + 0.5 * (1 + t) * xb[:, None]
        qy = 0.5 * (1 - t) * ya[:, None] + 0.5 * (1 + t) * yb[:, None]
        Wq = (0.5 * length)[:, None] * w[None, :]               # (nF, q)
        rm, sm = m.to_ref(ef[:, None], qx, qy)
        Vm, Lrm, Lsm = ref.lagrange(rm.ravel(), sm.ravel())
        nF, q = qx.shape
        Vm = Vm.reshape(nF, q, Np)
        gxm, gym = _physical_grad(m, ef, Lrm.reshape(nF, q, Np), Lsm.reshape(nF, q, Np))
        Dm = nx[:, None, None] * gxm + ny[:, None, None] * gym   # d_n l^- (nF,q,Np)
        km = kap[ef]
        interior = bc == BC_INTERIOR
        # penalty
        hm = length / m.area[ef]
        nbs = np.where(interior, nb, 0)
        hp = length / m.area[nbs]
        tau = np.where(interior, ctau * np.maximum(km * hm, kap[nbs] * hp), ctau * km * hm)
        WV = Wq[:, :, None] * Vm
        VtWV = np.einsum("fqi,fqj->fij", WV, Vm)
        VtWD = np.einsum("fqi,fqj->fij", WV, Dm)
        # diagonal block: interior (+1/2 weights, tau), Dirichlet (full, 2 tau)
        cons = np.where(interior, 0.5, 1.0)[:, None, None]
        pen = np.where(interior, tau, 2.0 * tau)[:, None, None]
        blk = -cons * km[:, None, None] * (VtWD + VtWD.transpose(0, 2, 1)) + pen * VtWV
        rows.append(ef)
        cols.append(ef)
        blks.append(blk)
        # coupling block to the neighbour (interior faces only)
        if np.any(interior):
            ei = ef[interior]
            ni = nb[interior]
            rp, spp = m.to_ref(ni[:, None], qx[interior], qy[interior])
            Vp, Lrp, Lsp = ref.lagrange(rp.ravel(), spp.ravel())
            nI = ei.size
            Vp = Vp.reshape(nI, q, Np)
            gxp, gyp = _physical_grad(m, ni, Lrp.reshape(nI, q, Np), Lsp.reshape(nI, q, Np))
            Dp = nx[interior][:, None, None] * gxp + ny[interior][:, None, None] * gyp
            kp = kap[ni]
            WVm = WV[interior]
            WDm = Wq[interior][:, :, None] * Dm[interior]
            cpl = (-0.5 * kp[:, None, None] * np.einsum("fqi,fqj->fij", WVm, Dp)
                   + 0.5 * km[interior][:, None, None] * np.einsum("fqi,fqj->fij", WDm, Vp)
                   - tau[interior][:, None, None] * np.einsum("fqi,fqj->fij", WVm, Vp))
            rows.append(ei)
            cols.append(ni)
            blks.append(cpl)
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(blks, axis=0)


def assemble(m: OracleMesh, lam: float, ctau: float, kappa=None) -> sp.csr_matrix:
    """Global sparse matrix A (K*Np square), element-major unknowns."""
    Np = m.Np
    r, c, b = block_rows(m, lam, ctau, kappa=kappa)
    ii = (r[:, None, None] * Np + np.arange(Np)[None, :, None])
    jj = (c[:, None, None] * Np + np.arange(Np)[None, None, :])
    ii = np.broadcast_to(ii, b.shape).ravel()
    jj = np.broadcast_to(jj, b.shape).ravel()
    n = m.K * Np
    return sp.csr_matrix((b.ravel(), (ii, jj)), shape=(n, n))


def apply_rows(m: OracleMesh, lam: float, ctau: float, x: np.ndarray, elems, kappa=None):
    """(A x) restricted to the nodes of ``elems``: shape (len(elems), Np)."""
    Np = m.Np
    elems = np.asarray(elems, dtype=np.int64)
    r, c, b = block_rows(m, lam, ctau, elems=elems, kappa=kappa)
    X = np.asarray(x, dtype=np.float64).reshape(m.K, Np)
    contrib = np.einsum("kij,kj->ki", b, X[c])
    pos_of = np.full(m.K, -1, dtype=np.int64)
    pos_of[elems] = np.arange(elems.size)
    out = np.zeros((elems.size, Np))
    np.add.at(out, pos_of[r], contrib)
    return out


def mass_matrix(m: OracleMesh) -> sp.csr_matrix:
    """Block-diagonal mass matrix, blocks J_e (l_i, l_j) on the reference."""
    ref = m.ref
    Np = ref.Np
    Mref = (ref.qL * ref.qw[:, None]).T @ ref.qL
    blocks = m.J[:, None, None] * Mref[None]
    return _block_diag(blocks, Np)


def _block_diag(blocks, Np):
    K = blocks.shape[0]
    ii = np.broadcast_to((np.arange(K)[:, None, None] * Np + np.arange(Np)[None, :, None]), blocks.shape)
    jj = np.broadcast_to((np.arange(K)[:, None, None] * Np + np.arange(Np)[None, None, :]), blocks.shape)
    n = K * Np
    return sp.csr_matrix((blocks.ravel(), (ii.ravel(), jj.ravel())), shape=(n, n))


def mass_apply(m: OracleMesh, f: np.ndarray) -> np.ndarray:
    """b = M f element by element (f nodal, element-major)."""
    ref = m.ref
    Mref = (ref.qL * ref.qw[:, None]).T @ ref.qL
    F = np.asarray(f, dtype=np.float64).reshape(m.K, m.Np)
    return (m.J[:, None] * (F @ Mref.T)).ravel()


def kappa_grad(m: OracleMesh, ctau: float, kappa, u, w) -> np.ndarray:
    """g_e = -w^T (dA/dkappa_e) u for the kappa-weighted form of block_rows.

    With <v> = v- - v+ seen from element e (its outward normal n):
      d a / d kappa_e = (grad u, grad w)_E
        + sum_{interior F of e} -1/2 (d_n u_e, <w>)_F - 1/2 (d_n w_e, <u>)_F
                               + dtau_F/dkappa_e (<u>, <w>)_F
        + sum_{Dirichlet F of e} -(d_n u, w)_F - (d_n w, u)_F + 2 c_tau (|F|/|E|) (u, w)_F
    where dtau_F/dkappa_e = c_tau |F|/|E| if kappa_e |F|/|E| attains the max
    in tau_F (ties: the element with the lower id), else 0.  Integrals by
    the same quadratures as block_rows.
    """
    ref = m.ref
    Np = ref.Np
    K = m.K
    kap = np.asarray(kappa, dtype=np.float64)
    U = np.asarray(u, dtype=np.float64).reshape(K, Np)
    Wv = np.asarray(w, dtype=np.float64).reshape(K, Np)
    e = np.arange(K)
    # volume: integral of grad u . grad w
    W = ref.qw
    ur, us = U @ ref.qLr.T, U @ ref.qLs.T                  # (K, nq)
    wr, ws = Wv @ ref.qLr.T, Wv @ ref.qLs.T
    ux = m.rx[:, None] * ur + m.sx[:, None] * us
    uy = m.ry[:, None] * ur + m.sy[:, None] * us
    wx = m.rx[:, None] * wr + m.sx[:, None] * ws
    wy = m.ry[:, None] * wr + m.sy[:, None] * ws
    g = m.J * ((ux * wx + uy * wy) @ W)
    gq, gw = ref.g1, ref.w1
    for f in range(3):
        bc = m.EToB[e, f]
        nb = m.EToE[e, f]
        xa, ya, xb, yb, length, nx, ny = m.face_geometry(e, f)
        t = gq[None, :]
        qx = 0.5 * (1 - t) * xa[:, None] + 0.5 * (1 + t) * xb[:, None]
        qy = 0.5 * (1 - t) * ya[:, None] + 0.5 * (1 + t) * yb[:, None]
        Wq = (0.5 * length)[:, None] * gw[None, :]
        rm, sm = m.to_ref(e[:, None], qx, qy)
        L0, Lr0, Ls0 = ref.lagrange(rm.ravel(), sm.ravel())
        q = qx.shape[1]
        L0 = L0.reshape(K, q, Np)
        Lr0 = Lr0.reshape(K, q, Np)
        Ls0 = Ls0.reshape(K, q, Np)
        um = np.einsum("kqi,ki->kq", L0, U)
        wm = np.einsum("kqi,ki->kq", L0, Wv)
        gxu = m.rx[:, None] * np.einsum("kqi,ki->kq", Lr0, U) + m.sx[:, None] * np.einsum("kqi,ki->kq", Ls0, U)
        gyu = m.ry[:, None] * np.einsum("kqi,ki->kq", Lr0, U) + m.sy[:, None] * np.einsum("kqi,ki->kq", Ls0, U)
        gxw = m.rx[:, None] * np.einsum("kqi,ki->kq", Lr0, Wv) + m.sx[:, None] * np.einsum("kqi,ki->kq", Ls0, Wv)
        gyw = m.ry[:, None] * np.einsum("kqi,ki->kq", Lr0, Wv) + m.sy[:, None] * np.einsum("kqi,ki->kq", Ls0, Wv)
        dnu = nx[:, None] * gxu + ny[:, None] * gyu
        dnw = nx[:, None] * gxw + ny[:, None] * gyw
        hm = length / m.area
        inner = bc == BC_INTERIOR
        if np.any(inner):
            ei = e[inner]
            ni = nb[inner]
            rp, sp_ = m.to_ref(ni[:, None], qx[inner], qy[inner])
            Lp, _, _ = ref.lagrange(rp.ravel(), sp_.ravel())
            Lp = Lp.reshape(ei.size, q, Np)
            up = np.einsum("kqi,ki->kq", Lp, U[ni])
            wp = np.einsum("kqi,ki->kq", Lp, Wv[ni])
            ju = um[inner] - up
            jw = wm[inner] - wp
            mine = kap[ei] * hm[inner]
            other = kap[ni] * length[inner] / m.area[ni]
            owns = (mine > other) | ((mine == other) & (ei < ni))
            dtau = np.where(owns, ctau * hm[inner], 0.0)
            Wi = Wq[inner]
            val = (-0.5 * np.sum(Wi * dnu[inner] * jw, 1) - 0.5 * np.sum(Wi * dnw[inner] * ju, 1)
                   + dtau * np.sum(Wi * ju * jw, 1))
            np.add.at(g, ei, val)
        dirf = bc == BC_DIRICHLET
        if np.any(dirf):
            Wd = Wq[dirf]
            val = (-np.sum(Wd * dnu[dirf] * wm[dirf], 1) - np.sum(Wd * dnw[dirf] * um[dirf], 1)
                   + 2 * ctau * hm[dirf] * np.sum(Wd * um[dirf] * wm[dirf], 1))
            np.add.at(g, e[dirf], val)
    return -g
