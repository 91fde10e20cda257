"""Semi-Lagrangian subcycling advection of the oracle (TEST INFRASTRUCTURE
ONLY: imported by tests/ and the benchmark's CPU leg).

Sec. 2.3, Eq. SS_2 / SS_3 / INS_CUB_N: the subproblem dU~/dt = -N~(Ubar, U~)
with, per element and for every test function v of P_N,

    (v, N~)_E = -(grad v, F~)_E + (v, n . F~*)_dE,     F~ = Ubar (x) U~,
    n . F~* = {n . F~} + (Lambda / 2) (U~- - U~+),
    Lambda  = max(|n . Ubar-|, |n . Ubar+|),

the integrals taken by cubature (Sec. 5.3, Eq. KSS_3): interpolation to the
volume and face cubature nodes, the combined differentiation-and-projection
operators P_r, P_s and the cubature lifts L_c^f.  Readings:

  * Lambda: n . dF~/dU~ = (n . Ubar) I does not depend on U~, so the maximum of
    the flux Jacobian over the segment [U~-, U~+] is taken at the two traces
    of the advecting field, as the surface kernel of Alg. SSS computes it, at
    each face cubature node.
  * Sign: Eq. KSS_3 carries -G P . F~ for the volume term (integration by
    parts); the volume kernel of Alg. SSV prints its sum without the sign.
    The equation is followed, so that N~ approximates Ubar . grad U~.
  * Cubature: the paper does not print its rules.  The face rule is the
    q-point Gauss-Legendre rule with q = floor(3 N / 2) + 1, exact for the
    degree-3N face integrand; it is part of the operator's definition because
    Lambda is evaluated pointwise.  The volume integrand (degree 3N - 1 on an
    affine element) is integrated exactly, so any rule exact to that degree
    gives the same operator; the oracle uses a collapsed-coordinate
    Gauss-Legendre product one point richer than needed.
  * Boundary faces: the advecting field is given on the whole domain, so its
    exterior trace is its interior one (Ubar+ = Ubar-) on every boundary
    face; the advected field takes U~+ = g on Dirichlet faces (the boundary
    velocity data, read at the face cubature nodes from a nodal field) and
    U~+ = U~- on Neumann faces.
  * Time stepping (Sec. 2.3): the five-stage fourth-order low-storage
    Runge-Kutta scheme of Carpenter and Kennedy, the method the paper cites
    without printing its coefficients; the advecting field is linear in the
    substep time, Ubar(t) = Ubar0 + t Ubar1 (S <= 1 in the paper's notation),
    and so is the boundary data, g(t) = g0 + t g1.
"""
from __future__ import annotations

import numpy as np

from .assemble import BC_DIRICHLET, BC_NEUMANN, OracleMesh
from .refelem import RefTriangle, gauss_legendre

# Carpenter & Kennedy (1994), five-stage fourth-order 2N-storage Runge-Kutta:
# du = a_k du + dt R(t + c_k dt, u);  u = u + b_k du.
LSERK_A = (0.0,
           -567301805773.0 / 1357537059087.0,
           -2404267990393.0 / 2016746695238.0,
           -3550918686646.0 / 2091501179385.0,
           -1275806237668.0 / 842570457699.0)
LSERK_B = (1432997174477.0 / 9575080441755.0,
           5161836677717.0 / 13612068292357.0,
           1720146321549.0 / 2090206949498.0,
           3134564353537.0 / 4481467310338.0,
           2277821191437.0 / 14882151754819.0)
LSERK_C = (0.0,
           1432997174477.0 / 9575080441755.0,
           2526269341429.0 / 6820363962896.0,
           2006345519317.0 / 3224310063776.0,
           2802321613138.0 / 2924317926251.0)

def face_points(N: int) -> int:
    """Face cubature size: Gauss-Legendre exact for the degree-3N integrand."""
    return (3 * N) // 2 + 1

def lserk_butcher():
    """Butcher tableau (A, b, c) of the 2N-storage scheme, by tracking the
    coefficients of the stage evaluations through its two registers."""
    s = len(LSERK_A)
    A = np.zeros((s, s))
    du = np.zeros(s)
    u = np.zeros(s)
    for k in range(s):
        A[k] = u
        du = LSERK_A[k] * du
        du[k] += 1.0
        u = u + LSERK_B[k] * du
    return A, u, A.sum(axis=1)

class CubatureOps:
    """Reference cubature operators of Sec. 5.3 for the oracle's degree-N
    triangle: volume nodes and weights with I, P_r, P_s; per face the Gauss
    points with I^f and the cubature lift L_c^f."""

    def __init__(self, N: int, extra_volume: int = 1):
        ref = RefTriangle(N)
        self.ref = ref
        q = face_points(N) + extra_volume
        ga, wa = gauss_legendre(q)
        A, B = np.meshgrid(ga, ga, indexing="ij")
        WA, WB = np.meshgrid(wa, wa, indexing="ij")
        self.rc = ((1.0 + A) * (1.0 - B) / 2.0 - 1.0).ravel()
        self.sc = B.ravel()
        self.wc = (WA * WB * (1.0 - B) / 2.0).ravel()
        self.I, Ir, Is = ref.lagrange(self.rc, self.sc)           # (Nc, Np)
        Minv = np.linalg.inv(ref.mass())
        self.Pr = Minv @ (Ir * self.wc[:, None]).T                  # (Np, Nc)
        self.Ps = Minv @ (Is * self.wc[:, None]).T
        self.tf, self.wf = gauss_legendre(face_points(N))
        self.If, self.Lc = [], []
        for f in range(3):
            Lf, _, _ = ref.lagrange(*ref.face_points(f, self.tf))   # (Nfc, Np)
            self.If.append(Lf)
            self.Lc.append(Minv @ (Lf * self.wf[:, None]).T)        # (Np, Nfc)

def face_maps(m: OracleMesh, ops: CubatureOps, e, f):
    """Interpolation of face f of element e to its cubature points: the
    interior trace matrix (Nfc x Np, in element e), the exterior one (in the
    neighbour, at the same physical points mapped back to its reference
    coordinates; None on a boundary face), the face length and the outward
    unit normal."""
    xa, ya, xb, yb, length, nx, ny = m.face_geometry(e, f)
    t = ops.tf
    px = xa + 0.5 * (1.0 + t) * (xb - xa)
    py = ya + 0.5 * (1.0 + t) * (yb - ya)
    L, _, _ = ops.ref.lagrange(*m.to_ref(e, px, py))
    nb = m.EToE[e, f]
    Ln = ops.ref.lagrange(*m.to_ref(nb, px, py))[0] if nb >= 0 else None
    return L, Ln, length, nx, ny


def _face_traces(m: OracleMesh, fm, fields, g, e, f):
    """Interior and exterior values of the nodal fields (Ubar, Vbar, U~, V~)
    at the face cubature nodes of face f of element e, from its face maps
    ``fm``; on a boundary face the exterior trace follows the boundary rule
    (g: the data of U~, V~)."""
    L, Ln, length, nx, ny = fm
    minus = [L @ F[e] for F in fields]
    bc = m.EToB[e, f]
    nb = m.EToE[e, f]
    if nb >= 0:
        plus = [Ln @ F[nb] for F in fields]
    elif bc == BC_DIRICHLET:
        plus = [minus[0].copy(), minus[1].copy()] + [L @ G[e] for G in g]
    elif bc == BC_NEUMANN:
        plus = [x.copy() for x in minus]
    else:
        raise ValueError("unmatched face without a boundary rule")
    return minus, plus, length, nx, ny


def advection_operator(m: OracleMesh, ubar, vbar, u, v, gu=None, gv=None, parts=3, ops=None, elems=None,
                       maps=None):
    """N~(Ubar, U~) of Eq. KSS_3 for both velocity components, as nodal
    fields (K Np each): parts = 1 the volume term, 2 the surface term, 3 both.
    Dirichlet data (gu, gv) give the exterior trace of U~ there (None = 0).
    ``elems``: compute only these elements' rows (returned in that order).
    ``maps``: the face maps of every (e, f) from ``face_maps``, if already
    built (they depend only on the mesh)."""
    ops = ops or CubatureOps(m.N)
    K, Np = m.K, m.Np
    E = np.arange(K) if elems is None else np.asarray(elems, dtype=np.int64)
    sh = lambda a: np.zeros((K, Np)) if a is None else np.asarray(a, dtype=np.float64).reshape(K, Np)
    UB, VB, U, V, GU, GV = (sh(a) for a in (ubar, vbar, u, v, gu, gv))
    Nu = np.zeros((E.size, Np))
    Nv = np.zeros((E.size, Np))
    if parts & 1:
        # volume: -(grad l_n, Ubar U~) at the cubature nodes, divided by J M
        ub, vb = UB[E] @ ops.I.T, VB[E] @ ops.I.T                 # (|E|, Nc)
        uc, vc = U[E] @ ops.I.T, V[E] @ ops.I.T
        rx, sx, ry, sy = (a[E][:, None] for a in (m.rx, m.sx, m.ry, m.sy))
        # the u row of F~ is (ub uc, vb uc), the v row (ub vc, vb vc)
        Nu -= (rx * ub * uc + ry * vb * uc) @ ops.Pr.T + (sx * ub * uc + sy * vb * uc) @ ops.Ps.T
        Nv -= (rx * ub * vc + ry * vb * vc) @ ops.Pr.T + (sx * ub * vc + sy * vb * vc) @ ops.Ps.T
    if parts & 2:
        for row, e in enumerate(E):
            for f in range(3):
                fm = maps[e][f] if maps is not None else face_maps(m, ops, e, f)
                (ubm, vbm, um, vm), (ubp, vbp, up, vp), length, nx, ny = _face_traces(
                    m, fm, (UB, VB, U, V), (GU, GV), e, f)
                anm = nx * ubm + ny * vbm
                anp = nx * ubp + ny * vbp
                lam = np.maximum(np.abs(anm), np.abs(anp))
                fu = 0.5 * (anm * um + anp * up) + 0.5 * lam * (um - up)
                fv = 0.5 * (anm * vm + anp * vp) + 0.5 * lam * (vm - vp)
                sc = length / m.area[e]                             # J^{ef} / J^e
                Nu[row] += sc * (ops.Lc[f] @ fu)
                Nv[row] += sc * (ops.Lc[f] @ fv)
    return Nu.ravel(), Nv.ravel()

def subcycle(m: OracleMesh, ubar0, vbar0, u, v, T, Ns, ubar1=None, vbar1=None, gu0=None, gv0=None, gu1=None,
             gv1=None):
    """Ns steps of the low-storage RK4 scheme over [0, T] for dU~/dt =
    -N~(Ubar(t), U~) with Ubar(t) = Ubar0 + t Ubar1 and Dirichlet data
    g(t) = g0 + t g1 (Sec. 2.3, Eq. SS_3).  Returns U~(T)."""
    ops = CubatureOps(m.N)
    maps = [[face_maps(m, ops, e, f) for f in range(3)] for e in range(m.K)]
    n = m.K * m.Np
    z = np.zeros(n)
    arr = lambda a: z if a is None else np.asarray(a, dtype=np.float64).ravel()
    UB0, VB0, UB1, VB1 = arr(ubar0), arr(vbar0), arr(ubar1), arr(vbar1)
    G0u, G0v, G1u, G1v = arr(gu0), arr(gv0), arr(gu1), arr(gv1)
    U = np.asarray(u, dtype=np.float64).ravel().copy()
    V = np.asarray(v, dtype=np.float64).ravel().copy()
    dt = T / Ns
    du = np.zeros(n)
    dv = np.zeros(n)
    for step in range(Ns):
        t0 = step * dt
        for k in range(5):
            t = t0 + LSERK_C[k] * dt
            Nu, Nv = advection_operator(m, UB0 + t * UB1, VB0 + t * VB1, U, V, G0u + t * G1u, G0v + t * G1v,
                                        ops=ops, maps=maps)
            du = LSERK_A[k] * du - dt * Nu
            dv = LSERK_A[k] * dv - dt * Nv
            U = U + LSERK_B[k] * du
            V = V + LSERK_B[k] * dv
    return U, V

def rk_order_residuals():
    """The eight order conditions of a fourth-order Runge-Kutta method,
    evaluated on the tableau (each residual is zero for an exact method)."""
    A, b, c = lserk_butcher()
    return {
        "b": b.sum() - 1.0,
        "bc": b @ c - 1.0 / 2.0,
        "bc2": b @ c ** 2 - 1.0 / 3.0,
        "bAc": b @ A @ c - 1.0 / 6.0,
        "bc3": b @ c ** 3 - 1.0 / 4.0,
        "bcAc": (b * c) @ A @ c - 1.0 / 8.0,
        "bAc2": b @ A @ c ** 2 - 1.0 / 12.0,
        "bAAc": b @ A @ A @ c - 1.0 / 24.0,
    }
