"""Pins of the oracle's subcycling advection (Sec. 2.3, Eq. SS_3 and
INS_CUB_N; Sec. 5.3, Eq. KSS_3) and of its Runge-Kutta scheme.

Fixed by the mathematics rather than by the oracle's own formulas:
  * the five-stage low-storage coefficients satisfy the eight order
    conditions of a fourth-order method, and the stage times are the row sums
    of the tableau they generate;
  * the volume rule integrates the monomials (1 + r)^a (1 + s)^b over the
    reference triangle exactly (closed form 2^(a+b+2) a! b! / (a+b+2)!) up to
    the degree the operator needs;
  * for a linear divergence-free advecting field and a global polynomial of
    degree <= N there are no jumps, so N~ is the interpolant of
    Ubar . grad U~ (degree N), with Neumann faces and with Dirichlet faces
    whose data is the advected field itself;
  * on a two-triangle mesh the operator times J M equals the variational form
    of Eq. INS_CUB_N integrated by adaptive quadrature (scipy), for
    discontinuous random fields, every boundary rule, and an advecting field
    constant per element (so that Lambda is constant along each face);
  * a polynomial of degree <= 4 carried by a constant velocity stays a
    polynomial, the semi-discrete operator is exact on it and nilpotent, and
    a fourth-order five-stage step reproduces the exact translation; a
    velocity linear in time and time-linear Dirichlet data are carried
    exactly as well (checks the stage times c_k).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import synth
from oracle.assemble import BC_DIRICHLET, BC_INTERIOR, BC_NEUMANN, OracleMesh
from oracle.subcycle import (LSERK_C, CubatureOps, advection_operator, face_points, lserk_butcher,
                             rk_order_residuals, subcycle)


def test_lserk_order_conditions():
    res = rk_order_residuals()
    for k, v in res.items():
        assert abs(v) < 1e-14, (k, v)
    _, _, c = lserk_butcher()
    assert np.allclose(c, LSERK_C, rtol=0, atol=1e-15)


@pytest.mark.parametrize("N", [1, 3, 5, 8])
def test_volume_rule_integrates_monomials(N):
    ops = CubatureOps(N)
    x, y = 1.0 + ops.rc, 1.0 + ops.sc
    deg = 3 * N + 1
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            exact = 2.0 ** (a + b + 2) * math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = ops.wc @ (x ** a * y ** b)
            assert abs(got - exact) <= 1e-13 * exact, (a, b)


@pytest.mark.parametrize("N", [1, 4, 7])
def test_face_rule_is_exact_to_3N(N):
    ops = CubatureOps(N)
    assert ops.tf.size == face_points(N)
    for k in range(3 * N + 1):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(ops.wf @ ops.tf ** k - exact) < 1e-14


def poly(x, y, N, seed):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((N + 1, N + 1))
    f = np.zeros_like(x)
    fx = np.zeros_like(x)
    fy = np.zeros_like(x)
    for a in range(N + 1):
        for b in range(N + 1 - a):
            f += c[a, b] * x ** a * y ** b
            if a:
                fx += c[a, b] * a * x ** (a - 1) * y ** b
            if b:
                fy += c[a, b] * b * x ** a * y ** (b - 1)
    return f, fx, fy


def linear_divfree(x, y, seed):
    a, b, c, d, e = np.random.default_rng(seed).standard_normal(5)
    return a + b * x + c * y, d + e * x - b * y


@pytest.mark.parametrize("N", [1, 2, 4, 6])
def test_polynomials_are_advected_exactly_neumann(N):
    msh = synth.permuted(synth.square_mesh(3, jitter=0.2, seed=5, bc="neumann"), seed=6)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    x, y = m.node_coords()
    ub, vb = linear_divfree(x, y, seed=N)
    u, ux, uy = poly(x, y, N, seed=10 + N)
    v, vx, vy = poly(x, y, N, seed=20 + N)
    Nu, Nv = advection_operator(m, ub, vb, u, v)
    eu = (ub * ux + vb * uy).ravel()
    ev = (ub * vx + vb * vy).ravel()
    assert np.abs(Nu - eu).max() <= 1e-10 * np.abs(eu).max()
    assert np.abs(Nv - ev).max() <= 1e-10 * np.abs(ev).max()


@pytest.mark.parametrize("bc", ["dirichlet", "mixed"])
@pytest.mark.parametrize("N", [2, 5])
def test_polynomials_with_dirichlet_data_are_advected_exactly(N, bc):
    msh = synth.permuted(synth.square_mesh(3, jitter=0.2, seed=7, bc=bc), seed=8)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    x, y = m.node_coords()
    ub, vb = linear_divfree(x, y, seed=30 + N)
    u, ux, uy = poly(x, y, N, seed=31 + N)
    v, vx, vy = poly(x, y, N, seed=32 + N)
    Nu, Nv = advection_operator(m, ub, vb, u, v, gu=u, gv=v)
    eu = (ub * ux + vb * uy).ravel()
    ev = (ub * vx + vb * vy).ravel()
    assert np.abs(Nu - eu).max() <= 1e-10 * np.abs(eu).max()
    assert np.abs(Nv - ev).max() <= 1e-10 * np.abs(ev).max()


def _two_triangles():
    VX = np.array([0.0, 1.1, 0.2, 1.3])
    VY = np.array([0.0, 0.1, 0.9, 1.2])
    EToV = np.array([[0, 1, 2], [1, 3, 2]])
    # element 0: faces (0,1) Dirichlet, (1,2) shared, (2,0) Neumann
    # element 1: faces (1,3) Neumann, (3,2) Dirichlet, (2,1) shared
    EToB = np.array([[BC_DIRICHLET, BC_INTERIOR, BC_NEUMANN], [BC_NEUMANN, BC_DIRICHLET, BC_INTERIOR]])
    return VX, VY, EToV, EToB


@pytest.mark.parametrize("N", [1, 2, 3])
def test_operator_matches_adaptive_quadrature_of_the_weak_form(N):
    VX, VY, EToV, EToB = _two_triangles()
    m = OracleMesh(VX, VY, EToV, EToB, N)
    K, Np = m.K, m.Np
    rng = np.random.default_rng(40 + N)
    U, V, GU, GV = (rng.standard_normal((K, Np)) for _ in range(4))
    vel = rng.standard_normal((K, 2))                       # advecting field, constant per element
    UB = np.repeat(vel[:, :1], Np, axis=1)
    VB = np.repeat(vel[:, 1:], Np, axis=1)
    Nu, Nv = advection_operator(m, UB, VB, U, V, GU, GV)
    M = m.ref.mass()
    got_u = (m.J[:, None] * (Nu.reshape(K, Np) @ M.T))
    got_v = (m.J[:, None] * (Nv.reshape(K, Np) @ M.T))

    def at(e, F, x, y):
        r, s = m.to_ref(e, np.atleast_1d(x), np.atleast_1d(y))
        L, _, _ = m.ref.lagrange(r, s)
        return (L @ F[e])[0]

    def basis(e, n, x, y):
        r, s = m.to_ref(e, np.atleast_1d(x), np.atleast_1d(y))
        L, Lr, Ls = m.ref.lagrange(r, s)
        gx = m.rx[e] * Lr[0, n] + m.sx[e] * Ls[0, n]
        gy = m.ry[e] * Lr[0, n] + m.sy[e] * Ls[0, n]
        return L[0, n], gx, gy

    for e in range(K):
        xs = np.array([m.x0[e], m.x1[e], m.x2[e]])
        ys = np.array([m.y0[e], m.y1[e], m.y2[e]])

        def tri_integral(fn):
            # x = x0 + a (x1 - x0) + b (x2 - x0), 0 <= b <= 1 - a
            jac = abs((xs[1] - xs[0]) * (ys[2] - ys[0]) - (xs[2] - xs[0]) * (ys[1] - ys[0]))
            g = lambda b, a: fn(xs[0] + a * (xs[1] - xs[0]) + b * (xs[2] - xs[0]),
                                ys[0] + a * (ys[1] - ys[0]) + b * (ys[2] - ys[0]))
            return jac * integrate.dblquad(g, 0.0, 1.0, 0.0, lambda a: 1.0 - a, epsabs=1e-13, epsrel=1e-13)[0]

        for n in range(Np):
            for comp, F, got in ((0, U, got_u), (1, V, got_v)):
                def vol(x, y):
                    _, gx, gy = basis(e, n, x, y)
                    w = at(e, F, x, y)
                    return -(gx * vel[e, 0] * w + gy * vel[e, 1] * w)
                total = tri_integral(vol)
                for f in range(3):
                    pa, pb = EToV[e, f], EToV[e, (f + 1) % 3]
                    xa, ya, xb, yb = VX[pa], VY[pa], VX[pb], VY[pb]
                    length = math.hypot(xb - xa, yb - ya)
                    nx, ny = (yb - ya) / length, -(xb - xa) / length
                    nb = -1 if EToB[e, f] != BC_INTERIOR else 1 - e
                    G = (GU, GV)[comp]

                    def surf(t):
                        x = xa + t * (xb - xa)
                        y = ya + t * (yb - ya)
                        wm = at(e, F, x, y)
                        anm = nx * vel[e, 0] + ny * vel[e, 1]
                        if nb >= 0:
                            wp = at(nb, F, x, y)
                            anp = nx * vel[nb, 0] + ny * vel[nb, 1]
                        elif EToB[e, f] == BC_DIRICHLET:
                            wp, anp = at(e, G, x, y), anm
                        else:
                            wp, anp = wm, anm
                        lam = max(abs(anm), abs(anp))
                        flux = 0.5 * (anm * wm + anp * wp) + 0.5 * lam * (wm - wp)
                        return basis(e, n, x, y)[0] * flux

                    total += length * integrate.quad(surf, 0.0, 1.0, epsabs=1e-13, epsrel=1e-13)[0]
                assert abs(got[e, n] - total) <= 1e-9 * max(1.0, abs(total)), (e, n, comp)


@pytest.mark.parametrize("N", [3, 4])
def test_subcycle_translates_polynomials_exactly(N):
    msh = synth.permuted(synth.square_mesh(3, jitter=0.15, seed=9, bc="neumann"), seed=10)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    x, y = m.node_coords()
    a, b = 0.7, -0.4
    u0, _, _ = poly(x, y, N, seed=50)
    v0, _, _ = poly(x, y, N, seed=51)
    # substeps inside the scheme's stability region for this mesh and degree
    # (rounding noise in the unresolved modes must not grow)
    T = 0.1
    U, V = subcycle(m, np.full(x.size, a), np.full(x.size, b), u0, v0, T, Ns=8)
    eu, _, _ = poly(x - a * T, y - b * T, N, seed=50)
    ev, _, _ = poly(x - a * T, y - b * T, N, seed=51)
    assert np.abs(U - eu.ravel()).max() <= 1e-11 * np.abs(eu).max()
    assert np.abs(V - ev.ravel()).max() <= 1e-11 * np.abs(ev).max()


def test_subcycle_with_time_linear_velocity_and_data():
    # u~(x, t) = x - a t - alpha t^2 / 2 under Ubar = (a + alpha t, 0), v~ = y
    # not moved (Neumann boundary)
    msh = synth.permuted(synth.square_mesh(3, jitter=0.1, seed=11, bc="neumann"), seed=12)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, 2)
    x, y = (c.ravel() for c in m.node_coords())
    a, alpha, T = 0.8, 0.5, 0.4
    one = np.ones_like(x)
    U, V = subcycle(m, a * one, 0 * one, x, y, T, Ns=2, ubar1=alpha * one, vbar1=0 * one)
    assert np.abs(U - (x - a * T - 0.5 * alpha * T * T)).max() < 1e-12
    assert np.abs(V - y).max() < 1e-12
    # Dirichlet data linear in time on the whole boundary: u~ = x - a t
    mshd = synth.permuted(synth.square_mesh(3, jitter=0.1, seed=13, bc="dirichlet"), seed=14)
    md = OracleMesh(mshd.VX, mshd.VY, mshd.EToV, mshd.EToB, 2)
    x, y = (c.ravel() for c in md.node_coords())
    one = np.ones_like(x)
    U, V = subcycle(md, a * one, 0 * one, x, y, T, Ns=2, gu0=x, gv0=y, gu1=-a * one, gv1=0 * one)
    assert np.abs(U - (x - a * T)).max() < 1e-12
    assert np.abs(V - y).max() < 1e-12


def test_subcycled_splitting_step_converges_to_the_taylor_vortex():
    """The splitting step with the subcycled advection stage (Sec. 2.3, first
    order) against the analytic Taylor vortex: halving dt about halves the
    velocity error (first order; the ratio approaches 2 from above as dt falls,
    2.32, 2.15, 2.05 for dt = 0.02 ... 0.0025 over a longer run, an O(dt^2)
    part riding on the first-order error).  Its error constant is about twice
    that of the step with the explicit nodal advection (the frozen-velocity
    transport carries a second-order term the explicit step does not)."""
    from oracle.assemble import mass_matrix
    from oracle.gradiv import ins_step, swapped_bc

    def taylor(x, y, t, nu):
        f = np.exp(-2 * np.pi ** 2 * nu * t)
        return (-np.cos(np.pi * x) * np.sin(np.pi * y) * f, np.sin(np.pi * x) * np.cos(np.pi * y) * f,
                -0.25 * (np.cos(2 * np.pi * x) + np.cos(2 * np.pi * y)) * f * f)

    def run(dt, sub, nu=0.05, T=0.06, N=6, n=6):
        msh = synth.square_mesh(n, jitter=0.1, seed=60)
        m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
        mp = OracleMesh(msh.VX, msh.VY, msh.EToV, swapped_bc(msh.EToB), N)
        x, y = (a.ravel() for a in m.node_coords())
        t = 0.05
        u, v, p = taylor(x, y, t, nu)
        pm1 = taylor(x, y, t - dt, nu)[2]
        for _ in range(int(round(T / dt))):
            gn, g1 = taylor(x, y, t, nu), taylor(x, y, t + dt, nu)
            u, v, p_new = ins_step(m, mp, nu, dt, float((N + 1) ** 2), u, v, p, pm1, gn[0], gn[1], g1[0], g1[1],
                                   subcycles=sub)
            pm1, p = p, p_new
            t += dt
        ue, ve, _ = taylor(x, y, t, nu)
        M = mass_matrix(m)
        nrm = lambda a: np.sqrt(a @ (M @ a))
        return np.sqrt(nrm(u - ue) ** 2 + nrm(v - ve) ** 2) / np.sqrt(nrm(ue) ** 2 + nrm(ve) ** 2)

    e1, e2 = run(0.01, 1), run(0.005, 2)
    print(f"subcycled velocity error {e1:.2e} (dt 0.01) -> {e2:.2e} (dt 0.005)")
    assert e2 < 1e-4
    assert 1.8 < e1 / e2 < 2.3
