"""Pins of the oracle's DG gradient and divergence (Sec. 2.1, Eq. INS_SD_4_1
and INS_SD_4_2) and of the projection half of the splitting step (Sec. 2.2,
Eq. INS_TD_3_3 and INS_TD_3_4).

Fixed by the mathematics rather than by the oracle's own formulas:
  * a global polynomial of degree <= N has no jumps, so central fluxes give
    the exact gradient (Dirichlet faces take p* = p-) and the exact
    divergence (Dirichlet data equal to the field itself, Neumann faces
    u* = u-);
  * with central fluxes and the paper's boundary rules the divergence is
    minus the adjoint of the gradient in the mass inner product,
    M D = -(M G)^T, for every boundary mix (integration by parts);
  * a constant pressure c has a gradient only through the Neumann faces
    (p* = 0): 1^T M G_x c = -c times the sum of n_x |F| over those faces;
  * projecting grad(phi) + curl(psi) (phi = 0 on the boundary, where the
    pressure is fixed) returns curl(psi) and phi, with errors falling at
    high order under refinement.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle.assemble import BC_DIRICHLET, BC_NEUMANN, OracleMesh, assemble
from oracle.gradiv import GradDiv, swapped_bc


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


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_gradient_of_a_global_polynomial_is_exact(N):
    msh = synth.permuted(synth.square_mesh(4, jitter=0.2, seed=1), seed=2)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    x, y = m.node_coords()
    p, px, py = (a.ravel() for a in poly(x, y, N, seed=N))
    gx, gy = GradDiv(m).grad(p)
    assert np.abs(gx - px).max() <= 1e-10 * np.abs(px).max()
    assert np.abs(gy - py).max() <= 1e-10 * np.abs(py).max()


@pytest.mark.parametrize("bc", ["dirichlet", "neumann", "mixed"])
@pytest.mark.parametrize("N", [1, 3, 4])
def test_divergence_of_a_global_polynomial_field_is_exact(N, bc):
    msh = synth.permuted(synth.square_mesh(4, jitter=0.2, seed=3, bc=bc), seed=4)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    x, y = m.node_coords()
    u, ux, _ = (a.ravel() for a in poly(x, y, N, seed=10 + N))
    v, _, vy = (a.ravel() for a in poly(x, y, N, seed=20 + N))
    d = GradDiv(m).div(u, v, u, v)
    ref = ux + vy
    assert np.abs(d - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("bc", ["dirichlet", "neumann", "mixed"])
@pytest.mark.parametrize("N", [1, 2, 3])
def test_divergence_is_minus_the_adjoint_of_the_gradient(N, bc):
    msh = synth.permuted(synth.square_mesh(3, jitter=0.2, seed=5, bc=bc), seed=6)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    gd = GradDiv(m)
    for D, G in ((gd.Dx, gd.Gx), (gd.Dy, gd.Gy)):
        MD = (gd.M @ D).toarray()
        MG = (gd.M @ G).toarray()
        assert np.abs(MD + MG.T).max() <= 1e-12 * np.abs(MG).max()


@pytest.mark.parametrize("bc", ["neumann", "mixed"])
def test_constant_pressure_sees_only_neumann_faces(bc):
    msh = synth.square_mesh(5, jitter=0.2, seed=7, bc=bc)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, 2)
    gd = GradDiv(m)
    c = 1.7
    gx, gy = gd.grad(np.full(m.K * m.Np, c))
    one = np.ones(m.K * m.Np)
    sx = sy = 0.0
    for e in range(m.K):
        for f in range(3):
            if m.EToB[e, f] == BC_NEUMANN:
                _, _, _, _, length, nx, ny = m.face_geometry(e, f)
                sx += nx * length
                sy += ny * length
    assert one @ (gd.M @ gx) == pytest.approx(-c * sx, abs=1e-12)
    assert one @ (gd.M @ gy) == pytest.approx(-c * sy, abs=1e-12)


def projection_error(n, N):
    """Project U = grad(phi) + curl(psi) on the unit square with velocity
    Neumann (outflow) boundaries, i.e. pressure Dirichlet p = 0, gamma / dt = 1."""
    msh = synth.square_mesh(n, jitter=0.1, seed=8, bc="neumann")
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    mp = OracleMesh(msh.VX, msh.VY, msh.EToV, swapped_bc(msh.EToB), N)
    x, y = (a.ravel() for a in m.node_coords())
    pi = np.pi
    phi = np.sin(pi * x) * np.sin(pi * y)
    psi = np.cos(pi * x) * np.cos(2 * pi * y)
    gpx, gpy = pi * np.cos(pi * x) * np.sin(pi * y), pi * np.sin(pi * x) * np.cos(pi * y)
    cx = -2 * pi * np.cos(pi * x) * np.sin(2 * pi * y)     # curl psi = (psi_y, -psi_x)
    cy = pi * np.sin(pi * x) * np.cos(2 * pi * y)
    gd = GradDiv(m)
    b = gd.pressure_rhs(1.0, 1.0, gpx + cx, gpy + cy)
    S = assemble(mp, 0.0, float((N + 1) ** 2))
    dp = spla.spsolve(S.tocsc(), b)
    u, v, p = gd.correct(1.0, 1.0, gpx + cx, gpy + cy, dp, np.zeros_like(dp))
    M = gd.M
    nrm = lambda a: np.sqrt(a @ (M @ a))
    eu = np.sqrt(nrm(u - cx) ** 2 + nrm(v - cy) ** 2) / np.sqrt(nrm(cx) ** 2 + nrm(cy) ** 2)
    ep = nrm(p - phi) / nrm(phi)
    return eu, ep


@pytest.mark.parametrize("N", [2, 3])
def test_projection_recovers_the_solenoidal_part(N):
    eu1, ep1 = projection_error(6, N)
    eu2, ep2 = projection_error(12, N)
    print(f"N={N}: velocity {eu1:.2e} -> {eu2:.2e}, pressure {ep1:.2e} -> {ep2:.2e}")
    assert eu2 < 5e-2 and ep2 < 5e-2
    assert eu1 / eu2 > 2 ** (N - 0.5)
    assert ep1 / ep2 > 2 ** (N - 0.5)


@pytest.mark.parametrize("bc", ["dirichlet", "mixed"])
@pytest.mark.parametrize("N", [1, 2, 4])
def test_dirichlet_data_reproduce_global_polynomials(N, bc):
    """SIPDG is consistent: for a global polynomial u of degree <= N,
    A u = M (-lap u + lambda u) + b_g(u) holds exactly once the Dirichlet data
    g = u enter through dirichlet_rhs.  On Neumann faces the natural condition
    would need the normal derivative as data, which is not supplied here, so
    on the mixed mesh only the rows of elements without Neumann faces are
    checked."""
    from oracle.assemble import mass_apply
    from oracle.gradiv import dirichlet_rhs
    msh = synth.permuted(synth.square_mesh(4, jitter=0.2, seed=40, bc=bc), seed=41)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    x, y = m.node_coords()
    x, y = x.ravel(), y.ravel()
    rng = np.random.default_rng(42 + N)
    c = rng.standard_normal((N + 1, N + 1))
    u = np.zeros_like(x)
    lap = np.zeros_like(x)
    for a in range(N + 1):
        for bb in range(N + 1 - a):
            u += c[a, bb] * x ** a * y ** bb
            if a >= 2:
                lap += c[a, bb] * a * (a - 1) * x ** (a - 2) * y ** bb
            if bb >= 2:
                lap += c[a, bb] * bb * (bb - 1) * x ** a * y ** (bb - 2)
    lam, ctau = 0.7, float((N + 1) ** 2)
    A = assemble(m, lam, ctau)
    r = A @ u - mass_apply(m, -lap + lam * u) - dirichlet_rhs(m, ctau, u)
    scale = np.abs(A @ u).max()
    if bc == "dirichlet":
        assert np.abs(r).max() <= 1e-10 * scale
    else:
        # rows of elements without Neumann faces see only interior and
        # Dirichlet faces: consistent there
        clean = np.all(m.EToB != BC_NEUMANN, axis=1)
        rr = r.reshape(m.K, m.Np)[clean]
        assert clean.any() and np.abs(rr).max() <= 1e-10 * scale


@pytest.mark.parametrize("bc", ["dirichlet", "neumann", "mixed"])
@pytest.mark.parametrize("N", [2, 4])
def test_advection_of_a_linear_field_is_exact(N, bc):
    """u linear: u (x) u is quadratic, represented exactly at the nodes when
    N >= 2, and continuous, so with the Dirichlet data equal to u every jump
    and flux difference vanishes and N(u) = div(u (x) u) exactly (Neumann
    faces copy u- as the outer state)."""
    from oracle.gradiv import advection
    msh = synth.permuted(synth.square_mesh(4, jitter=0.2, seed=50, bc=bc), seed=51)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    x, y = (a.ravel() for a in m.node_coords())
    a, b, c, d, e, f = 0.3, -1.2, 0.7, 0.5, 1.1, -0.4
    u = a + b * x + c * y
    v = d + e * x + f * y
    nu, nv = advection(m, u, v, u, v)
    # div(u u, u v) = 2 u u_x + u_y v + u v_y; div(v u, v v) = v_x u + v u_x + 2 v v_y
    ru = 2 * u * b + c * v + u * f
    rv = e * u + v * b + 2 * v * f
    assert np.abs(nu - ru).max() <= 1e-10 * np.abs(ru).max()
    assert np.abs(nv - rv).max() <= 1e-10 * np.abs(rv).max()


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_advection_flux_term_dissipates_jumps(bc):
    """The Lax-Friedrichs part of the flux, (Lambda/2)(c- - c+), adds to the
    energy rate (U, N(U))_M exactly sum_F int_F (Lambda/2) |u- - u+|^2 >= 0
    (each interior face seen from both sides; on Dirichlet faces with zero
    data, int (Lambda/2) |u-|^2): positive for a discontinuous field, zero
    for a continuous one whose data match it."""
    from oracle.gradiv import advection
    from oracle.assemble import mass_matrix
    msh = synth.square_mesh(5, jitter=0.2, seed=52, bc=bc)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, 3)
    M = mass_matrix(m)
    rng = np.random.default_rng(53)
    n = m.K * m.Np
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    rate = lambda lax: sum(a @ (M @ b) for a, b in zip((u, v), advection(m, u, v, lax=lax)))
    assert rate(1.0) - rate(0.0) > 0.0
    x, y = (a.ravel() for a in m.node_coords())
    u, v = 0.3 + x - y, -0.2 + 0.5 * x + y                       # continuous, data = itself
    rate = lambda lax: sum(a @ (M @ b) for a, b in zip((u, v), advection(m, u, v, u, v, lax=lax)))
    assert abs(rate(1.0) - rate(0.0)) <= 1e-12 * abs(rate(0.0))


def test_splitting_step_converges_to_the_taylor_vortex():
    """The whole step (advection, Dirichlet data, gradient, divergence, both
    solves) against the analytic Taylor vortex: at a spatial resolution far
    finer than the time error, halving dt halves the velocity error (first
    order in time)."""
    from oracle.assemble import mass_matrix
    from oracle.gradiv import ins_step

    def taylor(x, y, t, nu):
        f = np.exp(-2 * np.pi ** 2 * nu * t)
        return (-np.cos(np.pi * x) * np.sin(np.pi * y) * f, np.sin(np.pi * x) * np.cos(np.pi * y) * f,
                -0.25 * (np.cos(2 * np.pi * x) + np.cos(2 * np.pi * y)) * f * f)

    def run(dt, nu=0.05, T=0.1, N=6, n=8):
        msh = synth.square_mesh(n, jitter=0.1, seed=60)
        m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
        mp = OracleMesh(msh.VX, msh.VY, msh.EToV, swapped_bc(msh.EToB), N)
        x, y = (a.ravel() for a in m.node_coords())
        t = 0.05
        u, v, p = taylor(x, y, t, nu)
        pm1 = taylor(x, y, t - dt, nu)[2]
        for _ in range(int(round(T / dt))):
            gn, g1 = taylor(x, y, t, nu), taylor(x, y, t + dt, nu)
            u1, v1, p1 = ins_step(m, mp, nu, dt, float((N + 1) ** 2), u, v, p, pm1, gn[0], gn[1], g1[0], g1[1])
            pm1, u, v, p = p, u1, v1, p1
            t += dt
        ue, ve, _ = taylor(x, y, t, nu)
        M = mass_matrix(m)
        nrm = lambda a: np.sqrt(a @ (M @ a))
        return np.sqrt(nrm(u - ue) ** 2 + nrm(v - ve) ** 2) / np.sqrt(nrm(ue) ** 2 + nrm(ve) ** 2)

    e1, e2 = run(0.02), run(0.01)
    print(f"velocity error {e1:.2e} (dt 0.02) -> {e2:.2e} (dt 0.01)")
    assert e2 < 2e-4
    assert 1.8 < e1 / e2 < 2.2
