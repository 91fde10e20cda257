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
