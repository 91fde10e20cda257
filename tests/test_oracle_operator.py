"""Pins of the oracle's assembled SIPDG operator (Eq. INS_SD_5, Eq.
ellipticOp1, penalty Eq. Ch2.PenaltyParameter) against closed forms.

Each expected value is computed here from vertex coordinates or from calculus,
not by the oracle: a dropped term, a wrong sign, a wrong 1/2 or a transposed
block in the oracle fails at least one of these tests.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle.assemble import (OracleMesh, MeshError, assemble, mass_apply, mass_matrix,
                             apply_rows)


def omesh(msh, N):
    return OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)


def geom(msh, e, f):
    """Face f of element e straight from the vertex arrays."""
    a = msh.EToV[e, f]
    b = msh.EToV[e, (f + 1) % 3]
    xa, ya, xb, yb = msh.VX[a], msh.VY[a], msh.VX[b], msh.VY[b]
    L = math.hypot(xb - xa, yb - ya)
    return xa, ya, xb, yb, L, (yb - ya) / L, -(xb - xa) / L


def area(msh, e):
    x = msh.VX[msh.EToV[e]]
    y = msh.VY[msh.EToV[e]]
    return 0.5 * ((x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]))


def neighbours(msh):
    """(e, f) -> e' by brute force over all element pairs (tiny meshes)."""
    out = {}
    K = msh.K
    for e in range(K):
        for f in range(3):
            key = {msh.EToV[e, f], msh.EToV[e, (f + 1) % 3]}
            for e2 in range(K):
                if e2 == e:
                    continue
                for f2 in range(3):
                    if {msh.EToV[e2, f2], msh.EToV[e2, (f2 + 1) % 3]} == key:
                        out[(e, f)] = e2
    return out


def unit(K, Np, e, vals=1.0):
    x = np.zeros(K * Np)
    x[e * Np:(e + 1) * Np] = vals
    return x


# -- P-D: symmetry, positive-definiteness, Neumann null space ---------------

@pytest.mark.parametrize("N", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("bc", ["dirichlet", "mixed"])
def test_symmetric_positive_definite(N, bc):
    msh = synth.square_mesh(3, jitter=0.2, seed=7, bc=bc)
    m = omesh(msh, N)
    A = assemble(m, 0.0, (N + 1) ** 2).toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0


@pytest.mark.parametrize("N", [1, 3, 6])
def test_pure_neumann_null_space_is_constants(N):
    msh = synth.square_mesh(3, jitter=0.2, seed=8, bc="neumann")
    m = omesh(msh, N)
    A = assemble(m, 0.0, (N + 1) ** 2).toarray()
    one = np.ones(A.shape[0])
    assert np.abs(A @ one).max() < 1e-11 * np.abs(A).max()
    ev = np.linalg.eigvalsh(A)
    assert abs(ev[0]) < 1e-10 * ev[-1] and ev[1] > 1e-8 * ev[-1]
    # with lambda: sum_i (A x)_i = lambda 1^T M x
    lam = 3.7
    Al = assemble(m, lam, (N + 1) ** 2)
    x = np.random.default_rng(1).standard_normal(A.shape[0])
    assert one @ (Al @ x) == pytest.approx(lam * one @ mass_apply(m, x), rel=1e-11)


@pytest.mark.parametrize("N", [2, 4])
def test_lambda_enters_as_mass(N):
    msh = synth.square_mesh(3, jitter=0.2, seed=9)
    m = omesh(msh, N)
    A0 = assemble(m, 0.0, 9.0)
    A1 = assemble(m, 100.0, 9.0)
    M = mass_matrix(m)
    assert abs((A1 - A0 - 100.0 * M)).max() < 1e-11 * abs(A1).max()


# -- P-A: a smooth function vanishing on the boundary ------------------------

@pytest.mark.parametrize("N", [4, 5, 8])
@pytest.mark.parametrize("lam", [0.0, 100.0])
@pytest.mark.parametrize("jit", [0.0, 0.2])
def test_bubble_closed_form(N, lam, jit):
    """u = x(1-x)y(1-y) lies in V_N for N >= 4 and has no jumps and no
    boundary trace, so A u = M (-Lap u + lam u) element by element and
    u^T A u = int |grad u|^2 + lam int u^2 = 1/45 + lam/900 on any mesh of the
    unit square, for any penalty."""
    msh = synth.square_mesh(4, jitter=jit, seed=3)
    msh = synth.permuted(msh, seed=11)
    m = omesh(msh, N)
    x, y = m.node_coords()
    u = (x * (1 - x) * y * (1 - y)).ravel()
    g = (2 * y * (1 - y) + 2 * x * (1 - x)).ravel() + lam * u
    for ctau in (1.0 * (N + 1) ** 2, 50.0):
        A = assemble(m, lam, ctau)
        Au = A @ u
        np.testing.assert_allclose(Au, mass_apply(m, g), atol=1e-12 * np.abs(Au).max())
        assert u @ Au == pytest.approx(1 / 45 + lam / 900, rel=1e-12)


# -- P-C: N = 1 continuous hats reproduce the 5-point stencil ----------------

def test_p1_hats_give_five_point_stencil():
    n = 5
    msh = synth.square_mesh(n, bc="dirichlet")
    m = omesh(msh, 1)
    A = assemble(m, 0.0, 4.0)
    K = msh.K

    def hat(i, j):
        k = j * (n + 1) + i
        return (msh.EToV == k).astype(np.float64).ravel()   # node order = v0, v1, v2

    for (i, j) in [(1, 1), (2, 3), (4, 4)]:
        hij = hat(i, j)
        assert hij @ A @ hij == pytest.approx(4.0, abs=1e-12)
        for (di, dj) in [(1, 0), (-1, 0), (0, 1), (0, -1)]:
            ii, jj = i + di, j + dj
            if 0 < ii < n and 0 < jj < n:
                assert hat(ii, jj) @ A @ hij == pytest.approx(-1.0, abs=1e-12)
        for (di, dj) in [(1, 1), (-1, -1), (1, -1), (-1, 1)]:
            ii, jj = i + di, j + dj
            if 0 < ii < n and 0 < jj < n:
                assert hat(ii, jj) @ A @ hij == pytest.approx(0.0, abs=1e-12)


# -- penalty and consistency terms on single elements ------------------------

@pytest.mark.parametrize("N", [1, 3, 7])
@pytest.mark.parametrize("bc", ["neumann", "dirichlet", "mixed"])
def test_penalty_term_from_piecewise_constants(N, bc):
    """For u = 1 on element e and 0 elsewhere, grad u = 0 everywhere, so
    u^T A u = sum over e's interior faces of tau_F |F| + sum over its
    Dirichlet faces of 2 tau_F |F| (lambda = 0), and the coupling with a
    neighbour e' across F is -tau_F |F|."""
    msh = synth.square_mesh(3, jitter=0.25, seed=5, bc=bc)
    m = omesh(msh, N)
    Np = m.Np
    ctau = 7.5
    A = assemble(m, 0.0, ctau)
    nb = neighbours(msh)
    for e in range(msh.K):
        exp = 0.0
        for f in range(3):
            *_, L, _, _ = geom(msh, e, f)
            if (e, f) in nb:
                e2 = nb[(e, f)]
                tau = ctau * max(L / area(msh, e), L / area(msh, e2))
                exp += tau * L
                got = unit(msh.K, Np, e2) @ A @ unit(msh.K, Np, e)
                assert got == pytest.approx(-tau * L, rel=1e-12)
            elif msh.EToB[e, f] == synth.BC_DIRICHLET:
                exp += 2 * ctau * L / area(msh, e) * L
        ue = unit(msh.K, Np, e)
        assert ue @ A @ ue == pytest.approx(exp, rel=1e-12)


@pytest.mark.parametrize("N", [1, 2, 5])
@pytest.mark.parametrize("lam", [0.0, 2.5])
def test_consistency_terms_from_linear_functions(N, lam):
    """u = x and v = y on element e only (zero elsewhere), w = 1 on e, z = 1 on
    a neighbour.  Their forms follow from the face terms alone:
      a(u, w) over e's faces: interior -|F| n_x/2 + tau |F| x_mid,
                              Dirichlet -|F| n_x + 2 tau |F| x_mid
      a(u, z) across F:       |F| n_x/2 - tau |F| x_mid
      a(u, v): (grad x, grad y) = 0, interior faces
               -(n_x int_F y + n_y int_F x)/2 + tau int_F x y,
               Dirichlet faces -(n_x int_F y + n_y int_F x) + 2 tau int_F x y
    plus lam times the element integrals."""
    msh = synth.square_mesh(3, jitter=0.25, seed=6, bc="mixed")
    m = omesh(msh, N)
    Np = m.Np
    ctau = 5.0
    A = assemble(m, lam, ctau)
    X, Y = m.node_coords()
    nb = neighbours(msh)
    for e in range(msh.K):
        u = unit(msh.K, Np, e, X[e])
        v = unit(msh.K, Np, e, Y[e])
        w = unit(msh.K, Np, e)
        ex = msh.VX[msh.EToV[e]]
        ey = msh.VY[msh.EToV[e]]
        ar = area(msh, e)
        # element integrals of x, xy over a triangle (exact vertex formulas)
        int_x = ar * ex.mean()
        int_xy = ar / 12 * (np.sum(ex * ey) + np.sum(ex) * np.sum(ey))
        exp_uw = lam * int_x
        exp_uv = lam * int_xy
        for f in range(3):
            xa, ya, xb, yb, L, nx, ny = geom(msh, e, f)
            fx = L * (xa + xb) / 2
            fy = L * (ya + yb) / 2
            fxy = L * ((xa * ya + xb * yb) / 3 + (xa * yb + xb * ya) / 6)
            if (e, f) in nb:
                e2 = nb[(e, f)]
                tau = ctau * max(L / ar, L / area(msh, e2))
                exp_uw += -0.5 * L * nx + tau * fx
                exp_uv += -0.5 * (nx * fy + ny * fx) + tau * fxy
                z = unit(msh.K, Np, e2)
                assert z @ A @ u == pytest.approx(0.5 * L * nx - tau * fx, rel=1e-11, abs=1e-12)
            elif msh.EToB[e, f] == synth.BC_DIRICHLET:
                tau = ctau * L / ar
                exp_uw += -L * nx + 2 * tau * fx
                exp_uv += -(nx * fy + ny * fx) + 2 * tau * fxy
        assert w @ A @ u == pytest.approx(exp_uw, rel=1e-11, abs=1e-12)
        assert u @ A @ w == pytest.approx(exp_uw, rel=1e-11, abs=1e-12)
        assert v @ A @ u == pytest.approx(exp_uv, rel=1e-11, abs=1e-12)


def test_apply_rows_matches_full_assembly():
    msh = synth.permuted(synth.square_mesh(5, jitter=0.2, seed=2, bc="mixed"), seed=3)
    m = omesh(msh, 4)
    A = assemble(m, 3.0, 25.0)
    x = np.random.default_rng(0).standard_normal(A.shape[0])
    y = (A @ x).reshape(msh.K, m.Np)
    sel = np.array([7, 0, 33, 12, 49])
    np.testing.assert_allclose(apply_rows(m, 3.0, 25.0, x, sel), y[sel], rtol=0, atol=1e-13 * np.abs(y).max())


# -- O11: manufactured solution converges at order N+1 in L2 ----------------

def l2_error(m, u, exact):
    ref = m.ref
    U = u.reshape(m.K, m.Np) @ ref.qL.T                 # values at quadrature points
    r, s = ref.qr, ref.qs
    qx = (-(r + s)[None] * m.x0[:, None] + (1 + r)[None] * m.x1[:, None] + (1 + s)[None] * m.x2[:, None]) / 2
    qy = (-(r + s)[None] * m.y0[:, None] + (1 + r)[None] * m.y1[:, None] + (1 + s)[None] * m.y2[:, None]) / 2
    err = (U - exact(qx, qy)) ** 2
    return math.sqrt(np.sum(err * ref.qw[None] * m.J[:, None]))


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_manufactured_poisson_converges_at_order_N_plus_1(N):
    exact = lambda x, y: np.sin(np.pi * x) * np.sin(np.pi * y)
    errs = []
    ns = [4, 8, 16]
    for n in ns:
        msh = synth.square_mesh(n, jitter=0.0)
        m = omesh(msh, N)
        A = assemble(m, 0.0, (N + 1) ** 2).tocsc()
        x, y = m.node_coords()
        b = mass_apply(m, (2 * np.pi ** 2 * exact(x, y)).ravel())
        u = spla.spsolve(A, b)
        errs.append(l2_error(m, u, exact))
    rate = math.log(errs[-2] / errs[-1], 2)
    assert rate >= N + 1 - 0.2, (errs, rate)


# -- mesh validation ---------------------------------------------------------

def test_mesh_errors():
    msh = synth.square_mesh(2)
    bad = msh.EToV.copy()
    bad[0] = bad[0][::-1]                       # clockwise element
    with pytest.raises(MeshError):
        OracleMesh(msh.VX, msh.VY, bad, msh.EToB, 2)
    b = msh.EToB.copy()
    b[0, 0] = synth.BC_INTERIOR if b[0, 0] else synth.BC_DIRICHLET
    with pytest.raises(MeshError):
        OracleMesh(msh.VX, msh.VY, msh.EToV, b, 2)
    # a face shared by three elements
    VX = np.array([0.0, 1.0, 0.5, 0.5, 0.5])
    VY = np.array([0.0, 0.0, 1.0, -1.0, 2.0])
    EToV = np.array([[0, 1, 2], [1, 0, 3], [0, 1, 4]])
    with pytest.raises(MeshError):
        OracleMesh(VX, VY, EToV, np.zeros((3, 3), np.int8), 1)
