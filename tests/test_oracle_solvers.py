"""Pins of the oracle's solvers and preconditioners (Sec. 3).

Expected values come from a direct sparse solve, from the closed-form
Chebyshev error polynomial, from polynomial reproduction and from dense
eigen-decompositions, never from the solver under test.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import solvers as S
from oracle.assemble import OracleMesh, assemble, mass_apply
from oracle.refelem import RefTriangle


def omesh(msh, N):
    return OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)


def config1():
    """16 x 16 squares, N = 3, Dirichlet, c_tau = 16, f = 2 pi^2 sin sin."""
    msh = synth.square_mesh(16)
    m = omesh(msh, 3)
    A = assemble(m, 0.0, 16.0)
    x, y = m.node_coords()
    b = mass_apply(m, (2 * np.pi ** 2 * np.sin(np.pi * x) * np.sin(np.pi * y)).ravel())
    return msh, m, A, b


def test_jacobi_pcg_reaches_direct_solution_on_config1():
    msh, m, A, b = config1()
    xd = spla.spsolve(A.tocsc(), b)
    # 1e-12 is the attainable floor here: the direct solution's own relative
    # residual is ~1e-12 (cond(A) ~ 1.3e4)
    x, it, rel, _ = S.pcg(A, b, S.jacobi(A), tol=1e-12, max_iters=5000)
    assert rel <= 1e-12
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)
    # the 1e-10 run of the workload: residual bound holds
    x10, it10, rel10, _ = S.pcg(A, b, S.jacobi(A), tol=1e-10)
    assert rel10 <= 1e-10 and it10 < it


def test_flexible_equals_textbook_cg_for_fixed_spd_preconditioner():
    msh, m, A, b = config1()
    P = S.jacobi(A)
    _, _, _, i1 = S.pcg(A, b, P, tol=1e-9, keep_iterates=True)
    _, _, _, i2 = S.pcg(A, b, P, tol=1e-9, keep_iterates=True, flexible=True)
    for k in range(20):
        np.testing.assert_allclose(i2["iterates"][k], i1["iterates"][k],
                                   atol=1e-10 * np.abs(i1["iterates"][k]).max())


def test_block_mass_preconditioner_is_exact_inverse_of_mass_and_scale_free():
    msh = synth.square_mesh(6, jitter=0.2, seed=1)
    m = omesh(msh, 4)
    B = S.block_mass_inverse(m)
    v = np.random.default_rng(0).standard_normal(m.K * m.Np)
    np.testing.assert_allclose(mass_apply(m, B(v)), v, atol=1e-11 * np.abs(v).max())
    A = assemble(m, 1000.0, 25.0)
    b = mass_apply(m, np.random.default_rng(1).standard_normal(m.K * m.Np))
    _, it1, _, _ = S.pcg(A, b, B, tol=1e-8)
    _, it2, _, _ = S.pcg(A, b, lambda r: 7.0 * B(r), tol=1e-8)
    assert it1 == it2
    # mass dominated: few iterations as lambda grows
    A6 = assemble(m, 1e6, 25.0)
    _, it3, _, _ = S.pcg(A6, b, B, tol=1e-8)
    assert it3 < it1 and it3 <= 12


def test_pcg_breakdown_is_detected_on_an_indefinite_matrix():
    A = sp.diags([1.0, -1.0, 2.0])
    with pytest.raises(S.Breakdown):
        S.pcg(A, np.array([1.0, 1.0, 0.0]), tol=1e-12)


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_chebyshev_matches_closed_form_error_polynomial(degree):
    lam = np.linspace(0.05, 2.0, 40)
    A = sp.diags(lam).tocsr()
    dinv = np.ones_like(lam)
    xs = np.random.default_rng(3).standard_normal(lam.size)
    f = A @ xs
    lo, hi = 0.3, 2.2
    x = S.chebyshev(A, dinv, f, None, lo, hi, degree)
    theta, delta = (hi + lo) / 2, (hi - lo) / 2
    T = np.polynomial.chebyshev.Chebyshev.basis(degree)
    factor = T((theta - lam) / delta) / T(theta / delta)
    np.testing.assert_allclose(xs - x, factor * xs, atol=1e-13)


@pytest.mark.parametrize("Nc,Nf", [(1, 3), (3, 7), (2, 5), (7, 8)])
def test_interpolation_reproduces_coarse_polynomials(Nc, Nf):
    I = S.interpolation(Nc, Nf)
    rc, rf = RefTriangle(Nc), RefTriangle(Nf)
    for a in range(Nc + 1):
        for b in range(Nc + 1 - a):
            np.testing.assert_allclose(I @ (rc.r ** a * rc.s ** b), rf.r ** a * rf.s ** b, atol=1e-12)


def test_lanczos_estimate_brackets_the_spectrum():
    msh = synth.square_mesh(6, jitter=0.2, seed=2)
    m = omesh(msh, 3)
    A = assemble(m, 0.0, 16.0)
    d = A.diagonal()
    Ad = (A.toarray() / np.sqrt(d)[:, None]) / np.sqrt(d)[None, :]
    true = np.linalg.eigvalsh(Ad).max()
    est = S.lanczos_rho(A, steps=20, seed=0)
    assert 0.95 * true <= est <= true * (1 + 1e-12)


def pmg_setup(n=6, degrees=(5, 3, 1), exact=True):
    msh = synth.square_mesh(n, jitter=0.2, seed=4)
    ctau = (degrees[0] + 1) ** 2
    rho = []
    for Nl in degrees:
        ml = omesh(msh, Nl)
        rho.append(S.lanczos_rho(assemble(ml, 0.0, ctau * ((Nl + 1) / (degrees[0] + 1)) ** 2)))
    return msh, S.PMG(msh, degrees, 0.0, ctau, rho, coarse_exact=exact)


def test_vcycle_with_exact_coarse_solve_is_symmetric_positive_definite():
    msh, B = pmg_setup()
    n = B.levels[0]["A"].shape[0]
    rng = np.random.default_rng(5)
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    assert u @ B(v) == pytest.approx(v @ B(u), rel=1e-10)
    assert u @ B(u) > 0 and v @ B(v) > 0


def test_pmg_pcg_solves_and_beats_jacobi():
    msh, B = pmg_setup(n=8, exact=False)
    A = B.levels[0]["A"]
    b = np.random.default_rng(6).standard_normal(A.shape[0])
    x, it, rel, _ = S.pcg(A, b, B, tol=1e-8, flexible=True)
    xd = spla.spsolve(A.tocsc(), b)
    assert rel <= 1e-8
    assert np.linalg.norm(x - xd) <= 1e-5 * np.linalg.norm(xd)
    _, itj, _, _ = S.pcg(A, b, S.jacobi(A), tol=1e-8)
    assert it * 4 < itj
