"""Pins of the oracle's reference triangle against closed forms.

None of the expected values below is produced by the oracle: they are
lattice points, Gauss-Lobatto-Legendre abscissae in closed form, exact monomial
integrals over the bi-unit triangle and exact derivatives of monomials.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle.refelem import RefTriangle, wb_nodes, face_node_ids, gll_points


def tri_monomial_integral(a: int, b: int) -> float:
    """Exact integral of r^a s^b over {-1 <= r, s; r + s <= 0}.

    r = 2 xi - 1, s = 2 eta - 1 maps the unit simplex onto it (Jacobian 4), and
    int xi^k eta^l over the unit simplex is k! l! / (k + l + 2)!.
    """
    tot = Fraction(0)
    for k in range(a + 1):
        for l in range(b + 1):
            c = (math.comb(a, k) * 2**k * (-1) ** (a - k)
                 * math.comb(b, l) * 2**l * (-1) ** (b - l))
            tot += Fraction(c * math.factorial(k) * math.factorial(l), math.factorial(k + l + 2))
    return float(4 * tot)


@pytest.mark.parametrize("N", [1, 2])
def test_low_order_nodes_are_the_equispaced_lattice(N):
    r, s = wb_nodes(N)
    k = 0
    for j in range(N + 1):
        for i in range(N + 1 - j):
            assert r[k] == pytest.approx(-1 + 2 * i / N, abs=1e-14)
            assert s[k] == pytest.approx(-1 + 2 * j / N, abs=1e-14)
            k += 1


def test_edge_nodes_are_gll_in_closed_form():
    # N = 3: +-1, +-1/sqrt(5);  N = 4: 0, +-1, +-sqrt(3/7)
    exp3 = [-1, -1 / math.sqrt(5), 1 / math.sqrt(5), 1]
    exp4 = [-1, -math.sqrt(3 / 7), 0, math.sqrt(3 / 7), 1]
    for N, exp in ((3, exp3), (4, exp4)):
        r, s = wb_nodes(N)
        f0 = face_node_ids(N)[0]
        np.testing.assert_allclose(r[f0], exp, atol=1e-14)
        np.testing.assert_allclose(s[f0], -1.0, atol=1e-14)
        np.testing.assert_allclose(gll_points(N), exp, atol=1e-14)


@pytest.mark.parametrize("N", range(1, 9))
def test_node_set_has_triangle_symmetry(N):
    r, s = wb_nodes(N)
    assert r.size == (N + 1) * (N + 2) // 2
    # barycentric (l0, l1, l2) of v0=(-1,-1), v1=(1,-1), v2=(-1,1)
    l1 = (1 + r) / 2
    l2 = (1 + s) / 2
    l0 = 1 - l1 - l2
    pts = np.stack([l0, l1, l2], 1)
    assert np.all(pts > -1e-13)

    def same_set(p, q):
        d = np.abs(p[:, None, :] - q[None, :, :]).max(-1)
        return np.all(d.min(1) < 1e-12)

    assert same_set(pts, pts[:, [1, 2, 0]])   # rotation
    assert same_set(pts, pts[:, [0, 2, 1]])   # reflection


@pytest.mark.parametrize("N", range(1, 9))
def test_face_nodes_lie_on_their_faces_in_ccw_order(N):
    r, s = wb_nodes(N)
    F = face_node_ids(N)
    np.testing.assert_allclose(s[F[0]], -1, atol=1e-14)
    np.testing.assert_allclose(r[F[1]] + s[F[1]], 0, atol=1e-14)
    np.testing.assert_allclose(r[F[2]], -1, atol=1e-14)
    assert np.all(np.diff(r[F[0]]) > 0)      # v0 -> v1
    assert np.all(np.diff(s[F[1]]) > 0)      # v1 -> v2
    assert np.all(np.diff(s[F[2]]) < 0)      # v2 -> v0


@pytest.mark.parametrize("N", range(1, 9))
def test_mass_matrix_integrates_monomials_exactly(N):
    ref = RefTriangle(N)
    M = ref.mass()
    assert np.ones(ref.Np) @ M @ np.ones(ref.Np) == pytest.approx(2.0, rel=1e-14)
    mons = [(a, b) for a in range(N + 1) for b in range(N + 1 - a)]
    vals = {m: ref.r ** m[0] * ref.s ** m[1] for m in mons}
    for (a, b) in mons:
        for (c, d) in mons:
            got = vals[(a, b)] @ M @ vals[(c, d)]
            exp = tri_monomial_integral(a + c, b + d)
            assert got == pytest.approx(exp, rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("N", range(1, 9))
def test_derivative_matrices_are_exact_on_monomials(N):
    ref = RefTriangle(N)
    Dr, Ds = ref.deriv_matrices()
    r, s = ref.r, ref.s
    for a in range(N + 1):
        for b in range(N + 1 - a):
            u = r ** a * s ** b
            dur = a * r ** max(a - 1, 0) * s ** b if a else 0 * r
            dus = b * r ** a * s ** max(b - 1, 0) if b else 0 * r
            np.testing.assert_allclose(Dr @ u, dur, atol=1e-11 * max(1, np.abs(dur).max()))
            np.testing.assert_allclose(Ds @ u, dus, atol=1e-11 * max(1, np.abs(dus).max()))


@pytest.mark.parametrize("N", range(1, 9))
def test_lagrange_basis_is_cardinal(N):
    ref = RefTriangle(N)
    L, _, _ = ref.lagrange(ref.r, ref.s)
    np.testing.assert_allclose(L, np.eye(ref.Np), atol=1e-12)
