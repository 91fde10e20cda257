"""Pins of the oracle's aggregation AMG (the algebraic levels below degree 1)."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import amg as G
from oracle import solvers as S
from oracle.assemble import OracleMesh, assemble


def test_aggregation_of_a_path_by_hand():
    # 0-1-2-3-4-5-6: seeds 0 ({0,1}), 3 ({2,3,4}), 6 ({5,6}); nothing left for pass 2
    adj = [[1], [0, 2], [1, 3], [2, 4], [3, 5], [4, 6], [5]]
    agg, na = G.aggregate(adj)
    assert na == 3
    assert list(agg) == [0, 0, 1, 1, 1, 2, 2]


def test_aggregation_pass_two_by_hand():
    # star 0-{1,2,3} plus a tail 3-4-5: seed 0 takes {0,1,2,3}; 4 is free but
    # touches 3; 5's only neighbour 4 is free -> seed {4,5}
    adj = [[1, 2, 3], [0], [0], [0, 4], [3, 5], [4]]
    agg, na = G.aggregate(adj)
    assert list(agg) == [0, 0, 0, 0, 1, 1] and na == 2
    # 2-0-1-3-4: seed 0 takes {0,1,2}; 3 touches 1 (taken) -> free; 4 touches
    # 3 (free) -> seed {3,4}
    adj = [[1, 2], [0, 3], [0], [1, 4], [3]]
    agg, na = G.aggregate(adj)
    assert list(agg) == [0, 0, 0, 1, 1] and na == 2
    # 0-1-2-3: seed 0 {0,1}; 2 touches 1 -> free; 3 touches 2 (free) -> seed {2,3}
    adj = [[1], [0, 2], [1, 3], [2]]
    assert list(G.aggregate(adj)[0]) == [0, 0, 1, 1]
    # triangle chain where pass 2 is needed: 0-1, 1-2, 2-3, 1-3; seed 0 {0,1};
    # 2 and 3 touch 1 (taken) -> both free after pass 1; pass 2 joins them to
    # the aggregate of their lowest-index neighbour, 1 -> aggregate 0
    adj = [[1], [0, 2, 3], [1, 3], [1, 2]]
    agg, na = G.aggregate(adj)
    assert list(agg) == [0, 0, 0, 0] and na == 1


def mesh_and_amg(n=12, lam=1.0, bc="dirichlet", coarse_size=16, seed=0):
    msh = synth.square_mesh(n, jitter=0.2, seed=seed, bc=bc)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, 1)
    A = assemble(m, lam, 4.0)
    return m, A, G.AMG(m, A, S.lanczos_rho(A), coarse_size=coarse_size)


def test_aggregates_are_connected_and_cover_the_graph():
    msh = synth.permuted(synth.square_mesh(10, jitter=0.2, seed=3), seed=4)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, 1)
    adj = G.element_graph(m)
    agg, na = G.aggregate(adj)
    assert agg.min() == 0 and agg.max() == na - 1 and np.all(agg >= 0)
    for a in range(na):
        members = set(np.flatnonzero(agg == a))
        seen, stack = set(), [min(members)]
        while stack:
            i = stack.pop()
            if i in seen:
                continue
            seen.add(i)
            stack.extend(j for j in adj[i] if j in members)
        assert seen == members


def test_galerkin_levels_are_spd_and_shrink():
    m, A, amg = mesh_and_amg()
    sizes = amg.sizes
    assert sizes[0] == 3 * m.K and sizes[1] == m.K
    assert all(b < a for a, b in zip(sizes, sizes[1:]))
    assert sizes[-1] <= 16
    for Al in amg.A[1:]:
        D = Al.toarray()
        assert np.allclose(D, D.T, rtol=0, atol=1e-12 * abs(D).max())
        assert np.linalg.eigvalsh(D).min() > 0


def test_element_level_is_the_sum_of_element_blocks():
    m, A, amg = mesh_and_amg(n=6)
    AE = amg.A[1].toarray()
    Ad = A.toarray()
    for e in range(m.K):
        for f in range(m.K):
            assert AE[e, f] == pytest.approx(Ad[3 * e:3 * e + 3, 3 * f:3 * f + 3].sum(), abs=1e-12)


def test_neumann_constants_stay_in_the_null_space_of_every_level():
    m, A, amg = mesh_and_amg(n=8, lam=0.0, bc="neumann", coarse_size=4)
    scale = abs(A).max()
    for Al in amg.A:
        ones = np.ones(Al.shape[0])
        assert abs(Al @ ones).max() <= 1e-10 * scale


def test_gershgorin_bounds_the_spectrum():
    m, A, amg = mesh_and_amg()
    for Al, rho in zip(amg.A[1:], amg.rho[1:]):
        D = Al.toarray()
        d = np.sqrt(np.diag(D))
        ev = np.linalg.eigvalsh(D / d[:, None] / d[None, :]).max()
        assert ev <= rho * (1 + 1e-12)


def test_vcycle_is_symmetric_positive_definite():
    m, A, amg = mesh_and_amg()
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal(A.shape[0]), rng.standard_normal(A.shape[0])
    assert a @ amg.vcycle(0, b) == pytest.approx(b @ amg.vcycle(0, a), rel=1e-10)
    assert a @ amg.vcycle(0, a) > 0


def test_amg_preconditions_much_better_than_jacobi():
    m, A, amg = mesh_and_amg(n=24, lam=0.0)
    b = np.random.default_rng(2).standard_normal(A.shape[0])
    _, it_j, _, _ = S.pcg(A, b, S.jacobi(A), tol=1e-8)
    _, it_a, rel, _ = S.pcg(A, b, lambda r: amg.vcycle(0, r), tol=1e-8)
    assert rel <= 1e-8
    assert it_a * 4 < it_j


def test_pmg_with_amg_coarse_level_solves():
    msh = synth.square_mesh(10, jitter=0.2, seed=5)
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, 4)
    A = assemble(m, 0.0, 25.0)
    rho = []
    for N in (4, 2, 1):
        mN = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
        rho.append(S.lanczos_rho(assemble(mN, 0.0, 25.0 * ((N + 1) / 5) ** 2)))
    b = np.random.default_rng(3).standard_normal(A.shape[0])
    its = {}
    for cycles in (1, 2):
        B = S.PMG(msh, [4, 2, 1], 0.0, 25.0, rho, coarse_amg=True, amg_cycles=cycles, amg_coarse_size=16)
        _, its[cycles], rel, _ = S.pcg(A, b, B, tol=1e-8, flexible=True)
        assert rel <= 1e-8
    _, it_j, _, _ = S.pcg(A, b, S.jacobi(A), tol=1e-8)
    assert its[2] <= its[1] < it_j / 10


def test_kcycle_without_krylov_levels_is_the_vcycle():
    m, A, amg = mesh_and_amg()
    amg.kcycle_levels = 0
    r = np.random.default_rng(5).standard_normal(A.shape[0])
    assert np.array_equal(amg.cycle(0, r), amg.vcycle(0, r))


def test_krylov_correction_is_the_a_norm_projection_on_the_krylov_space():
    """With a fixed SPD preconditioner B in place of the inner cycle, the two
    flexible-CG steps give the A-norm best approximation of A^-1 rc in
    span{B rc, B A B rc}: solved here from the 2 x 2 Galerkin system."""
    m, A, amg = mesh_and_amg(n=10)
    l = 1
    Al = amg.A[l].toarray()
    rng = np.random.default_rng(6)
    d = 1.0 / np.diag(Al) * (1.0 + 0.5 * rng.random(Al.shape[0]))   # SPD diagonal B, not A's inverse
    amg.cycle = lambda lev, q: d * q
    rc = rng.standard_normal(Al.shape[0])
    amg.kcycle_t = 0.0                                                # always take both steps
    e = amg.krylov_correction(l, rc)
    V = np.stack([d * rc, d * (Al @ (d * rc))], axis=1)
    c = np.linalg.solve(V.T @ Al @ V, V.T @ rc)
    assert np.linalg.norm(e - V @ c) <= 1e-12 * np.linalg.norm(V @ c)


def test_krylov_correction_with_an_exact_inner_solve_is_exact():
    m, A, amg = mesh_and_amg(n=10)
    l = 1
    Al = amg.A[l].toarray()
    Ainv = np.linalg.inv(Al)
    amg.cycle = lambda lev, q: Ainv @ q
    rc = np.random.default_rng(7).standard_normal(Al.shape[0])
    e = amg.krylov_correction(l, rc)                                 # early exit after one step
    assert np.linalg.norm(e - Ainv @ rc) <= 1e-10 * np.linalg.norm(Ainv @ rc)


def test_kcycle_preconditions_better_than_the_vcycle():
    m, A, amg = mesh_and_amg(n=24, lam=0.0)
    b = np.random.default_rng(8).standard_normal(A.shape[0])
    _, it_v, _, _ = S.pcg(A, b, lambda r: amg.vcycle(0, r), tol=1e-8)
    _, it_k, rel, _ = S.pcg(A, b, lambda r: amg.cycle(0, r), tol=1e-8, flexible=True)
    assert rel <= 1e-8
    assert it_k < it_v


def test_top_krylov_step_on_the_degree_one_level():
    """The two flexible-CG steps on the degree-1 level itself (each
    preconditioned by one AMG cycle) give the A-norm best approximation over
    the span of their two preconditioned directions (a linear SPD stand-in
    for the cycle, as above), and in p-multigrid a solve needs no more
    iterations than with one cycle."""
    m, A, amg = mesh_and_amg(n=10)
    Ad = A.toarray()
    rng = np.random.default_rng(9)
    d = 1.0 / np.diag(Ad) * (1.0 + 0.5 * rng.random(Ad.shape[0]))
    cyc = amg.cycle
    amg.cycle = lambda lev, q: d * q
    amg.kcycle_t = 0.0
    rc = rng.standard_normal(Ad.shape[0])
    e = amg.krylov_correction(0, rc)
    V = np.stack([d * rc, d * (Ad @ (d * rc))], axis=1)
    c = np.linalg.solve(V.T @ Ad @ V, V.T @ rc)
    assert np.linalg.norm(e - V @ c) <= 1e-12 * np.linalg.norm(V @ c)
    amg.cycle = cyc
    msh = synth.square_mesh(10, jitter=0.2, seed=5)
    mk = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, 4)
    A4 = assemble(mk, 0.0, 25.0)
    rho = []
    for N in (4, 2, 1):
        mN = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
        rho.append(S.lanczos_rho(assemble(mN, 0.0, 25.0 * ((N + 1) / 5) ** 2)))
    b = np.random.default_rng(3).standard_normal(A4.shape[0])
    its = {}
    for top in (False, True):
        B = S.PMG(msh, [4, 2, 1], 0.0, 25.0, rho, coarse_amg=True, amg_coarse_size=16, amg_top_krylov=top)
        _, its[top], rel, _ = S.pcg(A4, b, B, tol=1e-8, flexible=True)
        assert rel <= 1e-8
    assert its[True] <= its[False]
