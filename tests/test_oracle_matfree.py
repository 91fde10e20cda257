"""Pins of the oracle's matrix-free operator (Alg. AxG + Alg. AxKernel,
Eq. ellipticOp3): it must equal the assembled bilinear form, the plain
definition of A, to round-off on every degree, boundary mix, lambda and
coefficient, also when only some elements' rows are computed.  Plausible
mistakes in its inputs (a missing neighbour trace, swapped normal components,
a wrong surface factor, swapped derivative matrices) each fail the pin."""
import numpy as np
import pytest

import synth
from oracle.assemble import OracleMesh, assemble
from oracle.matfree import MatFree


def omesh(msh, N):
    return OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)


CASES = [(N, bc, lam, kap) for N in range(1, 9)
         for (bc, lam, kap) in (("dirichlet", 0.0, False), ("mixed", 100.0, False),
                                ("neumann", 3.5, True), ("mixed", 1.0, True))]


@pytest.mark.parametrize("N,bc,lam,use_kappa", CASES)
def test_matrix_free_equals_assembled(N, bc, lam, use_kappa):
    msh = synth.permuted(synth.square_mesh(4, jitter=0.2, seed=N, bc=bc), seed=100 + N)
    kap = synth.kappa_draw(msh.K, seed=N) if use_kappa else None
    m = omesh(msh, N)
    ctau = float((N + 1) ** 2)
    x = synth.nodal_normal(msh.K, m.Np, seed=N)
    yo = assemble(m, lam, ctau, kappa=kap) @ x
    mf = MatFree(m)
    y = mf.apply(lam, ctau, x, kappa=kap)
    assert np.linalg.norm(y - yo) <= 1e-13 * np.linalg.norm(yo)
    # rows of a subset of elements (the sampled-row form)
    sel = np.array([0, 5, msh.K - 1])
    ys = mf.apply(lam, ctau, x, kappa=kap, elems=sel).reshape(sel.size, m.Np)
    assert np.abs(ys - yo.reshape(msh.K, m.Np)[sel]).max() <= 1e-13 * np.abs(yo).max()


def test_lift_is_inverse_mass_times_face_mass():
    """M LIFT restricted to face f's columns is the face mass on that face,
    and LIFT applied to a constant face trace integrates it: 1^T M LIFT g =
    integral of g along the face (length 2 in the face parameter)."""
    from oracle.refelem import RefTriangle
    for N in (1, 3, 6):
        ref = RefTriangle(N)
        L = ref.lift()
        ML = ref.mass() @ L
        for f in range(3):
            cols = ML[:, f * ref.Nfp:(f + 1) * ref.Nfp]
            assert np.allclose(np.ones(ref.Np) @ cols @ np.ones(ref.Nfp), 2.0, atol=1e-13)
            # rows of nodes off face f vanish: the trace of their basis is 0
            off = np.setdiff1d(np.arange(ref.Np), ref.Fmask[f])
            assert np.abs(cols[off]).max() <= 1e-13


@pytest.mark.parametrize("mistake", ["no_neighbour", "normal_swap", "fscale", "deriv_swap"])
def test_planted_mistakes_fail_the_pin(mistake):
    N = 3
    msh = synth.permuted(synth.square_mesh(4, jitter=0.2, seed=2, bc="mixed"), seed=3)
    m = omesh(msh, N)
    x = synth.nodal_normal(msh.K, m.Np, seed=4)
    yo = assemble(m, 2.0, 16.0) @ x
    mf = MatFree(m)
    if mistake == "no_neighbour":
        mf.vmapP = mf.vmapM.copy()
    elif mistake == "normal_swap":
        mf.nx, mf.ny = mf.ny.copy(), mf.nx.copy()
    elif mistake == "fscale":
        mf.fscale = 1.0 / mf.fscale
    else:
        mf.Dr, mf.Ds = mf.Ds, mf.Dr
    y = mf.apply(2.0, 16.0, x)
    assert np.linalg.norm(y - yo) > 1e-6 * np.linalg.norm(yo)
