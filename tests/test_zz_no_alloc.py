"""ipdg_pcg_solve_noalloc (the solve that allocates no device memory) against
ipdg_pcg_solve, through the C ABI: two calls in a row, the second on a
smaller mesh, for the identity, Jacobi and block inverse-mass
preconditioners.  Both run the same kernels on the same data, so iteration
counts agree exactly and the solutions to 1e-12; the true residual of each
solution under the oracle's assembled operator meets the tolerance.  Device
memory in use does not change across the allocation-free calls once the
stream has run each problem's kernels once (the HIP runtime reserves a
queue's private-segment memory at the first launch of a kernel that spills
registers; that reservation is the runtime's, not the library's)."""
import numpy as np
import pytest

import synth
from oracle.assemble import OracleMesh, assemble, mass_apply

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1801_00246_amd")

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def case(n, N, lam, seed):
    msh = synth.square_mesh(n, jitter=0.2, seed=seed, bc="mixed")
    m = OracleMesh(msh.VX, msh.VY, msh.EToV, msh.EToB, N)
    ctau = float((N + 1) ** 2)
    A = assemble(m, lam, ctau)
    b = mass_apply(m, synth.nodal_normal(msh.K, m.Np, seed=seed + 1))
    return dict(msh=msh, N=N, lam=lam, A=A, b=b, ctau=ctau)


@pytest.mark.parametrize("pc", ["none", "jacobi", "block_mass"])
def test_noalloc_solve_matches_pcg_solve(pc):
    pcv = {"none": P.PC_NONE, "jacobi": P.PC_JACOBI, "block_mass": P.PC_BLOCK_MASS}[pc]
    o = P.default_opts(pc=pcv)
    # the larger problem first, then a smaller one (the scratch keeps the
    # previous call's contents)
    cases = [case(26, 5, 40.0, 3), case(11, 3, 2.0, 7)]
    for c in cases:
        c["g"] = P.Mesh.from_synth(c["N"], c["msh"])
        c["bd"] = dev(c["b"])
        c["x"] = torch.zeros_like(c["bd"])
        c["x_ref"], c["info_ref"], c["st_ref"] = c["g"].pcg(c["bd"], lam=c["lam"], tau=c["ctau"],
                                                           tol=1e-9, opts=o)
    # warm-up of the stream (see the module docstring)
    for c in cases:
        xw = torch.zeros_like(c["bd"])
        c["g"].pcg_noalloc(c["bd"], xw, lam=c["lam"], tau=c["ctau"], tol=1e-9, opts=o)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for c in cases:
        print(f"noalloc {pc}: N={c['N']} K={c['msh'].K}", flush=True)
        c["info"], c["st"] = c["g"].pcg_noalloc(c["bd"], c["x"], lam=c["lam"], tau=c["ctau"], tol=1e-9,
                                                opts=o)
        torch.cuda.synchronize()
        print(f"  free device memory changed by {(torch.cuda.mem_get_info()[0] - free0) / 2**20:.1f} MiB",
              flush=True)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    for c in cases:
        xh, xr = host(c["x"]), host(c["x_ref"])
        rel = np.linalg.norm(xh - xr) / np.linalg.norm(xr)
        rr = np.linalg.norm(c["b"] - c["A"] @ xh) / np.linalg.norm(c["b"])
        print(f"  iters {c['info']['iters']} (pcg_solve {c['info_ref']['iters']}), rel diff {rel:.2e}, "
              f"true relres {rr:.2e}")
        assert c["st"] == c["st_ref"] == 0
        assert c["info"]["iters"] == c["info_ref"]["iters"]
        assert rel <= 1e-12
        assert rr <= 1e-9
        c["g"].close()


def test_noalloc_rejects_what_it_cannot_do():
    big = P.Mesh.from_synth(3, synth.square_mesh(256))      # K*Np = 1,310,720 > 2^20
    b = torch.ones(big.ndof, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(P.IpdgError) as e:
        big.pcg_noalloc(b, x, opts=P.default_opts(pc=P.PC_JACOBI))
    assert e.value.status == -1 and "limit" in str(e.value)
    small = P.Mesh.from_synth(2, synth.square_mesh(6))
    b = torch.ones(small.ndof, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    for bad in (dict(pc=P.PC_PMG), dict(prec=P.PREC_MIXED), dict(reliable_drop=1e-3)):
        with pytest.raises(P.IpdgError) as e:
            small.pcg_noalloc(b, x, opts=P.default_opts(**bad))
        assert e.value.status == -5
    # a zero right-hand side gives x = 0 without iterating
    x.fill_(3.0)
    info, st = small.pcg_noalloc(torch.zeros_like(b), x, opts=P.default_opts(pc=P.PC_JACOBI))
    assert st == 0 and info["iters"] == 0 and float(x.abs().max()) == 0.0
