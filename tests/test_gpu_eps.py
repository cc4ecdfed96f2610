"""GPU parity with a per-cell relative permittivity eps (the block benchmark of Sec. 4.1:
a centre square of refractive index 1.516 in air, eps = n^2 in the mass term), against
the oracle on the same inputs: matrices, FP64 and FP32-refinement solutions, the DDM fixed
point, and the block-preconditioned GMRES iteration counts over the benchmark's w sweep.

Each test prints its case before touching the GPU.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads
from oracle import gmres, system
from tests._gpu_helpers import csr, ddm_fp64, ddm_mixed, problem, rel, spec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def thm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2105_11993_amd as t
    return t


@pytest.mark.parametrize("d", [spec(2, 6, 1, 7.0), spec(2, 5, 2, 5.0), spec(3, 3, 1, 4.0)],
                         ids=lambda c: f"d{c['dim']}m{c['n'][0]}p{c['p']}")
def test_random_eps_matches_oracle(thm, d):
    rng = np.random.default_rng(60)
    nc = d["n"][0] ** d["dim"]
    d = dict(d, mu=rng.uniform(1.0, 2.0, nc), eps=rng.uniform(1.0, 3.0, nc))
    print("case", d["dim"], d["n"][0], d["p"], flush=True)
    S = thm.thm_assemble(d)
    so = system.assemble(problem(d))
    (kr, kc, kv), _ = thm.thm_export_matrices(S)
    assert np.abs(csr((kr, kc, kv), S.n) - so.K).max() <= 1e-13 * np.abs(so.K).max()
    el = thm.thm_export_elements(S, 0, 3, so.Mhat.shape[0])
    for c in range(3):
        ref = so.Ahat / so.mu[c] - d["omega"] ** 2 * d["eps"][c] * so.Mhat
        assert np.abs(el[c] - ref).max() <= 1e-13 * np.abs(ref).max()
    Eo = system.solve_lu(so)
    (E,), (st,) = thm.thm_gmres_solve([S], thm.default_opts(rtol=1e-13))
    assert st["status"] == 0 and rel(E.cpu().numpy(), Eo) <= 1e-10
    (E3,), (st3,) = thm.thm_gmres_solve([S], thm.default_opts(rtol=1e-11, precision=thm.THM_FP32_IR))
    assert st3["status"] == 0 and rel(E3.cpu().numpy(), Eo) <= 1e-8


@pytest.mark.parametrize("parts", [(2, 2, 1), (4, 2, 1)])
def test_block_benchmark_ddm(thm, parts):
    """DDM on the block benchmark (eps cut per subdomain with its cells) reaches the global
    LU solution, in FP64 and FP32 + refinement."""
    d = dict(workloads.block(m=16, omega=10.0), subdomains=parts)
    print("case block ddm", parts, flush=True)
    S = thm.thm_assemble(d)
    Eg = system.solve_lu(system.assemble(problem(d)))
    E, st = ddm_fp64(thm, S)
    assert st["rel_residual"] <= 1e-12 and rel(E, Eg) <= 1e-10
    E3, st3 = ddm_mixed(thm, S)
    assert st3["status"] == 0 and rel(E3, Eg) <= 1e-8


def test_block_benchmark_sweep_iterations_match_oracle(thm):
    """Block-preconditioned GMRES(50) to 1e-8 over w in {5, 10, 20, 40, 80} on a 24^2 block
    benchmark: the GPU's iteration counts equal the oracle's GMRES with the same exact
    preconditioner diag(K, K)^{-1} (LU), up to two steps of rounding."""
    print("case block sweep 24", flush=True)
    for w in workloads.BLOCK_OMEGAS:
        d = workloads.block(m=24, omega=w)
        S = thm.thm_assemble(d)
        (_,), (st,) = thm.thm_gmres_solve([S], thm.default_opts(rtol=1e-8, restart=50))
        so = system.assemble(problem(d))
        A = so.S[so.F][:, so.F]
        lu = spla.splu(so.K[so.F][:, so.F].tocsc())
        prec = lambda v: lu.solve(np.ascontiguousarray(v.real)) + 1j * lu.solve(np.ascontiguousarray(v.imag))
        _, it, _ = gmres.gmres(lambda v: A @ v, so.rhs_free(), prec, rtol=1e-8, restart=50)
        print(f"  w={w}: gpu {st['iters']} oracle {it}", flush=True)
        assert st["status"] == 0
        assert abs(st["iters"] - it) <= 2


def test_adjoint_gradient_with_eps(thm):
    """dJ/dmu on the block benchmark (eps in the mass term, random mu): the adjoint kernel's
    gradient equals the oracle's exact discrete gradient and central differences."""
    from oracle import adjoint
    d = workloads.block(m=16, omega=12.0)
    d = dict(d, mu=np.random.default_rng(61).uniform(1.0, 2.0, 256))
    print("case block adjoint 16", flush=True)
    S = thm.thm_assemble(d)
    opts = thm.default_opts(rtol=1e-13)
    (E,), _ = thm.thm_gmres_solve([S], opts)
    lo, hi = (0.6, 0.6, 0.0), (0.9, 0.9, 1.0)
    g, J = thm.thm_adjoint_grad(S, E, lo, hi, opts)
    so = system.assemble(problem(d))
    Eo = system.solve_lu(so)
    MT = adjoint.target_mass(so, lo, hi)
    go, _ = adjoint.gradient(so, Eo, MT)
    assert abs(J - adjoint.objective(so, Eo, MT)) <= 1e-10 * abs(J)
    assert rel(g.cpu().numpy(), go) <= 1e-8
    cells = workloads.fd_cells(so.mesh.n_cells, 6)
    fd = adjoint.fd_gradient(problem(d), cells, lo, hi)
    gc = g.cpu().numpy()[cells]
    assert (np.abs(gc - fd) / np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max())).max() <= 1e-6
