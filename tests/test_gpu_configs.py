"""GPU parity on the benchmark configurations (full size where the oracle is fast enough,
otherwise the same recipe at reduced size) against the oracle."""
import numpy as np
import pytest

import workloads
from oracle import adjoint, system
from tests._gpu_helpers import problem, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def thm():
    import torch
    assert torch.cuda.is_available()
    import paper_2105_11993_amd as t
    return t


def test_c5_adjoint_full_size(thm):
    """128^2 quads, p = 1, w = 30, mu from the Gaussian random field: forward solve and the
    adjoint gradient (16,384 parameters) against the oracle's LU solve and exact gradient."""
    d = workloads.c5()
    print("case c5 full", flush=True)
    S = thm.thm_assemble(d)
    opts = thm.default_opts(rtol=1e-13, restart=100)
    (E,), (st,) = thm.thm_gmres_solve([S], opts)
    lo, hi = workloads.C5_TARGET
    g, J = thm.thm_adjoint_grad(S, E, lo, hi, opts)
    so = system.assemble(problem(d))
    Eo = system.solve_lu(so)
    assert rel(E.cpu().numpy(), Eo) <= 1e-10
    MT = adjoint.target_mass(so, lo, hi)
    go, _ = adjoint.gradient(so, Eo, MT)
    assert abs(J - adjoint.objective(so, Eo, MT)) <= 1e-9 * abs(J)
    assert rel(g.cpu().numpy(), go) <= 1e-7
    # central differences of J with GPU solves on a few of the seeded cells
    import torch
    cells = workloads.fd_cells(so.mesh.n_cells)[:4]
    mu0 = np.asarray(d["mu"], dtype=np.float64)
    for c in cells:
        h = 1e-5 * mu0[c]
        Js = []
        for sgn in (1, -1):
            mu = mu0.copy()
            mu[c] += sgn * h
            thm.thm_system_set_mu(S, torch.from_numpy(mu))
            (Ec,), _ = thm.thm_gmres_solve([S], opts)
            _, Jc = thm.thm_adjoint_grad(S, Ec, lo, hi, opts)
            Js.append(Jc)
        fd = (Js[0] - Js[1]) / (2 * h)
        gc = g.cpu().numpy()[c]
        assert abs(gc - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(go).max()), (c, gc, fd)


def test_c4_uneven_batch_reduced(thm):
    """The 256-problem recipe (seed 4) at 1/4 mesh size, first 24 problems, one batched solve."""
    specs = workloads.c4(count=24, scale=4)
    print("case c4 reduced", flush=True)
    systems = [thm.thm_assemble(d) for d in specs]
    refs = [system.solve_lu(system.assemble(problem(d))) for d in specs]
    Es, sts = thm.thm_gmres_solve(systems, thm.default_opts(rtol=1e-13, restart=60))
    for E, st, Eo in zip(Es, sts, refs):
        assert st["status"] == 0
        assert rel(E.cpu().numpy(), Eo) <= 1e-10
    Es, sts = thm.thm_gmres_solve(systems, thm.default_opts(rtol=1e-11, restart=60, precision=thm.THM_FP32_IR))
    for E, Eo in zip(Es, refs):
        assert rel(E.cpu().numpy(), Eo) <= 1e-8


def test_c3_ddm_reduced(thm):
    """3D recipe (mu ~ U[1,2] per cell, seed 3, w = 20, 2x2x2 subdomains) on 8^3 hexes."""
    d = workloads.c3(m=8)
    print("case c3 reduced", flush=True)
    S = thm.thm_assemble(d)
    Eg = system.solve_lu(system.assemble(problem(d)))
    E, st = thm.thm_ddm_solve(S, thm.default_opts(rtol=1e-11, inner_rtol=1e-12, restart=80))
    assert st["rel_residual"] <= 1e-11
    assert rel(E.cpu().numpy(), Eg) <= 1e-9
    E, st = thm.thm_ddm_solve(S, thm.default_opts(rtol=1e-10, inner_rtol=1e-11, restart=80,
                                                  precision=thm.THM_FP32_IR))
    assert rel(E.cpu().numpy(), Eg) <= 1e-8


def test_c2_full_size_sampled(thm):
    """The benchmark configuration at full size (1.18M DoFs): the glued DDM field's global
    residual, recomputed on the CPU from the oracle's own assembled matrices, is below the
    solver tolerance; sampled DoFs on Gamma^inc equal the oracle's Dirichlet values."""
    d = workloads.c2()
    print("case c2 full", flush=True)
    S = thm.thm_assemble(d)
    E, st = thm.thm_ddm_solve(S, thm.default_opts(rtol=1e-8, inner_rtol=1e-10, restart=64,
                                                  precision=thm.THM_FP32_IR))
    assert st["status"] == 0
    so = system.assemble(problem(d))
    Eh = E.cpu().numpy()
    assert system.relative_residual(so, Eh) <= 1.5e-8
    assert rel(Eh[so.D], so.gD) <= 1e-13


def test_refinement_fallback_is_fp64_accurate(thm):
    """With no refinement steps allowed, every system is finished by FP64 GMRES from its
    iterate: FP64 accuracy, and the stats report the fallback."""
    from tests._gpu_helpers import spec
    d = spec(2, 12, 2, 12.0)
    print("case forced fp64 finish", flush=True)
    S = thm.thm_assemble(d)
    Eo = system.solve_lu(system.assemble(problem(d)))
    (E,), (st,) = thm.thm_gmres_solve([S], thm.default_opts(rtol=1e-13, restart=40, precision=thm.THM_FP32_IR,
                                                            max_refine=0))
    assert st["status"] == 0 and st["fp64_fallback"] == 1
    assert rel(E.cpu().numpy(), Eo) <= 1e-10


def test_c4_half_size_batch_reaches_tolerance_in_fp32_refinement(thm):
    """All 256 problems of the uneven batch (meshes halved) reach 1e-8 in the FP32 +
    refinement form; problems whose FP32 factor is too inaccurate (high w, near-resonant
    K) are detected by the refinement safeguard and finished in FP64."""
    specs = workloads.c4(256, scale=2)
    print("case c4 half size fp32", flush=True)
    systems = [thm.thm_assemble(d) for d in specs]
    Es, sts = thm.thm_gmres_solve(systems, thm.default_opts(rtol=1e-8, restart=64, precision=thm.THM_FP32_IR),
                                  allow_not_converged=True)
    bad = [(i, s["rel_residual"]) for i, s in enumerate(sts) if not (s["status"] == 0 and s["rel_residual"] <= 1e-8)]
    print("fp64 fallbacks:", sum(s["fp64_fallback"] for s in sts), flush=True)
    assert not bad, bad[:5]
