"""GPU parity of the complete-inverse preconditioner (K + iC)^{-1} (THM_PREC_FULL).

Sec. 3.2 names the complete inverse of the block system as the alternative to the
block-diagonal preconditioner. The library applies it exactly through K^{-1} and a
boundary correction (Woodbury). Each result is checked against the oracle's Dirichlet-
modified complex system on the same input: the residual of the inverse, the GMRES
iteration count it gives (one step in exact arithmetic), the solution, and the DDM fixed
point. Each test prints its case before touching the GPU.
"""
import numpy as np
import pytest

from oracle import system
from tests._gpu_helpers import ddm_fp64, ddm_mixed, dirichletized, problem, rel, spec

pytestmark = pytest.mark.gpu

CASES = [spec(2, 4, 0, 6.0), spec(2, 5, 1, 7.0), spec(2, 4, 2, 9.0), spec(3, 2, 0, 4.0), spec(3, 3, 1, 5.0)]


def _ids(c):
    return f"d{c['dim']}m{c['n'][0]}p{c['p']}"


def _randomize(d, seed):
    rng = np.random.default_rng(seed)
    m = d["n"][0]
    d = dict(d)
    d["mu"] = rng.uniform(1.0, 2.0, m ** d["dim"])
    th = 0.29
    d["inc_dir"] = (np.cos(th), np.sin(th), 0.1 if d["dim"] == 3 else 0.0)
    d["inc_pol"] = (-np.sin(th), np.cos(th), 0.3j if d["dim"] == 3 else 0.0)
    return d


@pytest.fixture(scope="module")
def thm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2105_11993_amd as t
    return t


def _backward_error(A, z, x):
    an = abs(A).sum(axis=1).max()
    return np.linalg.norm(A @ z - x, np.inf) / (an * np.linalg.norm(z, np.inf) + np.linalg.norm(x, np.inf))


@pytest.mark.parametrize("d", CASES, ids=_ids)
def test_full_preconditioner_inverts_the_system(thm, d):
    """z = (K + iC)^{-1} x to FP64 rounding (and (K - iC)^{-1} for the transpose); the FP32
    form agrees to FP32 accuracy; repeated application is bitwise reproducible."""
    import torch
    d = _randomize(d, 5)
    print("case", _ids(d), flush=True)
    S = thm.thm_assemble(d)
    so = system.assemble(problem(d))
    Sd, _ = dirichletized(so)
    rng = np.random.default_rng(6)
    x = rng.standard_normal(S.n) + 1j * rng.standard_normal(S.n)
    xt = torch.from_numpy(x).cuda()
    for tr in (False, True):
        A = Sd.conj() if tr else Sd
        z = thm.thm_apply_precond_full(S, xt, transpose=tr).cpu().numpy()
        # normwise backward error at FP64 rounding; the relative residual is that error
        # times ||A|| ||z|| / ||x||, which reaches 1e2..1e4 on the degree-2 cases
        assert _backward_error(A, z, x) <= 1e-12
        assert rel(A @ z, x) <= 1e-9
        z2 = thm.thm_apply_precond_full(S, xt, transpose=tr).cpu().numpy()
        assert np.array_equal(z, z2)
        z32 = thm.thm_apply_precond_full(S, xt, transpose=tr, precision=thm.THM_FP32_IR).cpu().numpy()
        # FP32: unit roundoff 6e-8 times the growth of the explicit block inverses and of the
        # cancellation in z - K^{-1} P^T t, where both terms can exceed the result by orders
        # of magnitude (measured 2e-4 on d2m4p2); a wrong sign, index or boundary set gives
        # an O(1) error
        assert _backward_error(A, z32, x) <= 1e-3
    # differs from the block preconditioner wherever C acts
    zb = thm.thm_apply_precond(S, xt).cpu().numpy()
    zf = thm.thm_apply_precond_full(S, xt).cpu().numpy()
    assert rel(zb, zf) > 1e-6


def test_full_preconditioner_on_subdomain_shape(thm):
    """The 64 x 64, degree-2 square of one subdomain of the 4x4-split 256x256 square (576 boundary DoFs carry C): the
    correction inverts K + iC to FP64 rounding and to FP32 accuracy in FP32."""
    import torch
    d = _randomize(spec(2, 64, 2, 50.0), 42)
    print("case subdomain shape d2m64p2", flush=True)
    S = thm.thm_assemble(d)
    so = system.assemble(problem(d))
    Sd, _ = dirichletized(so)
    rng = np.random.default_rng(43)
    x = rng.standard_normal(S.n) + 1j * rng.standard_normal(S.n)
    xt = torch.from_numpy(x).cuda()
    z = thm.thm_apply_precond_full(S, xt).cpu().numpy()
    assert _backward_error(Sd, z, x) <= 1e-11
    z32 = thm.thm_apply_precond_full(S, xt, precision=thm.THM_FP32_IR).cpu().numpy()
    # FP32 rounding amplified by the explicit block inverses (as for the block form) and
    # by the cancellation in the correction; a wrong boundary set or sign leaves an O(1)
    # residual
    assert _backward_error(Sd, z32, x) <= 1e-3


@pytest.mark.parametrize("d", CASES[:3] + CASES[4:], ids=_ids)
def test_gmres_with_full_preconditioner(thm, d):
    """Right-preconditioned GMRES with the exact complete inverse stops after one or two
    steps and returns the LU solution (FP64, and FP32 + FP64 refinement)."""
    d = _randomize(d, 7)
    print("case", _ids(d), flush=True)
    S = thm.thm_assemble(d)
    so = system.assemble(problem(d))
    Eo = system.solve_lu(so)
    (E,), (st,) = thm.thm_gmres_solve([S], thm.default_opts(rtol=1e-12, precond=thm.THM_PREC_FULL))
    assert st["status"] == 0, st
    assert st["iters"] <= 2, st
    assert rel(E.cpu().numpy(), Eo) <= 1e-10
    (E3,), (st3,) = thm.thm_gmres_solve([S], thm.default_opts(rtol=1e-11, precond=thm.THM_PREC_FULL,
                                                               precision=thm.THM_FP32_IR))
    assert st3["status"] == 0, st3
    assert rel(E3.cpu().numpy(), Eo) <= 1e-8
    # GMRES-based refinement with the FP32 complete inverse as the preconditioner of FP64 GMRES
    (E4,), (st4,) = thm.thm_gmres_solve([S], thm.default_opts(rtol=1e-12, precond=thm.THM_PREC_FULL,
                                                               precision=thm.THM_FP32_IR, ir_mode=thm.THM_IR_GMRES))
    assert st4["status"] == 0 and st4["gmres_ir"] == 1 and st4["fp64_fallback"] == 0, st4
    assert rel(E4.cpu().numpy(), Eo) <= 1e-10
    # the block preconditioner needs many more steps on the same system
    (_,), (stb,) = thm.thm_gmres_solve([S], thm.default_opts(rtol=1e-12))
    assert stb["iters"] > st["iters"]


@pytest.mark.parametrize("case", [(2, 8, 1, (2, 2, 1), 6.0), (3, 4, 1, (2, 1, 1), 4.0)],
                         ids=lambda c: f"d{c[0]}m{c[1]}p{c[2]}s{c[3][0]}{c[3][1]}{c[3][2]}")
def test_ddm_with_full_preconditioner(thm, case):
    """The DDM fixed point with complete-inverse subdomain solves (batched, FP64 and FP32 +
    refinement) is the global LU solution; every subdomain solve takes at most two steps."""
    dim, m, p, parts, om = case
    print("case", case, flush=True)
    d = spec(dim, m, p, om, subdomains=parts)
    d = _randomize(d, 8)
    S = thm.thm_assemble(d)
    Eg = system.solve_lu(system.assemble(problem(d)))
    E, st = ddm_fp64(thm, S, precond=thm.THM_PREC_FULL, max_outer=200)
    assert st["rel_residual"] <= 1e-12, st
    assert rel(E, Eg) <= 1e-10
    # at the default tolerances every subdomain solve takes at most two steps (iters: the
    # largest inner iteration count of each outer application, summed)
    _, st = thm.thm_ddm_solve(S, thm.default_opts(precond=thm.THM_PREC_FULL))
    assert st["status"] == 0 and st["iters"] <= 2 * (st["outer_iters"] + 2), st
    E32, st32 = ddm_mixed(thm, S, precond=thm.THM_PREC_FULL, max_outer=200)
    assert st32["rel_residual"] <= 1e-10, st32
    assert rel(E32, Eg) <= 1e-8
