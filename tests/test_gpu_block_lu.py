"""The block-LU form of the factorised K^{-1} (chosen for thick layers, forced here on small
problems with THM_FACTOR_FORM=lu) against the oracle: the preconditioner inverts the
Dirichlet-modified K (eq. (11)) to the same bar as the cyclic-reduction form and agrees with
it, FP32 stays within its rounding, and a DDM solve whose subdomain factors are block LU
matches the oracle's global LU solution.

Each test prints its case before touching the GPU.
"""
import numpy as np
import pytest

import workloads
from oracle import system
from tests._gpu_helpers import FP64_TIGHT, dirichletized, problem, rel, spec

pytestmark = pytest.mark.gpu

CASES = [spec(2, 6, 1, 7.0), spec(2, 5, 2, 9.0), spec(3, 3, 1, 5.0), spec(3, 4, 0, 6.0)]


def _ids(c):
    return f"d{c['dim']}m{c['n'][0]}p{c['p']}"


@pytest.fixture(scope="module")
def thm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2105_11993_amd as t
    return t


def _precond(thm, d, form, x, monkeypatch, precision=None):
    import torch
    monkeypatch.setenv("THM_FACTOR_FORM", form)
    S = thm.thm_assemble(d)
    xt = torch.from_numpy(x).cuda()
    if precision is None:
        return thm.thm_apply_precond(S, xt).cpu().numpy()
    return thm.thm_apply_precond(S, xt, precision=precision).cpu().numpy()


@pytest.mark.parametrize("d", CASES, ids=_ids)
def test_block_lu_inverts_k_like_cyclic_reduction(thm, d, monkeypatch):
    rng = np.random.default_rng(81)
    m = d["n"][0]
    d = dict(d, mu=rng.uniform(1.0, 2.0, m ** d["dim"]))
    print("case block lu", _ids(d), flush=True)
    so = system.assemble(problem(d))
    K = dirichletized(so)[0].real
    x = rng.standard_normal(so.n) + 1j * rng.standard_normal(so.n)
    z_lu = _precond(thm, d, "lu", x, monkeypatch)
    z_bcr = _precond(thm, d, "bcr", x, monkeypatch)
    assert rel(K @ z_lu, x) <= 1e-10
    assert rel(z_lu, z_bcr) <= 1e-10
    z32 = _precond(thm, d, "lu", x, monkeypatch, precision=thm.THM_FP32_IR)
    assert rel(z32, z_lu) <= 1e-3


def test_ddm_with_block_lu_factors_matches_oracle(thm, monkeypatch):
    d = workloads.c3(m=8)
    print("case block lu ddm c3-8", flush=True)
    monkeypatch.setenv("THM_FACTOR_FORM", "lu")
    S = thm.thm_assemble(d)
    # the outer iteration stagnates near 3e-13 on this case, so it stops at 1e-12
    E, st = thm.thm_ddm_solve(S, thm.default_opts(**dict(FP64_TIGHT, rtol=1e-12)), allow_not_converged=True)
    Eo = system.solve_lu(system.assemble(problem(d)))
    print("block lu ddm:", st, rel(E.cpu().numpy(), Eo), flush=True)
    assert st["status"] == 0 and st["rel_residual"] <= 1e-12
    assert rel(E.cpu().numpy(), Eo) <= 1e-10


def test_invalid_factor_form_is_rejected(thm, monkeypatch):
    import torch
    print("case invalid factor form", flush=True)
    monkeypatch.setenv("THM_FACTOR_FORM", "dense")
    S = thm.thm_assemble(spec(2, 3, 0, 4.0))
    with pytest.raises(thm.ThmError):
        thm.thm_apply_precond(S, torch.zeros(S.n, dtype=torch.complex128, device="cuda"))


SMALLEST = [spec(2, 1, p, 3.0) for p in (0, 1, 2, 3)] + [spec(3, 1, p, 2.0) for p in (0, 1)]


@pytest.mark.parametrize("d", SMALLEST, ids=_ids)
def test_block_lu_on_smallest_meshes(thm, d, monkeypatch):
    """One-cell meshes (two layers): the block-LU factor inverts K, the complete inverse built on
    it inverts K + iC, and the allocation-free apply gives the same bits as the allocating one."""
    import torch
    rng = np.random.default_rng(82)
    d = dict(d, mu=rng.uniform(1.0, 2.0, d["n"][0] ** d["dim"]))
    print("case block lu smallest", _ids(d), flush=True)
    monkeypatch.setenv("THM_FACTOR_FORM", "lu")
    S = thm.thm_assemble(d)
    so = system.assemble(problem(d))
    Sd = dirichletized(so)[0]
    x = rng.standard_normal(S.n) + 1j * rng.standard_normal(S.n)
    xt = torch.from_numpy(x).cuda()

    def eta(A, z):
        an = abs(A).sum(axis=1).max()
        return np.linalg.norm(A @ z - x, np.inf) / (an * np.linalg.norm(z, np.inf) + np.linalg.norm(x, np.inf))

    z = thm.thm_apply_precond(S, xt)
    assert eta(Sd.real, z.cpu().numpy()) <= 1e-12
    assert eta(Sd, thm.thm_apply_precond_full(S, xt).cpu().numpy()) <= 1e-12
    y = torch.full_like(xt, complex(float("nan"), float("nan")))
    thm.thm_apply_precond_noalloc(S, xt, y)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), z.cpu().numpy())
