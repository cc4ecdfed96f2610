"""GPU edge cases against the oracle on the same inputs: single-cell meshes at every
supported degree (2D degree 0..3, 3D degree 0..1), one-cell subdomains, a batch mixing
the smallest and a ragged system, and the error paths for an empty batch, a partition that
does not divide the mesh, an unsupported degree and an unknown preconditioner.

Each test prints its case before touching the GPU.
"""
import numpy as np
import pytest

from oracle import system
from tests._gpu_helpers import csr, ddm_fp64, dirichletized, problem, rel, spec

pytestmark = pytest.mark.gpu

SMALL = [spec(2, 1, p, 3.0) for p in (0, 1, 2, 3)] + [spec(3, 1, p, 2.0) for p in (0, 1)]


def _ids(c):
    return f"d{c['dim']}m{c['n'][0]}p{c['p']}"


@pytest.fixture(scope="module")
def thm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2105_11993_amd as t
    return t


def _eta(A, z, x):
    an = abs(A).sum(axis=1).max()
    return np.linalg.norm(A @ z - x, np.inf) / (an * np.linalg.norm(z, np.inf) + np.linalg.norm(x, np.inf))


@pytest.mark.parametrize("d", SMALL, ids=_ids)
def test_smallest_meshes(thm, d):
    """Matrices, both preconditioners and the GMRES solution on the smallest meshes."""
    import torch
    rng = np.random.default_rng(50)
    d = dict(d, mu=rng.uniform(1.0, 2.0, d["n"][0] ** d["dim"]))
    print("case", _ids(d), flush=True)
    S = thm.thm_assemble(d)
    so = system.assemble(problem(d))
    assert S.n == so.n
    (kr, kc, kv), (cr, cc, cv) = thm.thm_export_matrices(S)
    assert np.abs(csr((kr, kc, kv), S.n) - so.K).max() <= 1e-13 * np.abs(so.K).max()
    assert np.abs(csr((cr, cc, cv), S.n) - so.C).max() <= 1e-13 * max(np.abs(so.C).max(), 1.0)
    Sd, _ = dirichletized(so)
    x = rng.standard_normal(S.n) + 1j * rng.standard_normal(S.n)
    xt = torch.from_numpy(x).cuda()
    z = thm.thm_apply_precond(S, xt).cpu().numpy()
    assert _eta(Sd.real, z, x) <= 1e-12
    zf = thm.thm_apply_precond_full(S, xt).cpu().numpy()
    assert _eta(Sd, zf, x) <= 1e-12
    Eo = system.solve_lu(so)
    (E,), (st,) = thm.thm_gmres_solve([S], thm.default_opts(rtol=1e-13))
    assert st["status"] == 0, st
    assert rel(E.cpu().numpy(), Eo) <= 1e-10
    (E3,), (st3,) = thm.thm_gmres_solve([S], thm.default_opts(rtol=1e-11, precision=thm.THM_FP32_IR))
    assert st3["status"] == 0, st3
    assert rel(E3.cpu().numpy(), Eo) <= 1e-8


def test_batch_of_smallest_and_ragged_systems(thm):
    """A batch mixing single-cell systems of every 2D degree with a 7x7 system (not a
    multiple of any tile) gives each system its own LU solution."""
    specs = [spec(2, 1, p, 3.0 + p) for p in (0, 1, 2, 3)] + [spec(2, 7, 1, 9.0)]
    print("case batch of smallest + ragged", flush=True)
    systems = [thm.thm_assemble(d) for d in specs]
    Es, sts = thm.thm_gmres_solve(systems, thm.default_opts(rtol=1e-13, restart=30))
    for d, E, st in zip(specs, Es, sts):
        assert st["status"] == 0, st
        assert rel(E.cpu().numpy(), system.solve_lu(system.assemble(problem(d)))) <= 1e-10


@pytest.mark.parametrize("case", [(2, 2, 1, (2, 2, 1), 5.0), (2, 4, 2, (4, 1, 1), 6.0), (3, 2, 1, (2, 2, 2), 3.0)],
                         ids=lambda c: f"d{c[0]}m{c[1]}p{c[2]}s{c[3][0]}{c[3][1]}{c[3][2]}")
def test_one_cell_subdomains(thm, case):
    """DDM with one-cell subdomains (2D 2x2, a 4x1 strip of 1-cell-wide subdomains, 3D 2x2x2)
    reaches the global LU solution."""
    dim, m, p, parts, om = case
    print("case", case, flush=True)
    d = spec(dim, m, p, om, subdomains=parts)
    S = thm.thm_assemble(d)
    Eg = system.solve_lu(system.assemble(problem(d)))
    E, st = ddm_fp64(thm, S)
    assert st["rel_residual"] <= 1e-12, st
    assert rel(E, Eg) <= 1e-10


def test_empty_batch_and_uneven_partition_are_rejected(thm):
    print("case error paths", flush=True)
    with pytest.raises(thm.ThmError) as e:
        thm.thm_gmres_solve([], thm.default_opts())
    assert e.value.code == -1
    with pytest.raises(thm.ThmError) as e:
        thm.thm_assemble(spec(2, 5, 1, 4.0, subdomains=(2, 1, 1)))
    assert e.value.code == -2
    for bad in (spec(3, 1, 2, 2.0), spec(2, 1, 4, 2.0)):
        with pytest.raises(thm.ThmError) as e:
            thm.thm_assemble(bad)
        assert e.value.code == -2
    # an unknown preconditioner kind is an invalid option
    S = thm.thm_assemble(spec(2, 2, 0, 3.0))
    with pytest.raises(thm.ThmError) as e:
        thm.thm_gmres_solve([S], thm.default_opts(precond=7))
    assert e.value.code == -1
