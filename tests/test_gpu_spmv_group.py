"""The grouped SELL-64 product of a batch (systems with the same K read it once per
product, each applies its own C): on a homogeneous partition the subdomains off the x = 0
side form one group, and the DDM solution with the grouped product is bitwise the one with
the per-system SELL-64 product (the sums run in the same order) and equals the global LU
solution; on a partition with random mu every subdomain is its own group and the result
still equals the oracle's.  The single-system form is covered with every other variant in
test_every_spmv_variant_matches_oracle.

Each test prints its case before touching the GPU.
"""
import numpy as np
import pytest

import workloads
from oracle import system
from tests._gpu_helpers import problem, rel, spec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def thm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2105_11993_amd as t
    return t


def _solve_pinned(thm, S, variant, o):
    for p in (thm.THM_FP64, thm.THM_FP32_IR):
        thm.thm_set_spmv_variant(S, p, variant)
    E, st = thm.thm_ddm_solve(S, o)
    return E.cpu().numpy(), st


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32ir"])
def test_grouped_product_is_bitwise_sell_on_homogeneous_partition(thm, fp32):
    d = dict(workloads.c2(32))
    print("case c2-32 grouped spmv", "fp32ir" if fp32 else "fp64", flush=True)
    S = thm.thm_assemble(d)
    o = thm.default_opts(rtol=1e-11, inner_rtol=1e-12, restart=80,
                         precision=thm.THM_FP32_IR if fp32 else thm.THM_FP64)
    thm.thm_ddm_solve(S, o)  # builds the batched subdomain context
    groups = S.fresh_info()["ddm_spmv_groups"]
    # the 4 subdomains on x = 0 carry Dirichlet rows, the other 12 share one K
    assert groups == 2
    E19, st19 = _solve_pinned(thm, S, thm.THM_SPMV_SELL, o)
    E20, st20 = _solve_pinned(thm, S, thm.THM_SPMV_SELL_GROUP, o)
    assert S.fresh_info()["ddm_spmv_variant"] == thm.THM_SPMV_SELL_GROUP
    assert st19["status"] == 0 and st20["status"] == 0
    assert st19["iters"] == st20["iters"] and st19["outer_iters"] == st20["outer_iters"]
    assert np.array_equal(E19, E20)
    Eg = system.solve_lu(system.assemble(problem(d)))
    assert rel(E20, Eg) <= (1e-8 if fp32 else 1e-9)


def test_grouped_product_with_distinct_subdomains(thm):
    rng = np.random.default_rng(70)
    d = spec(2, 12, 2, 8.0, mu=rng.uniform(1, 2, 144), subdomains=(3, 2, 1),
             inc_dir=(np.cos(0.3), np.sin(0.3), 0.0), inc_pol=(-np.sin(0.3), np.cos(0.3), 0.0))
    print("case random-mu 3x2 grouped spmv", flush=True)
    S = thm.thm_assemble(d)
    o = thm.default_opts(rtol=1e-11, inner_rtol=1e-13)
    thm.thm_ddm_solve(S, o)
    assert S.fresh_info()["ddm_spmv_groups"] == 6
    E, st = _solve_pinned(thm, S, thm.THM_SPMV_SELL_GROUP, o)
    assert st["status"] == 0
    Eg = system.solve_lu(system.assemble(problem(d)))
    assert rel(E, Eg) <= 1e-9
