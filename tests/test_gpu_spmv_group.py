"""The grouped SELL-64 product of a batch (systems with the same K read it once per
product, each applies its own C): on a homogeneous partition the subdomains off the x = 0
side form one group, and the DDM solution with the grouped product -- also in the form whose
Arnoldi steps read the member-interleaved copy that the preconditioner writes -- is bitwise
the one with the per-system SELL-64 product (the sums run in the same order) and equals the
global LU solution; on a partition with random mu every subdomain is its own group and the result
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
    E, st = thm.thm_ddm_solve(S, o, allow_not_converged=True)
    return E.cpu().numpy(), st


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32ir"])
def test_grouped_product_is_bitwise_sell_on_homogeneous_partition(thm, fp32):
    d = dict(workloads.c2(32))
    print("case c2-32 grouped spmv", "fp32ir" if fp32 else "fp64", flush=True)
    S = thm.thm_assemble(d)
    from tests._gpu_helpers import FP64_TIGHT, MIXED_TIGHT
    o = thm.default_opts(restart=80, **(dict(MIXED_TIGHT, precision=thm.THM_FP32_IR) if fp32 else FP64_TIGHT))
    thm.thm_ddm_solve(S, o, allow_not_converged=True)  # builds the batched subdomain context
    groups = S.fresh_info()["ddm_spmv_groups"]
    # the 4 subdomains on x = 0 carry Dirichlet rows, the other 12 share one K
    assert groups == 2
    E19, st19 = _solve_pinned(thm, S, thm.THM_SPMV_SELL, o)
    E20, st20 = _solve_pinned(thm, S, thm.THM_SPMV_SELL_GROUP, o)
    assert S.fresh_info()["ddm_spmv_variant"] == thm.THM_SPMV_SELL_GROUP
    # the Arnoldi steps with the preconditioner writing the member-interleaved copy
    E29, st29 = _solve_pinned(thm, S, thm.THM_SPMV_SELL_GROUP_IL, o)
    assert S.fresh_info()["ddm_spmv_variant"] == thm.THM_SPMV_SELL_GROUP_IL
    assert st19["rel_residual"] <= (1e-10 if fp32 else 1e-12) and st20["rel_residual"] == st19["rel_residual"]
    assert st19["iters"] == st20["iters"] and st19["outer_iters"] == st20["outer_iters"]
    assert st29["iters"] == st20["iters"] and st29["rel_residual"] == st20["rel_residual"]
    assert np.array_equal(E19, E20) and np.array_equal(E20, E29)
    Eg = system.solve_lu(system.assemble(problem(d)))
    assert rel(E20, Eg) <= (1e-8 if fp32 else 1e-10)


def test_grouped_product_with_distinct_subdomains(thm):
    rng = np.random.default_rng(70)
    d = spec(2, 12, 2, 8.0, mu=rng.uniform(1, 2, 144), subdomains=(3, 2, 1),
             inc_dir=(np.cos(0.3), np.sin(0.3), 0.0), inc_pol=(-np.sin(0.3), np.cos(0.3), 0.0))
    print("case random-mu 3x2 grouped spmv", flush=True)
    S = thm.thm_assemble(d)
    from tests._gpu_helpers import FP64_TIGHT
    o = thm.default_opts(**FP64_TIGHT)
    thm.thm_ddm_solve(S, o, allow_not_converged=True)
    assert S.fresh_info()["ddm_spmv_groups"] == 6
    E, st = _solve_pinned(thm, S, thm.THM_SPMV_SELL_GROUP, o)
    assert st["rel_residual"] <= 1e-12
    Eg = system.solve_lu(system.assemble(problem(d)))
    assert rel(E, Eg) <= 1e-10


def test_batched_spmv_timing_counts_each_distinct_k_once(thm):
    """thm_time_spmv_batch needs the DDM's subdomain batch; its algorithmic bytes are the
    same for every variant: the two distinct K of the homogeneous 4x4 partition once each,
    and per subdomain its C, row pointers, x read once and y written once.  The counts are
    the stored (structural) patterns, taken from the oracle's subdomain meshes: K has one
    entry per pair of DoFs that share a cell, and C (2D, degree p) p + 1 entries in each
    row it touches, since an edge's trace DoFs couple only to each other.  The oracle's
    own matrices drop the entries that Legendre orthogonality makes exactly zero."""
    import scipy.sparse as sps
    from oracle import ddm
    d = dict(workloads.c2(32))
    print("case c2-32 batched spmv timing", flush=True)
    S = thm.thm_assemble(d)
    with pytest.raises(thm.ThmError):
        thm.thm_time_spmv_batch(S)
    thm.thm_ddm_solve(S, thm.default_opts(rtol=1e-8, inner_rtol=1e-10))
    subs = ddm.DDM(problem(d)).subs

    def k_pattern(s):
        T = s.mesh.table()
        r = np.repeat(T, T.shape[1], axis=1).ravel()
        c = np.tile(T, (1, T.shape[1])).ravel()
        return sps.coo_matrix((np.ones(r.size), (r, c)), shape=(s.n, s.n)).tocsr().nnz

    def c_pattern(s):
        return (d["p"] + 1) * int((np.diff(s.C.tocsr().indptr) > 0).sum())

    nk = {k_pattern(s) for s in subs}
    assert len(nk) == 1
    nk = nk.pop()
    assert nk > subs[0].K.nnz  # the orthogonality zeros the oracle's sparse sums drop
    for prec, w in ((thm.THM_FP64, 8), (thm.THM_FP32_IR, 4)):
        ref = 2 * ((w + 4) * nk + 4 * (subs[0].n + 1))
        ref += sum((w + 4) * c_pattern(s) + 4 * (s.n + 1) + 4 * s.n * w for s in subs)
        for v in (thm.THM_SPMV_SELL, thm.THM_SPMV_SELL_GROUP, thm.THM_SPMV_SELL_GROUP_IL):
            ms, by = thm.thm_time_spmv_batch(S, prec, v, reps=3)
            print(f"  prec {prec} variant {v}: {ms * 1e3:.1f} us, {by / 1e6:.3f} MB (oracle sizes {ref / 1e6:.3f})",
                  flush=True)
            assert ms > 0.0
            assert by == pytest.approx(ref, rel=1e-12)
    with pytest.raises(thm.ThmError):
        thm.thm_time_spmv_batch(S, thm.THM_FP64, 17)
