"""The allocation-free preconditioner apply (thm_apply_precond_noalloc) gives the same result
as thm_apply_precond on the same inputs, on consecutive calls that share the library's static
scratch array: a larger system, then a smaller one, then the larger one again (the second and
third calls find the previous call's contents in the array).  Both precisions."""
import numpy as np
import pytest

from tests._gpu_helpers import spec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def thm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2105_11993_amd as t
    return t


def _system(thm, d, seed):
    rng = np.random.default_rng(seed)
    d = dict(d)
    d["mu"] = rng.uniform(1.0, 2.0, int(np.prod(d["n"][:d["dim"]])))
    return thm.thm_assemble(d)


def _vec(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return torch.from_numpy(v).cuda()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_apply_equals_allocating_apply(thm, prec):
    import torch
    p = thm.THM_FP64 if prec == "fp64" else thm.THM_FP32_IR
    big = _system(thm, spec(2, 20, 2, 9.0), 11)
    small = _system(thm, spec(3, 3, 1, 5.0), 12)
    assert small.n < big.n
    # not prepared yet: rejected, nothing launched
    with pytest.raises(thm.ThmError) as e:
        thm.thm_apply_precond_noalloc(small, _vec(small.n, 0), _vec(small.n, 0), precision=p)
    assert e.value.code == -1
    for k, S in enumerate((big, small, big)):
        print(f"case noalloc {prec} call {k} n={S.n}", flush=True)
        x = _vec(S.n, 100 + k)
        ref = thm.thm_apply_precond(S, x, precision=p)
        y = torch.full_like(x, complex(float("nan"), float("nan")))
        thm.thm_apply_precond_noalloc(S, x, y, precision=p)
        torch.cuda.synchronize()
        a, b = y.cpu().numpy(), ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b), np.abs(a - b).max() / np.abs(b).max()
