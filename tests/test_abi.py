"""The C-ABI library loads and exports every entry point declared in include/thm.h (no GPU needed)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "thm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(thm_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_four_entry_points():
    names = declared()
    for n in ("thm_assemble", "thm_gmres_solve", "thm_ddm_solve", "thm_adjoint_grad"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2105_11993_amd as thm
    lib = ctypes.CDLL(thm.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(thm.EXPORTS) == declared()


def test_default_opts_and_error_string():
    import paper_2105_11993_amd as thm
    o = thm.default_opts()
    assert o.restart == 50 and o.rtol == 1e-8 and o.inner_rtol == 1e-10 and o.batched == 1
    assert isinstance(thm._lib.thm_last_error(), bytes)


def test_invalid_problem_is_rejected_without_gpu_work():
    import paper_2105_11993_amd as thm
    p, keep = thm.make_problem(dict(dim=4, n=(2, 2, 2), p=0, omega=1.0))
    h = ctypes.c_void_p()
    rc = thm._lib.thm_assemble(ctypes.byref(p), None, ctypes.byref(h))
    assert rc == -2 and h.value is None
    assert b"dim" in thm._lib.thm_last_error()
