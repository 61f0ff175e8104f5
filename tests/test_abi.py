"""Host-side checks of the C-ABI library (no GPU work): it loads, exports
every entry point include/obem.h declares, reports the same physical
constants as the oracle, and rejects calls without a valid context."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "obem.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:obem_status|void|const char \*)\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    from paper_2110_09214_amd import binding

    lib = binding.load()
    names = _declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(binding.SYMBOLS)


def test_constants_match_oracle(orc):
    from paper_2110_09214_amd import binding

    a = binding.obem_constants()
    b = orc.constants()
    for k in a:
        assert a[k] == pytest.approx(b[k], rel=1e-15)


def test_null_context_is_rejected():
    from paper_2110_09214_amd import binding

    lib = binding.load()
    assert lib.field_eval(None, None, None, 0, None, None, None, None, 1, None, None, None, 0.0, 0, 0,
                          None, None, None, None) == -1
    assert lib.bem_solve_charges(None, None, None, None, 0, None) == -1
    assert lib.obem_create(None, 0, None) == -1
    assert lib.obem_last_error(None) == b"null context"


def test_create_fails_cleanly_without_gpu():
    import torch

    from paper_2110_09214_amd import binding

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = binding.load()
    h = C.c_void_p()
    assert lib.obem_create(C.byref(h), 0, None) != 0
    assert not h.value
