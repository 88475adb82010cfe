"""Host-side checks of the C ABI (no GPU work): the library loads, exports
every function include/pmc.h declares, and rejects bad arguments before
touching a device."""
import ctypes as C
import os
import re

import pytest

from paper_1409_8336_amd import pmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "pmc.h")).read()
    return sorted(set(re.findall(r"^\s*(?:pmc_status|const char\*)\s+(pmc_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pmc.LIB_PATH):
        from paper_1409_8336_amd import _build
        _build.build()
    return pmc.lib()


def test_header_declares_the_binding_names():
    assert _declared() == sorted(pmc.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_default_params_and_version(lib):
    p = pmc.pmc_default_params()
    assert p.f_mcs == 1.07 and p.s_min_cm == 1e-4 and p.k_batches == 10 and p.flags == 0
    assert lib.pmc_default_params(None) == pmc.PMC_ERR_ARG
    assert pmc.pmc_version().startswith("pmc")


def test_create_rejects_bad_params_before_device(lib):
    h = C.c_void_p()
    assert lib.pmc_create(None, 0, None) == pmc.PMC_ERR_ARG
    for bad in (dict(k_batches=1), dict(k_batches=65), dict(block_threads=100),
                dict(s_min_cm=0.0), dict(flags=64)):
        p = pmc.pmc_default_params(**bad)
        assert lib.pmc_create(C.byref(h), 0, C.byref(p)) == pmc.PMC_ERR_ARG
        assert pmc.pmc_last_error(None) != ""


def test_null_context_is_an_argument_error(lib):
    assert lib.pmc_destroy(None) == pmc.PMC_OK
    assert lib.pmc_load_physics(None, None) == pmc.PMC_ERR_ARG
    assert lib.pmc_run_spots(None, None, 0, 0, 0, None, None, None) == pmc.PMC_ERR_ARG
    assert lib.pmc_inspect_tables(None, None, None, None, None, None) == pmc.PMC_ERR_ARG
