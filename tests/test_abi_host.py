"""Host-side checks of the C ABI (no GPU work): the library loads, exports
every function include/pmc.h declares, and rejects bad arguments before
touching a device."""
import ctypes as C
import os
import re

import pytest

from paper_1409_8336_amd import pmc, unet

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="pmc.h"):
    text = open(os.path.join(ROOT, "include", header)).read()
    return sorted(set(re.findall(r"^\s*(?:pmc_status|const char\*)\s+(pmc_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pmc.LIB_PATH):
        from paper_1409_8336_amd import _build
        _build.build()
    return pmc.lib()


def test_header_declares_the_binding_names():
    assert _declared() == sorted(pmc.EXPORTS)
    assert _declared("pmc_unet.h") == sorted(unet.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in _declared() + _declared("pmc_unet.h"):
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
                dict(s_min_cm=0.0), dict(flags=32), dict(flags=64)):
        p = pmc.pmc_default_params(**bad)
        assert lib.pmc_create(C.byref(h), 0, C.byref(p)) == pmc.PMC_ERR_ARG
        assert pmc.pmc_last_error(None) != ""


def test_null_context_is_an_argument_error(lib):
    assert lib.pmc_destroy(None) == pmc.PMC_OK
    assert lib.pmc_load_physics(None, None) == pmc.PMC_ERR_ARG
    assert lib.pmc_run_spots(None, None, 0, 0, 0, None, None, None) == pmc.PMC_ERR_ARG
    assert lib.pmc_inspect_tables(None, None, None, None, None, None) == pmc.PMC_ERR_ARG
    assert lib.pmc_run_spots_let(None, None, 0, 0, 0, None, None, None, None) == pmc.PMC_ERR_ARG
    assert lib.pmc_run_spots_let_dev(None, None, 0, 0, 0, None, None, None, None, None) == pmc.PMC_ERR_ARG
    buf = (C.c_float * 16)()
    assert lib.pmc_vavilov_table(None, 20000) == pmc.PMC_ERR_ARG
    assert lib.pmc_vavilov_table(buf, 16) == pmc.PMC_ERR_ARG


def test_engine_vavilov_table_matches_oracle():
    """The engine's Vavilov quantile table (closed-form sine/cosine integrals,
    density inversion and running integral) against the oracle's (running
    integrals of the defining integrands, Gil-Pelaez inversion): two
    independent numerical routes to the same quantiles.  Both carry
    integration errors of about 1e-3 sigma; the bar is 5e-3 sigma for normal
    scores within 4.5 and 1e-2 sigma in the far tails."""
    import numpy as np
    from oracle import oracle as O
    eng = pmc.pmc_vavilov_table().astype(np.float64)
    ora = O.vavilov_table()
    z = np.arange(97) / 8.0 - 6.0
    core = np.abs(z) <= 4.5
    assert np.all(np.isfinite(eng)) and np.all(np.diff(eng, axis=-1) > 0)
    assert np.max(np.abs(eng - ora)[:, :, core]) < 5e-3
    assert np.max(np.abs(eng - ora)) < 1e-2


def test_denoiser_and_gamma_reject_bad_arguments(lib):
    L = unet.lib()
    u = C.c_void_p()
    assert L.pmc_unet_create(None, 0, 1, 8, 8, 8, 0) == pmc.PMC_ERR_ARG
    for shape in ((0, 8, 8, 8), (1, 12, 8, 8), (1, 8, 4, 8), (1, 8, 8, 9)):
        assert L.pmc_unet_create(C.byref(u), 0, *shape, 0) == pmc.PMC_ERR_ARG
    assert L.pmc_unet_destroy(None) == pmc.PMC_OK
    assert L.pmc_unet_forward(None, None, None, None, None) == pmc.PMC_ERR_ARG
    assert L.pmc_unet_adam_step(None, 1e-3, 1.0, None) == pmc.PMC_ERR_ARG
    assert L.pmc_unet_grad_norm(None, None, None) == pmc.PMC_ERR_ARG
    # channel counts must be multiples of 8
    assert L.pmc_nn_conv3d_forward(None, None, None, None, 1, 8, 8, 8, 8, 16, 0, None) == pmc.PMC_ERR_ARG
    one = C.c_void_p(1)
    assert L.pmc_nn_conv3d_forward(one, one, None, one, 1, 8, 8, 8, 12, 16, 0, None) == pmc.PMC_ERR_ARG
    rate, n = C.c_double(), C.c_int64()
    assert L.pmc_gamma_index(one, one, 4, 4, 4, 0.2, 0.2, 0.2, 0.02, 0.0, 0.1, 0.6, 0.05, None,
                             C.byref(rate), C.byref(n), None) == pmc.PMC_ERR_ARG
    assert L.pmc_gamma_index(one, one, 4, 4, 4, 0.2, 0.2, 0.2, 0.02, 0.2, 0.1, 10.0, 0.05, None,
                             C.byref(rate), C.byref(n), None) == pmc.PMC_ERR_ARG


def test_engine_moliere_table_matches_oracle():
    """The engine's Molière table (J0 densities on a v grid, running Simpson
    integrals) against the oracle's (J1 running integrals in closed form,
    Simpson in u): ln(v^2/q) within 5e-4 everywhere, i.e. the sampled angles
    within 0.025%."""
    import numpy as np
    from oracle import oracle as O
    eng = pmc.pmc_moliere_table().astype(np.float64)
    ora = O.moliere_table()
    assert np.all(np.isfinite(eng))
    assert np.max(np.abs(eng - ora)) < 5e-4
    buf = (C.c_float * 16)()
    assert pmc.lib().pmc_moliere_table(buf, 16) == pmc.PMC_ERR_ARG
