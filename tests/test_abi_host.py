"""Host-side checks of the C ABI (no GPU work): the library loads, exports
every function include/pmc.h declares, and rejects bad arguments before
touching a device."""
import ctypes as C
import os
import re

import numpy as np

import pytest

from paper_1409_8336_amd import pmc, unet

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="pmc.h"):
    text = open(os.path.join(ROOT, "include", header)).read()
    return sorted(set(re.findall(r"^\s*(?:pmc_status|const char\*|double)\s+(pmc_\w+)\s*\(", text, re.M)))


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
                dict(s_min_cm=0.0), dict(flags=32), dict(flags=128)):
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


def test_cascade_nucleus_matches_the_oracle(lib):
    """The engine's Woods-Saxon shells (Gauss-Legendre) against the oracle's
    (Simpson): shell radii, densities of both species and Fermi energies."""
    from oracle import oracle as O
    for el in range(1, 7):
        e = pmc.pmc_inc_nucleus(el)
        o = O.inc_nucleus(el)
        assert e["a"] == o["a"]
        np.testing.assert_allclose(e["r"], o["r"], rtol=1e-14, atol=0)
        assert abs(e["radius_ws"] - o["radius_ws"]) < 1e-13
        for k in ("rho_p", "rho_n", "tf_p", "tf_n"):
            np.testing.assert_allclose(e[k], o[k], rtol=1e-9, err_msg="element %d %s" % (el, k))
    assert lib.pmc_inc_nucleus(0, None, 78) == pmc.PMC_ERR_ARG
    assert lib.pmc_inc_nucleus(7, None, 78) == pmc.PMC_ERR_ARG


def test_evaporation_widths_match_the_oracle(lib):
    """The engine's closed-form level-density integral against the oracle's
    quadrature, with separation energies and barriers, over open and closed
    channels of light and heavy residuals."""
    from oracle import oracle as O
    rng = np.random.default_rng(5)
    cases = [(8, 17, 30.0), (22, 49, 120.0), (6, 13, 9.0), (20, 41, 2.0), (15, 32, 0.3), (3, 6, 40.0)]
    cases += [(int(z), int(z) + int(rng.integers(0, 8)), float(rng.uniform(0.1, 200.0)))
              for z in rng.integers(3, 23, size=40)]
    n_open = 0
    for z, a, es in cases:
        for kind in range(6):
            we, se, be = pmc.pmc_inc_width(z, a, es, kind)
            wo, so, bo = O.evap_width(z, a, es, kind)
            if wo == 0.0:
                assert we == 0.0, (z, a, es, kind)
                continue
            n_open += 1
            assert abs(se - so) < 1e-9 and abs(be - bo) < 1e-12, (z, a, es, kind)
            assert abs(we / wo - 1.0) < 1e-8, (z, a, es, kind, we, wo)
    assert n_open > 100
