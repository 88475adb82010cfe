"""Molière multiple scattering (arXiv:1409.8336 Sec. II.A.2 option) in the
HIP engine, through the C ABI, against the FP64 oracle with the same option.

Bars: those of the Highland parity tests (integrated depth-dose within 1% of
its maximum, R80 within 0.2 mm, voxels above 10% of the maximum dose within
3 sigma or at the t-tail rate where histories diverged, ledger residual
below 1e-5), plus lateral profiles: the dose-weighted lateral RMS at every
depth no farther from the oracle's than the oracle's own seed-to-seed spread
(or 1%): an r^2-weighted width is carried by a few far-scattered protons, and
histories that diverge through FP32-vs-FP64 decisions are independent
realisations.  Against the scaled Highland default the
Molière core is within 7% (Highland x 1.07 was fitted to a Molière-like
model) and its single-scattering tail carries more dose far off axis."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1409_8336_amd import pmc, synth

from parity_tools import compare, density_grid, ledger_residual

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nd():
    return synth.nuclear_data()


@pytest.fixture(scope="module")
def mt():
    return synth.material_table()


def _consistent(m):
    """Same seed: every voxel at or above 10% of the maximum within 3 sigma."""
    return m["all_within_3sigma"]


def _gpu(nd, mt, hu, spots, n, seed, flags):
    e = pmc.Engine(0, flags=flags)
    e.load_physics(nd)
    e.load_geometry(hu, (0.2, 0.2, 0.2), mt)
    d, v, s = e.run_spots(spots, n, seed)
    e.close()
    return d, v, s


def _lateral_rms(dose, rho, cx, cy):
    """Dose-weighted RMS distance from the beam axis (cm) per depth slice."""
    nz, ny, nx = dose.shape
    y, x = np.meshgrid((np.arange(ny) + 0.5) * 0.2 - cy, (np.arange(nx) + 0.5) * 0.2 - cx, indexing="ij")
    e = dose * rho
    w = e.sum(axis=(1, 2))
    ok = w > 0.2 * w.max()
    r2 = (e * (x * x + y * y)).sum(axis=(1, 2)) / np.where(w > 0, w, 1.0)
    return np.sqrt(r2[ok]), ok


@pytest.mark.parametrize("case", ["water100", "ct150"])
def test_moliere_parity(nd, mt, case):
    if case == "water100":
        cfg = synth.config_water_pencil(100_000)
    else:
        cfg = synth.config_ct_spots(150.0, 60_000)
    _say("case: Moliere parity %s" % case)
    gd, gv, gs = _gpu(nd, mt, cfg["hu"], cfg["spots"], cfg["n_histories"], 1, pmc.PMC_MOLIERE)
    o = O.Oracle(flags=O.MOLIERE)
    o.load_physics(nd)
    o.load_geometry(cfg["hu"], (0.2, 0.2, 0.2), mt)
    r = o.run_spots(cfg["spots"], cfg["n_histories"], 1)
    r2 = o.run_spots(cfg["spots"], cfg["n_histories"], 2)
    rho = density_grid(cfg["hu"])
    m = compare(gd, gv, r["dose"], r["var"], rho, (0.2, 0.2, 0.2), gs["total_weight"],
                r["summary"]["total_weight"])
    m.update(gpu_res=ledger_residual(gs), ora_res=ledger_residual(r["summary"]))
    sp = cfg["spots"][0]
    la, _ = _lateral_rms(gd, rho, sp[0], sp[1])
    lb, _ = _lateral_rms(r["dose"], rho, sp[0], sp[1])
    lc, _ = _lateral_rms(r2["dose"], rho, sp[0], sp[1])
    m["lateral_max_rel"] = float(np.max(np.abs(la / lb - 1.0)))
    m["lateral_seed_spread"] = float(np.max(np.abs(lc / lb - 1.0)))
    _say("metrics %s: %s" % (case, m))
    assert m["idd_max_rel"] <= 0.01, m
    assert m["r80_diff_mm"] <= 0.2, m
    assert _consistent(m), m
    assert m["gpu_res"] < 1e-5 and m["ora_res"] < 1e-5, m
    assert m["lateral_max_rel"] <= max(0.01, m["lateral_seed_spread"]), m


def test_moliere_against_highland(nd, mt):
    """Same beam with the default scaled Highland: the depth-dose barely
    moves, and the lateral variance that scattering adds to the beam's own
    (r^2 at depth minus r^2 at the entrance) is of the same size — the
    Molière core is a few per cent narrower than Highland x 1.07, its
    single-scattering tail adds to r^2."""
    _say("case: Moliere vs Highland")
    cfg = synth.config_water_pencil(200_000)
    hu = cfg["hu"]
    a = _gpu(nd, mt, hu, cfg["spots"], cfg["n_histories"], 3, pmc.PMC_MOLIERE)
    b = _gpu(nd, mt, hu, cfg["spots"], cfg["n_histories"], 3, 0)
    rho = density_grid(hu)
    sp = cfg["spots"][0]
    la, _ = _lateral_rms(a[0], rho, sp[0], sp[1])
    lb, _ = _lateral_rms(b[0], rho, sp[0], sp[1])
    add_a, add_b = la ** 2 - la[0] ** 2, lb ** 2 - lb[0] ** 2
    deep = add_b > 0.2 * lb[0] ** 2
    ratio = np.sqrt(add_a[deep] / add_b[deep])
    m = compare(a[0], a[1], b[0], b[1], rho, (0.2, 0.2, 0.2), a[2]["total_weight"], b[2]["total_weight"])
    _say("Moliere vs Highland: added lateral RMS ratio %s; idd %s r80 %s"
         % (np.round(ratio, 3).tolist(), m["idd_max_rel"], m["r80_diff_mm"]))
    assert deep.sum() >= 5
    assert np.all((ratio > 0.85) & (ratio < 1.3)), ratio
    assert m["idd_max_rel"] <= 0.02 and m["r80_diff_mm"] <= 0.3, m
    assert ledger_residual(a[2]) < 1e-9
