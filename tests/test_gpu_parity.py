"""GPU parity: the HIP engine (through the C ABI) against the FP64 CPU
oracle on the same seeded inputs (arXiv:1409.8336 Sec. II.A transport,
Sec. II.B.2 statistics).

Tolerances (the acceptance bar):
  integrated depth-dose within 1% of its maximum, R80 within 0.2 mm,
  voxels above 10% of the maximum dose consistent within 3 sigma of the two
  10-group variance estimates, energy-ledger residual below 1e-5.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1409_8336_amd import pmc, synth

from parity_tools import assert_same_seed, compare, density_grid, ledger_residual, r80

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


def _engine(nd, mt, hu, voxel=(0.2, 0.2, 0.2), **params):
    e = pmc.Engine(0, **params)
    e.load_physics(nd)
    e.load_geometry(hu, voxel, mt)
    return e


def _oracle(nd, mt, hu, voxel=(0.2, 0.2, 0.2), flags=0):
    o = O.Oracle(flags=flags)
    o.load_physics(nd)
    o.load_geometry(hu, voxel, mt)
    return o


# ---------------------------------------------------------------- tables

def test_tables_match_oracle(nd, mt):
    _say("case: tables")
    hu = synth.water_phantom(8, 8, 8)
    e = _engine(nd, mt, hu)
    t = pmc.pmc_inspect_tables(e.ctx)
    o = _oracle(nd, mt, hu)
    grid = synth.energy_grid()
    want = np.log([o.range(x) for x in grid[1:]])
    np.testing.assert_allclose(t["lnr_water"][1:], want, rtol=0, atol=2e-6 * np.abs(want).max())
    assert t["lnr_water"][0] == -np.inf
    ti = int(np.nonzero(mt["own_table"])[0][0])
    want_ti = np.log([o.range(x, table=ti + 1) for x in grid[1:]])
    np.testing.assert_allclose(t["lnr_own"][1:], want_ti, rtol=0, atol=2e-6 * np.abs(want_ti).max())
    for m in range(len(mt["hu_lo"])):
        info = o.material_info(m)
        f, x0, za, own = t["material"][m]
        assert abs(f / info["f"] - 1) < 1e-9 and abs(x0 / info["x0_g_cm2"] - 1) < 1e-9
        assert abs(za / info["z_over_a"] - 1) < 1e-9 and own == info["own"]
        sig = np.array([sum(o.sigma(p, el, x) * 6.02214076e23 / (1.00794, 12.0107, 14.0067, 15.9994,
                                                                30.973762, 40.078, 47.867)[el]
                            * float(mt["mass_frac"][m][el]) * 1e-24
                            for p in (0, 1) for el in range(7)) for x in grid[::97]])
        np.testing.assert_allclose(t["sigma_per_g"][m][::97], sig, rtol=2e-6, atol=1e-12)
    e.close()


# ------------------------------------------------- deterministic special case

@pytest.mark.parametrize("hu_val,e0", [(0, 100.0), (1000, 150.0), (3000, 70.0)])
def test_deterministic_depth_dose(nd, mt, hu_val, e0):
    _say("case: deterministic hu=%d e0=%g" % (hu_val, e0))
    nz = 100 if hu_val != 3000 else 40
    hu = synth.uniform_phantom(hu_val, 3, 3, nz)
    flags = pmc.PMC_NO_STRAGGLE | pmc.PMC_NO_MCS | pmc.PMC_NO_NUCLEAR
    e = _engine(nd, mt, hu, flags=flags)
    o = _oracle(nd, mt, hu, flags=flags)
    spot = synth.pencil_spot(0.3, 0.3, e0, 0.0)
    n = 64
    gd, gv, gs = e.run_spots(spot, n, 1)
    od = o.run_spots(spot, n, 1)
    rho = density_grid(hu)
    g_idd = (gd * rho).sum(axis=(1, 2))
    o_idd = (od["dose"] * rho).sum(axis=(1, 2))
    conv = 1.602176634e-10 / float(np.prod(np.float32([0.2, 0.2, 0.2]).astype(np.float64)))
    g_e, o_e = g_idd / conv, o_idd / conv          # MeV per history
    assert np.nonzero(g_e)[0][-1] == np.nonzero(o_e)[0][-1]
    assert np.max(np.abs(g_e - o_e)) <= 3e-4 * e0, np.max(np.abs(g_e - o_e))
    assert abs(g_e.sum() - e0) <= 1e-5 * e0
    assert ledger_residual(gs) < 1e-9
    e.close()


# ------------------------------------------------------- statistical parity

def _parity(nd, mt, hu, spots, n, seed_gpu=1, seed_ora=1, tag=""):
    _say("case: parity %s n=%d" % (tag, n))
    e = _engine(nd, mt, hu)
    gd, gv, gs = e.run_spots(spots, n, seed_gpu)
    e.close()
    o = _oracle(nd, mt, hu)
    r = o.run_spots(spots, n, seed_ora)
    os_ = r["summary"]
    rho = density_grid(hu)
    m = compare(gd, gv, r["dose"], r["var"], rho, (0.2, 0.2, 0.2), gs["total_weight"],
                os_["total_weight"])
    m.update(gpu_steps_per_hist=gs["steps"] / n, ora_steps_per_hist=os_["steps"] / n,
             gpu_ne=gs["n_nonelastic"], ora_ne=os_["n_nonelastic"],
             gpu_el=gs["n_elastic"], ora_el=os_["n_elastic"],
             gpu_res=ledger_residual(gs), ora_res=ledger_residual(os_))
    _say("metrics %s: %s" % (tag, m))
    return m, gs, os_


def _assert_parity(m):
    assert m["idd_max_rel"] <= 0.01, m
    assert m["r80_diff_mm"] <= 0.2, m
    assert_same_seed(m)
    assert m["gpu_res"] < 1e-5 and m["ora_res"] < 1e-5, m
    assert abs(m["gpu_steps_per_hist"] / m["ora_steps_per_hist"] - 1) < 0.01, m


def test_water_pencil_parity(nd, mt):
    cfg = synth.config_water_pencil(100_000)
    m, gs, os_ = _parity(nd, mt, cfg["hu"], cfg["spots"], cfg["n_histories"], tag="water100")
    _assert_parity(m)
    for key in ("n_nonelastic", "n_elastic"):
        a, b = gs[key], os_[key]
        assert abs(a - b) <= 4 * math.sqrt(a + b) + 2, (key, a, b)


@pytest.mark.parametrize("energy", [70.0, 150.0, 230.0])
def test_ct_spot_parity(nd, mt, energy):
    """The heterogeneous CT with one spot per energy at its configured 1e6
    histories."""
    cfg = synth.config_ct_spots(energy, 1_000_000)
    m, gs, os_ = _parity(nd, mt, cfg["hu"], cfg["spots"], cfg["n_histories"], tag="ct%g" % energy)
    _assert_parity(m)


def test_half_slab_with_anisotropic_voxels(nd, mt):
    """Water with 2 cm of bone (HU 1000) at 4-6 cm depth over the half x >= 6
    cm, in 2 x 2 x 1 mm voxels (every other test uses 2 mm cubes), two
    150 MeV pencils, one through each half: same-seed dose parity with the
    oracle, and on the GPU's dose the slab half's R80 shorter than the water
    half's by the slab's t (rho f - 1) within 0.2 mm (the oracle's own pin of
    the composed transport)."""
    nx, ny, dz = 60, 30, 0.1
    nz = int(round(20.0 / dz))
    hu = np.zeros((nz, ny, nx), np.int16)
    hu[int(round(4.0 / dz)):int(round(6.0 / dz)), :, nx // 2:] = 1000
    voxel = (0.2, 0.2, dz)
    spots = np.concatenate([synth.pencil_spot(3.0, 3.0, 150.0, 0.3), synth.pencil_spot(9.0, 3.0, 150.0, 0.3)])
    n = 200_000
    _say("case: half slab, anisotropic voxels, n=%d" % n)
    e = _engine(nd, mt, hu, voxel)
    gd, gv, gs = e.run_spots(spots, n, 3)
    e.close()
    o = _oracle(nd, mt, hu, voxel)
    r = o.run_spots(spots, n, 3)
    lo = mt["hu_lo"].astype(int)
    b = int(np.searchsorted(lo, 1000, side="right") - 1)
    f = o.material_info(b)["f"]
    o.close()
    rho_grid = density_grid(hu)
    m = compare(gd, gv, r["dose"], r["var"], rho_grid, voxel, gs["total_weight"], r["summary"]["total_weight"])
    m.update(gpu_res=ledger_residual(gs), ora_res=ledger_residual(r["summary"]),
             gpu_steps_per_hist=gs["steps"] / n, ora_steps_per_hist=r["summary"]["steps"] / n)
    _say("metrics half slab: %s" % m)
    _assert_parity(m)
    rho = float(rho_grid[int(round(5.0 / dz)), 0, nx - 1])
    edep = gd * rho_grid
    r_water = r80(edep[:, :, : nx // 2].sum(axis=(1, 2)), dz)
    r_slab = r80(edep[:, :, nx // 2:].sum(axis=(1, 2)), dz)
    want = 2.0 * (rho * f - 1.0)
    _say("R80 water %.4f slab %.4f shift %.4f want %.4f cm" % (r_water, r_slab, r_water - r_slab, want))
    assert abs((r_water - r_slab) - want) < 0.02


def _random_case(k):
    """Seeded small heterogeneous case k: grid 12-48 x 12-48 x 20-120 voxels,
    anisotropic voxels of 0.1-0.3 cm, random lung / soft tissue / bone /
    titanium boxes, 1-6 spots anywhere over the entrance face (some near or
    past its edges), 5-250 MeV, sigma 0-1 cm, lognormal weights."""
    rng = np.random.default_rng(500 + k)
    nx, ny, nz = int(rng.integers(12, 49)), int(rng.integers(12, 49)), int(rng.integers(20, 121))
    vox = tuple(float(v) for v in rng.uniform(0.1, 0.3, size=3).round(3))
    hu = np.zeros((nz, ny, nx), np.int16)
    for _ in range(int(rng.integers(0, 6))):
        lo = [int(rng.integers(0, n)) for n in (nz, ny, nx)]
        hi = [int(rng.integers(l + 1, n + 1)) for l, n in zip(lo, (nz, ny, nx))]
        hu[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = rng.choice([-800, 40, 300, 1000, 2500, 3000])
    n_sp = int(rng.integers(1, 7))
    sp = np.zeros((n_sp, 6), np.float32)
    sp[:, 0] = rng.uniform(-0.1, 1.1, n_sp) * nx * vox[0]
    sp[:, 1] = rng.uniform(-0.1, 1.1, n_sp) * ny * vox[1]
    sp[:, 2] = rng.uniform(5.0, 250.0, n_sp)
    sp[:, 3] = rng.uniform(0.0, 1.0, n_sp)
    sp[:, 4] = rng.uniform(0.0, 1.0, n_sp)
    sp[:, 5] = rng.lognormal(0.0, 0.5, n_sp)
    return hu, vox, sp


@pytest.mark.parametrize("k", range(10))
def test_random_small_cases_close_and_agree(nd, mt, k):
    """Seeded random small cases (the edges of what the path accepts:
    anisotropic voxels, spots off the phantom, every material, 5 MeV
    protons that stop in the first voxels): on the GPU the ledger closes to
    rounding and the dose is finite and non-negative; against the oracle on
    the same seed the deposited, escaped and neutral energy fractions agree
    within 1% of the incident energy, the steps per history within 2%, and
    the nuclear event counts within their counting noise."""
    hu, vox, sp = _random_case(k)
    n = 20_000
    _say("case: random %d grid %s voxels %s spots %d" % (k, hu.shape, vox, len(sp)))
    e = _engine(nd, mt, hu, vox)
    gd, gv, gs = e.run_spots(sp, n, 9)
    e.close()
    o = _oracle(nd, mt, hu, vox)
    r = o.run_spots(sp, n, 9)
    o.close()
    os_ = r["summary"]
    assert np.all(np.isfinite(gd)) and np.all(gd >= 0) and np.all(np.isfinite(gv))
    assert ledger_residual(gs) < 1e-9 and ledger_residual(os_) < 1e-9, (gs, os_)
    for key in ("deposited", "escaped", "neutral"):
        a, b = gs[key] / gs["incident"], os_[key] / os_["incident"]
        assert abs(a - b) <= 0.01, (key, a, b)
    assert abs(gs["steps"] / max(os_["steps"], 1) - 1) < 0.02, (gs["steps"], os_["steps"])
    for key in ("n_nonelastic", "n_elastic"):
        a, b = gs[key], os_[key]
        assert abs(a - b) <= 4 * math.sqrt(a + b) + 3, (key, a, b)


@pytest.mark.parametrize("k,flag", [(0, "vavilov"), (3, "vavilov"), (6, "vavilov"),
                                    (1, "moliere"), (4, "moliere"), (9, "moliere")])
def test_random_small_cases_with_options(nd, mt, k, flag):
    """The same random cases with Vavilov-Gaussian straggling or Molière
    scattering on both sides: ledger, energy fractions, steps and event
    counts as for the defaults."""
    hu, vox, sp = _random_case(k)
    n = 20_000
    gflag, oflag = {"vavilov": (pmc.PMC_VAVILOV, O.VAVILOV), "moliere": (pmc.PMC_MOLIERE, O.MOLIERE)}[flag]
    _say("case: random %d with %s" % (k, flag))
    e = _engine(nd, mt, hu, vox, flags=gflag)
    gd, gv, gs = e.run_spots(sp, n, 9)
    e.close()
    o = _oracle(nd, mt, hu, vox, flags=oflag)
    r = o.run_spots(sp, n, 9)
    o.close()
    os_ = r["summary"]
    assert np.all(np.isfinite(gd)) and np.all(gd >= 0)
    assert ledger_residual(gs) < 1e-9 and ledger_residual(os_) < 1e-9, (gs, os_)
    for key in ("deposited", "escaped", "neutral"):
        a, b = gs[key] / gs["incident"], os_[key] / os_["incident"]
        assert abs(a - b) <= 0.01, (key, a, b)
    assert abs(gs["steps"] / max(os_["steps"], 1) - 1) < 0.02, (gs["steps"], os_["steps"])
    for key in ("n_nonelastic", "n_elastic"):
        a, b = gs[key], os_[key]
        assert abs(a - b) <= 4 * math.sqrt(a + b) + 3, (key, a, b)


def test_independent_seeds_are_consistent(nd, mt):
    cfg = synth.config_water_pencil(60_000)
    m, _, _ = _parity(nd, mt, cfg["hu"], cfg["spots"], cfg["n_histories"], seed_gpu=2, seed_ora=3,
                      tag="indep")
    n = m["n_sel"]
    assert m["frac_z_gt3"] <= 0.008 + 3.0 * math.sqrt(0.008 / n), m
    assert abs(m["z_mean"]) <= 0.1 and 0.85 <= m["z_std"] <= 1.2, m
    assert m["idd_max_rel"] <= 0.01 and m["r80_diff_mm"] <= 0.2, m


# ---------------------------------------------------------------- edge cases

def test_zero_histories_and_escaping_spot(nd, mt):
    _say("case: edges")
    hu = synth.water_phantom(16, 16, 32)
    e = _engine(nd, mt, hu)
    d, v, s = e.run_spots(synth.pencil_spot(1.6, 1.6, 80.0), 0, 1)
    assert not d.any() and not v.any() and s["incident"] == 0 and s["steps"] == 0
    d, v, s = e.run_spots(synth.pencil_spot(-5.0, 1.6, 80.0, 0.1), 1000, 1)
    assert not d.any() and s["steps"] == 0
    assert abs(s["escaped"] - s["incident"]) < 1e-9 * s["incident"]
    # one history, ragged against every wave
    d, v, s = e.run_spots(synth.pencil_spot(1.6, 1.6, 80.0), 1, 1)
    assert s["histories"] == 1 and d.sum() > 0 and ledger_residual(s) < 1e-9
    e.close()


def test_argument_errors(nd, mt):
    _say("case: errors")
    hu = synth.water_phantom(8, 8, 8)
    e = _engine(nd, mt, hu)
    with pytest.raises(pmc.PMCError) as ei:
        e.run_spots(synth.pencil_spot(0.8, 0.8, 300.0), 10, 1)
    assert ei.value.status == pmc.PMC_ERR_RANGE
    with pytest.raises(pmc.PMCError) as ei:
        e.run_spots(np.array([[0.8, 0.8, 50.0, 0.1, 0.1, -1.0]], np.float32), 10, 1)
    assert ei.value.status == pmc.PMC_ERR_RANGE
    with pytest.raises(pmc.PMCError) as ei:
        pmc.pmc_load_geometry(e.ctx, np.zeros((0, 4, 4), np.int16), (0.2, 0.2, 0.2), mt)
    assert ei.value.status == pmc.PMC_ERR_ARG
    bad = dict(mt)
    bad["mass_frac"] = mt["mass_frac"] * 2
    with pytest.raises(pmc.PMCError):
        pmc.pmc_load_geometry(e.ctx, hu, (0.2, 0.2, 0.2), bad)
    fresh = pmc.Engine(0)
    with pytest.raises(pmc.PMCError) as ei:
        pmc.pmc_run_spots(fresh.ctx, synth.pencil_spot(0.8, 0.8, 50.0), 10, 1, (8, 8, 8))
    assert ei.value.status == pmc.PMC_ERR_STATE
    fresh.close()
    e.close()


def test_queue_overflow_is_reported_and_ledger_closes(nd, mt):
    _say("case: overflow")
    hu = synth.water_phantom(32, 32, 170)
    # the generation queue's overflow: workgroup queues off, so that every
    # secondary goes through it
    e = _engine(nd, mt, hu, queue_capacity=8, local_queue=-1)
    with pytest.raises(pmc.PMCError) as ei:
        e.run_spots(synth.pencil_spot(3.2, 3.2, 230.0, 0.3), 20000, 1)
    assert ei.value.status == pmc.PMC_ERR_QUEUE_OVERFLOW
    s = pmc.summary_dict(pmc.pmc_summary())
    e.close()
    e = _engine(nd, mt, hu, queue_capacity=8, local_queue=4)
    dose = np.zeros(hu.shape)
    var = np.zeros(hu.shape)
    summ = pmc.pmc_summary()
    import ctypes as C
    st = pmc.lib().pmc_run_spots(e.ctx, pmc._ptr(synth.pencil_spot(3.2, 3.2, 230.0, 0.3)), 1, 20000,
                                 1, pmc._ptr(dose), pmc._ptr(var), C.byref(summ))
    s = pmc.summary_dict(summ)
    assert st == pmc.PMC_ERR_QUEUE_OVERFLOW and s["n_overflow"] > 0 and s["overflow"] > 0
    assert ledger_residual(s) < 1e-9
    assert dose.sum() > 0
    e.close()


def test_launch_shape_does_not_change_results(nd, mt):
    _say("case: launch shapes")
    cfg = synth.config_ct_spots(150.0, 20_000)
    ref = None
    for params in (dict(), dict(block_threads=64, refill_lanes=1, batch_events=1),
                   dict(block_threads=512, refill_lanes=48, batch_events=16, blocks_per_cu=1)):
        e = _engine(nd, mt, cfg["hu"], **params)
        d, v, s = e.run_spots(cfg["spots"], cfg["n_histories"], 5)
        e.close()
        if ref is None:
            ref = (d, s)
            continue
        np.testing.assert_allclose(d, ref[0], rtol=1e-9, atol=1e-9 * ref[0].max())
        for k in ("steps", "n_elastic", "n_nonelastic", "secondaries"):
            assert s[k] == ref[1][k], (k, params)


def test_workgroup_queues_preserve_results(nd, mt):
    """Secondaries a workgroup takes from its own queue within the launch give
    the dose, variance and counts of the generation-by-generation schedule
    (queues off); a 4-entry queue sends most of them on to the generation
    queue, mixing both paths; the ledger closes in every case."""
    _say("case: workgroup queues")
    cfg = synth.config_ct_spots(150.0, 30_000)
    runs = []
    fixed = dict(refill_lanes=8, batch_events=4)   # no autotuning
    for params in (dict(fixed, block_threads=1024, local_queue=-1), dict(fixed, block_threads=1024),
                   dict(fixed, block_threads=1024, local_queue=4),
                   dict(fixed, block_threads=256, local_queue=64, epoch_steps=5)):
        e = _engine(nd, mt, cfg["hu"], **params)
        d, v, s = e.run_spots(cfg["spots"], cfg["n_histories"], 8)
        e.close()
        _say("  %s: generations %d secondaries %d" % (params, s["generations"], s["secondaries"]))
        runs.append((params, d, v, s))
    p0, d0, v0, s0 = runs[0]
    assert s0["secondaries"] > 100 and s0["generations"] >= 3
    assert runs[1][3]["generations"] <= 2        # everything inside the first launch
    for params, d, v, s in runs[1:]:
        np.testing.assert_allclose(d, d0, rtol=1e-9, atol=1e-9 * d0.max())
        np.testing.assert_allclose(v, v0, rtol=1e-6, atol=1e-9 * v0.max())
        for k in ("steps", "n_elastic", "n_nonelastic", "secondaries", "tally_atomics", "n_overflow"):
            assert s[k] == s0[k], (k, params)
        assert ledger_residual(s) < 1e-9


def test_deposit_cache_preserves_results(nd, mt):
    """The workgroup LDS deposit cache only regroups FP64 additions: dose,
    step and event counts equal the uncached run; with the cache on fewer
    atomics reach device memory, and a tiny cache flushed every 7 iterations
    (many misses and evictions) gives the same results."""
    _say("case: deposit cache")
    cfg = synth.config_ct_spots(150.0, 30_000)
    runs = []
    fixed = dict(refill_lanes=16, batch_events=4)   # no autotuning
    for params in (dict(fixed, block_threads=1024, tally_cache=-1), dict(fixed, block_threads=1024),
                   dict(fixed, block_threads=1024, tally_cache=512, epoch_steps=7),
                   dict(fixed, block_threads=512, tally_cache=2048, epoch_steps=300)):
        e = _engine(nd, mt, cfg["hu"], **params)
        d, v, s = e.run_spots(cfg["spots"], cfg["n_histories"], 6)
        e.close()
        runs.append((params, d, v, s))
    p0, d0, v0, s0 = runs[0]
    assert s0["global_atomics"] == s0["tally_atomics"]
    for params, d, v, s in runs[1:]:
        np.testing.assert_allclose(d, d0, rtol=1e-9, atol=1e-9 * d0.max())
        np.testing.assert_allclose(v, v0, rtol=1e-6, atol=1e-9 * v0.max())
        for k in ("steps", "n_elastic", "n_nonelastic", "secondaries", "tally_atomics"):
            assert s[k] == s0[k], (k, params)
        assert abs(s["deposited"] - s0["deposited"]) <= 1e-12 * s0["deposited"]
        assert s["global_atomics"] < s0["global_atomics"], params
        _say("%s: global atomics %d of %d deposits" % (params, s["global_atomics"], s["tally_atomics"]))


def test_device_buffers_match_host_buffers(nd, mt):
    import torch
    _say("case: device buffers")
    cfg = synth.config_water_pencil(20_000)
    e = _engine(nd, mt, cfg["hu"])
    d, v, s = e.run_spots(cfg["spots"], cfg["n_histories"], 9)
    dd = torch.zeros(cfg["hu"].shape, dtype=torch.float64, device="cuda")
    dv = torch.zeros_like(dd)
    stream = torch.cuda.Stream()
    s2 = e.run_spots_dev(cfg["spots"], cfg["n_histories"], 9, dd, dv, stream)
    torch.cuda.synchronize()
    np.testing.assert_allclose(dd.cpu().numpy(), d, rtol=1e-9, atol=1e-9 * d.max())
    np.testing.assert_allclose(dv.cpu().numpy(), v, rtol=1e-6, atol=1e-9 * v.max())
    assert s2["steps"] == s["steps"]
    e.close()


# --------------------------------------------- full-size treatment field

def test_full_size_field_same_seed_parity(nd, mt):
    """The 256x256x200 CT with the 2000-spot field at its configured 1e7
    histories, in the benchmark's launch configuration (device buffers on
    the current stream, autotuned launch shape), against the oracle on the
    same seed: IDD within 1%, R80 within 0.2 mm, every voxel at or above 10%
    of the maximum dose within 3 sigma, the variance voxel by voxel, the
    ledger, steps per history; and properties that hold at any size."""
    import torch
    cfg = synth.config_field(10_000_000)
    n = cfg["n_histories"]
    _say("case: full field same seed n=%d (GPU)" % n)
    e = _engine(nd, mt, cfg["hu"])
    dd = torch.empty(cfg["hu"].shape, dtype=torch.float64, device="cuda")
    dv = torch.empty_like(dd)
    gs = e.run_spots_dev(cfg["spots"], n, cfg["seed"], dd, dv, torch.cuda.current_stream())
    torch.cuda.synchronize()
    e.close()
    gd, gv = dd.cpu().numpy(), dv.cpu().numpy()
    del dd, dv
    _say("full field GPU summary %s" % gs)
    assert gs["histories"] == n and (gd >= 0).all() and (gv >= 0).all()
    _say("case: full field same seed n=%d (oracle)" % n)
    o = _oracle(nd, mt, cfg["hu"])
    r = o.run_spots(cfg["spots"], n, cfg["seed"])
    o.close()
    os_ = r["summary"]
    _say("oracle %.1f s on %d threads" % (os_["wall_s"], os_["threads"]))
    m = compare(gd, gv, r["dose"], r["var"], density_grid(cfg["hu"]), (0.2, 0.2, 0.2),
                gs["total_weight"], os_["total_weight"])
    m.update(gpu_steps_per_hist=gs["steps"] / n, ora_steps_per_hist=os_["steps"] / n,
             gpu_res=ledger_residual(gs), ora_res=ledger_residual(os_))
    _say("metrics field: %s" % m)
    _assert_parity(m)
    for key in ("n_nonelastic", "n_elastic"):
        a, b = gs[key], os_[key]
        assert abs(a - b) <= 4 * math.sqrt(a + b) + 2, (key, a, b)


def test_geometry_density_matches_hu_calibration(nd, mt):
    """pmc_geometry_density returns the density the transport uses: the
    piecewise-linear HU calibration (Sec. II.A.1) restated on the host, to
    float32 rounding, for the main geometry and an extra geometry slot."""
    import torch
    _say("case: geometry density")
    hu = synth.ct_phantom(40, 36, 30, 0.2, seed=9)
    hu2 = synth.scaled_ct_phantom(24, 20, 16, seed=10)
    e = _engine(nd, mt, hu)
    gid = pmc.pmc_load_geometry_slot(e.ctx, hu2, (0.2, 0.2, 0.2), mt)
    for g, h in ((0, hu), (gid, hu2)):
        rho = torch.empty(h.shape, dtype=torch.float32, device="cuda")
        pmc.pmc_geometry_density(e.ctx, g, rho)
        torch.cuda.synchronize()
        ref = density_grid(h)
        np.testing.assert_allclose(rho.cpu().numpy(), ref, rtol=2.0 ** -23, atol=0)
    with pytest.raises(pmc.PMCError):
        pmc.pmc_geometry_density(e.ctx, 99, torch.empty(hu.shape, dtype=torch.float32, device="cuda"))
    e.close()


def test_group_count_leaves_the_dose_unchanged(nd, mt):
    """K only splits the histories into groups for the variance: the total
    dose is the same realisation for K = 3, 10 and 64 (FP64 summation order
    aside), the variance is non-negative and its mean over the dose region
    agrees between K = 10 and K = 64 within their sampling spread."""
    _say("case: group counts")
    cfg = synth.config_ct_spots(150.0, 40_000)
    res = {}
    for k in (3, 10, 64):
        e = _engine(nd, mt, cfg["hu"], k_batches=k)
        d, v, s = e.run_spots(cfg["spots"], cfg["n_histories"], 4)
        e.close()
        res[k] = (d, v, s)
        assert (v >= 0).all()
    d10, v10, _ = res[10]
    for k in (3, 64):
        np.testing.assert_allclose(res[k][0], d10, rtol=1e-9, atol=1e-12 * d10.max())
    m = d10 > 0.1 * d10.max()
    r = res[64][1][m].mean() / v10[m].mean()
    # the mean of many voxel variances: each has relative spread sqrt(2/(K-1))
    assert 0.8 < r < 1.25, r


def test_hundred_million_histories_without_variance(nd, mt):
    """The launch shape of the one GPU fault on record, run on the fixed
    code: a denoiser-target run of 1e8 histories on the 128x128x160 CT
    through pmc_run_spots_dev with no variance output (d_var NULL), 512-lane
    workgroups two per CU with the deposit cache.  Its ledger closes, the
    dose is finite and non-negative, and its depth-dose agrees with an
    independent 1e6-history oracle run within the oracle's noise."""
    import torch
    case = synth.denoiser_case(0)
    n = 100_000_000
    _say("case: 1e8 histories, d_var NULL, 512-lane workgroups (GPU)")
    e = _engine(nd, mt, case["hu"], block_threads=512, blocks_per_cu=2, refill_lanes=16,
                batch_events=4)
    dd = torch.empty(case["hu"].shape, dtype=torch.float64, device="cuda")
    s = e.run_spots_dev(case["spots"], n, 20_000, dd, None)
    torch.cuda.synchronize()
    e.close()
    d = dd.cpu().numpy()
    _say("1e8 summary %s" % s)
    assert s["histories"] == n and s["block_threads"] == 512 and s["cache_slots"] > 0
    assert s["grid_blocks"] == 2 * torch.cuda.get_device_properties(0).multi_processor_count
    assert ledger_residual(s) < 1e-5
    assert np.isfinite(d).all() and (d >= 0).all() and d.max() > 0
    o = _oracle(nd, mt, case["hu"])
    r = o.run_spots(case["spots"], 1_000_000, 3)
    o.close()
    rho = density_grid(case["hu"])
    g_idd = (d * rho).sum(axis=(1, 2))
    o_idd = (r["dose"] * rho).sum(axis=(1, 2))
    o_sd = np.sqrt((r["var"] * rho ** 2).sum(axis=(1, 2)))
    diff = np.abs(g_idd - o_idd)
    assert np.all(diff <= 4 * o_sd + 0.01 * o_idd.max()), float((diff / o_idd.max()).max())
