"""Pins of the oracle's non-elastic model (arXiv:1409.8336 Sec. II.A.4:
Bertini-style intranuclear cascade in a two-component Fermi gas with a
Woods-Saxon density in 15 constant-density shells, Pauli blocking,
refraction and reflection at the shell boundaries, elastic NN collisions,
then evaporation) against facts that do not come from the oracle: the
Woods-Saxon integral by independent quadrature, the Fermi-gas closed forms,
conservation laws (baryon number, charge, energy, four-momentum),
closed-form evaporation widths and spectra, and Snell's law at a potential
step."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import oracle as O

HBARC = 197.3269804
M_N = 938.918754
ZA = {1: (6, 12), 2: (7, 14), 3: (8, 16), 4: (15, 31), 5: (20, 40), 6: (22, 48)}


@pytest.mark.parametrize("el", [1, 3, 5, 6])
def test_woods_saxon_shells_hold_the_nucleons(el):
    """15 equal-thickness shells out to R + 5a, each at the Woods-Saxon
    average density over its volume (scipy quadrature here), normalised to
    A nucleons; protons Z/A of it."""
    nu = O.inc_nucleus(el)
    z, a = ZA[el]
    assert (nu["z"], nu["a"]) == (z, a)
    R = 1.16 * a ** (1 / 3) * (1 - 1.16 * a ** (-2 / 3))
    assert abs(nu["radius_ws"] - R) < 1e-12 and abs(nu["r_out"] - (R + 5 * 0.55)) < 1e-12
    r = nu["r"]
    vol = 4 / 3 * math.pi * (r[1:] ** 3 - r[:-1] ** 3)
    rho = nu["rho_p"] + nu["rho_n"]
    assert abs((rho * vol).sum() - a) < 1e-9 * a
    np.testing.assert_allclose(nu["rho_p"] / rho, z / a, rtol=1e-12)
    ws = lambda x: 4 * math.pi * x * x / (1 + math.exp((x - R) / 0.55))
    full = integrate.quad(ws, 0, r[-1], epsabs=0, epsrel=1e-12)[0]
    for k in range(15):
        want = a * integrate.quad(ws, r[k], r[k + 1], epsabs=0, epsrel=1e-12)[0] / full
        assert abs(rho[k] * vol[k] - want) < 1e-7 * a, (k, rho[k] * vol[k], want)
    # density falls outward; the central density is nuclear-matter-like
    assert np.all(np.diff(rho) < 0) and 0.12 < rho[0] < 0.22


@pytest.mark.parametrize("el", [3, 6])
def test_fermi_energies_follow_the_shell_densities(el):
    nu = O.inc_nucleus(el)
    for sp in ("p", "n"):
        pf = HBARC * np.cbrt(3 * math.pi ** 2 * nu["rho_" + sp])
        np.testing.assert_allclose(nu["tf_" + sp], np.sqrt(pf ** 2 + M_N ** 2) - M_N, rtol=1e-12)


def test_fermi_sea_momentum_sampling():
    """A full Fermi sphere: |p|^3 / p_F^3 uniform, directions isotropic."""
    rng = np.random.default_rng(5)
    pf = 250.0
    u = rng.random((40000, 3))
    p = np.array([O.fermi_momentum(pf, x) for x in u])
    m = np.linalg.norm(p, axis=1)
    assert m.max() <= pf * (1 + 1e-12)
    assert stats.kstest((m / pf) ** 3, "uniform").pvalue > 1e-3
    ct = p[:, 2] / m
    assert stats.kstest((ct + 1) / 2, "uniform").pvalue > 1e-3
    phi = np.arctan2(p[:, 1], p[:, 0])
    assert stats.kstest((phi + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-3


def test_refraction_is_snell_at_a_potential_step():
    """Crossing a spherical boundary: total energy (kinetic minus well depth)
    and the momentum along the surface are kept; below the critical angle the
    particle is reflected with unchanged energy."""
    rng = np.random.default_rng(6)
    for _ in range(300):
        x = rng.normal(size=3)
        x *= rng.uniform(1, 5) / np.linalg.norm(x)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        t, v1, v2 = rng.uniform(1, 200), rng.uniform(0, 50), rng.uniform(0, 50)
        crossed, t2, d2 = O.inc_refract(t, v1, v2, x, d)
        n = x / np.linalg.norm(x)
        p1 = math.sqrt(t * (t + 2 * M_N)) * d
        if crossed:
            assert abs((t2 - v2) - (t - v1)) < 1e-9 * t
            p2 = math.sqrt(t2 * (t2 + 2 * M_N)) * np.array(d2)
            np.testing.assert_allclose(p2 - np.dot(p2, n) * n, p1 - np.dot(p1, n) * n, atol=1e-8 * np.abs(p1).max())
            assert np.sign(np.dot(p2, n)) == np.sign(np.dot(p1, n))
        else:
            assert t2 == t
            np.testing.assert_allclose(np.dot(d2, n), -np.dot(d, n), atol=1e-12)
            pn2 = (t - v1 + v2) * (t - v1 + v2 + 2 * M_N) - np.dot(p1 - np.dot(p1, n) * n, p1 - np.dot(p1, n) * n)
            assert t - v1 + v2 <= 0 or pn2 <= 1e-6 * t * t
        assert abs(np.linalg.norm(d2) - 1) < 1e-12


def test_nn_collision_conserves_four_momentum_and_follows_exp_bt():
    rng = np.random.default_rng(7)
    for _ in range(200):
        p1 = rng.normal(size=3) * 400
        p2 = rng.normal(size=3) * 150
        o1, o2 = O.nn_collide(p1, p2, rng.random(), rng.random())
        e = lambda p: math.sqrt(np.dot(p, p) + M_N ** 2)
        np.testing.assert_allclose(np.add(o1, o2), np.add(p1, p2), atol=1e-8 * 400)
        assert abs(e(o1) + e(o2) - e(p1) - e(p2)) < 1e-9 * (e(p1) + e(p2))
    # on a nucleon at rest, the CM polar angle: t = -2 p*^2 (1 - cos) with
    # density ~ exp(B t) on [-4 p*^2, 0]
    p1 = np.array([0.0, 0.0, 1500.0])
    s = (math.sqrt(1500.0 ** 2 + M_N ** 2) + M_N) ** 2 - 1500.0 ** 2
    ps2 = (s / 4 - M_N ** 2) * 1e-6
    B = O.lib().oracle_nn_slope(1.5)
    assert abs(B - 5.5 * 1.5 ** 8 / (7.7 + 1.5 ** 8)) < 1e-12
    ts = []
    for ut in rng.random(20000):
        o1, o2 = O.nn_collide(p1, [0.0, 0.0, 0.0], ut, rng.random())
        # back to the CM: the momentum transfer is invariant, t = (p1 - o1)^2 (GeV^2)
        e1, f1 = math.sqrt(1500.0 ** 2 + M_N ** 2), math.sqrt(np.dot(o1, o1) + M_N ** 2)
        ts.append(((e1 - f1) ** 2 - np.dot(p1 - np.array(o1), p1 - np.array(o1))) * 1e-6)
    ts = np.array(ts)
    cdf = lambda t: (np.exp(B * t) - np.exp(-4 * ps2 * B)) / (1 - np.exp(-4 * ps2 * B))
    assert stats.kstest(ts, cdf).pvalue > 1e-3


@pytest.mark.parametrize("el,t", [(1, 70.0), (3, 150.0), (3, 230.0), (5, 100.0), (6, 200.0)])
def test_cascade_conserves_baryons_charge_and_energy(el, t):
    """Per event: A + 1 = A_res + escaped nucleons, Z + 1 = Z_res + escaped
    protons; the energy balance T = sum T_out + (n_esc - 1) S + E* matches
    the excitation summed independently over holes (Fermi energy minus the
    struck nucleon's kinetic energy) and trapped particles; after
    evaporation T = sum of all kinetic energies + separation energies + the
    excitation left, and the fragment numbers add up."""
    z, a = ZA[el]
    for uid in range(300):
        r = O.inc_event(el, t, 9, uid)
        inc = r["stage"] == 0
        n_p = int(np.sum((r["kind"] == 1) & inc))
        assert r["a_res"] + int(inc.sum()) == a + 1 and r["z_res"] + n_p == z + 1
        assert r["n_esc"] == int(inc.sum())
        assert abs(r["e_star"] - r["e_star_sum"]) < 1e-9 * t, (uid, r["e_star"], r["e_star_sum"])
        assert r["e_star"] >= -1e-9
        assert abs(t - r["t"].sum() - r["binding"] - r["e_star_fin"]) < 1e-9 * t
        ev = ~inc
        zj = np.array([0, 1, 1, 1, 2, 2])[r["kind"][ev]]
        aj = np.array([1, 1, 2, 3, 3, 4])[r["kind"][ev]]
        assert r["a_fin"] == r["a_res"] - aj.sum() and r["z_fin"] == r["z_res"] - zj.sum()
        assert r["e_star_fin"] >= -1e-9 and np.all(r["t"] > 0)
        # Pauli: every allowed collision's products lie above their Fermi energies
        assert r["n_coll"] >= 1 or r["compound"]
        assert r["pauli_min"] > 0


def test_pauli_blocking_suppresses_low_energy_collisions():
    """Blocking grows as the incident energy approaches the Fermi surface
    (slow cascade secondaries are blocked at any incident energy)."""
    lo = [O.inc_event(3, 15.0, 3, u, evaporate=False) for u in range(200)]
    hi = [O.inc_event(3, 200.0, 3, u, evaporate=False) for u in range(200)]
    frac = lambda rs: sum(r["n_blocked"] for r in rs) / max(1, sum(r["n_blocked"] + r["n_coll"] for r in rs))
    assert frac(lo) > frac(hi) + 0.05 and frac(lo) > 0.75, (frac(lo), frac(hi))


def _width_closed_form(x, la):
    """integral_0^X (X - U) exp(2 sqrt(la U)) dU = (e^Y (2Y^2 - 6Y + 6) + Y^2 - 6) / (8 la^2), Y = 2 sqrt(la X)"""
    y = 2 * math.sqrt(la * x)
    if y < 1e-2:
        return x * x / 2
    return (math.exp(y) * (2 * y * y - 6 * y + 6) + y * y - 6) / (8 * la * la)


@pytest.mark.parametrize("z,a,e", [(8, 16, 30.0), (20, 40, 60.0), (6, 12, 25.0), (22, 48, 10.0)])
def test_evaporation_widths_match_the_closed_form(z, a, e):
    ez = [0, 1, 1, 1, 2, 2]
    ea = [1, 1, 2, 3, 3, 4]
    g = [2, 2, 3, 2, 2, 1]
    for j in range(6):
        w, sep, bar = O.evap_width(z, a, e, j)
        zd, ad = z - ez[j], a - ea[j]
        bd = O.lib().oracle_binding_energy(zd, ad)
        bp = O.lib().oracle_binding_energy(z, a)
        be_j = 0.0 if ea[j] == 1 else O.lib().oracle_binding_energy(ez[j], ea[j])
        assert abs(sep - (bp - bd - be_j)) < 1e-9
        rad = 1.5 * (ad ** (1 / 3) + ea[j] ** (1 / 3))
        assert abs(bar - (1.439964548 * ez[j] * zd / rad if ez[j] else 0.0)) < 1e-9
        x = e - sep - bar
        if x <= 0:
            assert w == 0.0
            continue
        mu = ea[j] * ad / (ea[j] + ad)
        want = g[j] * mu * rad * rad * _width_closed_form(x, ad / 8.0)
        assert abs(w / want - 1) < 1e-6, (j, w, want)


def test_weizsaecker_binding_energies():
    """The liquid-drop formula with its stated coefficients, and measured
    values for the light ejectiles."""
    assert abs(O.lib().oracle_binding_energy(2, 4) - 28.295673) < 1e-9
    assert abs(O.lib().oracle_binding_energy(1, 2) - 2.224566) < 1e-9
    for z, a in [(8, 16), (20, 40), (6, 12), (13, 27)]:
        n = a - z
        b = 15.75 * a - 17.8 * a ** (2 / 3) - 0.711 * z * (z - 1) / a ** (1 / 3) - 23.7 * (n - z) ** 2 / a
        b += 11.18 / math.sqrt(a) * (1 if (z % 2 == 0 and n % 2 == 0) else (-1 if (z % 2 and n % 2) else 0))
        assert abs(O.lib().oracle_binding_energy(z, a) - b) < 1e-9
    # measured binding energies of O-16 and Ca-40 (127.6, 342.1 MeV) within the formula's few per cent
    assert abs(O.lib().oracle_binding_energy(8, 16) / 127.62 - 1) < 0.05
    assert abs(O.lib().oracle_binding_energy(20, 40) / 342.05 - 1) < 0.05


def test_evaporation_first_emission_spectrum_and_channels():
    """For one excited nucleus, the first emission's channel frequencies
    follow the widths, its kinetic energy above the barrier the integrand
    y exp(2 sqrt(a (X - y))), and directions are isotropic."""
    z, a, e = 20, 40, 40.0
    widths = np.array([O.evap_width(z, a, e, j)[0] for j in range(6)])
    n = 6000
    first = [O.evaporate(z, a, e, 11, uid) for uid in range(n)]
    kinds = np.array([f["kind"][0] for f in first])
    counts = np.bincount(kinds, minlength=6)
    expect = widths / widths.sum() * n
    ok = expect > 5
    chi2 = (((counts - expect) ** 2 / np.where(ok, expect, 1))[ok]).sum()
    assert chi2 < stats.chi2.ppf(0.999, ok.sum() - 1), (counts, expect)
    for j in (0, 1):
        _, sep, bar = O.evap_width(z, a, e, j)
        x = e - sep - bar
        la = (a - [1, 1][j]) / 8.0
        y = np.array([f["t"][0] for f in first if f["kind"][0] == j]) - bar
        norm = integrate.quad(lambda v: v * math.exp(2 * math.sqrt(la * (x - v))), 0, x)[0]
        cdf = np.vectorize(lambda s: integrate.quad(lambda v: v * math.exp(2 * math.sqrt(la * (x - v))),
                                                    0, min(max(s, 0), x))[0] / norm)
        assert stats.kstest(y, cdf).pvalue > 1e-3
    ct = np.array([f["dir"][0][2] for f in first])
    assert stats.kstest((ct + 1) / 2, "uniform").pvalue > 1e-3


def test_nn_cross_section_stand_ins():
    assert abs(O.lib().oracle_nn_sigma_mb(1, 100.0) - 32.0) < 1e-12
    assert abs(O.lib().oracle_nn_sigma_mb(0, 100.0) - 60.0) < 1e-12
    assert O.lib().oracle_nn_sigma_mb(1, 0.5) == O.lib().oracle_nn_sigma_mb(1, 1.0)


def test_inc_transport_ledger_closes():
    """In the transport with the cascade on (water pencil, 150 MeV): incident
    = deposited + escaped + neutral (neutrons, separation energies,
    photon excitation) exactly, and secondaries are produced."""
    from paper_1409_8336_amd import synth
    o = O.Oracle(flags=O.INC)
    o.load_physics(synth.nuclear_data())
    o.load_geometry(synth.water_phantom(32, 32, 100), (0.2, 0.2, 0.2), synth.material_table())
    out = o.run_spots(synth.pencil_spot(3.2, 3.2, 150.0, 0.3), 4000, 1)
    s = out["summary"]
    res = abs(s["incident"] - s["deposited"] - s["escaped"] - s["neutral"]) / s["incident"]
    assert res < 1e-12 and s["n_nonelastic"] > 50 and s["secondaries"] > 20
