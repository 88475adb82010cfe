"""Seeded synthetic inputs shared by the HIP engine, the CPU oracle, the tests
and the benchmark.

This module only *generates data*: HU phantoms, beam-spot lists, the HU ->
material table, the per-element nuclear cross-section tables and the
non-elastic secondary-proton table.  It performs none of the transport
arithmetic (no stopping powers, ranges, scattering or sampling of the method)
so that both implementations of the method stay independent of each other.

The paper's own inputs (Schneider's HU conversion, Geant4 cross-section
tables, the INC/evaporation model, TOPAS phase space; Sec. II.A) are not
available, so every table here is a documented synthetic stand-in with the
shape of the paper's workloads (Sec. II.D, III.B-C).  Every tabulated value is
rounded to a float32-representable number so that the float32 device engine
and the float64 oracle start from bit-identical inputs.
"""
from __future__ import annotations

import math

import numpy as np

# Element order of every per-element array (mass fractions, cross sections).
ELEMENTS = ("H", "C", "N", "O", "P", "Ca", "Ti")
# Molar masses (g/mol) used only to build the water composition below.
_MOLAR_MASS = {"H": 1.00794, "O": 15.9994}
# Mass numbers and charges used only to shape the synthetic cross sections.
_MASS_NUMBER = (1, 12, 14, 16, 31, 40, 48)
_CHARGE = (1, 6, 7, 8, 15, 20, 22)

# Energy grid of every tabulated quantity: E_i = E_MIN*(E_MAX/E_MIN)**(i/(N_E-1)).
E_MIN_MEV = 0.1
E_MAX_MEV = 250.0
N_E = 1000

# Non-elastic secondary table: nuclei C..Ti (element indices 1..6), 25 bins
# of 10 MeV in incident energy, multiplicity 0..4, 32-bin CDFs.
SEC_NUCLEI = ELEMENTS[1:]
SEC_N_EBINS = 25
SEC_EBIN_MEV = 10.0
SEC_N_MULT = 5
SEC_N_CDF = 32

HU_MIN = -1000
HU_MAX = 3000


def _f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32)


def energy_grid() -> np.ndarray:
    """The shared log-spaced energy grid (float64, MeV)."""
    i = np.arange(N_E, dtype=np.float64)
    return E_MIN_MEV * (E_MAX_MEV / E_MIN_MEV) ** (i / (N_E - 1))


# ---------------------------------------------------------------------------
# HU -> material table (stand-in for Schneider et al.; Sec. II.A.1)
# ---------------------------------------------------------------------------

def _normalise(fr):
    fr = np.asarray(fr, dtype=np.float64)
    return fr / fr.sum()


def _water_fractions():
    mh, mo = _MOLAR_MASS["H"], _MOLAR_MASS["O"]
    m = 2 * mh + mo
    fr = np.zeros(7)
    fr[0] = 2 * mh / m
    fr[3] = mo / m
    return fr


def material_table() -> dict:
    """Piecewise HU -> (density, composition) table with 8 bins.

    Bin b covers HU in [hu_lo[b], hu_lo[b+1]) (the last bin ends at HU_MAX);
    density is linear in HU from rho_lo[b] to rho_hi[b] across the bin and the
    composition is constant within it.  The titanium bin is flagged to use its
    own stopping/range table instead of water scaling (Sec. II.A.2).
    Returns float32 arrays (int16 for hu_lo, int32 for own_table).
    """
    rows = [
        # name, hu_lo, rho_lo, rho_hi, I (eV), fractions H C N O P Ca Ti, own
        ("lung", -1000, 0.0012, 0.93, 75.3,
         [0.103, 0.105, 0.031, 0.749, 0.002, 0.0, 0.0], 0),
        ("adipose", -150, 0.93, 0.98, 63.2,
         [0.114, 0.598, 0.007, 0.278, 0.0, 0.0, 0.0], 0),
        ("water", -20, 1.0, 1.0, 75.0, list(_water_fractions()), 0),
        ("soft_tissue", 20, 1.02, 1.10, 74.9,
         [0.102, 0.143, 0.034, 0.708, 0.002, 0.0, 0.0], 0),
        ("spongy_bone", 150, 1.10, 1.40, 80.0,
         [0.085, 0.404, 0.028, 0.367, 0.034, 0.074, 0.0], 0),
        ("cortical_bone", 600, 1.40, 2.20, 106.4,
         [0.034, 0.155, 0.042, 0.435, 0.103, 0.225, 0.0], 0),
        ("dense_bone", 2000, 2.20, 2.90, 110.0,
         [0.034, 0.155, 0.042, 0.435, 0.103, 0.225, 0.0], 0),
        ("titanium", 3000, 4.50, 4.50, 233.0,
         [0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0], 1),
    ]
    names = [r[0] for r in rows]
    hu_lo = np.array([r[1] for r in rows], dtype=np.int16)
    rho_lo = _f32([r[2] for r in rows])
    rho_hi = _f32([r[3] for r in rows])
    i_ev = _f32([r[4] for r in rows])
    frac = np.stack([_normalise(r[5]) for r in rows]).astype(np.float32)
    own = np.array([r[6] for r in rows], dtype=np.int32)
    return {"names": names, "hu_lo": hu_lo, "rho_lo": rho_lo, "rho_hi": rho_hi,
            "mass_frac": frac, "i_ev": i_ev, "own_table": own}


# ---------------------------------------------------------------------------
# Nuclear data: cross sections (Sec. II.A.4-5) and secondary table
# ---------------------------------------------------------------------------

def _threshold_mev(z, a):
    # Coulomb-barrier-like threshold: 7 MeV for 16-O, scaled by Z/A^(1/3).
    return 7.0 * (z / a ** (1.0 / 3.0)) / (8.0 / 16.0 ** (1.0 / 3.0))


def cross_sections() -> tuple[np.ndarray, np.ndarray]:
    """Smooth parametric stand-ins for the tabulated cross sections.

    Returns (sigma_ne, sigma_el), each float32 [7, N_E] in barn on
    energy_grid().  Non-elastic: 0.30 b (A/16)^(2/3) (1 - exp(-(E-E_th)/15))
    above a Coulomb-like threshold, zero for hydrogen (no channel below the
    pion threshold).  Nuclear elastic: a third of the non-elastic magnitude,
    without threshold.  p-p elastic: 22 mb + 350 mb exp(-E/15).
    """
    e = energy_grid()
    ne = np.zeros((7, N_E))
    el = np.zeros((7, N_E))
    for k in range(7):
        a, z = _MASS_NUMBER[k], _CHARGE[k]
        if k == 0:
            el[k] = 0.022 + 0.35 * np.exp(-e / 15.0)
            continue
        scale = 0.30 * (a / 16.0) ** (2.0 / 3.0)
        eth = _threshold_mev(z, a)
        ne[k] = scale * np.clip(1.0 - np.exp(-(e - eth) / 15.0), 0.0, None)
        el[k] = scale / 3.0 * (1.0 - np.exp(-e / 15.0))
    return _f32(ne), _f32(el)


def constant_cross_sections(sigma_ne_barn: float, sigma_el_barn: float = 0.0):
    """Energy-independent cross sections for every nucleus with A >= 2
    (hydrogen gets none): the attenuation special case."""
    ne = np.zeros((7, N_E))
    el = np.zeros((7, N_E))
    ne[1:] = sigma_ne_barn
    el[1:] = sigma_el_barn
    return _f32(ne), _f32(el)


def _cdf_from_weights(w):
    w = np.asarray(w, dtype=np.float64)
    c = np.concatenate([[0.0], np.cumsum(w) / w.sum()])
    c = c.astype(np.float32)
    c[0] = 0.0
    c[-1] = 1.0
    c = np.maximum.accumulate(c)
    return c


def secondary_table(seed: int = 7) -> dict:
    """Seeded synthetic energy/angle table of non-elastic secondary protons.

    For nucleus n (C..Ti) and incident-energy bin j (E in [10j, 10j+10) MeV):
      mult_cdf[n,j,m]  P(number of protons <= m), m = 0..4
      f_local[n,j]     fraction of the incident energy deposited locally
      x_cdf[n,j,:]     CDF of x = E_secondary/E_incident at x = i/32
      mu_cdf[n,j,:]    CDF of cos(theta) at mu = -1 + 2i/32
    Shapes: a forward, high-x knock-out component plus an isotropic low-energy
    evaporation component, perturbed by seeded noise.
    """
    rng = np.random.default_rng(seed)
    nn, nb = len(SEC_NUCLEI), SEC_N_EBINS
    mult = np.zeros((nn, nb, SEC_N_MULT), dtype=np.float32)
    floc = np.zeros((nn, nb), dtype=np.float32)
    xcdf = np.zeros((nn, nb, SEC_N_CDF + 1), dtype=np.float32)
    mucdf = np.zeros((nn, nb, SEC_N_CDF + 1), dtype=np.float32)
    xm = (np.arange(SEC_N_CDF) + 0.5) / SEC_N_CDF
    mum = -1.0 + 2.0 * xm
    for n in range(nn):
        a = _MASS_NUMBER[n + 1]
        for j in range(nb):
            ec = SEC_EBIN_MEV * (j + 0.5)
            mean = (0.2 + 1.6 * ec / E_MAX_MEV) * (1.0 + 0.15 * math.log(a / 16.0))
            mean *= rng.uniform(0.9, 1.1)
            pm = np.array([math.exp(-mean) * mean ** m / math.factorial(m)
                           for m in range(SEC_N_MULT)])
            mult[n, j] = _cdf_from_weights(pm)[1:]
            floc[n, j] = np.float32(np.clip(0.10 + 0.05 * a / 48.0
                                            + rng.uniform(-0.02, 0.02), 0.02, 0.3))
            wko = min(0.9, 0.3 + 0.5 * ec / E_MAX_MEV)
            ko = xm ** 3 * (1.0 - xm) ** 0.8
            ko /= ko.sum()
            ev = np.exp(-xm * ec / 6.0)
            ev /= ev.sum()
            wx = (wko * ko + (1.0 - wko) * ev) * np.clip(
                1.0 + 0.1 * rng.standard_normal(SEC_N_CDF), 0.05, None)
            xcdf[n, j] = _cdf_from_weights(wx)
            kappa = 2.0 + 8.0 * ec / E_MAX_MEV
            fw = np.exp(kappa * (mum - 1.0))
            fw /= fw.sum()
            wmu = (wko * fw + (1.0 - wko) / SEC_N_CDF) * np.clip(
                1.0 + 0.1 * rng.standard_normal(SEC_N_CDF), 0.05, None)
            mucdf[n, j] = _cdf_from_weights(wmu)
    return {"mult_cdf": mult, "f_local": floc, "x_cdf": xcdf, "mu_cdf": mucdf}


def nuclear_data(seed: int = 7, sigma=None) -> dict:
    """Cross sections plus secondary table, in the layout both engines take."""
    ne, el = cross_sections() if sigma is None else sigma
    d = {"sigma_ne": ne, "sigma_el": el}
    d.update(secondary_table(seed))
    return d


# ---------------------------------------------------------------------------
# Phantoms (HU grids, [nz][ny][nx] with x fastest)
# ---------------------------------------------------------------------------

def water_phantom(nx=64, ny=64, nz=128) -> np.ndarray:
    return np.zeros((nz, ny, nx), dtype=np.int16)


def uniform_phantom(hu, nx, ny, nz) -> np.ndarray:
    return np.full((nz, ny, nx), hu, dtype=np.int16)


def ct_phantom(nx=128, ny=128, nz=160, voxel_cm=0.2, seed=2,
               counts=(2, 3, 4), ti_depth_cm=10.0, ti_offset_cm=1.0) -> np.ndarray:
    """Heterogeneous synthetic CT: water background, seeded axis-aligned
    ellipsoids of lung (-800 HU), soft tissue (+40) and cortical bone (+1000)
    painted in that order (semi-axes 1-4 cm), and a 1 cm diameter titanium
    cylinder (+3000 HU) along y at the given depth, offset laterally."""
    rng = np.random.default_rng(seed)
    lx, ly, lz = nx * voxel_cm, ny * voxel_cm, nz * voxel_cm
    xs = (np.arange(nx) + 0.5) * voxel_cm
    ys = (np.arange(ny) + 0.5) * voxel_cm
    zs = (np.arange(nz) + 0.5) * voxel_cm
    hu = np.zeros((nz, ny, nx), dtype=np.int16)
    for count, value in zip(counts, (-800, 40, 1000)):
        for _ in range(count):
            c = rng.uniform([0.15 * lx, 0.15 * ly, 0.1 * lz],
                            [0.85 * lx, 0.85 * ly, 0.9 * lz])
            r = rng.uniform(1.0, 4.0, size=3)
            # evaluate only inside the ellipsoid's bounding box
            i0 = [max(0, int(math.floor((c[a] - r[a]) / voxel_cm)) - 1) for a in range(3)]
            i1 = [min(n, int(math.ceil((c[a] + r[a]) / voxel_cm)) + 1)
                  for a, n in zip(range(3), (nx, ny, nz))]
            q = (((xs[None, None, i0[0]:i1[0]] - c[0]) / r[0]) ** 2
                 + ((ys[None, i0[1]:i1[1], None] - c[1]) / r[1]) ** 2
                 + ((zs[i0[2]:i1[2], None, None] - c[2]) / r[2]) ** 2)
            sub = hu[i0[2]:i1[2], i0[1]:i1[1], i0[0]:i1[0]]
            sub[q <= 1.0] = value
    if ti_depth_cm is not None and ti_depth_cm < lz:
        cx = 0.5 * lx + ti_offset_cm
        q = ((xs[None, None, :] - cx) ** 2 + (zs[:, None, None] - ti_depth_cm) ** 2)
        mask = np.broadcast_to(q <= 0.5 ** 2, hu.shape)
        hu[mask] = HU_MAX
    return hu


def scaled_ct_phantom(nx, ny, nz, seed, voxel_cm=0.2) -> np.ndarray:
    """The ct_phantom recipe with ellipsoid counts scaled by volume."""
    vol = nx * ny * nz / (128 * 128 * 160)
    counts = tuple(max(1, int(round(c * vol))) for c in (2, 3, 4))
    return ct_phantom(nx, ny, nz, voxel_cm, seed, counts)


# ---------------------------------------------------------------------------
# Beam spots: rows (x_cm, y_cm, e_mev, sigma_x_cm, sigma_y_cm, weight)
# ---------------------------------------------------------------------------

def pencil_spot(x_cm, y_cm, e_mev, sigma_cm=0.3, weight=1.0) -> np.ndarray:
    return _f32([[x_cm, y_cm, e_mev, sigma_cm, sigma_cm, weight]])


def hex_points(n, pitch_cm):
    """The n points of a hexagonal lattice (pitch p) nearest the origin,
    ordered by distance then angle."""
    pts = []
    for j in range(-40, 41):
        for i in range(-40, 41):
            x = pitch_cm * (i + 0.5 * j)
            y = pitch_cm * j * math.sqrt(3.0) / 2.0
            pts.append((round(math.hypot(x, y), 9), round(math.atan2(y, x), 9), x, y))
    pts.sort()
    return [(p[2], p[3]) for p in pts[:n]]


def spot_field(center_xy, n_layers=40, n_per_layer=50, e_lo=70.0, e_hi=230.0,
               pitch_cm=0.5, seed=4) -> np.ndarray:
    """Treatment-field stand-in: n_layers energy layers from e_lo to e_hi, each
    with the n_per_layer hexagonal-grid points nearest the centre; spot sigma
    falls linearly from 6 mm (lowest energy) to 3 mm (highest); weights are
    lognormal(0, 0.5)."""
    rng = np.random.default_rng(seed)
    pts = hex_points(n_per_layer, pitch_cm)
    rows = []
    for l in range(n_layers):
        e = e_lo + (e_hi - e_lo) * l / max(1, n_layers - 1)
        sig = 0.1 * (6.0 - 3.0 * (e - e_lo) / (e_hi - e_lo))
        for (x, y) in pts:
            rows.append([center_xy[0] + x, center_xy[1] + y, e, sig, sig, 0.0])
    spots = np.array(rows, dtype=np.float64)
    spots[:, 5] = rng.lognormal(0.0, 0.5, size=len(rows))
    return _f32(spots)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def config_water_pencil(n_histories=100_000):
    """64x64x128 water voxels of 2 mm, one 100 MeV spot (sigma 3 mm)."""
    hu = water_phantom(64, 64, 128)
    spots = pencil_spot(6.4, 6.4, 100.0, 0.3)
    return {"hu": hu, "voxel_cm": (0.2, 0.2, 0.2), "spots": spots,
            "n_histories": n_histories, "seed": 1}


def config_ct_spots(energy_mev, n_histories=1_000_000):
    """128x128x160 heterogeneous CT of 2 mm voxels, one centred spot."""
    hu = ct_phantom(128, 128, 160, 0.2, seed=2)
    spots = pencil_spot(12.8, 12.8, energy_mev, 0.3)
    return {"hu": hu, "voxel_cm": (0.2, 0.2, 0.2), "spots": spots,
            "n_histories": n_histories, "seed": 1}


def config_field(n_histories=10_000_000):
    """256x256x200 CT of 2 mm voxels with a 2000-spot, 40-layer field."""
    hu = scaled_ct_phantom(256, 256, 200, seed=3)
    spots = spot_field((25.6, 25.6), seed=4)
    return {"hu": hu, "voxel_cm": (0.2, 0.2, 0.2), "spots": spots,
            "n_histories": n_histories, "seed": 1}


def random_field(rng, n_spots, center_xy, e_lo=70.0, e_hi=230.0, pitch_cm=0.5):
    """A field of about n_spots spots: a seeded number of energy layers in
    [e_lo, e_hi], each a hexagonal patch of equal size, lognormal weights."""
    n_layers = int(rng.integers(4, 21))
    per = max(1, int(round(n_spots / n_layers)))
    pts = hex_points(per, pitch_cm)
    lo = rng.uniform(e_lo, 0.5 * (e_lo + e_hi))
    hi = rng.uniform(lo + 10.0, e_hi)
    rows = []
    for l in range(n_layers):
        e = lo + (hi - lo) * l / max(1, n_layers - 1)
        sig = 0.1 * (6.0 - 3.0 * (e - e_lo) / (e_hi - e_lo))
        for (x, y) in pts:
            rows.append([center_xy[0] + x, center_xy[1] + y, e, sig, sig, 0.0])
    spots = np.array(rows, dtype=np.float64)
    spots[:, 5] = rng.lognormal(0.0, 0.5, size=len(rows))
    return _f32(spots)


def plan_set(n_plans=16, seed=100, hist_scale=1.0, max_grid=(256, 256, 200), min_grid=(96, 96, 96)):
    """Uneven multi-plan batch: per plan a CT grid between min_grid and
    max_grid (2 mm voxels, the ct_phantom recipe with counts scaled by
    volume), 200-3000 spots (uniform) and 1e6-1e7 histories (log-uniform),
    times hist_scale.  Plan i uses seed + i."""
    plans = []
    for i in range(n_plans):
        rng = np.random.default_rng(seed + i)
        dims = [int(rng.integers(lo, hi + 1)) for lo, hi in zip(min_grid, max_grid)]
        nx, ny, nz = dims
        hu = scaled_ct_phantom(nx, ny, nz, seed=seed + i)
        n_spots = int(rng.integers(200, 3001))
        spots = random_field(rng, n_spots, (0.1 * nx, 0.1 * ny))
        n_hist = int(round(10 ** rng.uniform(6.0, 7.0) * hist_scale))
        plans.append({"hu": hu, "voxel_cm": (0.2, 0.2, 0.2), "spots": spots,
                      "n_histories": max(1, n_hist)})
    return plans


# ---------------------------------------------------------------------------
# Denoiser inputs
# ---------------------------------------------------------------------------

def bf16_bits(a) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); the bit
    patterns as uint16."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16_values(bits) -> np.ndarray:
    """float64 values of bfloat16 bit patterns."""
    return (np.asarray(bits, np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_normal(rng, shape, sd=1.0):
    """Normal samples rounded to bfloat16: (bits uint16, exact float64 values)."""
    bits = bf16_bits(rng.normal(0.0, sd, size=shape).astype(np.float32))
    return bits, bf16_values(bits)


def conv_weights(rng, cin, cout, sd=None):
    """A convolution weight matrix [cout][Kp] (Kp = 27*cin rounded up to 32,
    index tap*cin + ci, zero padding columns) of bfloat16 values."""
    k = (27 * cin + 31) // 32 * 32
    sd = sd if sd is not None else (2.0 / (27 * cin)) ** 0.5
    bits = np.zeros((cout, k), np.uint16)
    bits[:, :27 * cin] = bf16_bits(rng.normal(0.0, sd, size=(cout, 27 * cin)).astype(np.float32))
    return bits, bf16_values(bits)


def training_field(rng, center_xy, e_lo=70.0, e_hi=230.0, pitch_cm=0.5):
    """A small random field for denoiser data: 1-3 energy layers of 10-60
    hexagonal-lattice spots each around a seeded offset from the centre,
    lognormal(0, 0.5) weights."""
    n_layers = int(rng.integers(1, 4))
    rows = []
    cx = center_xy[0] + rng.uniform(-3.0, 3.0)
    cy = center_xy[1] + rng.uniform(-3.0, 3.0)
    for _ in range(n_layers):
        e = rng.uniform(e_lo, e_hi)
        sig = 0.1 * (6.0 - 3.0 * (e - e_lo) / (e_hi - e_lo))
        for (x, y) in hex_points(int(rng.integers(10, 61)), pitch_cm):
            rows.append([cx + x, cy + y, e, sig, sig, 0.0])
    spots = np.array(rows, dtype=np.float64)
    spots[:, 5] = rng.lognormal(0.0, 0.5, size=len(rows))
    return _f32(spots)


def denoiser_case(index, nx=128, ny=128, nz=160):
    """Case `index` of the denoiser data set: a ct_phantom-recipe CT with seed
    1000 + index (2 mm voxels, titanium rod included) and a training_field
    drawn from the same seed."""
    seed = 1000 + index
    rng = np.random.default_rng(seed)
    hu = ct_phantom(nx, ny, nz, 0.2, seed=seed)
    spots = training_field(rng, (0.1 * nx, 0.1 * ny))
    return {"hu": hu, "voxel_cm": (0.2, 0.2, 0.2), "spots": spots}
