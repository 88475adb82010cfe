"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
this module.  It compiles ``liboracle.so`` from ``pmc_oracle.c`` with gcc when
the library is missing or older than its source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pmc_oracle.c")
SRC_INC = os.path.join(HERE, "pmc_oracle_inc.c")
LIB = os.path.join(HERE, "liboracle.so")

NO_STRAGGLE, NO_MCS, NO_NUCLEAR, VAVILOV, MOLIERE = 1, 2, 4, 8, 16
PLAIN_HINGE = 32   # test only: no landing of the second hinge segment on the face
INC = 64           # non-elastic events by the intranuclear cascade and evaporation
INC_SHELLS, INC_MAX_OUT = 15, 96
EJ_NAMES = ("n", "p", "d", "t", "He3", "alpha")


class Nucleus(C.Structure):
    _fields_ = [("z", C.c_int32), ("a", C.c_int32), ("radius_ws", C.c_double), ("diffuseness", C.c_double),
                ("r_out", C.c_double), ("r", C.c_double * (INC_SHELLS + 1)),
                ("rho_p", C.c_double * INC_SHELLS), ("rho_n", C.c_double * INC_SHELLS),
                ("tf_p", C.c_double * INC_SHELLS), ("tf_n", C.c_double * INC_SHELLS)]


class IncResult(C.Structure):
    _fields_ = [("n", C.c_int32), ("kind", C.c_int32 * INC_MAX_OUT), ("stage", C.c_int32 * INC_MAX_OUT),
                ("id", C.c_uint32 * INC_MAX_OUT), ("t", C.c_double * INC_MAX_OUT),
                ("dir", (C.c_double * 3) * INC_MAX_OUT), ("z_res", C.c_int32), ("a_res", C.c_int32),
                ("e_star", C.c_double), ("e_star_sum", C.c_double), ("n_coll", C.c_int32),
                ("n_blocked", C.c_int32), ("attempts", C.c_int32), ("n_esc", C.c_int32),
                ("compound", C.c_int32), ("z_fin", C.c_int32), ("a_fin", C.c_int32),
                ("e_star_fin", C.c_double), ("binding", C.c_double), ("pauli_min", C.c_double)]
MOL_SHAPE = (13, 161)     # [1/B = 1/20 + j (2/9 - 1/20)/12][q = k/8]
VAV_SHAPE = (5, 31, 97)   # [beta^2 = k/10][log10 kappa = -2 + j/10][z = -6 + i/8]
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle (gcc -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(SRC_INC), os.path.getmtime(os.path.join(HERE, "pmc_oracle.h"))):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC",
                               "-shared", "-Wall", "-Wno-unknown-pragmas", SRC, SRC_INC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [("f_mcs", C.c_double), ("s_min_cm", C.c_double), ("k_batches", C.c_int32),
                ("flags", C.c_uint32), ("n_threads", C.c_int32)]


class MaterialTable(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("hu_lo", C.c_void_p), ("rho_lo", C.c_void_p),
                ("rho_hi", C.c_void_p), ("mass_frac", C.c_void_p), ("i_ev", C.c_void_p),
                ("own_table", C.c_void_p)]


class NuclearData(C.Structure):
    _fields_ = [("sigma_ne", C.c_void_p), ("sigma_el", C.c_void_p), ("mult_cdf", C.c_void_p),
                ("f_local", C.c_void_p), ("x_cdf", C.c_void_p), ("mu_cdf", C.c_void_p)]


class Summary(C.Structure):
    _fields_ = [("incident", C.c_double), ("deposited", C.c_double), ("escaped", C.c_double),
                ("neutral", C.c_double), ("histories", C.c_uint64), ("steps", C.c_uint64),
                ("secondaries", C.c_uint64), ("n_elastic", C.c_uint64),
                ("n_nonelastic", C.c_uint64), ("interactions", (C.c_uint64 * 7) * 2),
                ("total_weight", C.c_double), ("wall_s", C.c_double), ("threads", C.c_int32),
                ("n_short_steps", C.c_uint64)]


class Diag(C.Structure):
    _fields_ = [("uid_begin", C.c_uint64), ("uid_end", C.c_uint64), ("batch_tally", C.c_void_p),
                ("first_nuclear_z_cm", C.c_void_p), ("escape_log", C.c_void_p),
                ("escape_cap", C.c_uint64), ("escape_count", C.c_uint64)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(LIB)
            d, u32p = C.c_double, C.POINTER(C.c_uint32)
            L.oracle_create.argtypes = [C.POINTER(C.c_void_p), C.POINTER(Params)]
            L.oracle_destroy.argtypes = [C.c_void_p]
            L.oracle_load_physics.argtypes = [C.c_void_p, C.POINTER(NuclearData)]
            L.oracle_load_geometry.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int,
                                               C.c_float, C.c_float, C.c_float,
                                               C.POINTER(MaterialTable)]
            L.oracle_run_spots.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_uint64, C.c_uint64,
                                           C.c_void_p, C.c_void_p, C.POINTER(Summary),
                                           C.POINTER(Diag)]
            L.oracle_run_spots_let.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_uint64,
                                               C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p,
                                               C.POINTER(Summary), C.POINTER(Diag)]
            L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
            L.oracle_philox4x32_10.restype = None
            L.oracle_u01.argtypes = [C.c_uint32]
            for name, args in [("oracle_normal_quantile", [d]),
                               ("oracle_bethe_bloch", [d, d, d]),
                               ("oracle_stopping_power", [d, d, d]),
                               ("oracle_bb_peak_energy", [d, d]),
                               ("oracle_radiation_length", [C.POINTER(C.c_double)]),
                               ("oracle_water_z_over_a", []),
                               ("oracle_range", [C.c_void_p, C.c_int, d]),
                               ("oracle_energy_at_range", [C.c_void_p, C.c_int, d]),
                               ("oracle_highland_theta0", [d, d, d, d]),
                               ("oracle_straggling_variance", [d, d, d, d]),
                               ("oracle_sigma", [C.c_void_p, C.c_int, C.c_int, d]),
                               ("oracle_u01", [C.c_uint32])]:
                f = getattr(L, name)
                f.argtypes = args
                f.restype = d
            for name, args in [("oracle_vavilov_cdf", [d, d, d]),
                               ("oracle_vavilov_kappa", [d, d, d, d]),
                               ("oracle_vavilov_quantile", [C.c_void_p, d, d, d])]:
                f = getattr(L, name)
                f.argtypes = args
                f.restype = d
            L.oracle_vavilov_table.argtypes = [C.c_void_p]
            L.oracle_moliere_f.argtypes = [C.c_int, d]
            L.oracle_moliere_f.restype = d
            L.oracle_moliere_survival.argtypes = [d, d]
            L.oracle_moliere_survival.restype = d
            L.oracle_moliere_table.argtypes = [C.c_void_p]
            L.oracle_moliere_theta.argtypes = [C.c_void_p, C.c_int, d, d, d, d, C.POINTER(d)]
            L.oracle_moliere_theta.restype = d
            L.oracle_material_info.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_double)]
            L.oracle_elastic_sample.argtypes = [C.c_int, d, d, d, C.POINTER(C.c_double)]
            L.oracle_secondary_sample.argtypes = [C.c_void_p, C.c_int, d, C.c_uint64, C.c_uint32,
                                                  C.c_uint64, d, C.POINTER(C.c_int),
                                                  C.POINTER(C.c_double), C.POINTER(C.c_double),
                                                  C.POINTER(C.c_double)]
            L.oracle_rotate.argtypes = [C.POINTER(C.c_double), d, d, d]
            L.oracle_rotate.restype = None
            L.oracle_inc_nucleus.argtypes = [C.c_int, C.POINTER(Nucleus)]
            L.oracle_nn_sigma_mb.argtypes = [C.c_int, d]
            L.oracle_nn_sigma_mb.restype = d
            L.oracle_nn_slope.argtypes = [d]
            L.oracle_nn_slope.restype = d
            L.oracle_inc_event.argtypes = [C.c_int, d, C.c_uint64, C.c_uint64, C.c_uint32, C.c_int,
                                           C.POINTER(IncResult)]
            L.oracle_evaporate.argtypes = [C.c_int, C.c_int, d, C.c_uint64, C.c_uint64, C.c_uint32,
                                           C.POINTER(IncResult)]
            L.oracle_binding_energy.argtypes = [C.c_int, C.c_int]
            L.oracle_binding_energy.restype = d
            L.oracle_evap_width.argtypes = [C.c_int, C.c_int, d, C.c_int, C.POINTER(d), C.POINTER(d)]
            L.oracle_evap_width.restype = d
            L.oracle_fermi_momentum.argtypes = [d, C.POINTER(d), C.POINTER(d)]
            L.oracle_fermi_momentum.restype = None
            L.oracle_inc_refract.argtypes = [d, d, d, C.POINTER(d), C.POINTER(d), C.POINTER(d)]
            L.oracle_nn_collide.argtypes = [C.POINTER(d), C.POINTER(d), d, d, C.POINTER(d), C.POINTER(d)]
            L.oracle_nn_collide.restype = None
            _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def philox(key, ctr):
    """Philox4x32-10 block for key (2 u32) and counter (4 u32)."""
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    o = (C.c_uint32 * 4)()
    lib().oracle_philox4x32_10(k, c, o)
    return list(o)


def elastic_sample(mass_number, t_mev, u_comp, u_t):
    out = (C.c_double * 7)()
    lib().oracle_elastic_sample(int(mass_number), t_mev, u_comp, u_t, out)
    return list(out)


def vavilov_cdf(kappa, beta2, x):
    """P(X <= x), X = (energy loss - mean) / T_max in Vavilov's model."""
    return lib().oracle_vavilov_cdf(float(kappa), float(beta2), float(x))


def vavilov_table():
    """Quantile nodes G of the standardised Vavilov variable, VAV_SHAPE."""
    out = np.zeros(VAV_SHAPE, dtype=np.float64)
    rc = lib().oracle_vavilov_table(_ptr(out))
    if rc:
        raise ValueError("oracle_vavilov_table failed: %d" % rc)
    return out


def moliere_f(n, v):
    """Bethe's f0, f1, f2 of the Molière expansion at reduced angle v."""
    return lib().oracle_moliere_f(int(n), float(v))


def moliere_survival(x, v):
    """P(V > v) of the reduced angle for 1/B = x."""
    return lib().oracle_moliere_survival(float(x), float(v))


def moliere_table():
    out = np.zeros(MOL_SHAPE, dtype=np.float64)
    if lib().oracle_moliere_table(_ptr(out)):
        raise ValueError("oracle_moliere_table failed")
    return out


def vavilov_kappa(t_mev, s_cm, rho, za):
    return lib().oracle_vavilov_kappa(float(t_mev), float(s_cm), float(rho), float(za))


def rotate(d, ct, st, phi_rev):
    arr = (C.c_double * 3)(*d)
    lib().oracle_rotate(arr, ct, st, phi_rev)
    return list(arr)


def inc_nucleus(element):
    """The cascade's nucleus for element 1..6 (C, N, O, P, Ca, Ti) as a dict."""
    nu = Nucleus()
    if lib().oracle_inc_nucleus(int(element), C.byref(nu)):
        raise ValueError("bad element")
    out = {"z": nu.z, "a": nu.a, "radius_ws": nu.radius_ws, "diffuseness": nu.diffuseness, "r_out": nu.r_out}
    for k in ("r", "rho_p", "rho_n", "tf_p", "tf_n"):
        out[k] = np.array(getattr(nu, k)[:], dtype=np.float64)
    return out


def _inc_dict(r):
    n = r.n
    out = {k: getattr(r, k) for k in ("z_res", "a_res", "e_star", "e_star_sum", "n_coll", "n_blocked",
                                       "attempts", "n_esc", "compound", "z_fin", "a_fin", "e_star_fin",
                                       "binding", "pauli_min")}
    out.update(kind=np.array(r.kind[:n]), stage=np.array(r.stage[:n]), id=np.array(r.id[:n]),
               t=np.array(r.t[:n]), dir=np.array([list(r.dir[i]) for i in range(n)]).reshape(n, 3))
    return out


def inc_event(element, t_mev, seed, uid, ks=0, evaporate=True):
    """One non-elastic event (cascade, then evaporation) as a dict."""
    r = IncResult()
    if lib().oracle_inc_event(int(element), float(t_mev), int(seed), int(uid), int(ks), int(evaporate),
                              C.byref(r)):
        raise ValueError("oracle_inc_event failed")
    return _inc_dict(r)


def evaporate(z, a, e_star, seed, uid, ks=0):
    r = IncResult()
    lib().oracle_evaporate(int(z), int(a), float(e_star), int(seed), int(uid), int(ks), C.byref(r))
    return _inc_dict(r)


def evap_width(z, a, e_star, kind):
    """(relative width, separation energy, Coulomb barrier) of ejectile kind."""
    s, v = C.c_double(), C.c_double()
    w = lib().oracle_evap_width(int(z), int(a), float(e_star), int(kind), C.byref(s), C.byref(v))
    return w, s.value, v.value


def fermi_momentum(p_fermi, u):
    uu = (C.c_double * 3)(*u)
    p = (C.c_double * 3)()
    lib().oracle_fermi_momentum(float(p_fermi), uu, p)
    return list(p)


def inc_refract(t, v_from, v_to, x, d):
    """(crossed, new kinetic energy, new direction) at a shell boundary."""
    xx = (C.c_double * 3)(*x)
    dd = (C.c_double * 3)(*d)
    to = C.c_double()
    crossed = lib().oracle_inc_refract(float(t), float(v_from), float(v_to), xx, dd, C.byref(to))
    return crossed, to.value, list(dd)


def nn_collide(p1, p2, u_t, u_phi):
    a = (C.c_double * 3)(*p1)
    b = (C.c_double * 3)(*p2)
    o1, o2 = (C.c_double * 3)(), (C.c_double * 3)()
    lib().oracle_nn_collide(a, b, float(u_t), float(u_phi), o1, o2)
    return list(o1), list(o2)


def radiation_length(w):
    arr = (C.c_double * 7)(*[float(x) for x in w])
    return lib().oracle_radiation_length(arr)


class Oracle:
    """One oracle context: physics tables + one geometry."""

    def __init__(self, f_mcs=1.07, s_min_cm=1e-4, k_batches=10, flags=0, n_threads=0):
        L = lib()
        self._p = Params(f_mcs, s_min_cm, k_batches, flags, n_threads)
        h = C.c_void_p()
        rc = L.oracle_create(C.byref(h), C.byref(self._p))
        if rc:
            raise ValueError("oracle_create failed: %d" % rc)
        self.h = h
        self.k_batches = k_batches
        self._keep = []
        self.shape = None

    def close(self):
        if self.h:
            lib().oracle_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_physics(self, nd: dict):
        arrs = [np.ascontiguousarray(nd[k], dtype=np.float32)
                for k in ("sigma_ne", "sigma_el", "mult_cdf", "f_local", "x_cdf", "mu_cdf")]
        self._phys = arrs
        s = NuclearData(*[_ptr(a) for a in arrs])
        rc = lib().oracle_load_physics(self.h, C.byref(s))
        if rc:
            raise ValueError("oracle_load_physics failed: %d" % rc)

    def load_geometry(self, hu, voxel_cm, mt: dict):
        hu = np.ascontiguousarray(hu, dtype=np.int16)
        nz, ny, nx = hu.shape
        arrs = [np.ascontiguousarray(mt["hu_lo"], dtype=np.int16),
                np.ascontiguousarray(mt["rho_lo"], dtype=np.float32),
                np.ascontiguousarray(mt["rho_hi"], dtype=np.float32),
                np.ascontiguousarray(mt["mass_frac"], dtype=np.float32),
                np.ascontiguousarray(mt["i_ev"], dtype=np.float32),
                np.ascontiguousarray(mt["own_table"], dtype=np.int32)]
        t = MaterialTable(len(arrs[0]), *[_ptr(a) for a in arrs])
        rc = lib().oracle_load_geometry(self.h, _ptr(hu), nx, ny, nz, float(voxel_cm[0]),
                                        float(voxel_cm[1]), float(voxel_cm[2]), C.byref(t))
        if rc:
            raise ValueError("oracle_load_geometry failed: %d" % rc)
        self.shape = (nz, ny, nx)

    def run_spots(self, spots, n_histories, seed, batch_tally=False, first_nuclear=False,
                  escape_cap=0, uid_range=None, let=False):
        """Dose, variance and summary; with let=True also the dose-averaged
        LET per voxel in keV/um (key "let")."""
        spots = np.ascontiguousarray(spots, dtype=np.float32).reshape(-1, 6)
        dose = np.zeros(self.shape, dtype=np.float64)
        var = np.zeros(self.shape, dtype=np.float64)
        s = Summary()
        dg = Diag()
        out = {}
        if uid_range is not None:
            dg.uid_begin, dg.uid_end = int(uid_range[0]), int(uid_range[1])
        if batch_tally:
            bt = np.zeros(self.shape + (self.k_batches,), dtype=np.float64)
            dg.batch_tally = _ptr(bt)
            out["batch_tally"] = bt
        if first_nuclear:
            fz = np.zeros(int(n_histories), dtype=np.float64)
            dg.first_nuclear_z_cm = _ptr(fz)
            out["first_nuclear_z"] = fz
        if escape_cap:
            el = np.zeros((int(escape_cap), 8), dtype=np.float64)
            dg.escape_log = _ptr(el)
            dg.escape_cap = int(escape_cap)
        if let:
            lt = np.zeros(self.shape, dtype=np.float64)
            out["let"] = lt
            rc = lib().oracle_run_spots_let(self.h, _ptr(spots), len(spots), int(n_histories),
                                            int(seed), _ptr(dose), _ptr(var), _ptr(lt),
                                            C.byref(s), C.byref(dg))
        else:
            rc = lib().oracle_run_spots(self.h, _ptr(spots), len(spots), int(n_histories),
                                        int(seed), _ptr(dose), _ptr(var), C.byref(s), C.byref(dg))
        if rc:
            raise ValueError("oracle_run_spots failed: %d" % rc)
        if escape_cap:
            out["escapes"] = el[:min(int(dg.escape_count), int(escape_cap))]
        summ = {f[0]: getattr(s, f[0]) for f in Summary._fields_ if f[0] != "interactions"}
        summ["interactions"] = np.array([[s.interactions[a][e] for e in range(7)]
                                         for a in range(2)], dtype=np.int64)
        out.update(dose=dose, var=var, summary=summ)
        return out

    # ---- pieces for pins ----
    def moliere_theta(self, material, t_mev, rho, s_cm, u):
        """(polar angle, B) of the transport's Molière draw (flags MOLIERE);
        angle NaN and B 0 where the step keeps Highland."""
        b = C.c_double()
        th = lib().oracle_moliere_theta(self.h, int(material), float(t_mev), float(rho), float(s_cm),
                                        float(u), C.byref(b))
        return th, b.value

    def vavilov_quantile(self, kappa, beta2, z):
        """The transport's Vavilov draw for normal score z (flags VAVILOV)."""
        return lib().oracle_vavilov_quantile(self.h, float(kappa), float(beta2), float(z))

    def range(self, t_mev, table=0):
        return lib().oracle_range(self.h, table, float(t_mev))

    def energy_at_range(self, r, table=0):
        return lib().oracle_energy_at_range(self.h, table, float(r))

    def material_info(self, m):
        out = (C.c_double * 6)()
        if lib().oracle_material_info(self.h, m, out):
            raise ValueError("bad material index")
        keys = ("z_over_a", "i_ev", "f", "x0_g_cm2", "own", "nuclei_per_g")
        return dict(zip(keys, list(out)))

    def sigma(self, process, element, t_mev):
        return lib().oracle_sigma(self.h, process, element, float(t_mev))

    def secondary_sample(self, element, t_mev, uid, k, seed, u_mult):
        n = C.c_int()
        e = (C.c_double * 4)()
        mu = (C.c_double * 4)()
        fl = C.c_double()
        lib().oracle_secondary_sample(self.h, element, t_mev, uid, k, seed, u_mult, C.byref(n),
                                      e, mu, C.byref(fl))
        return n.value, list(e)[:n.value], list(mu)[:n.value], fl.value
