"""Thin ctypes binding of the engine's C ABI (``include/pmc.h``).

Function names match the C entry points; this module only marshals
arguments.  Every step of the transport runs in the HIP library
``libpmc.so`` next to this file; importing fails loudly when it is missing.
PyTorch is used only for device buffers and streams (``pmc_run_spots_dev``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmc.so")

PMC_OK, PMC_ERR_ARG, PMC_ERR_RANGE, PMC_ERR_NOMEM = 0, -1, -2, -3
PMC_ERR_DEVICE, PMC_ERR_QUEUE_OVERFLOW, PMC_ERR_STATE = -4, -5, -6
PMC_NO_STRAGGLE, PMC_NO_MCS, PMC_NO_NUCLEAR, PMC_VAVILOV, PMC_MOLIERE, PMC_INC = 1, 2, 4, 8, 16, 64
INC_MAX_OUT = 96   # emitted particles per cascade event
MOL_SHAPE = (13, 161)     # [1/B = 1/20 + j (2/9 - 1/20)/12][q = k/8]
VAV_SHAPE = (5, 31, 97)   # [beta^2 = k/10][log10 kappa = -2 + j/10][z = -6 + i/8]

# every symbol include/pmc.h declares
EXPORTS = ("pmc_default_params", "pmc_create", "pmc_destroy", "pmc_last_error",
           "pmc_load_physics", "pmc_load_geometry", "pmc_run_spots", "pmc_run_spots_dev",
           "pmc_inspect_tables", "pmc_atomic_probe", "pmc_load_geometry_slot", "pmc_run_plans",
           "pmc_geometry_density", "pmc_version", "pmc_run_spots_let", "pmc_run_spots_let_dev",
           "pmc_vavilov_table", "pmc_moliere_table", "pmc_plan_launch", "pmc_roofline_replay",
           "pmc_stream_probe", "pmc_inc_events", "pmc_inc_nucleus", "pmc_inc_width")


class PMCError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("pmc status %d: %s" % (status, message))
        self.status = status


class pmc_params(C.Structure):
    _fields_ = [("f_mcs", C.c_double), ("s_min_cm", C.c_double), ("k_batches", C.c_int32),
                ("flags", C.c_uint32), ("queue_capacity", C.c_uint32),
                ("block_threads", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("refill_lanes", C.c_int32), ("batch_events", C.c_int32),
                ("tally_cache", C.c_int32), ("epoch_steps", C.c_int32),
                ("cache_probes", C.c_int32), ("claim_run_log2", C.c_int32),
                ("local_queue", C.c_int32)]


class pmc_spot(C.Structure):
    _fields_ = [("x_cm", C.c_float), ("y_cm", C.c_float), ("e_mev", C.c_float),
                ("sigma_x_cm", C.c_float), ("sigma_y_cm", C.c_float), ("weight", C.c_float)]


class pmc_material_table(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("hu_lo", C.c_void_p), ("rho_lo", C.c_void_p),
                ("rho_hi", C.c_void_p), ("mass_frac", C.c_void_p), ("i_ev", C.c_void_p),
                ("own_table", C.c_void_p)]


class pmc_nuclear_data(C.Structure):
    _fields_ = [("sigma_ne_barn", C.c_void_p), ("sigma_el_barn", C.c_void_p),
                ("mult_cdf", C.c_void_p), ("f_local", C.c_void_p), ("x_cdf", C.c_void_p),
                ("mu_cdf", C.c_void_p)]


class pmc_summary(C.Structure):
    _fields_ = [("incident", C.c_double), ("deposited", C.c_double), ("escaped", C.c_double),
                ("neutral", C.c_double), ("overflow", C.c_double), ("histories", C.c_uint64),
                ("steps", C.c_uint64), ("secondaries", C.c_uint64), ("n_elastic", C.c_uint64),
                ("n_nonelastic", C.c_uint64), ("n_overflow", C.c_uint64),
                ("n_short_steps", C.c_uint64), ("tally_atomics", C.c_uint64),
                ("total_weight", C.c_double), ("device_ms", C.c_double),
                ("transport_ms", C.c_double), ("generations", C.c_int32),
                ("launches", C.c_int32), ("global_atomics", C.c_uint64),
                ("block_threads", C.c_int32), ("grid_blocks", C.c_int32),
                ("cache_slots", C.c_int32), ("epoch_steps", C.c_int32),
                ("cache_flush_atomics", C.c_uint64), ("refill_lanes", C.c_int32),
                ("batch_events", C.c_int32), ("first_launch_ms", C.c_double),
                ("inc_events", C.c_uint64), ("inc_secondaries", C.c_uint64),
                ("inc_collisions", C.c_uint64), ("inc_ms", C.c_double)]


class pmc_inc_result(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("n_out", "n_coll", "n_blocked", "attempts", "n_esc", "compound",
                                         "z_res", "a_res", "z_fin", "a_fin", "n_flights", "reserved")] + [
        (n, C.c_double) for n in ("e_star", "e_star_sum", "e_star_fin", "binding")]


class pmc_inc_particle(C.Structure):
    _fields_ = [("kind", C.c_int32), ("stage", C.c_int32), ("id", C.c_uint32), ("reserved", C.c_int32),
                ("t_mev", C.c_double), ("dir", C.c_double * 3)]


class pmc_launch_query(C.Structure):
    _fields_ = [("block_threads", C.c_int32), ("grid_blocks", C.c_int32), ("n_plans", C.c_int32),
                ("batched", C.c_int32), ("score_let", C.c_int32), ("k_batches", C.c_int32),
                ("n_mat", C.c_int32), ("tally_cache", C.c_int32), ("local_queue", C.c_int32),
                ("n_spots", C.c_int32), ("queue_capacity", C.c_uint64), ("n_histories", C.c_uint64),
                ("max_plan_histories", C.c_uint64), ("max_nvox", C.c_uint64)]


class pmc_launch_layout(C.Structure):
    _fields_ = [("lds_bytes", C.c_uint64)] + [(n, C.c_int32) for n in (
        "blob_words", "plan_desc_off", "cache_off", "key_off", "num_off", "ctl_off", "args_off",
        "ledger_off", "counter_off", "end_words", "cache_slots", "key_words", "tally_planes",
        "local_queue_cap", "args_bytes", "reserved")] + [
        ("queue_cap", C.c_uint64), ("local_queue_words", C.c_uint64), ("claim_words", C.c_uint64),
        ("order_words", C.c_uint64)]


class pmc_replay_result(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("transport_ms", "trace_only_ms", "gather_ms", "atomic_ms",
                                          "cached_atomic_ms", "combined_ms")] + [
        (n, C.c_uint64) for n in ("steps", "steps_traced", "deposits", "trace_iters")] + [
        (n, C.c_int32) for n in ("grid_blocks", "block_threads", "cache_slots", "epoch_steps")]


class pmc_plan(C.Structure):
    _fields_ = [("geometry_id", C.c_int32), ("n_spots", C.c_int32), ("spots", C.c_void_p),
                ("n_histories", C.c_uint64), ("d_dose", C.c_void_p), ("d_var", C.c_void_p),
                ("summary", C.c_void_p), ("d_let", C.c_void_p)]


_lib = None
# voxel count of every loaded geometry, per (context, geometry id): the C calls
# take bare device pointers, so the binding checks tensor sizes against it
_geom_numel = {}


def _need_numel(ctx, gid, t, name):
    want = _geom_numel.get((ctx.value if hasattr(ctx, "value") else ctx, int(gid)))
    if want is None:
        raise ValueError("no geometry %d is loaded in this context" % gid)
    if t.numel() != want:
        raise ValueError("%s has %d elements, geometry %d has %d voxels" % (name, t.numel(), gid, want))


def lib():
    """Load libpmc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpmc.so is not built: run __graft_entry__.build()")
        # PyTorch ships its own HIP runtime; load it first so that this
        # library binds to the same runtime (one HIP runtime per process)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i32, u64 = C.c_void_p, C.c_int, C.c_uint64
        L.pmc_default_params.argtypes = [C.POINTER(pmc_params)]
        L.pmc_create.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(pmc_params)]
        L.pmc_destroy.argtypes = [vp]
        L.pmc_last_error.argtypes = [vp]
        L.pmc_last_error.restype = C.c_char_p
        L.pmc_load_physics.argtypes = [vp, C.POINTER(pmc_nuclear_data)]
        L.pmc_load_geometry.argtypes = [vp, vp, i32, i32, i32, C.c_float, C.c_float, C.c_float,
                                        C.POINTER(pmc_material_table)]
        L.pmc_run_spots.argtypes = [vp, vp, i32, u64, u64, vp, vp, C.POINTER(pmc_summary)]
        L.pmc_run_spots_dev.argtypes = [vp, vp, i32, u64, u64, vp, vp, vp, C.POINTER(pmc_summary)]
        L.pmc_run_spots_let.argtypes = [vp, vp, i32, u64, u64, vp, vp, vp, C.POINTER(pmc_summary)]
        L.pmc_run_spots_let_dev.argtypes = [vp, vp, i32, u64, u64, vp, vp, vp, vp,
                                            C.POINTER(pmc_summary)]
        L.pmc_inspect_tables.argtypes = [vp, vp, vp, vp, vp, vp]
        L.pmc_atomic_probe.argtypes = [vp, u64, vp, C.POINTER(C.c_double)]
        L.pmc_load_geometry_slot.argtypes = [vp, C.POINTER(C.c_int), vp, i32, i32, i32, C.c_float,
                                             C.c_float, C.c_float, C.POINTER(pmc_material_table)]
        L.pmc_run_plans.argtypes = [vp, C.POINTER(pmc_plan), i32, u64, vp]
        L.pmc_geometry_density.argtypes = [vp, i32, vp, vp]
        L.pmc_vavilov_table.argtypes = [vp, C.c_int32]
        L.pmc_moliere_table.argtypes = [vp, C.c_int32]
        L.pmc_plan_launch.argtypes = [C.POINTER(pmc_launch_query), C.POINTER(pmc_launch_layout), C.c_char_p,
                                      C.c_int32]
        L.pmc_roofline_replay.argtypes = [vp, vp, i32, u64, u64, vp, C.POINTER(pmc_replay_result)]
        L.pmc_stream_probe.argtypes = [vp, u64, vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.pmc_inc_events.argtypes = [vp, vp, vp, vp, vp, C.c_int32, u64, C.c_int32, vp, vp]
        L.pmc_inc_nucleus.argtypes = [C.c_int32, vp, C.c_int32]
        L.pmc_inc_width.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_int32, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]
        L.pmc_version.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("pmc_last_error", "pmc_version", "pmc_inc_width"):
                getattr(L, name).restype = C.c_int
        L.pmc_inc_width.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a):
    return C.c_void_p(a.ctypes.data)


def _check(ctx, status):
    if status != PMC_OK:
        raise PMCError(status, pmc_last_error(ctx))


def pmc_version() -> str:
    return lib().pmc_version().decode()


def pmc_last_error(ctx=None) -> str:
    return lib().pmc_last_error(ctx).decode()


def pmc_default_params(**overrides) -> pmc_params:
    p = pmc_params()
    lib().pmc_default_params(C.byref(p))
    names = {f[0] for f in pmc_params._fields_}
    for k, v in overrides.items():
        if k not in names:
            raise ValueError("unknown engine parameter %r" % k)
        setattr(p, k, v)
    return p


def pmc_create(device: int = 0, params: pmc_params | None = None):
    h = C.c_void_p()
    st = lib().pmc_create(C.byref(h), int(device), C.byref(params) if params is not None else None)
    _check(None, st)
    return h


def pmc_destroy(ctx):
    cv = getattr(ctx, "value", ctx)
    for key in [k for k in _geom_numel if k[0] == cv]:
        del _geom_numel[key]
    lib().pmc_destroy(ctx)


def pmc_load_physics(ctx, nd: dict):
    arrs = [np.ascontiguousarray(nd[k], dtype=np.float32)
            for k in ("sigma_ne", "sigma_el", "mult_cdf", "f_local", "x_cdf", "mu_cdf")]
    s = pmc_nuclear_data(*[a.ctypes.data for a in arrs])
    _check(ctx, lib().pmc_load_physics(ctx, C.byref(s)))


def pmc_load_geometry(ctx, hu, voxel_cm, mt: dict):
    hu = np.ascontiguousarray(hu, dtype=np.int16)
    nz, ny, nx = hu.shape
    arrs = _material_arrays(mt)
    t = pmc_material_table(len(arrs[0]), *[a.ctypes.data for a in arrs])
    _check(ctx, lib().pmc_load_geometry(ctx, _ptr(hu), nx, ny, nz, float(voxel_cm[0]),
                                        float(voxel_cm[1]), float(voxel_cm[2]), C.byref(t)))
    _geom_numel[(ctx.value, 0)] = nx * ny * nz
    return (nz, ny, nx)


def _material_arrays(mt):
    return [np.ascontiguousarray(mt["hu_lo"], dtype=np.int16),
            np.ascontiguousarray(mt["rho_lo"], dtype=np.float32),
            np.ascontiguousarray(mt["rho_hi"], dtype=np.float32),
            np.ascontiguousarray(mt["mass_frac"], dtype=np.float32),
            np.ascontiguousarray(mt["i_ev"], dtype=np.float32),
            np.ascontiguousarray(mt["own_table"], dtype=np.int32)]


def pmc_load_geometry_slot(ctx, hu, voxel_cm, mt: dict) -> int:
    """Load a further geometry; returns its slot id."""
    hu = np.ascontiguousarray(hu, dtype=np.int16)
    nz, ny, nx = hu.shape
    arrs = _material_arrays(mt)
    t = pmc_material_table(len(arrs[0]), *[a.ctypes.data for a in arrs])
    gid = C.c_int()
    _check(ctx, lib().pmc_load_geometry_slot(ctx, C.byref(gid), _ptr(hu), nx, ny, nz,
                                             float(voxel_cm[0]), float(voxel_cm[1]),
                                             float(voxel_cm[2]), C.byref(t)))
    _geom_numel[(ctx.value, gid.value)] = nx * ny * nz
    return gid.value


def pmc_run_plans(ctx, plans, seed, stream=None):
    """Batched run.  plans: list of dicts with geometry_id, spots, n_histories,
    d_dose (and optional d_var, d_let) torch float64 device tensors.  Returns
    the per-plan summaries."""
    import torch
    arr = (pmc_plan * len(plans))()
    keep, sums = [], []
    for i, p in enumerate(plans):
        sp = _spots(p["spots"])
        keep.append(sp)
        d = p["d_dose"]
        if d.dtype != torch.float64 or not d.is_cuda or not d.is_contiguous():
            raise ValueError("d_dose must be a contiguous float64 device tensor")
        _need_numel(ctx, p["geometry_id"], d, "d_dose")
        opt = {}
        for name in ("d_var", "d_let"):
            v = p.get(name)
            if v is not None:
                if v.dtype != torch.float64 or not v.is_cuda or not v.is_contiguous():
                    raise ValueError("%s must be a contiguous float64 device tensor" % name)
                _need_numel(ctx, p["geometry_id"], v, name)
                opt[name] = v.data_ptr()
        sm = pmc_summary()
        sums.append(sm)
        arr[i] = pmc_plan(int(p["geometry_id"]), len(sp), sp.ctypes.data, int(p["n_histories"]),
                          d.data_ptr(), opt.get("d_var"), C.addressof(sm), opt.get("d_let"))
    if stream is None:
        stream = torch.cuda.current_stream()
    handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    _check(ctx, lib().pmc_run_plans(ctx, arr, len(plans), int(seed), C.c_void_p(handle)))
    return [summary_dict(s) for s in sums]


def summary_dict(s: pmc_summary) -> dict:
    return {f[0]: getattr(s, f[0]) for f in pmc_summary._fields_}


def _spots(spots):
    return np.ascontiguousarray(np.asarray(spots, dtype=np.float32).reshape(-1, 6))


def pmc_run_spots(ctx, spots, n_histories, seed, shape):
    """Host-buffer run: returns (dose, var, summary)."""
    sp = _spots(spots)
    dose = np.zeros(shape, np.float64)
    var = np.zeros(shape, np.float64)
    s = pmc_summary()
    st = lib().pmc_run_spots(ctx, _ptr(sp), len(sp), int(n_histories), int(seed), _ptr(dose),
                             _ptr(var), C.byref(s))
    _check(ctx, st)
    return dose, var, summary_dict(s)


def pmc_run_spots_let(ctx, spots, n_histories, seed, shape):
    """Host-buffer run with dose-averaged LET: returns (dose, var, let in
    keV/um, summary)."""
    sp = _spots(spots)
    dose = np.zeros(shape, np.float64)
    var = np.zeros(shape, np.float64)
    let = np.zeros(shape, np.float64)
    s = pmc_summary()
    st = lib().pmc_run_spots_let(ctx, _ptr(sp), len(sp), int(n_histories), int(seed), _ptr(dose),
                                 _ptr(var), _ptr(let), C.byref(s))
    _check(ctx, st)
    return dose, var, let, summary_dict(s)


def pmc_run_spots_let_dev(ctx, spots, n_histories, seed, d_dose, d_let, d_var=None, stream=None):
    """As pmc_run_spots_dev, with LET_d (keV/um) into the float64 device
    tensor d_let of the geometry's voxel count."""
    import torch
    sp = _spots(spots)
    for name, t in (("d_dose", d_dose), ("d_let", d_let), ("d_var", d_var)):
        if t is None and name == "d_var":
            continue
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("%s must be a contiguous float64 device tensor" % name)
        _need_numel(ctx, 0, t, name)
    if stream is None:
        stream = torch.cuda.current_stream(d_dose.device)
    handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    s = pmc_summary()
    st = lib().pmc_run_spots_let_dev(ctx, _ptr(sp), len(sp), int(n_histories), int(seed),
                                     C.c_void_p(d_dose.data_ptr()),
                                     C.c_void_p(d_var.data_ptr()) if d_var is not None else None,
                                     C.c_void_p(d_let.data_ptr()), C.c_void_p(handle), C.byref(s))
    _check(ctx, st)
    return summary_dict(s)


def pmc_run_spots_dev(ctx, spots, n_histories, seed, d_dose, d_var=None, stream=None):
    """Device-buffer run into torch tensors (float64, nz*ny*nx elements) on
    ``stream`` (a torch.cuda.Stream or raw handle; None = current stream)."""
    import torch
    sp = _spots(spots)
    if d_dose.dtype != torch.float64 or not d_dose.is_cuda or not d_dose.is_contiguous():
        raise ValueError("d_dose must be a contiguous float64 device tensor")
    if d_var is not None and (d_var.dtype != torch.float64 or not d_var.is_contiguous()
                              or not d_var.is_cuda or d_var.numel() != d_dose.numel()):
        raise ValueError("d_var must match d_dose")
    _need_numel(ctx, 0, d_dose, "d_dose")
    if stream is None:
        stream = torch.cuda.current_stream(d_dose.device)
    handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    s = pmc_summary()
    st = lib().pmc_run_spots_dev(ctx, _ptr(sp), len(sp), int(n_histories), int(seed),
                                 C.c_void_p(d_dose.data_ptr()),
                                 C.c_void_p(d_var.data_ptr()) if d_var is not None else None,
                                 C.c_void_p(handle), C.byref(s))
    _check(ctx, st)
    return summary_dict(s)


def pmc_vavilov_table():
    """The engine's Vavilov straggling quantile table, VAV_SHAPE (host only)."""
    out = np.zeros(VAV_SHAPE, np.float32)
    _check(None, lib().pmc_vavilov_table(_ptr(out), out.size))
    return out


def pmc_moliere_table():
    """The engine's Molière sampling table, MOL_SHAPE (host only)."""
    out = np.zeros(MOL_SHAPE, np.float32)
    _check(None, lib().pmc_moliere_table(_ptr(out), out.size))
    return out


def pmc_inspect_tables(ctx):
    lnr_w = np.zeros(1000, np.float32)
    lnr_o = np.zeros(1000, np.float32)
    n = C.c_int32()
    _check(ctx, lib().pmc_inspect_tables(ctx, None, None, None, None, C.byref(n)))
    sig = np.zeros((n.value, 1000), np.float32)
    mat = np.zeros((n.value, 4), np.float64)
    _check(ctx, lib().pmc_inspect_tables(ctx, _ptr(lnr_w), _ptr(lnr_o), _ptr(sig), _ptr(mat),
                                         C.byref(n)))
    return {"lnr_water": lnr_w, "lnr_own": lnr_o, "sigma_per_g": sig, "material": mat}


def pmc_atomic_probe(ctx, n_atomics, stream=None):
    """Device milliseconds for n_atomics tally-pattern FP64 atomics."""
    ms = C.c_double()
    handle = None
    if stream is not None:
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    _check(ctx, lib().pmc_atomic_probe(ctx, int(n_atomics), C.c_void_p(handle) if handle else None,
                                       C.byref(ms)))
    return ms.value


def pmc_plan_launch(**query):
    """Launch layout for the query fields (pmc_launch_query); host only.
    Returns (status, layout fields as a dict, reason)."""
    q = pmc_launch_query(**query)
    out = pmc_launch_layout()
    why = C.create_string_buffer(256)
    rc = lib().pmc_plan_launch(C.byref(q), C.byref(out), why, 256)
    return rc, {f[0]: getattr(out, f[0]) for f in pmc_launch_layout._fields_}, why.value.decode()


def _stream_handle(stream):
    if stream is None:
        return None
    h = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    return C.c_void_p(h) if h else None


def pmc_roofline_replay(ctx, spots, n_histories, seed, stream=None):
    """Replay timings of the transport's own address stream (pmc_replay_result
    fields as a dict)."""
    sp = np.ascontiguousarray(spots, dtype=np.float32).reshape(-1, 6)
    out = pmc_replay_result()
    _check(ctx, lib().pmc_roofline_replay(ctx, _ptr(sp), len(sp), int(n_histories), int(seed),
                                          _stream_handle(stream), C.byref(out)))
    return {f[0]: getattr(out, f[0]) for f in pmc_replay_result._fields_}


def pmc_stream_probe(ctx, n_bytes, stream=None):
    """(read ms, copy ms) of a plain read and a plain copy of n_bytes."""
    r, cp = C.c_double(), C.c_double()
    _check(ctx, lib().pmc_stream_probe(ctx, int(n_bytes), _stream_handle(stream), C.byref(r), C.byref(cp)))
    return r.value, cp.value


def pmc_inc_events(ctx, element, t_mev, uid, ks, seed, evaporate=True):
    """Cascade and evaporation of n non-elastic events on the GPU.  Returns
    (results: list of dicts of pmc_inc_result fields, particles: structured
    array [n][INC_MAX_OUT] with kind, stage, id, t_mev, dir)."""
    el = np.ascontiguousarray(element, dtype=np.int32).ravel()
    n = el.size
    t = np.ascontiguousarray(np.broadcast_to(np.asarray(t_mev, np.float64), (n,)))
    u = np.ascontiguousarray(np.broadcast_to(np.asarray(uid, np.uint64), (n,)))
    k = np.ascontiguousarray(np.broadcast_to(np.asarray(ks, np.uint32), (n,)))
    res = (pmc_inc_result * max(n, 1))()
    pdt = np.dtype([("kind", np.int32), ("stage", np.int32), ("id", np.uint32), ("reserved", np.int32),
                    ("t_mev", np.float64), ("dir", np.float64, 3)])
    parts = np.zeros((max(n, 1), INC_MAX_OUT), pdt)
    _check(ctx, lib().pmc_inc_events(ctx, _ptr(el), _ptr(t), _ptr(u), _ptr(k), n, int(seed),
                                     1 if evaporate else 0, C.cast(res, C.c_void_p), _ptr(parts)))
    out = [{f[0]: getattr(res[i], f[0]) for f in pmc_inc_result._fields_} for i in range(n)]
    return out, parts[:n]


def pmc_inc_nucleus(element):
    """The cascade's target nucleus (host only): shell radii, densities and
    Fermi energies of protons and neutrons, the Woods-Saxon radius and A."""
    out = np.zeros(78, np.float64)
    _check(None, lib().pmc_inc_nucleus(int(element), _ptr(out), out.size))
    return {"r": out[:16], "rho_p": out[16:31], "rho_n": out[31:46], "tf_p": out[46:61],
            "tf_n": out[61:76], "radius_ws": out[76], "a": int(out[77])}


def pmc_inc_width(z, a, e_star, kind):
    """(relative evaporation width, separation energy, barrier), host only."""
    sep, bar = C.c_double(), C.c_double()
    w = lib().pmc_inc_width(int(z), int(a), float(e_star), int(kind), C.byref(sep), C.byref(bar))
    return w, sep.value, bar.value


def pmc_geometry_density(ctx, geometry_id, d_rho, stream=None):
    """Voxel densities (g/cm^3) of a loaded geometry into a float32 device
    tensor of nz*ny*nx elements."""
    import torch
    if d_rho.dtype != torch.float32 or not d_rho.is_cuda or not d_rho.is_contiguous():
        raise ValueError("d_rho must be a contiguous float32 device tensor")
    if (ctx.value, int(geometry_id)) in _geom_numel:
        _need_numel(ctx, geometry_id, d_rho, "d_rho")
    if stream is None:
        stream = torch.cuda.current_stream(d_rho.device)
    handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    _check(ctx, lib().pmc_geometry_density(ctx, int(geometry_id), C.c_void_p(d_rho.data_ptr()),
                                           C.c_void_p(handle)))


class Engine:
    """Owns one context; convenience wrapper over the functions above."""

    def __init__(self, device=0, **params):
        self.params = pmc_default_params(**params)
        self.ctx = pmc_create(device, self.params)
        self.shape = None

    def close(self):
        if self.ctx:
            pmc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_physics(self, nd):
        pmc_load_physics(self.ctx, nd)

    def load_geometry(self, hu, voxel_cm, mt):
        self.shape = pmc_load_geometry(self.ctx, hu, voxel_cm, mt)

    def run_spots(self, spots, n_histories, seed):
        return pmc_run_spots(self.ctx, spots, n_histories, seed, self.shape)

    def run_spots_dev(self, spots, n_histories, seed, d_dose, d_var=None, stream=None):
        return pmc_run_spots_dev(self.ctx, spots, n_histories, seed, d_dose, d_var, stream)

    def run_spots_let(self, spots, n_histories, seed):
        return pmc_run_spots_let(self.ctx, spots, n_histories, seed, self.shape)

    def run_spots_let_dev(self, spots, n_histories, seed, d_dose, d_let, d_var=None, stream=None):
        return pmc_run_spots_let_dev(self.ctx, spots, n_histories, seed, d_dose, d_let, d_var,
                                     stream)
