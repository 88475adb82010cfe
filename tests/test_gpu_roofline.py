"""Roofline measurement entry points on the GPU (through the C ABI): the
replay of the transport's own address stream (one voxel-record gather and
one FP64 tally add per condensed-history step, Sec. II.A.3 / II.B.2) and the
plain read / copy bandwidth references."""
import sys

import numpy as np
import pytest

from paper_1409_8336_amd import pmc, synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_replay_reissues_the_transport_address_stream():
    """The traced run is the run (same steps), its trace holds every step of
    the first generation, the replays take positive time that grows with the
    work they re-issue, and the engine's results are unchanged afterwards."""
    _say("case: roofline replay (CT 150 MeV, 3e5 histories)")
    nd, mt = synth.nuclear_data(), synth.material_table()
    cfg = synth.config_ct_spots(150.0, 300_000)
    e = pmc.Engine(0)
    e.load_physics(nd)
    e.load_geometry(cfg["hu"], cfg["voxel_cm"], mt)
    d0, v0, s0 = e.run_spots(cfg["spots"], cfg["n_histories"], 5)
    r = pmc.pmc_roofline_replay(e.ctx, cfg["spots"], cfg["n_histories"], 5)
    _say("replay %s" % r)
    d1, v1, s1 = e.run_spots(cfg["spots"], cfg["n_histories"], 5)
    e.close()
    assert r["steps"] == s0["steps"]
    # the trace holds every evaluated step of generation 0 (all of them
    # unless a workgroup queue overflowed): the counted steps plus the last
    # step of every track that the residual range ends (counted as a
    # termination, not a step, but a gather and a deposit all the same)
    assert r["steps"] <= r["steps_traced"] <= r["steps"] + s0["histories"] + s0["secondaries"]
    assert r["deposits"] >= r["steps"]
    assert r["grid_blocks"] > 0 and r["block_threads"] > 0 and r["trace_iters"] > 0
    for k in ("transport_ms", "trace_only_ms", "gather_ms", "atomic_ms", "cached_atomic_ms", "combined_ms"):
        assert r[k] > 0, k
    assert r["gather_ms"] >= 0.9 * r["trace_only_ms"]
    assert r["combined_ms"] >= 0.9 * max(r["gather_ms"], r["cached_atomic_ms"])
    np.testing.assert_allclose(d1, d0, rtol=1e-9, atol=1e-12 * d0.max())
    assert s1["steps"] == s0["steps"]


def test_stream_probe_bandwidth_is_plausible():
    _say("case: stream probe")
    e = pmc.Engine(0)
    n = 1 << 30
    read_ms, copy_ms = pmc.pmc_stream_probe(e.ctx, n)
    e.close()
    read_gbs = n / (read_ms * 1e-3) / 1e9
    copy_gbs = 2 * n / (copy_ms * 1e-3) / 1e9
    _say("read %.0f GB/s, copy %.0f GB/s" % (read_gbs, copy_gbs))
    assert 500 < read_gbs < 8000 and 500 < copy_gbs < 8000
    with pytest.raises(pmc.PMCError):
        pmc.pmc_stream_probe(pmc.Engine(0).ctx, 1000)


def test_atomic_probe_rate_is_plausible_and_leaves_the_dose():
    """The tally-pattern atomic probe: a positive time that grows with the
    atomic count, a rate between 1e9 and 1e11 FP64 atomics per second, a
    geometry required, and the engine's next run unchanged (the probe adds
    zeros into the tally)."""
    _say("case: atomic probe")
    nd, mt = synth.nuclear_data(), synth.material_table()
    cfg = synth.config_water_pencil(50_000)
    e = pmc.Engine(0)
    e.load_physics(nd)
    with pytest.raises(pmc.PMCError):
        pmc.pmc_atomic_probe(e.ctx, 1000)          # no geometry yet
    e.load_geometry(cfg["hu"], cfg["voxel_cm"], mt)
    d0, v0, s0 = e.run_spots(cfg["spots"], cfg["n_histories"], 4)
    t1 = pmc.pmc_atomic_probe(e.ctx, 20_000_000)
    t2 = pmc.pmc_atomic_probe(e.ctx, 80_000_000)
    _say("probe %.3f ms for 2e7, %.3f ms for 8e7 atomics" % (t1, t2))
    assert 0 < t1 < t2
    rate = 8e7 / (t2 * 1e-3)
    assert 1e9 < rate < 1e11, rate
    d1, v1, s1 = e.run_spots(cfg["spots"], cfg["n_histories"], 4)
    e.close()
    np.testing.assert_allclose(d1, d0, rtol=1e-9, atol=1e-12 * d0.max())
    assert s1["steps"] == s0["steps"]
