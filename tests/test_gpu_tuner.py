"""The launch-shape autotuner (pmc_params with block_threads, refill_lanes
and batch_events left at 0): the shape it picks for a workload runs within
15% of the fastest shape of its own candidate grid, timed the same way
(median device time of five runs), and it is remembered per workload.
Results never depend on the shape (covered by the parity tests)."""
import sys

import numpy as np
import pytest

from paper_1409_8336_amd import pmc, synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _median_ms(e, spots, n, reps=5):
    ts = []
    for i in range(reps):
        _, _, s = e.run_spots(spots, n, 3 + i)
        ts.append(s["device_ms"])
    return float(np.median(ts)), s


@pytest.mark.parametrize("energy,n", [(150.0, 1_000_000), (70.0, 2_000_000)])
def test_tuned_shape_is_near_the_best_of_its_grid(energy, n):
    nd, mt = synth.nuclear_data(), synth.material_table()
    cfg = synth.config_ct_spots(energy, n)
    _say("case: autotuner, CT %g MeV spot, %d histories" % (energy, n))
    e = pmc.Engine(0)
    e.load_physics(nd)
    e.load_geometry(cfg["hu"], cfg["voxel_cm"], mt)
    e.run_spots(cfg["spots"], n, 2)                 # tunes
    t_tuned, s = _median_ms(e, cfg["spots"], n)
    picked = (s["block_threads"], s["refill_lanes"], s["batch_events"], s["cache_slots"] > 0)
    e.close()
    best = None
    for block in (256, 512, 1024):
        for refill in (8, 16):
            for batch in (4, 8):
                for cache in ((0, -1) if block >= 512 else (0,)):
                    f = pmc.Engine(0, block_threads=block, refill_lanes=refill, batch_events=batch,
                                   tally_cache=cache)
                    f.load_physics(nd)
                    f.load_geometry(cfg["hu"], cfg["voxel_cm"], mt)
                    f.run_spots(cfg["spots"], n, 2)
                    t, _ = _median_ms(f, cfg["spots"], n)
                    f.close()
                    if best is None or t < best[0]:
                        best = (t, (block, refill, batch, cache == 0))
    _say("tuned %s %.3f ms; best of grid %s %.3f ms" % (picked, t_tuned, best[1], best[0]))
    assert t_tuned <= 1.15 * best[0], (picked, t_tuned, best)
