"""Launch layout of the transport kernel, checked on the CPU through the
C ABI (pmc_plan_launch, host only): every LDS region of a workgroup inside
the dynamic allocation, aligned and disjoint, and every buffer the kernel
indexes sized for the indices it can form -- for every workgroup size, plan
count, LET_d scoring, statistical group count and material count, and for
history counts up to 1e8 and beyond.  The regions are recomputed here from
the returned offsets, independently of the library's own check."""
import itertools

import pytest

from paper_1409_8336_amd import pmc

LDS_PER_CU = 163840


@pytest.fixture(scope="module")
def plan():
    class O:
        def __init__(self, d):
            self.__dict__.update(d)

    def run(**kw):
        rc, out, why = pmc.pmc_plan_launch(**kw)
        return rc, O(out), why
    return run


def _regions(q, o):
    """(name, begin word, end word, alignment in bytes) as the kernel uses them."""
    np_ = q["n_plans"]
    s = o.cache_slots
    r = [("blob", 0, o.blob_words, 4)]
    if q["batched"]:
        r.append(("plans", o.plan_desc_off, o.plan_desc_off + 16 * np_, 16))
    if s:
        r.append(("sums", o.cache_off, o.cache_off + 2 * s, 8))
        r.append(("keys", o.key_off, o.key_off + o.key_words * s, 4 * o.key_words))
        if q["score_let"]:
            r.append(("nums", o.num_off, o.num_off + s, 4))
    r.append(("ctl", o.ctl_off, o.ctl_off + 8, 4))
    r.append(("args", o.args_off, o.args_off + o.args_bytes // 4, 8))
    if q["batched"]:
        r.append(("ledgers", o.ledger_off, o.ledger_off + 6 * np_, 8))
        r.append(("counters", o.counter_off, o.counter_off + 16 * np_, 8))
    return r


def _check(q, o):
    assert o.lds_bytes == 4 * o.end_words <= LDS_PER_CU
    # the table blob: range tables, inverse indices, n_mat cross-section rows, 4 constants per bin
    assert o.blob_words == 3024 + 1004 * q["n_mat"]
    prev = 0
    for name, b, e, al in sorted(_regions(q, o), key=lambda t: t[1]):
        assert b >= prev, (name, b, prev)
        assert (4 * b) % al == 0, (name, b, al)
        assert e <= o.end_words, (name, e, o.end_words)
        prev = e
    planes = q["k_batches"] + (2 if q["score_let"] else 0)
    assert o.tally_planes == planes
    if o.cache_slots:
        # every tally index is a cache key below the free-slot marker 0xFFFFFFFF
        assert q["max_nvox"] * planes - 1 < 0xFFFFFFFF
        assert 512 <= o.cache_slots <= 16384
    # generation queues hold every index the kernel writes (slot < cap)
    assert o.queue_cap >= 1
    if q["grid_blocks"]:
        assert o.local_queue_words == q["grid_blocks"] * o.local_queue_cap * 12
        assert o.local_queue_cap <= 65536
        if q["local_queue"] == 0:
            assert o.local_queue_words * 4 <= 1 << 30
        assert o.claim_words == 64 * q["grid_blocks"]
    ns = q["n_spots"]
    assert o.order_words == q["k_batches"] * (ns + 1) + q["k_batches"] * ns + 1


BLOCKS = [64, 128, 256, 512, 768, 1024]


@pytest.mark.parametrize("block,batched,let", list(itertools.product(BLOCKS, [0, 1], [0, 1])))
def test_layout_regions_fit_for_every_shape(plan, block, batched, let):
    for n_mat, k, n_plans, cache in itertools.product([1, 8, 16], [2, 10, 64], [1, 2, 16, 64],
                                                      [0, -1, 512, 4096]):
        if not batched and n_plans != 1:
            continue
        for grid in (0, 256, 256 * max(1, 1024 // block)):
            q = dict(block_threads=block, grid_blocks=grid, n_plans=n_plans, batched=batched,
                     score_let=let, k_batches=k, n_mat=n_mat, tally_cache=cache, local_queue=0,
                     n_spots=2000 * n_plans, queue_capacity=0, n_histories=10 ** 8 * n_plans,
                     max_plan_histories=10 ** 8, max_nvox=256 * 256 * 200)
            rc, o, why = plan(**q)
            if rc == 0:
                _check(q, o)
            else:
                # only an explicit cache request too large for the LDS may fail
                assert cache > 0 and "exceeds" in why, (q, why)


def test_automatic_cache_always_fits(plan):
    for block, n_mat, let, batched in itertools.product(BLOCKS, range(1, 17), [0, 1], [0, 1]):
        q = dict(block_threads=block, grid_blocks=256, n_plans=64 if batched else 1, batched=batched,
                 score_let=let, k_batches=10, n_mat=n_mat, tally_cache=0, local_queue=0, n_spots=100,
                 queue_capacity=0, n_histories=10 ** 6, max_plan_histories=10 ** 6, max_nvox=10 ** 6)
        rc, o, why = plan(**q)
        assert rc == 0, (q, why)
        _check(q, o)
        # the cache shares the CU with the other resident workgroups
        wgs = max(1, 1024 // block)
        if o.cache_slots:
            assert wgs * o.lds_bytes <= LDS_PER_CU


def test_layout_of_the_faulted_launch_shape(plan):
    """The launch shape of the one GPU fault on record (512-lane workgroups,
    two per CU, 8 material bins, one plan, 1e8 histories on the 128x128x160
    CT): every region and index fits."""
    q = dict(block_threads=512, grid_blocks=512, n_plans=1, batched=0, score_let=0, k_batches=10,
             n_mat=8, tally_cache=0, local_queue=0, n_spots=180, queue_capacity=0,
             n_histories=10 ** 8, max_plan_histories=10 ** 8, max_nvox=128 * 128 * 160)
    rc, o, why = plan(**q)
    assert rc == 0, why
    _check(q, o)
    assert o.queue_cap == 10 ** 8 and o.cache_slots > 0
    assert 2 * o.lds_bytes <= LDS_PER_CU


def test_cache_is_dropped_when_tally_indices_exceed_the_key(plan):
    # 256x256x200 x 10 groups fits 32 bits; 4e8 voxels x 12 planes does not
    q = dict(block_threads=1024, grid_blocks=256, n_plans=1, batched=0, score_let=1, k_batches=10,
             n_mat=8, tally_cache=0, local_queue=0, n_spots=10, queue_capacity=0,
             n_histories=10 ** 6, max_plan_histories=10 ** 6, max_nvox=400_000_000)
    rc, o, why = plan(**q)
    assert rc == 0 and o.cache_slots == 0, why
    _check(q, o)


@pytest.mark.parametrize("bad,frag", [
    (dict(block_threads=96), "multiple of 64"),
    (dict(n_plans=2, batched=0), "single-plan"),
    (dict(n_plans=65, batched=1), "n_plans"),
    (dict(k_batches=1), "k_batches"),
    (dict(n_mat=17), "n_mat"),
    (dict(max_plan_histories=1 << 32), "2^32"),
    (dict(max_nvox=0), "grid size"),
    (dict(tally_cache=16384, block_threads=1024), "exceeds"),
    (dict(n_mat=16, block_threads=1024, tally_cache=12000), "exceeds"),
    (dict(queue_capacity=1 << 41), "queue capacity"),
])
def test_impossible_launches_are_refused(plan, bad, frag):
    q = dict(block_threads=256, grid_blocks=512, n_plans=1, batched=0, score_let=0, k_batches=10,
             n_mat=8, tally_cache=0, local_queue=0, n_spots=10, queue_capacity=0,
             n_histories=10 ** 6, max_plan_histories=10 ** 6, max_nvox=10 ** 6)
    q.update(bad)
    rc, o, why = plan(**q)
    assert rc != 0 and frag in why, (rc, why)
