// Launch layout of the transport kernel (see layout.hpp) and its check.
// Host code only: the run driver lays out and checks every launch with these
// functions, and pmc_plan_launch exposes them without a device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "device.hpp"
#include "layout.hpp"
#include "pmc.h"

namespace pmc {

namespace {
std::string fmt(const char* f, unsigned long long a = 0, unsigned long long b = 0, unsigned long long c = 0)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, f, a, b, c);
    return buf;
}
}  // namespace

std::string plan_layout(const LayoutQuery& q, LaunchLayout* out)
{
    LaunchLayout L;
    if (q.block < 64 || q.block > 1024 || q.block % 64) return "block must be a multiple of 64 in [64, 1024]";
    if (q.n_plans < 1 || q.n_plans > kMaxPlans) return "n_plans must be in [1, 64]";
    if (!q.multi && q.n_plans != 1) return "a single-plan launch has one plan";
    if (q.k_batches < 2 || q.k_batches > 64) return "k_batches must be in [2, 64]";
    if (q.n_mat < 1 || q.n_mat > 16) return "n_mat must be in [1, 16]";
    const int np = q.n_plans;
    L.blob_words = kOffSigma + 1000 * q.n_mat + 4 * q.n_mat;
    L.pd_off = (L.blob_words + 3) & ~3;
    const int table_words = q.multi ? L.pd_off + 16 * np : L.blob_words;
    L.planes = q.k_batches + (q.score_let ? 2 : 0);
    L.key_words = q.multi ? 2 : 1;
    const int slot_words = 2 + L.key_words + (q.score_let ? 1 : 0);
    // the cache key is the tally index as u32 (0xFFFFFFFF marks a free slot)
    const bool keys_fit = q.max_nvox * (unsigned long long)L.planes < 0xFFFFFFFFull;
    L.cache_off = (table_words + 1) & ~1;
    const long plan_block_bytes = q.multi ? (long)kPlanLdsBytes * np : 0L;
    int slots = 0;
    if (q.cache_request >= 0 && keys_fit) {
        slots = q.cache_request;
        if (slots == 0) {
            // what the tables, control words, staged arguments (with their
            // alignment) and a batch's per-plan block leave of the CU's LDS
            // when 1024 / block workgroups share it
            const long wgs = std::max(1, 1024 / q.block);
            const long avail = (long)kLdsPerCu / wgs - 4L * L.cache_off - 4L * kWgCtlWords - 8 -
                               (long)sizeof(LdsArgs) - plan_block_bytes;
            slots = (int)std::min(16384L, std::max(0L, avail) / (4L * slot_words));
            if (slots < 512) slots = 0;
        }
    }
    L.cache_slots = slots;
    L.key_off = L.cache_off + 2 * slots;
    L.num_off = L.key_off + L.key_words * slots;
    L.ctl_off = L.num_off + (q.score_let ? slots : 0);
    L.args_off = (L.ctl_off + kWgCtlWords + 1) & ~1;
    L.led_off = L.args_off + (int)(sizeof(LdsArgs) / 4);
    L.cnt_off = L.led_off + (q.multi ? 6 * np : 0);
    L.end_words = L.cnt_off + (q.multi ? 2 * kWgCounters * np : 0);
    L.lds_bytes = (size_t)L.end_words * 4;
    L.q_cap = q.queue_capacity ? q.queue_capacity : std::max<unsigned long long>(65536ull, q.n_histories);
    if (q.grid > 0) {
        L.loc_cap = q.local_queue < 0 ? 0
                    : (q.local_queue ? q.local_queue
                                     : (int)std::min<long>(65536L, (1L << 30) / (48L * q.grid)));
        L.qloc_words = (unsigned long long)q.grid * (unsigned long long)L.loc_cap * kLocEntryWords;
        L.claim_words = (unsigned long long)kMaxGenerations * (unsigned long long)q.grid;
    }
    const unsigned long long K = (unsigned long long)q.k_batches, ns = (unsigned long long)std::max(q.n_spots, 0);
    L.order_words = K * (ns + 1) + K * ns + 1;
    *out = L;
    return check_layout(q, L);
}

std::string check_layout(const LayoutQuery& q, const LaunchLayout& L)
{
    // ---- LDS: every region aligned, inside the allocation, disjoint
    struct Region {
        const char* name;
        long begin, end;   // words
        int align;         // bytes
    };
    std::vector<Region> r;
    const int np = q.n_plans, s = L.cache_slots;
    r.push_back({"table blob", 0, L.blob_words, 4});
    if (q.multi) r.push_back({"plan descriptors", L.pd_off, L.pd_off + 16L * np, 16});
    if (s > 0) {
        r.push_back({"cache sums", L.cache_off, L.cache_off + 2L * s, 8});
        r.push_back({"cache keys", L.key_off, L.key_off + (long)L.key_words * s, 4 * L.key_words});
        if (q.score_let) r.push_back({"cache LET numerators", L.num_off, L.num_off + (long)s, 4});
    }
    r.push_back({"control words", L.ctl_off, L.ctl_off + kWgCtlWords, 4});
    r.push_back({"staged arguments", L.args_off, L.args_off + (long)(sizeof(LdsArgs) / 4), 8});
    if (q.multi) {
        r.push_back({"plan ledgers", L.led_off, L.led_off + 6L * np, 8});
        r.push_back({"plan counters", L.cnt_off, L.cnt_off + 2L * kWgCounters * np, 8});
    }
    if ((size_t)L.end_words * 4 != L.lds_bytes) return "LDS size does not match the last region";
    if (L.lds_bytes > kLdsPerCu)
        return fmt("LDS request of %llu bytes exceeds the %llu bytes of a CU", L.lds_bytes, kLdsPerCu);
    std::vector<Region> sorted = r;
    std::sort(sorted.begin(), sorted.end(), [](const Region& a, const Region& b) { return a.begin < b.begin; });
    long prev_end = 0;
    const char* prev = "start";
    for (const Region& g : sorted) {
        if (g.begin < 0 || g.end < g.begin) return std::string("LDS region ") + g.name + " is malformed";
        if ((g.begin * 4) % g.align) return std::string("LDS region ") + g.name + " is misaligned";
        if (g.begin < prev_end) return std::string("LDS region ") + g.name + " overlaps " + prev;
        if (g.end > L.end_words) return std::string("LDS region ") + g.name + " runs past the allocation";
        prev_end = g.end;
        prev = g.name;
    }
    // the kernel's control words: produced, claimed, published, busy, primaries done, done
    static_assert(kWgCtlWords >= 6, "the transport kernel uses six control words");
    static_assert(sizeof(LdsArgs) % 8 == 0, "the per-plan ledgers after the staged arguments are doubles");
    // ---- deposit cache keys and slots
    if (s < 0 || s > 16384) return "cache slots outside [0, 16384]";
    if (s > 0 && q.max_nvox * (unsigned long long)L.planes >= 0xFFFFFFFFull)
        return "a tally index does not fit the 32-bit cache key";
    // ---- tallies, work list, random streams
    if (q.max_nvox == 0 || q.max_nvox > 4000000000ull) return "grid size outside [1, 4e9] voxels";
    if (q.max_plan_histories >= (1ull << 32)) return "at most 2^32-1 histories per plan";
    if (q.n_histories > 64ull * 0xFFFFFFFFull) return "too many histories";
    if (q.n_spots < 0) return "negative spot count";
    // ---- queues and claims
    if (L.q_cap == 0 || L.q_cap > (1ull << 40)) return "generation queue capacity outside [1, 2^40]";
    if (q.grid > 0) {
        if (L.loc_cap < 0 || L.loc_cap > 65536) return "workgroup queue capacity outside [0, 65536]";
        if (L.qloc_words / kLocEntryWords / (unsigned long long)q.grid != (unsigned long long)L.loc_cap)
            return "workgroup queue size overflows";
        // the largest claim index: ((j >> c) G + b) << c with j <= N + 64
        const unsigned long long jmax = std::max(q.n_histories, L.q_cap) + 64ull;
        if (jmax > (1ull << 62) / (unsigned long long)q.grid) return "claim index overflows";
    }
    return std::string();
}

}  // namespace pmc

extern "C" pmc_status pmc_plan_launch(const pmc_launch_query* q, pmc_launch_layout* out, char* why, int32_t why_len)
{
    if (why && why_len > 0) why[0] = 0;
    if (!q || !out) return PMC_ERR_ARG;
    pmc::LayoutQuery lq;
    lq.block = q->block_threads;
    lq.grid = q->grid_blocks;
    lq.n_plans = q->n_plans;
    lq.multi = q->batched != 0;
    lq.score_let = q->score_let != 0;
    lq.k_batches = q->k_batches;
    lq.n_mat = q->n_mat;
    lq.cache_request = q->tally_cache;
    lq.local_queue = q->local_queue;
    lq.queue_capacity = q->queue_capacity;
    lq.n_histories = q->n_histories;
    lq.max_plan_histories = q->max_plan_histories;
    lq.n_spots = q->n_spots;
    lq.max_nvox = q->max_nvox;
    pmc::LaunchLayout L;
    const std::string e = pmc::plan_layout(lq, &L);
    std::memset(out, 0, sizeof(*out));
    out->lds_bytes = L.lds_bytes;
    out->blob_words = L.blob_words;
    out->plan_desc_off = L.pd_off;
    out->cache_off = L.cache_off;
    out->key_off = L.key_off;
    out->num_off = L.num_off;
    out->ctl_off = L.ctl_off;
    out->args_off = L.args_off;
    out->ledger_off = L.led_off;
    out->counter_off = L.cnt_off;
    out->end_words = L.end_words;
    out->cache_slots = L.cache_slots;
    out->key_words = L.key_words;
    out->tally_planes = L.planes;
    out->local_queue_cap = L.loc_cap;
    out->queue_cap = L.q_cap;
    out->local_queue_words = L.qloc_words;
    out->claim_words = L.claim_words;
    out->order_words = L.order_words;
    out->args_bytes = (int32_t)sizeof(pmc::LdsArgs);
    if (!e.empty()) {
        if (why && why_len > 0) {
            std::strncpy(why, e.c_str(), (size_t)why_len - 1);
            why[why_len - 1] = 0;
        }
        return PMC_ERR_ARG;
    }
    return PMC_OK;
}
