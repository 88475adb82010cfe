// Launch layout of the transport kernel: where every region of a
// workgroup's LDS lies, and the sizes of the device buffers a launch indexes.
// One host function computes it (the run driver and the kernel use exactly
// these offsets), another checks it before every launch: every LDS region
// inside the dynamic allocation, aligned and disjoint from the others, and
// every index the kernel can form inside its buffer.
#pragma once

#include <cstdint>
#include <string>

namespace pmc {

struct LayoutQuery {
    int block = 256;            // workgroup size (lanes)
    int grid = 0;               // workgroups of the launch (0: not yet known)
    int n_plans = 1;
    bool multi = false;         // batched-plan kernel
    bool score_let = false;     // LET_d planes and numerators
    int k_batches = 10;
    int n_mat = 8;              // material bins (table blob size)
    int cache_request = 0;      // slots: -1 off, 0 sized from the LDS left, else that many
    int local_queue = 0;        // per-workgroup queue entries: -1 off, 0 automatic, else that many
    unsigned long long queue_capacity = 0;   // generation queue entries (0: max(65536, N))
    unsigned long long n_histories = 0;      // all plans
    unsigned long long max_plan_histories = 0;
    int n_spots = 0;            // all plans
    unsigned long long max_nvox = 0;         // largest plan grid
};

struct LaunchLayout {
    // LDS, in 32-bit words from the start of the dynamic allocation
    int blob_words = 0;
    int pd_off = 0;       // plan descriptors (batched launch)
    int cache_off = 0;    // slot sums (double)
    int key_off = 0;      // slot keys (u32; u64 in a batched launch)
    int num_off = 0;      // slot LET numerators (float)
    int ctl_off = 0;      // control words
    int args_off = 0;     // staged arguments
    int led_off = 0;      // per-plan ledgers (batched)
    int cnt_off = 0;      // per-plan counters (batched)
    int end_words = 0;
    size_t lds_bytes = 0;
    int cache_slots = 0;
    int key_words = 1;
    // device buffers
    int planes = 0;                        // tally doubles per voxel
    unsigned long long q_cap = 0;          // generation queue entries
    int loc_cap = 0;                       // per-workgroup queue entries
    unsigned long long qloc_words = 0;     // all workgroup queues
    unsigned long long claim_words = 0;    // per-generation claim counters
    unsigned long long order_words = 0;    // primary work list
};

// Fills *out for q; returns an empty string, or why the launch cannot be laid out.
std::string plan_layout(const LayoutQuery& q, LaunchLayout* out);
// Checks a layout against q; empty string when every region and index fits.
std::string check_layout(const LayoutQuery& q, const LaunchLayout& L);

constexpr size_t kLdsPerCu = 163840;   // 160 KiB on gfx950, also the per-workgroup limit

}  // namespace pmc
