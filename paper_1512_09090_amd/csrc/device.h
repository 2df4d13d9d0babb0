// device.h - device-resident graph and the per-call launch sequence (sweep.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "prep.h"

void set_error(const std::string &msg);   // thread-local message behind iso_last_error()

namespace isodev {

constexpr size_t LDS_MAX = 160 * 1024;      // LDS of one gfx950 compute unit
constexpr size_t CELL_LDS_BUDGET = 80 * 1024;   // per cell workgroup: two workgroups per CU
constexpr size_t TOP_LDS_BUDGET = 144 * 1024;   // the single top-block workgroup
constexpr uint32_t MAX_LANES = 64;

struct RunArgs {
    uint32_t lanes = 1;          // real queries in this launch (<= k_pow2)
    uint32_t k_pow2 = 1;         // label row width (power of two >= lanes)
    uint32_t lane_base = 0;
    bool mode_plain = true;
    bool want_dist = false;
    size_t out_cap = 0;          // capacity of the edge-key buffer
    std::vector<uint32_t> taus;      // k_pow2 (padding lanes: INF)
    std::vector<uint32_t> src_cell;  // k_pow2 (padding lanes: NO_CELL)
    // upward-search labels of every lane, one entry each: position, lane, label
    std::vector<uint32_t> upos, ulane, uval;
};

struct RunResult {
    uint32_t count = 0;          // keys produced (may exceed the capacity)
    uint32_t active_cells = 0;   // length of the active-cell list (cells mode)
    bool overflow = false;
    std::vector<uint64_t> keys;  // sorted lane << 58 | tail << 29 | head
    std::vector<uint32_t> dcore, dist, active_list;   // only with want_dist
};

struct QueryBufs {
    uint32_t *d_dcore = nullptr, *d_uval = nullptr, *d_uin = nullptr, *d_taus = nullptr,
             *d_src_cell = nullptr, *d_flags = nullptr, *d_list = nullptr, *d_counters = nullptr,
             *d_dist = nullptr;
    uint64_t *d_keys = nullptr, *d_keys_sorted = nullptr;
    void *d_sort_tmp = nullptr, *h_pinned = nullptr;
    size_t sz_dcore = 0, sz_uval = 0, sz_uin = 0, sz_taus = 0, sz_src_cell = 0, sz_flags = 0, sz_list = 0,
           sz_counters = 0, sz_keys = 0, sz_keys_sorted = 0, sz_sort_tmp = 0, sz_dist = 0, sz_pinned = 0;
    void release();
};

struct Profile {
    bool on = false;
    double core_ms = 0, active_ms = 0, cell_ms = 0, sort_ms = 0;
    uint64_t core_launches = 0, cell_launches = 0, calls = 0, core_bytes = 0, cell_bytes = 0;
    uint64_t core_entries = 0, cell_entries = 0, cell_vertices = 0, cells_swept = 0;
    hipEvent_t ev[6] = {};
};

struct DevGraph {
    int device = -1;
    hipStream_t stream = nullptr;
    uint32_t n = 0, n_core = 0, num_cells = 0;
    // core levels (host copy), and prefix sums used to size the LDS top block
    std::vector<uint32_t> core_lvl;
    std::vector<uint32_t> core_lvl_entries;   // down_off at each core level boundary
    uint32_t *d_down_off = nullptr;
    uint2 *d_down_arc = nullptr;
    uint32_t *d_perm = nullptr, *d_core_cell = nullptr, *d_core_ecc = nullptr, *d_cell_off = nullptr,
             *d_uslot = nullptr, *d_top_lvl = nullptr;
    uint8_t *d_uncovered = nullptr;
    // per-cell blobs for the cell sweep: [offsets][level bounds][core refs][entries]
    uint32_t *d_blob = nullptr;
    uint32_t *d_cblob = nullptr;   // word offset of each cell's blob
    uint4 *d_cmeta = nullptr;      // (internal count, levels, core refs, entries)
    uint32_t max_blob_words = 0, max_cell_labels = 0;
    uint64_t bytes = 0;
    QueryBufs bufs;
    Profile prof;
    // per-cell sizes for the byte accounting
    std::vector<uint32_t> cell_cnt, cell_words, cell_core_refs;
    std::vector<uint64_t> cell_entries;
    uint64_t core_entries = 0;

    int upload(const iso::Prep &P, int device);
    int run(const RunArgs &A, RunResult &R);
    void release();
};

}  // namespace isodev
