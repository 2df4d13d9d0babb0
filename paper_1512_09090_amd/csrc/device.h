// device.h - device-resident graph and the per-call launch sequence (sweep.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <functional>
#include <map>
#include <mutex>
#include <vector>

#include "prep.h"

void set_error(const std::string &msg);   // thread-local message behind iso_last_error()

namespace isodev {

constexpr size_t LDS_MAX = 160 * 1024;          // LDS of one gfx950 compute unit
constexpr uint32_t TABLE_MAX = 16384;           // vertices of the top-of-hierarchy distance table built at load
constexpr uint32_t TABLE_DEFAULT = TABLE_MAX;   // vertices of the levels merged into it by default
constexpr uint32_t MAX_LANES = 64;
constexpr uint32_t MAX_CELLS = 1u << 24;   // cell ids share a 32-bit work item with a width shift and a lane chunk
// static device scratch of the no-allocation entry point (per GPU) and its pinned staging block
constexpr size_t SCRATCH_BYTES = size_t(64) << 20;
constexpr size_t FIXED_STAGE_BYTES = size_t(4) << 20;

struct TargetSet;

// Resident cell workgroups per CU for sweeps that overlap on two streams.
constexpr uint32_t OVERLAP_CELL_PER_CU = 3;

struct RunArgs {
    uint32_t lanes = 1;          // real queries in this launch (<= k_pow2)
    uint32_t k_pow2 = 1;         // label row width (power of two >= lanes)
    uint32_t lane_base = 0;
    uint32_t block = 256;            // threads per workgroup of the core level kernel
    uint32_t use_graph = 0;          // 1: replay the captured device sweep
    uint32_t cell_stage = 2;         // 0: level pipeline per work item, 1: a work item's cell staged in LDS,
                                     // 2: one workgroup per cell for all its lanes (k_cell_chunks)
    uint32_t cell_block = 512;       // threads per cell workgroup (cell_stage 0 and 1)
    size_t cell_lds_bytes = 40 * 1024;
    // resident cell workgroups per CU (0: as many as fit).  A sweep that overlaps another
    // sweep's kernels runs faster with fewer (measured: 2 of 3 on road18m), one alone with all.
    uint32_t cell_per_cu = 0;
    bool mode_plain = true;
    bool want_dist = false;
    bool debug = false;          // count rare kernel branches (QueryBufs::d_dbg)
    bool core64 = true;          // 64 queries per sweep: core levels one wavefront per vertex
    bool fill_uslot = false;     // refill the slot table first (its memory is shared with other calls)
    bool plain_stream = true;    // plain mode at 64 queries per sweep: the internal vertices as a stream of
                                 // levels across all cells (k_plain_level64) instead of cell by cell
    size_t out_cap = 0;          // capacity of the edge-key buffer
    uint32_t table_x = 0;        // top table used: core positions [0, table_x), the first table_levels levels
    uint32_t table_levels = 0;
    // isoPHAST-CD: the slot entries hold every core label a host search settled (no table
    // entries); the device fills the core labels from them instead of sweeping the core levels
    bool core_dijkstra = false;
    // vertices in range instead of edges (vbits set): per lane j < lanes, row j of ceil(n / 64)
    // words of vbits gets bit v % 64 of word v / 64 for every original id v in range; no edges
    uint64_t *vbits = nullptr;
    bool vmask_only = false;     // vertex output kept as lane masks by position only (polygons)
    // one-to-many instead (tg set): distances from each lane's source to the target set's
    // targets, row j of tg_out (tg->count words) for lane j < lanes; no cells, no edges
    const TargetSet *tg = nullptr;
    uint32_t *tg_out = nullptr;
    std::vector<uint32_t> taus;      // k_pow2 (padding lanes: INF)
    std::vector<uint32_t> src_cell;  // k_pow2 (padding lanes: NO_CELL)
    // upward-search labels per lane: positions and labels inside the top table X
    // (position < TX), and elsewhere
    std::vector<std::vector<uint32_t>> xpos, xval, spos, sval;
};

struct RunResult {
    uint32_t count = 0;          // isochrone edges produced (may exceed the capacity)
    uint32_t active_cells = 0;   // length of the active-cell list (cells mode)
    bool overflow = false;
    // The edges as (tail, head) pairs of original ids, sorted by lane, then tail, then head;
    // lane j's edges are [lane_off[j], lane_off[j + 1]).  They are copied to sink(count) if a
    // sink is given (2 * count words; nullptr = out of host memory), else into `edges`.
    std::function<uint32_t *(size_t)> sink;
    std::vector<uint32_t> edges, lane_off;
    // Device destination instead (dev_dst set): the pairs go to dev_pairs + 2 * dev_base and
    // dev_base + the lane starts to dev_off[0 .. dev_lanes]; dev_overflow if dev_base + count
    // exceeds dev_cap pairs, or if it was set beforehand (then nothing is written).
    uint32_t *dev_pairs = nullptr, *dev_off = nullptr;
    uint64_t dev_cap = 0;
    uint32_t dev_base = 0, dev_lanes = 0;
    bool dev_dst = false, dev_overflow = false;
    double t_result_ms = 0;      // host time of sorting, decoding and copying back the edges
    std::vector<uint32_t> dcore, dist, active_list;   // only with want_dist
};

// A target set's restricted downward graph (RPHAST) on the device.  Rows of the label array:
// [0, tx) the top-table vertices (rows = positions), then the restricted vertices below the
// table, grouped by level (core levels top first, then the cells' local levels top first, every
// cell's level l in one group) so that no entry joins two rows of one group.
struct TargetSet {
    int device = -1;
    uint32_t count = 0;                  // targets
    uint32_t tx = 0, table_levels = 0;   // top-table prefix the restriction was built for
    uint32_t nr = 0;                     // restricted vertices below the table
    uint64_t arcs = 0;                   // their entries (finite lengths only)
    std::vector<uint32_t> group;         // group bounds in rows, from tx to tx + nr
    uint32_t *d_off = nullptr;           // nr + 1: entries of row tx + i
    uint2 *d_arc = nullptr;              // (row of the tail, length)
    uint32_t *d_rpos = nullptr;          // nr: position of row tx + i
    uint32_t *d_row = nullptr;           // count: row of each target
    uint64_t bytes = 0;
    void release();
};

// Rotation system of the input graph for the polygon output (polygon.hip): darts are the
// ordered neighbour pairs (u, v) of the undirected input, numbered in (u, v) order over
// original ids (CSR d_off over u, n + 1 words).
struct Rotation {
    bool ready = false;
    uint64_t darts = 0, bytes = 0;
    uint32_t *d_off = nullptr;     // n + 1: first dart of each original id
    uint32_t *d_hpos = nullptr;    // per dart: sweep position of the head
    uint32_t *d_hid = nullptr;     // per dart: original id of the head
    uint32_t *d_twin = nullptr;    // per dart: the dart (v, u)
    uint32_t *d_fnext = nullptr;   // per dart (a, b): the next dart (b, c) of the face on its left
    void release();
};

// Work buffers of the polygon kernels (grown on demand, kept between calls).
struct PolyBufs {
    size_t cap = size_t(1) << 12;   // boundary-dart capacity of the enumeration (grown as calls need; small
                                    // at first, so that the first calls take the grow-and-repeat path)
    uint64_t *d_keys = nullptr, *d_keys2 = nullptr, *d_scan = nullptr, *d_scx = nullptr;
    uint32_t *d_nxt = nullptr, *d_mn = nullptr, *d_rk = nullptr, *d_w = nullptr, *d_cyc = nullptr,
             *d_small = nullptr;
    uint2 *d_out = nullptr;
    void *d_sort_tmp = nullptr, *d_scan_tmp = nullptr;
    size_t sz_keys = 0, sz_keys2 = 0, sz_scan = 0, sz_scx = 0, sz_nxt = 0, sz_mn = 0, sz_rk = 0, sz_w = 0,
           sz_cyc = 0, sz_small = 0, sz_out = 0, sz_sort_tmp = 0, sz_scan_tmp = 0;
    void release();
};

// Polygons of one sweep's lanes: darts as (tail, head) pairs in cycle order, lane j's darts
// [loff[j], loff[j + 1]); cycle starts (indices into the darts), lane j's cycles
// [lcyc[j], lcyc[j + 1]).
struct PolyResult {
    std::vector<uint32_t> darts, cyc, loff, lcyc;
};

struct QueryBufs {
    uint32_t *d_xin = nullptr;   // per-lane upward labels inside the table: ptr (k+1), pos, val
    size_t sz_xin = 0;
    uint32_t *d_uslot = nullptr; // n entries: slot of a position in the upward-label table, or none
    size_t sz_uslot = 0;
    uint32_t *d_dcore = nullptr, *d_uval = nullptr, *d_uin = nullptr, *d_taus = nullptr,
             *d_src_cell = nullptr, *d_flags = nullptr, *d_list = nullptr, *d_counters = nullptr,
             *d_dist = nullptr;
    uint64_t *d_keys = nullptr, *d_keys_sorted = nullptr;
    uint64_t *d_vmask = nullptr, *d_cin = nullptr;   // vertex output: lanes in range per position; per cell
    uint32_t *d_rlab = nullptr;                        // one-to-many: labels of a target set's rows
    uint64_t *d_prof = nullptr;                        // profile: cell-sweep sums (k_prof_cells)
    unsigned long long *d_dbg = nullptr;               // branch counters of the sweep kernels (8 words)
    uint32_t *d_lane_off = nullptr;   // MAX_LANES + 1 lane starts of the decoded edges
    void *d_sort_tmp = nullptr, *h_pinned = nullptr;
    bool fixed = false;   // carved from the static scratch (iso_query_batch_device_noalloc): never freed or grown
    size_t sz_dcore = 0, sz_uval = 0, sz_uin = 0, sz_taus = 0, sz_src_cell = 0, sz_flags = 0, sz_list = 0,
           sz_counters = 0, sz_keys = 0, sz_keys_sorted = 0, sz_sort_tmp = 0, sz_dist = 0, sz_pinned = 0,
           sz_lane_off = 0, sz_vmask = 0, sz_cin = 0, sz_rlab = 0, sz_prof = 0, sz_dbg = 0;
    void release();
};

struct Profile {
    bool on = false;
    bool acc_ready = false;   // the device sums (QueryBufs::d_prof) were cleared since enabling
    double core_ms = 0, active_ms = 0, cell_ms = 0, sort_ms = 0;
    uint64_t core_launches = 0, cell_launches = 0, calls = 0, core_bytes = 0, cell_bytes = 0;
    uint64_t core_entries = 0, cell_entries = 0, cell_vertices = 0, cells_swept = 0, cell_lanes = 0,
             cell_items = 0, cell_bytes_survey = 0, level_bytes = 0, level_launches = 0;
    double level_ms = 0;
    hipEvent_t ev[8] = {};   // phase marks: 0 core start, 1 core end, 2/3 cell sweep, 4/5 sort, 6/7 core levels
};

// Everything the captured sweep sequence depends on (kernel arguments and grid shapes).
struct GraphSig {
    uint32_t K, plain, dist, block, cell_lds, xcap, cell_stage, cell_block, table_x, table_levels;   // no padding
    uint64_t cap;
    uint64_t ptr[10];
};
static_assert(sizeof(GraphSig) == 10 * 4 + 8 + 10 * 8, "GraphSig is compared with memcmp: no padding");

// One sweep in flight: its stream, buffers, profile and the state kept between launch and
// finish.  Several contexts over one DevGraph run concurrently (the serving loop).
struct SweepCtx {
    hipGraphExec_t graph_exec = nullptr;   // captured device sweep (use_graph)
    GraphSig sig{};
    uint32_t xcap = 0;                     // capacity of the per-lane table lists
    int device = -1;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    QueryBufs bufs;
    Profile prof;
    bool pending = false;
    uint32_t K = 1, lk = 0, lg = 0, lanes = 0, lane_base = 0, nlev = 0, top = 0, cell_variant = 0;
    size_t cap = 0;
    bool mode_plain = true, want_dist = false, vertex_mode = false, one_to_many = false, levels_timed = false;
    bool pstream = false;          // the plain sweep ran as a stream of levels (k_plain_level64)
    uint32_t plain_launches = 0;   // its launches
    uint32_t *h_counters = nullptr;   // pinned: keys produced, active cells
    int create(int device);
    void release();
};

struct DevGraph {
    int device = -1;
    uint32_t n = 0, n_core = 0, num_cells = 0;
    // Edge keys: lane << rank_bits | the arc's rank among all arcs ordered by (tail, head) over
    // original ids, so that sorted keys are in (lane, tail, head) order
    uint32_t rank_bits = 1;
    uint2 *d_arc_rank = nullptr;   // per downward entry: ranks of its forward and reverse arcs (INF: none)
    uint2 *d_arc_pair = nullptr;   // per rank: (tail, head), original ids
    // core levels (host copy), and prefix sums used to size the LDS top block
    std::vector<uint32_t> core_lvl;
    std::vector<uint32_t> core_lvl_entries;   // down_off at each core level boundary
    uint32_t *d_down_off = nullptr;
    uint2 *d_core_rec = nullptr;   // per core vertex: entry offsets and its first entries (k_core_level64)
    uint2 *d_down_arc = nullptr;
    uint32_t *d_core_cell = nullptr, *d_core_ecc = nullptr, *d_cell_off = nullptr;
    uint32_t *d_pos = nullptr;   // original id -> position (vertex output)
    // plain sweep as a stream of levels across all cells (k_plain_level64): the internal positions'
    // records (position, entry range, whether an entry reads the label, first entries) grouped by
    // level from the top of their cell (launch l: records [plvl_ptr[l], plvl_ptr[l + 1])), and the
    // internal entries and read positions for the byte accounting
    uint2 *d_plvl_rec = nullptr;
    std::vector<uint32_t> plvl_ptr;
    uint64_t plain_entries = 0, plain_written = 0;
    uint32_t plain_per_cu = 0;   // resident k_plain_level64 blocks per compute unit (occupancy query)
    // top-of-hierarchy table: X = core positions [0, TX) covering the first nlev_table levels;
    // d_table[y * TX + x] = shortest downward path y -> x inside X
    uint32_t TX = 0, nlev_table = 0;
    // the largest prefix of the table's levels with at most `want` vertices (0 = TABLE_DEFAULT;
    // 1 = no table)
    void table_cut(uint32_t want, uint32_t &tx, uint32_t &levels) const {
        const uint32_t cap = want == 1 ? 0u : std::min(want ? want : TABLE_DEFAULT, TX);
        tx = 0;
        levels = 0;
        for (uint32_t l = 0; l < nlev_table && core_lvl[l + 1] <= cap; ++l) {
            tx = core_lvl[l + 1];
            levels = l + 1;
        }
    }
    uint32_t *d_table = nullptr;
    uint8_t *d_uncovered = nullptr;
    uint32_t *d_cell_core_off = nullptr, *d_cell_core = nullptr;   // core positions of each cell (CSR)
    // per-cell blobs for the cell sweep: [offsets][level bounds][core refs][entries]
    uint32_t *d_blob = nullptr;
    uint32_t *d_cblob = nullptr;   // word offset of each cell's blob
    // per-cell data of the one-workgroup-per-cell sweep (k_cell_chunks): offsets, level starts,
    // core refs, entries packed into one word each (packed2) or two
    uint32_t *d_blob2 = nullptr, *d_cblob2 = nullptr;
    uint32_t max_blob2_words = 0, max_rows2 = 0, lb2 = 16;
    bool packed2 = false;
    uint4 *d_cmeta = nullptr;      // (internal count, levels, core refs, entries)
    uint32_t *d_cell_ebase = nullptr;   // index of each cell's first downward entry
    uint32_t max_blob_words = 0, max_cell_labels = 0, max_cell_cnt = 0, max_cell_levels = 0;
    int num_cus = 0;                                   // compute units of the device
    std::map<uint64_t, uint32_t> occ_cache;            // cell-sweep workgroups per CU by (variant, LDS)
    std::mutex occ_mu;                                 // the serving loop's threads launch concurrently
    int cell_occupancy(uint32_t variant, uint32_t threads, size_t lds, uint32_t &per_cu);
    int upload_arc_ranks(const iso::Prep &P);
    int upload_cell_blobs2(const iso::Prep &P, const std::vector<std::vector<uint32_t>> &refs_of);
    uint64_t bytes = 0;
    SweepCtx main;   // context of the direct query calls
    SweepCtx fixed;  // context of the no-allocation entry point (buffers in the static scratch)
    void *scratch_ptr = nullptr;      // device address of this GPU's static scratch
    hipEvent_t fixed_wait = nullptr;  // for waiting on the caller's stream without creating an event
    int setup_fixed();
    int carve_fixed(uint32_t K, uint32_t nu, uint32_t nx, size_t min_cap, size_t &cap);
    SweepCtx aux;    // second context of a batch call, so that consecutive sweeps overlap (made on first use)
    bool aux_ready = false;
    // per-cell sizes for the byte accounting
    std::vector<uint32_t> cell_cnt, cell_words, cell_core_refs;
    std::vector<uint64_t> cell_entries;
    uint64_t core_entries = 0;

    // polygon output (polygon.hip): the rotation system built from the coordinates on first
    // use, and the polygon kernels after a vertex-mask sweep on C
    Rotation rot;
    PolyBufs poly;
    int upload_rotation(const iso::Prep &P, const double *xy, int threads);
    int polygons(SweepCtx &C, uint32_t lanes, PolyResult &out);

    int upload(const iso::Prep &P, int device);
    // launch: copies the inputs and enqueues the whole sweep on C.stream (asynchronous);
    // finish: waits for it, sorts the edge keys and copies them back.  A result with
    // overflow set must be launched again with a larger capacity.
    int launch(SweepCtx &C, const RunArgs &A);
    int finish(SweepCtx &C, RunResult &R);
    int sort_keys(SweepCtx &C, uint32_t cnt_all);
    // RPHAST target selection: the restricted graph of the targets (original ids) for the top
    // table prefix [0, tx) of table_levels levels, uploaded to the device.
    int select_targets(const iso::Prep &P, const uint32_t *targets, uint32_t count, uint32_t tx,
                       uint32_t table_levels, TargetSet &T);
    std::vector<uint32_t> sel_row;   // target selection scratch: position -> row
    int run(SweepCtx &C, const RunArgs &A, RunResult &R);
    // device bytes a context needs for k lanes and an edge capacity (admission control),
    // including the radix sort's temporary storage for that capacity
    size_t ctx_bytes(uint32_t k, size_t cap, size_t upward_entries, bool plain = false) const;
    void release();
};

}  // namespace isodev
