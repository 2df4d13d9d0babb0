// sweep.hip - HIP kernels (gfx950) of the isochrone query and their launch sequence.
//
// Query = upward CH search on the host (Section 2, PHAST upward phase), then on
// the device:
//   1. core sweep: the core block of the sweep order, level by level from the
//      top, each vertex taking min(upward label, tail label + length) over its
//      incoming downward arcs (Section 2, PHAST scanning phase; Section 5,
//      isoPHAST-CP second phase).  Every core vertex also sets its cell's flags
//      i (label <= tau) and o (label + ecc > tau) - the relaxed rule that
//      Section 5 gives for parallel queries - and tests the flagged original
//      arcs at it for isochrone edges (Section 5, output during the sweep).
//      The top levels, where the hierarchy narrows to a near-clique chain, are
//      answered from a precomputed table of downward distances (one (min,+)
//      product per query); the rest runs one launch per level.
//   2. active cells: i and (o or uncovered), plus the source's cell (Section 4
//      definition of an active cell; Section 5 source-cell case).
//   3. cell sweep: one workgroup per active cell for all the queries that
//      activate it (cells are independent, Section 5 parallelisation).  The
//      cell's data and the labels of its vertices and of the core vertices it
//      references live in LDS; levels are separated by workgroup barriers (the
//      narrow top levels by wavefront fences) and isochrone edges are extracted
//      as soon as a label is final.
// In the plain mode step 2 selects every cell (a PHAST one-to-all sweep); with 64
// queries per sweep step 3 is instead a stream of launches, one per cell level
// across all cells, with the labels in device memory.
//
// k queries share one sweep: labels are stored k-interleaved (row of k uint32
// per vertex).  Isochrone edges are collected per workgroup in LDS and appended
// with one output reservation per workgroup as 64-bit keys
// lane << 33 | downward entry << 1 | direction; before the sort each key becomes
// lane << r | rank, where rank is the arc's index among all arcs ordered by
// (tail, head) over original ids and r = ceil(log2 m), and a radix sort over
// r + log2 k bits orders them by (query, tail, head).
#include <hip/hip_runtime.h>

#include <chrono>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <thread>

#include "device.h"

namespace isodev {


constexpr uint32_t INF = 0xFFFFFFFFu;
constexpr uint32_t TAIL_MASK = 0x3FFFFFFFu;
constexpr uint32_t FLAG_FWD = 0x80000000u;
constexpr uint32_t FLAG_REV = 0x40000000u;
constexpr uint32_t FLAGS = FLAG_FWD | FLAG_REV;
constexpr uint32_t LOCAL_MASK = 0xFFFFu;   // cell-local tail index inside a blob entry
constexpr uint32_t NO_SLOT = 0xFFFFFFFFu;
constexpr uint32_t NO_CELL = 0xFFFFFFFFu;

// a + b saturated at INF (one v_add_u32 with the clamp bit)
__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) { return __builtin_elementwise_add_sat(a, b); }

// Output key of an isochrone edge as the sweep kernels write it: the lane, the downward entry
// and the direction (0: the entry's forward arc tail -> head, 1: its reverse arc).  Before the
// sort, k_rank_keys turns it into lane << rb | the arc's rank in (tail, head) order.
__device__ __forceinline__ uint64_t entry_key(uint32_t lane, uint32_t entry, uint32_t rev) {
    return (uint64_t(lane) << 33) | (uint64_t(entry) << 1) | rev;
}

// Sorted keys -> (tail, head) pairs (the rank's entry of arc_pair), and the first position of
// every lane: lane_off[l] = base + the first i whose lane is >= l (lane_off is filled with
// base + the key count beforehand).
__global__ void k_decode(const uint64_t *__restrict__ keys, uint32_t n, uint2 *__restrict__ pairs,
                         uint32_t *__restrict__ lane_off, uint32_t base, const uint2 *__restrict__ arc_pair,
                         uint32_t rb) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = keys[i];
    pairs[i] = arc_pair[uint32_t(k & ((uint64_t(1) << rb) - 1u))];
    const uint32_t j = uint32_t(k >> rb);
    const uint32_t from = i ? uint32_t(keys[i - 1] >> rb) + 1u : 0u;
    for (uint32_t l = from; l <= j; ++l) lane_off[l] = base + i;
}

// Phase profile of the cell sweep, summed on the device so that a sweep needs no copy back:
// per active cell its lanes, internal vertices and entries, and its algorithmic bytes (the
// cell's data streamed once, each active lane reading each referenced core label once), added
// into acc[0..4] = bytes, cells, lanes, vertices, entries.  Every thread reaches the reduction.
// Also acc[5]: the survey's algorithmic bytes of the swept cells (the graph stream at 8 bytes
// per entry plus the offsets, and per (cell, lane) each internal label written once and read
// back once), and acc[6]: chunks of 2^lg lanes (the one-workgroup-per-cell sweep).  words_mode:
// 0 per-item cell data, 1 / 2 per-cell data with wide / packed entries.
__host__ __device__ __forceinline__ uint32_t blob_words(uint32_t cnt, uint32_t nl, uint32_t nrefs, uint32_t ne);
__host__ __device__ __forceinline__ uint32_t c2_words(uint32_t cnt, uint32_t nl, uint32_t nrefs, uint32_t ne,
                                                      bool packed);
__global__ void k_prof_cells(const uint32_t *__restrict__ clist, const uint32_t *__restrict__ counters,
                             const uint64_t *__restrict__ cmask, const uint4 *__restrict__ cmeta,
                             unsigned long long *__restrict__ acc, uint32_t words_mode, uint32_t lg) {
    const uint32_t n = counters[1];
    unsigned long long v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t c = clist[i];
        const uint4 m = cmeta[c];
        const unsigned long long l = (unsigned long long)__popcll(cmask[c]);
        const uint32_t words = words_mode ? c2_words(m.x, m.y, m.z, m.w, words_mode == 2) : blob_words(m.x, m.y, m.z, m.w);
        v[0] += 4ull * words + l * 4ull * m.z;
        v[1] += 1;
        v[2] += l;
        v[3] += m.x;
        v[4] += m.w;
        v[5] += 4ull * (m.x + 1) + 8ull * m.w + 8ull * m.x * l;
        v[6] += (l + (1ull << lg) - 1) >> lg;
    }
#pragma unroll
    for (uint32_t k = 0; k < 7; ++k) {
        for (uint32_t o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], (int)o);
        if (__lane_id() == 0 && v[k]) atomicAdd(&acc[k], v[k]);
    }
}

__global__ void k_fill(uint32_t *__restrict__ p, uint32_t value, uint64_t count) {
    uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (; i < count; i += stride) p[i] = value;
}

// Upward labels: entry i = (position, lane, label).  The first entry to claim a
// position becomes its slot (row of k labels in uval); the table is filled with INF first.
__global__ void k_uset_claim(uint32_t *__restrict__ uslot, const uint32_t *__restrict__ upos, uint32_t nu) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nu) atomicCAS(&uslot[upos[i]], NO_SLOT, i);
}
__global__ void k_uset_write(const uint32_t *__restrict__ uslot, const uint32_t *__restrict__ upos,
                             const uint32_t *__restrict__ ulane, const uint32_t *__restrict__ ulab,
                             uint32_t *__restrict__ uval, uint32_t nu, uint32_t lk) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nu) uval[(uslot[upos[i]] << lk) + ulane[i]] = ulab[i];
}
__global__ void k_uset_clear(uint32_t *__restrict__ uslot, const uint32_t *__restrict__ upos, uint32_t nu) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nu) uslot[upos[i]] = NO_SLOT;
}

// isoPHAST-CD: the core labels come from the host's core search as slot entries; the label of
// core position v for lane j is its entry, or INF where the search did not settle v within the
// lane's limit (the query treats it as out of range).
__global__ void k_core_from_slots(const uint32_t *__restrict__ uslot, const uint32_t *__restrict__ uval,
                                  uint32_t *__restrict__ dcore, uint32_t n_core, uint32_t lk) {
    const uint64_t total = uint64_t(n_core) << lk;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += stride) {
        const uint32_t v = uint32_t(t >> lk), j = uint32_t(t) & ((1u << lk) - 1u);
        const uint32_t sl = uslot[v];
        dcore[t] = sl != NO_SLOT ? uval[(sl << lk) + j] : INF;
    }
}

// Cell flags of a core vertex v for the K lanes of its group (relaxed rule: d <= tau is "in",
// d + ecc > tau is "out"): two wavefront ballots; the group's first thread stores the group's
// K-bit slices as v's lane masks (plain stores, no atomics).  The lanes of a group are
// consecutive in the wavefront (K lanes x S sub-lanes, K * S <= 64), and only sub-lane 0
// holds the final label.  Every thread of the wavefront must call it.
__device__ __forceinline__ void store_vertex_masks(bool act, uint32_t v, uint32_t cell, uint32_t ecc, uint32_t dv,
                                                   uint32_t tau, uint32_t j, uint32_t sub, uint32_t lk,
                                                   uint32_t lgs, uint64_t *__restrict__ vin,
                                                   uint64_t *__restrict__ vout) {
    const bool mine = act && sub == 0 && cell != NO_CELL;
    const uint64_t bin = __ballot(mine && dv <= tau);
    const uint64_t bout = __ballot(mine && sat_add(dv, ecc) > tau);
    if (mine && j == 0) {
        const uint32_t sh = (__lane_id() >> lgs) << lgs;
        const uint64_t m = lk == 6 ? ~0ull : ((1ull << (1u << lk)) - 1ull);
        vin[v] = (bin >> sh) & m;
        vout[v] = (bout >> sh) & m;
    }
}

struct CoreArgs {
    const uint32_t *down_off;
    const uint2 *down_arc;
    uint32_t *dcore;
    const uint32_t *uslot, *uval, *core_cell, *core_ecc, *taus;
    uint64_t *vin, *vout;    // per core vertex: lanes with d <= tau, lanes with d + ecc > tau
    uint64_t *out_keys;
    uint32_t *out_count;
    uint32_t out_cap, lane_base, lk;
    unsigned long long *dbg;   // branch counters (nullptr: none)
};

// Per (vertex, lane, sub-lane): bit k of `in` / `flag` tells whether the sub-lane's k-th entry
// (beg + sub + k * S) has its tail in range / is flagged, for k < 32; `over` marks sub-lanes
// with more than 32 entries.
struct EntryBits {
    uint32_t in = 0, flag = 0;
    bool over = false;
};

// One core vertex v for lane j, sub-lane `sub` of S (= 1 << ls): partial minimum over
// entries beg+sub, beg+sub+S, ...; LAB(tail) gives the tail's label for lane j.  The
// partial minima are combined across the S sub-lanes (lanes K, 2K, ... apart).  Returns
// min(init, the minimum); eb records which entries can straddle tau once the label is known.
template <class ARC, class LAB>
__device__ __forceinline__ uint32_t relax_group(ARC arc, LAB lab, uint32_t beg, uint32_t end, uint32_t sub,
                                                uint32_t S, uint32_t K, uint32_t init, uint32_t tau,
                                                EntryBits &eb) {
    uint32_t m = INF;
    // chunks of up to 8 entries: every entry load of a chunk is issued, then every label load,
    // so a vertex of ordinary degree costs two memory latencies instead of two per entry
    uint32_t k = 0;
    for (uint32_t e = beg + sub; e < end; e += 8 * S, k += 8) {
        uint2 a[8];
        uint32_t l[8];
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) a[u] = e + u * S < end ? arc(e + u * S) : make_uint2(0u, INF);
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) l[u] = e + u * S < end ? lab(a[u].x & TAIL_MASK) : INF;
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) {
            m = min(m, sat_add(l[u], a[u].y));
            if (k + u < 32) {
                if (a[u].x & FLAGS) eb.flag |= 1u << (k + u);
                if (l[u] <= tau) eb.in |= 1u << (k + u);
            } else if (e + u * S < end) {
                eb.over = true;
            }
        }
    }
    for (uint32_t o = K; o < K * S; o <<= 1) m = min(m, (uint32_t)__shfl_xor((int)m, (int)o));
    return min(init, m);
}

// Block-wide list of output keys in LDS (count in *s_n, capacity CORE_KEYS); written out with
// one output reservation per workgroup.
constexpr uint32_t CORE_KEYS = 1024;

// Wavefront-aggregated append of a key to the block's list; a key that finds the list full is
// written out at once.  Every lane of the wavefront must call it.
__device__ __forceinline__ void push_key(bool pred, uint64_t key, uint64_t *s_keys, uint32_t *s_n,
                                         const CoreArgs &A) {
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    const uint32_t lane = __lane_id();
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if ((int)lane == leader) base = atomicAdd(s_n, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (pred) {
        const uint32_t k = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
        if (k < CORE_KEYS) {
            s_keys[k] = key;
        } else {
            if (A.dbg) atomicAdd(&A.dbg[3], 1ull);
            const uint32_t idx = atomicAdd(A.out_count, 1u);
            if (idx < A.out_cap) A.out_keys[idx] = key;
        }
    }
}

// Isochrone edges at core vertex v (label dv final) for lane j: the flagged entries of this
// sub-lane whose tails lie on the other side of tau, from the bits recorded while relaxing
// (one load of the entry's arc ranks for each, INF for a direction that is no arc);
// sub-lanes with more than 32 entries walk theirs again.  Wavefront-uniform loops.
template <class ARC, class LAB>
__device__ __forceinline__ void extract_group(ARC arc, LAB lab, const CoreArgs &A, bool act, uint32_t beg,
                                              uint32_t end, uint32_t sub, uint32_t S, uint32_t j, uint32_t dv,
                                              uint32_t tau, const EntryBits &eb, uint64_t *s_keys, uint32_t *s_n) {
    const bool vin = dv <= tau;
    uint32_t st = act && !eb.over ? (eb.flag & (vin ? ~eb.in : eb.in)) : 0u;
    const bool walk = act && eb.over;
    const uint32_t lane = A.lane_base + j;
    while (__any(st != 0)) {
        const bool have = st != 0;
        const uint32_t k = have ? uint32_t(__ffs(st) - 1) : 0u;
        st &= st - 1u;
        const uint32_t e = beg + sub + k * S;
        const uint32_t x = have ? arc(e).x : 0u;
        push_key(x & FLAG_FWD, entry_key(lane, e, 0u), s_keys, s_n, A);
        push_key(x & FLAG_REV, entry_key(lane, e, 1u), s_keys, s_n, A);
    }
    uint32_t e = walk ? beg + sub : 0, stop = walk ? end : 0;
    while (__any(e < stop)) {
        const bool have = e < stop;
        const uint2 a = have ? arc(e) : make_uint2(0u, 0u);
        const bool str = have && (a.x & FLAGS) && ((lab(a.x & TAIL_MASK) <= tau) != vin);
        if (A.dbg && str) atomicAdd(&A.dbg[2], 1ull);
        push_key(str && (a.x & FLAG_FWD), entry_key(lane, e, 0u), s_keys, s_n, A);
        push_key(str && (a.x & FLAG_REV), entry_key(lane, e, 1u), s_keys, s_n, A);
        e += S;
    }
}

// Start and end of a core kernel's block-wide key list (every thread calls both).
__device__ __forceinline__ void keys_begin(uint32_t *s_n) {
    if (threadIdx.x == 0) *s_n = 0;
    __syncthreads();
}
__device__ __forceinline__ void keys_end(uint64_t *s_keys, uint32_t *s_n, uint32_t *s_base, const CoreArgs &A) {
    __syncthreads();
    const uint32_t n = min(*s_n, CORE_KEYS);   // no key is added any more
    if (n == 0) return;
    if (threadIdx.x == 0) *s_base = atomicAdd(A.out_count, n);
    __syncthreads();
    const uint32_t base = *s_base;
    for (uint32_t k = threadIdx.x; k < n; k += blockDim.x)
        if (base + k < A.out_cap) A.out_keys[base + k] = s_keys[k];
}

// Top of the core as a table: X = positions [0, TX) (the top levels, where the
// hierarchy narrows to a near-clique chain of one-vertex levels).  D[y][x] is the
// length of a shortest path y -> x that uses only vertices of X (upward arcs and
// downward entries among them; 0 on the diagonal, INF if none), precomputed per
// graph.  The host's upward search stops at the first vertices of X it reaches
// (every upward path entering X stays in X), and a query's labels on X are
//   d(x) = min over reached y in X of up(y) + D[y][x]
// - a shortest up-down path to x (Section 2, CH) through its first vertex in X,
// written as one (min,+) product instead of a level-by-level sweep of X.
// The levels of X are a prefix of the table's levels, and a path between two vertices of a
// prefix stays inside it (it goes up, then down), so the table of a prefix is the top-left
// corner of the table (rows `stride` apart).  One wavefront per (64-column tile, lane, split
// of the lane's upward list); the splits are combined with atomicMin into dcore (pre-filled
// with INF).
__global__ void __launch_bounds__(64)
k_top_table(const uint32_t *__restrict__ D, uint32_t TX, uint32_t stride, const uint32_t *__restrict__ xptr,
            const uint32_t *__restrict__ xpos, const uint32_t *__restrict__ xval, uint32_t *__restrict__ dcore,
            uint32_t lk, uint32_t tiles, uint32_t splits) {
    const uint32_t K = 1u << lk;
    uint32_t b = blockIdx.x;
    uint32_t tile = b % tiles;
    uint32_t j = (b / tiles) & (K - 1);
    uint32_t q = b / (tiles * K);
    uint32_t x = tile * 64 + threadIdx.x;
    uint32_t lo = xptr[j], hi = xptr[j + 1];
    uint32_t len = hi - lo, per = (len + splits - 1) / splits;
    uint32_t e0 = lo + q * per, e1 = min(hi, e0 + per);
    uint32_t acc = INF;
    if (x < TX) {
        uint32_t e = e0;
        for (; e + 4 <= e1; e += 4) {
            uint32_t y0 = xpos[e], y1 = xpos[e + 1], y2 = xpos[e + 2], y3 = xpos[e + 3];
            uint32_t d0 = D[size_t(y0) * stride + x], d1 = D[size_t(y1) * stride + x];
            uint32_t d2 = D[size_t(y2) * stride + x], d3 = D[size_t(y3) * stride + x];
            acc = min(min(acc, min(sat_add(xval[e], d0), sat_add(xval[e + 1], d1))),
                      min(sat_add(xval[e + 2], d2), sat_add(xval[e + 3], d3)));
        }
        for (; e < e1; ++e) acc = min(acc, sat_add(xval[e], D[size_t(xpos[e]) * stride + x]));
        if (acc != INF) atomicMin(&dcore[(x << lk) + j], acc);
    }
}

// Flags and isochrone edges of the table vertices (all their labels are final).  S = 1 << ls
// sub-lanes per (vertex, lane) split the entry list: the first pass over the entries finds
// which sub-lanes can hold a straddling arc, the second emits them.
__global__ void __launch_bounds__(256) k_top_finish(CoreArgs A, uint32_t TX, uint32_t ls) {
    __shared__ uint64_t s_keys[CORE_KEYS];
    __shared__ uint32_t s_n, s_base;
    keys_begin(&s_n);
    const uint32_t lk = A.lk, K = 1u << lk, S = 1u << ls, lgs = lk + ls;
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t v = t >> lgs, j = t & (K - 1), sub = (t >> lk) & (S - 1);
    bool act = v < TX;
    uint32_t tau = A.taus[j];
    uint32_t dv = act ? A.dcore[(v << lk) + j] : INF;
    uint32_t beg = act ? A.down_off[v] : 0, end = act ? A.down_off[v + 1] : 0;
    const uint32_t cell = act && sub == 0 ? A.core_cell[v] : NO_CELL;
    const uint32_t ecc = cell != NO_CELL ? A.core_ecc[v] : 0u;
    store_vertex_masks(act, v, cell, ecc, dv, tau, j, sub, lk, lgs, A.vin, A.vout);
    const uint2 *__restrict__ darc = A.down_arc;
    const uint32_t *__restrict__ dc = A.dcore;
    auto arc = [&](uint32_t e) { return darc[e]; };
    auto lab = [&](uint32_t tl) { return dc[(tl << lk) + j]; };
    EntryBits eb;
    relax_group(arc, lab, beg, end, sub, S, K, INF, tau, eb);   // the labels are final: only the bits count
    extract_group(arc, lab, A, act, beg, end, sub, S, j, dv, tau, eb, s_keys, &s_n);
    keys_end(s_keys, &s_n, &s_base, A);
}

// One item of a core level: thread t of the level serves vertex vbeg + (t >> (lk + ls)),
// lane t & (K - 1), sub-lane (t >> lk) & (S - 1).  All lanes of a wavefront must call it.
__device__ __forceinline__ void core_item(const CoreArgs &A, uint32_t t, uint32_t ls, uint32_t vbeg,
                                          uint32_t vend, uint64_t *s_keys, uint32_t *s_n) {
    const uint32_t lk = A.lk, K = 1u << lk, S = 1u << ls, lgs = lk + ls;
    uint32_t v = vbeg + (t >> lgs);
    uint32_t j = t & (K - 1), sub = (t >> lk) & (S - 1);
    bool act = v < vend;
    uint32_t tau = A.taus[j];
    uint32_t init = INF, beg = 0, end = 0, cell = NO_CELL, ecc = 0;
    if (act) {
        beg = A.down_off[v];
        end = A.down_off[v + 1];
        uint32_t s = A.uslot[v];
        if (sub == 0) {
            cell = A.core_cell[v];
            ecc = A.core_ecc[v];
        }
        if (s != NO_SLOT) init = A.uval[(s << lk) + j];
    }
    const uint2 *__restrict__ darc = A.down_arc;
    const uint32_t *__restrict__ dc = A.dcore;
    auto arc = [&](uint32_t e) { return darc[e]; };
    auto lab = [&](uint32_t tl) { return dc[(tl << lk) + j]; };
    EntryBits eb;
    uint32_t dv = relax_group(arc, lab, beg, end, sub, S, K, init, tau, eb);
    if (act && sub == 0) A.dcore[(v << lk) + j] = dv;
    store_vertex_masks(act, v, cell, ecc, dv, tau, j, sub, lk, lgs, A.vin, A.vout);
    extract_group(arc, lab, A, act, beg, end, sub, S, j, dv, tau, eb, s_keys, s_n);
}

// Sub-lanes per vertex for a level: enough to cover its mean in-degree, at most 8, and the
// group (K lanes x S sub-lanes) within one wavefront.
__host__ __device__ __forceinline__ uint32_t level_ls(uint32_t vertices, uint32_t entries, uint32_t K) {
    uint32_t deg = (entries + vertices - 1) / vertices;
    uint32_t ls = 0;
    while ((1u << ls) < deg && (K << (ls + 1)) <= 64u && ls < 3) ++ls;
    return ls;
}

// One core level: positions [vbeg, vend).  The grid is a multiple of 8 blocks; block b takes
// the (b mod 8)-th eighth of the level, so each XCD (blocks are dealt to the 8 XCDs in turn)
// sweeps a contiguous run of positions.  Within a level the core is ordered by cell, so those
// vertices are neighbours and share many tails, whose label rows then meet in one XCD's L2.
__global__ void __launch_bounds__(1024)
k_core_level(CoreArgs A, uint32_t ls, uint32_t vbeg, uint32_t vend) {
    __shared__ uint64_t s_keys[CORE_KEYS];
    __shared__ uint32_t s_n, s_base;
    keys_begin(&s_n);
    const uint32_t b = (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    core_item(A, b * blockDim.x + threadIdx.x, ls, vbeg, vend, s_keys, &s_n);
    keys_end(s_keys, &s_n, &s_base, A);
}

// Vertices per wavefront of the plain sweep's stream (k_plain_level64): their loads are issued
// together, so that a wavefront keeps several label rows in flight.
constexpr uint32_t PV = 4;

// Straddling flagged entries of vertex v (label dv, final): the first 32 entries from their
// recorded bits, a vertex with more walks them again.  Every lane of the wavefront calls it.
__device__ __forceinline__ void plain_extract(const CoreArgs &A, const uint2 *__restrict__ darc,
                                              const uint32_t *__restrict__ lab, uint32_t beg, uint32_t end,
                                              uint32_t in, uint32_t flag, uint32_t dv, uint32_t tau, uint32_t j,
                                              uint64_t *s_keys, uint32_t *s_n) {
    const bool vin = dv <= tau;
    const uint32_t lane = A.lane_base + j;
    if (end - beg <= 32) {
        uint32_t st = flag & (vin ? ~in : in);
        while (__any(st != 0)) {
            const bool have = st != 0;
            const uint32_t k = have ? uint32_t(__ffs(st) - 1) : 0u;
            st &= st - 1u;
            const uint32_t xw = have ? darc[beg + k].x : 0u;
            push_key(xw & FLAG_FWD, entry_key(lane, beg + k, 0u), s_keys, s_n, A);
            push_key(xw & FLAG_REV, entry_key(lane, beg + k, 1u), s_keys, s_n, A);
        }
    } else {
        for (uint32_t e = beg; e < end; ++e) {   // uniform loop
            const uint2 a = darc[e];
            const bool str = (a.x & FLAGS) && ((lab[(uint64_t(a.x & TAIL_MASK) << 6) + j] <= tau) != vin);
            if (A.dbg && str) atomicAdd(&A.dbg[2], 1ull);
            push_key(str && (a.x & FLAG_FWD), entry_key(lane, e, 0u), s_keys, s_n, A);
            push_key(str && (a.x & FLAG_REV), entry_key(lane, e, 1u), s_keys, s_n, A);
        }
    }
}

// A core level for 64 queries per sweep: one wavefront per vertex, lane j = query j.  A core
// vertex's record (CORE_REC uint2 words: its entry offsets, then its first CORE_REC - 1 entries)
// is read by the wavefront's lanes in one coalesced load, together with its slot in the upward
// table, so that its entries' tail rows (one coalesced 256-byte load each, all issued together)
// follow after one memory round trip instead of two.  Entries beyond the record come from the
// downward CSR, eight at a time.  The first 32 entries' "tail in range" bits give the straddling
// entries once the label is final (a vertex with more entries walks them again).  Block b of
// the grid takes the (b mod 8)-th eighth of the level, as in k_core_level.
constexpr uint32_t CORE_REC = 16;

__global__ void __launch_bounds__(256) k_core_level64(CoreArgs A, const uint2 *__restrict__ rec, uint32_t vbeg,
                                                      uint32_t vend) {
    __shared__ uint64_t s_keys[CORE_KEYS];
    __shared__ uint32_t s_n, s_base;
    keys_begin(&s_n);
    const uint32_t b = (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t v = vbeg + b * (blockDim.x >> 6) + wv;   // uniform over the wavefront
    const uint32_t j = __lane_id();
    if (v < vend) {
        const uint32_t tau = A.taus[j];
        const uint2 r = rec[(uint64_t(v) * CORE_REC) + (j & (CORE_REC - 1))];   // lane u: record word u
        const uint32_t sl = A.uslot[v];
        const uint32_t beg = uint32_t(__builtin_amdgcn_readlane(int(r.x), 0));
        const uint32_t end = uint32_t(__builtin_amdgcn_readlane(int(r.y), 0));
        uint32_t dv = INF;
        uint32_t in = 0, flag = 0;   // per entry k < 32: tail in range (this lane), entry flagged
        const uint2 *__restrict__ darc = A.down_arc;
        const uint32_t *__restrict__ dc = A.dcore;
        {   // the record's entries: words 1 .. CORE_REC - 1 (padding: tail 0, length INF, no flags)
            uint32_t tx[CORE_REC - 1], tw[CORE_REC - 1], l[CORE_REC - 1];
#pragma unroll
            for (uint32_t u = 0; u < CORE_REC - 1; ++u) {
                tx[u] = uint32_t(__builtin_amdgcn_readlane(int(r.x), int(u + 1)));
                tw[u] = uint32_t(__builtin_amdgcn_readlane(int(r.y), int(u + 1)));
            }
#pragma unroll
            for (uint32_t u = 0; u < CORE_REC - 1; ++u) l[u] = dc[((tx[u] & TAIL_MASK) << 6) + j];
#pragma unroll
            for (uint32_t u = 0; u < CORE_REC - 1; ++u) {
                dv = min(dv, sat_add(l[u], tw[u]));
                flag |= ((tx[u] & FLAGS) ? 1u : 0u) << u;
                in |= uint32_t(l[u] <= tau) << u;
            }
            // the upward label, for the few vertices with a slot: a load only there
            if (sl != NO_SLOT) dv = min(dv, A.uval[(sl << 6) + j]);
            // the padding words' bits: cleared
            const uint32_t nrec = min(end - beg, CORE_REC - 1);
            const uint32_t keep = nrec >= 32 ? ~0u : ((1u << nrec) - 1u);
            in &= keep;
            flag &= keep;
        }
        for (uint32_t e = beg + CORE_REC - 1; e < end; e += 8) {
            uint2 a[8];
            uint32_t l[8];
#pragma unroll
            for (uint32_t u = 0; u < 8; ++u) a[u] = e + u < end ? darc[e + u] : make_uint2(0u, INF);
#pragma unroll
            for (uint32_t u = 0; u < 8; ++u) l[u] = e + u < end ? dc[((a[u].x & TAIL_MASK) << 6) + j] : INF;
#pragma unroll
            for (uint32_t u = 0; u < 8; ++u) {
                dv = min(dv, sat_add(l[u], a[u].y));
                const uint32_t k = e - beg + u;
                if (k < 32 && e + u < end) {
                    flag |= ((a[u].x & FLAGS) ? 1u : 0u) << k;
                    in |= uint32_t(l[u] <= tau) << k;
                }
            }
        }
        A.dcore[(v << 6) + j] = dv;
        const uint32_t cell = A.core_cell[v];
        if (cell != NO_CELL) {
            const uint32_t ecc = A.core_ecc[v];
            const uint64_t bin = __ballot(dv <= tau), bout = __ballot(sat_add(dv, ecc) > tau);
            if (j == 0) {
                A.vin[v] = bin;
                A.vout[v] = bout;
            }
        }
        // straddling flagged entries: the recorded bits, or a walk over every entry beyond 32
        const bool vin = dv <= tau;
        const uint32_t lane = A.lane_base + j;
        if (end - beg <= 32) {
            uint32_t st = flag & (vin ? ~in : in);
            while (__any(st != 0)) {
                const bool have = st != 0;
                const uint32_t k = have ? uint32_t(__ffs(st) - 1) : 0u;
                st &= st - 1u;
                const uint32_t x = have ? darc[beg + k].x : 0u;
                push_key(x & FLAG_FWD, entry_key(lane, beg + k, 0u), s_keys, &s_n, A);
                push_key(x & FLAG_REV, entry_key(lane, beg + k, 1u), s_keys, &s_n, A);
            }
        } else {
            for (uint32_t e = beg; e < end; ++e) {   // uniform loop
                const uint2 a = darc[e];
                const bool str = (a.x & FLAGS) && ((dc[((a.x & TAIL_MASK) << 6) + j] <= tau) != vin);
                if (A.dbg && str) atomicAdd(&A.dbg[2], 1ull);
                push_key(str && (a.x & FLAG_FWD), entry_key(lane, e, 0u), s_keys, &s_n, A);
                push_key(str && (a.x & FLAG_REV), entry_key(lane, e, 1u), s_keys, &s_n, A);
            }
        }
    }
    keys_end(s_keys, &s_n, &s_base, A);
}

// The plain sweep's internal vertices for 64 queries per sweep, one launch per level counted
// from the top of each cell (Section 2, PHAST: levels in descending order).  A cell's level l
// reads only the core and the cell's own higher levels, so the l-th levels of all cells form
// one launch, and the internal vertices become a stream of about 20 launches of up to millions
// of vertices each.  Labels are rows of 64 words in HBM (the core's rows, then the internal
// positions'), as in k_core_level64: lane j = query j, one coalesced 256-byte row per entry.
// The launch's vertices come as records in list order (PLAIN_REC uint2 words each: the
// position and its first entry, the entry end and whether an entry reads the label, then the
// first PLAIN_REC - 2 entries): a wavefront takes PV consecutive records with one coalesced
// load, issues the rows of their first four entries together, and reaches the rest of the
// entries from the record or the downward CSR.  So a vertex costs two dependent memory round
// trips (record, rows), with its upward slot fetched beside the rows.  The grid is resident (a
// few blocks per compute unit): the blocks of XCD x (block index mod 8) take the x-th eighth of
// the level's list and their wavefronts stride through it, so that the vertices of one cell,
// consecutive in the list, meet in one XCD's L2.  A label that no downward entry reads is not
// written back.
constexpr uint32_t PLAIN_REC = 16;
static_assert(PV * PLAIN_REC <= 64, "a wavefront loads its PV records in one instruction");

__global__ void __launch_bounds__(256)
k_plain_level64(CoreArgs A, const uint2 *__restrict__ prec, uint32_t lb, uint32_t le) {
    __shared__ uint64_t s_keys[CORE_KEYS];
    __shared__ uint32_t s_n, s_base;
    keys_begin(&s_n);
    const uint32_t x = blockIdx.x & 7u, bx = blockIdx.x >> 3, nbx = gridDim.x >> 3;
    const uint32_t len = le - lb, per = (len + 7u) >> 3;
    const uint32_t s0 = lb + min(len, x * per), s1 = lb + min(len, (x + 1u) * per);
    const uint32_t wpb = blockDim.x >> 6;
    const uint32_t w0 = bx * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = nbx * wpb;
    const uint32_t j = __lane_id(), tau = A.taus[j];
    const uint2 *__restrict__ darc = A.down_arc;
    uint32_t *__restrict__ lab = A.dcore;
    // lane j: word j mod PLAIN_REC of the record of list entry i + j / PLAIN_REC (a wavefront's
    // next records are loaded while it works on the current ones)
    uint32_t i = s0 + w0 * PV;
    uint2 r = i < s1 ? prec[uint64_t(min(i + j / PLAIN_REC, s1 - 1u)) * PLAIN_REC + (j % PLAIN_REC)]
                     : make_uint2(0u, 0u);
    for (; i < s1; i += nw * PV) {   // uniform over the wavefront
        uint32_t v[PV], beg[PV], end[PV], wr[PV], dv[PV], in[PV], flag[PV];
#pragma unroll
        for (uint32_t q = 0; q < PV; ++q) {
            const bool act = i + q < s1;
            v[q] = uint32_t(__builtin_amdgcn_readlane(int(r.x), int(q * PLAIN_REC)));
            beg[q] = uint32_t(__builtin_amdgcn_readlane(int(r.y), int(q * PLAIN_REC)));
            end[q] = uint32_t(__builtin_amdgcn_readlane(int(r.x), int(q * PLAIN_REC + 1)));
            wr[q] = uint32_t(__builtin_amdgcn_readlane(int(r.y), int(q * PLAIN_REC + 1)));
            if (!act) end[q] = beg[q];
        }
        // the next records (past the share: its last record again, whose load stays in bounds)
        const uint2 rn = prec[uint64_t(min(i + nw * PV + j / PLAIN_REC, s1 - 1u)) * PLAIN_REC + (j % PLAIN_REC)];
        uint32_t sl[PV];
#pragma unroll
        for (uint32_t q = 0; q < PV; ++q) sl[q] = A.uslot[v[q]];
        // the first four entries of every vertex, from the records: all rows issued together
        uint32_t l[PV][4], tw[PV][4];
#pragma unroll
        for (uint32_t q = 0; q < PV; ++q)
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                const uint32_t tx = uint32_t(__builtin_amdgcn_readlane(int(r.x), int(q * PLAIN_REC + 2 + u)));
                tw[q][u] = uint32_t(__builtin_amdgcn_readlane(int(r.y), int(q * PLAIN_REC + 2 + u)));
                l[q][u] = lab[(uint64_t(beg[q] + u < end[q] ? (tx & TAIL_MASK) : 0u) << 6) + j];
                if (u == 0) flag[q] = 0;
                flag[q] |= uint32_t(beg[q] + u < end[q] && (tx & FLAGS)) << u;
            }
#pragma unroll
        for (uint32_t q = 0; q < PV; ++q) {
            dv[q] = INF;
            in[q] = 0;
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                const bool ok = beg[q] + u < end[q];
                dv[q] = min(dv[q], ok ? sat_add(l[q][u], tw[q][u]) : INF);
                in[q] |= uint32_t(ok && l[q][u] <= tau) << u;
            }
            // the upward label, for the few vertices with a slot (the sources' cells): a load only there
            if (sl[q] != NO_SLOT) dv[q] = min(dv[q], A.uval[(uint64_t(sl[q]) << 6) + j]);
        }
        // further entries: from the record up to PLAIN_REC - 2, then from the downward CSR
#pragma unroll
        for (uint32_t q = 0; q < PV; ++q) {
            const uint32_t deg = end[q] - beg[q], nrec = min(deg, PLAIN_REC - 2);
            for (uint32_t u0 = 4; u0 < nrec; u0 += 4) {   // uniform loop, four rows in flight
                uint32_t tx[4], w[4], t[4];
#pragma unroll
                for (uint32_t k = 0; k < 4; ++k) {
                    const uint32_t u = min(u0 + k, PLAIN_REC - 3);   // a word of the record
                    tx[k] = uint32_t(__builtin_amdgcn_readlane(int(r.x), int(q * PLAIN_REC + 2 + u)));
                    w[k] = uint32_t(__builtin_amdgcn_readlane(int(r.y), int(q * PLAIN_REC + 2 + u)));
                }
#pragma unroll
                for (uint32_t k = 0; k < 4; ++k) t[k] = lab[(uint64_t(tx[k] & TAIL_MASK) << 6) + j];
#pragma unroll
                for (uint32_t k = 0; k < 4; ++k) {
                    const bool ok = u0 + k < nrec;
                    dv[q] = min(dv[q], ok ? sat_add(t[k], w[k]) : INF);
                    flag[q] |= uint32_t(ok && (tx[k] & FLAGS)) << (u0 + k);
                    in[q] |= uint32_t(ok && t[k] <= tau) << (u0 + k);
                }
            }
            for (uint32_t e = beg[q] + PLAIN_REC - 2; e < end[q]; e += 4) {
                uint2 bb[4];
                uint32_t t[4];
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u) bb[u] = darc[e + u < end[q] ? e + u : e];
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u) t[u] = lab[(uint64_t(bb[u].x & TAIL_MASK) << 6) + j];
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u) {
                    const bool ok = e + u < end[q];
                    dv[q] = min(dv[q], ok ? sat_add(t[u], bb[u].y) : INF);
                    const uint32_t k = e - beg[q] + u;
                    if (k < 32) {
                        flag[q] |= uint32_t(ok && (bb[u].x & FLAGS)) << k;
                        in[q] |= uint32_t(ok && t[u] <= tau) << k;
                    }
                }
            }
        }
#pragma unroll
        for (uint32_t q = 0; q < PV; ++q)
            if (i + q < s1 && wr[q]) lab[(uint64_t(v[q]) << 6) + j] = dv[q];
#pragma unroll
        for (uint32_t q = 0; q < PV; ++q)
            if (i + q < s1) plain_extract(A, darc, lab, beg[q], end[q], in[q], flag[q], dv[q], tau, j, s_keys, &s_n);
        r = rn;
    }
    keys_end(s_keys, &s_n, &s_base, A);
}

// Lanes for which each cell is active, one wavefront per cell: the flag rule of the
// cell-restricted sweep, i and (o or uncovered), or the cell holds the lane's source, with i
// and o the ORs of the lane masks of the cell's core vertices (cell_core lists them); in
// plain mode (all_cells = 1) every real lane.  Padding lanes have no source cell and are
// never active.
__global__ void k_cell_masks(const uint32_t *__restrict__ cell_core_off, const uint32_t *__restrict__ cell_core,
                             const uint64_t *__restrict__ vin, const uint64_t *__restrict__ vout,
                             const uint8_t *__restrict__ uncovered, const uint32_t *__restrict__ cell_off,
                             const uint32_t *__restrict__ src_cell, uint32_t k, uint32_t num_cells,
                             uint32_t all_cells, uint64_t *__restrict__ cmask, uint64_t *__restrict__ cin) {
    const uint32_t c = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, lane = __lane_id();
    if (c >= num_cells) return;   // uniform over the wavefront
    const uint32_t sc = lane < k ? src_cell[lane] : NO_CELL;
    const uint64_t real = __ballot(sc != NO_CELL), src = __ballot(sc == c);
    uint64_t m = 0, some_in = 0;
    if (cell_off[c + 1] > cell_off[c]) {
        if (all_cells) {
            m = real;
        } else {
            uint64_t in = 0, out = 0;
            for (uint32_t p = cell_core_off[c] + lane; p < cell_core_off[c + 1]; p += 64) {
                const uint32_t v = cell_core[p];
                in |= vin[v];
                out |= vout[v];
            }
            for (uint32_t o = 32; o > 0; o >>= 1) {
                in |= (uint64_t)__shfl_xor((unsigned long long)in, (int)o);
                out |= (uint64_t)__shfl_xor((unsigned long long)out, (int)o);
            }
            m = ((in & (uncovered[c] ? real : out)) | src) & real;
            some_in = in & real;
        }
    }
    if (lane == 0) {
        cmask[c] = m;
        if (cin) cin[c] = some_in;
    }
}

// Vertices in range, the alternative output of Section 3, as a 64-bit lane mask per position
// (bit j: d_j <= tau_j).  Core positions from their final labels (one ballot per group of K
// lanes; the loop count is the same for every lane of a wavefront).
__global__ void k_vmask_core(const uint32_t *__restrict__ dcore, const uint32_t *__restrict__ taus,
                             uint32_t n_core, uint32_t lk, uint64_t *__restrict__ vmask) {
    const uint32_t K = 1u << lk;
    const uint64_t total = ((uint64_t(n_core) << lk) + 63u) & ~uint64_t(63);
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += stride) {
        const uint32_t v = uint32_t(t >> lk), j = uint32_t(t) & (K - 1);
        const bool act = v < n_core;
        const uint64_t b = __ballot(act && dcore[(uint64_t(v) << lk) + j] <= taus[j]);
        if (act && j == 0) {
            const uint32_t sh = __lane_id() & ~(K - 1);
            vmask[v] = lk == 6 ? b : ((b >> sh) & ((1ull << K) - 1ull));
        }
    }
}

// Internal positions of every cell: the lanes for which the cell is not swept but some core
// vertex of it is in range.  For those the flag rule left o unset and the cell is covered, so
// every core vertex u has d(u) + ecc(u) <= tau and every internal vertex, reached inside the
// cell from some u, is in range.  (A cell with no core vertex in range has no internal vertex
// in range unless it is swept.)  The swept lanes are ORed in by the cell sweep.
__global__ void k_vmask_cells(const uint64_t *__restrict__ cin, const uint64_t *__restrict__ cmask,
                              const uint32_t *__restrict__ cell_off, uint32_t num_cells,
                              uint64_t *__restrict__ vmask) {
    const uint32_t c = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, lane = __lane_id();
    if (c >= num_cells) return;
    const uint64_t full = cin[c] & ~cmask[c];
    for (uint32_t p = cell_off[c] + lane; p < cell_off[c + 1]; p += 64) vmask[p] = full;
}

// Lane masks by position -> one bitmap row of W words per lane over the original ids: each
// wavefront takes 64 consecutive ids, i.e. one word of every row (one ballot per lane).
__global__ void k_vmask_out(const uint64_t *__restrict__ vmask, const uint32_t *__restrict__ pos, uint32_t n,
                            uint32_t W, uint32_t lanes, uint64_t *__restrict__ bits) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x, word = v >> 6, lane = __lane_id();
    const uint64_t w = v < n ? vmask[pos[v]] : 0ull;
    uint64_t mine = 0;
    for (uint32_t j = 0; j < lanes; ++j) {
        const uint64_t b = __ballot((w >> j) & 1ull);
        if (lane == j) mine = b;
    }
    if (lane < lanes && word < W) bits[uint64_t(lane) * W + word] = mine;
}

// One-to-many (RPHAST): one level group of a target set's restricted downward graph, thread per
// (row, lane): the row's upward label (slot table, by position) and the minimum over its
// entries of tail label + length.  Entries are read four at a time (loads issued together).
__global__ void __launch_bounds__(256) k_rphast_level(const uint32_t *__restrict__ off,
                                                      const uint2 *__restrict__ arc,
                                                      const uint32_t *__restrict__ rpos,
                                                      const uint32_t *__restrict__ uslot,
                                                      const uint32_t *__restrict__ uval, uint32_t *__restrict__ lab,
                                                      uint32_t tx, uint32_t rbeg, uint32_t rend, uint32_t lk) {
    const uint32_t K = 1u << lk;
    const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint32_t r = rbeg + uint32_t(t >> lk), j = uint32_t(t) & (K - 1);
    if (r >= rend) return;
    const uint32_t i = r - tx;
    const uint32_t s = uslot[rpos[i]];
    uint32_t d = s != NO_SLOT ? uval[(s << lk) + j] : INF;
    const uint32_t e1 = off[i + 1];
    for (uint32_t e = off[i]; e < e1; e += 4) {
        uint2 a[4];
        uint32_t l[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) a[u] = arc[min(e + u, e1 - 1)];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) l[u] = lab[(uint64_t(a[u].x) << lk) + j];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) d = min(d, sat_add(l[u], a[u].y));
    }
    lab[(uint64_t(r) << lk) + j] = d;
}

// Distances of the lanes to the targets: out[j * count + i] = label of target i's row.
__global__ void k_rphast_out(const uint32_t *__restrict__ lab, const uint32_t *__restrict__ row, uint32_t count,
                             uint32_t lk, uint32_t lanes, uint32_t *__restrict__ out) {
    const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint32_t j = uint32_t(t / count), i = uint32_t(t % count);
    if (j >= lanes) return;
    out[uint64_t(j) * count + i] = lab[(uint64_t(row[i]) << lk) + j];
}

// Sources of the cell sweep's per-cell header records (hdr == nullptr: work items instead).
constexpr uint32_t CELL_HDR = 16;   // words per record: cell, (cnt, nl, nrefs, ne), lanes, cb, ebase, blob
struct CellHdrSrc {
    const uint4 *cmeta;
    const uint32_t *cell_off, *cell_ebase, *cblob;
    uint32_t *hdr;
};

// Active cells (nonzero lane mask) in a list, and either work items or header records.  Items:
// the lanes of a cell are cut into items of at most G = 1 << lg lanes; item c << 6 | q covers
// the lanes of rank [qG, qG + G) in the mask, a cell's items consecutive in the item list.
// Header records (for the one-workgroup-per-cell sweep): the record at a cell's list position
// holds what its workgroup needs before it reads the cell's blob.

__global__ void k_active_cells(const uint64_t *__restrict__ cmask, uint32_t num_cells, uint32_t lg,
                               uint32_t *__restrict__ list, uint32_t *__restrict__ items,
                               uint32_t *__restrict__ counters, CellHdrSrc H) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t m = c < num_cells ? cmask[c] : 0ull;
    const bool act = m != 0;
    // full items of G = 1 << lg lanes, then the rest in one item of the fewest lane slots that
    // hold it, G / 2^shift with shift <= 3 (a workgroup spends about as long per item whatever
    // lanes it holds, and fewer lane slots leave more vertex slots per level)
    const uint32_t L = uint32_t(__popcll(m)), full = L >> lg, rest = L & ((1u << lg) - 1u);
    uint32_t shift = 0;
    while (shift < 3 && shift < lg && rest > 0 && rest <= (1u << (lg - shift - 1))) ++shift;
    const uint32_t nch = act ? full + (rest > 0 ? 1u : 0u) : 0u;
    const uint64_t amask = __ballot(act);
    if (amask == 0) return;
    const uint32_t lane = __lane_id();
    // inclusive scan of the item counts over the wavefront
    uint32_t incl = nch;
    for (uint32_t d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(incl, d);
        if (lane >= d) incl += t;
    }
    const uint32_t total = __shfl(incl, 63);
    uint32_t lbase = 0, ibase = 0;
    if (lane == 0) {
        lbase = atomicAdd(counters + 1, (uint32_t)__popcll(amask));
        ibase = atomicAdd(counters + 2, total);
    }
    lbase = __shfl(lbase, 0);
    ibase = __shfl(ibase, 0);
    if (act && H.hdr) {   // the cell sweep's header records instead of work items
        const uint32_t pos = lbase + (uint32_t)__popcll(amask & ((1ull << lane) - 1ull));
        list[pos] = c;
        const uint4 meta = H.cmeta[c];
        uint32_t *h = H.hdr + size_t(pos) * CELL_HDR;
        h[0] = c;
        h[1] = meta.x;
        h[2] = meta.y;
        h[3] = meta.z;
        h[4] = meta.w;
        h[5] = uint32_t(m);
        h[6] = uint32_t(m >> 32);
        h[7] = H.cell_off[c];
        h[8] = H.cell_ebase[c];
        h[9] = H.cblob[c];
    } else if (act) {
        list[lbase + (uint32_t)__popcll(amask & ((1ull << lane) - 1ull))] = c;
        const uint32_t first = ibase + incl - nch;
        for (uint32_t q = 0; q < full; ++q) items[first + q] = (c << 8) | q;
        if (rest) items[first + full] = (c << 8) | (shift << 6) | (full << shift);
    }
}

// Position of the set bit of rank r (0-based) in m; r must be below popcount(m).
__device__ __forceinline__ uint32_t nth_set_bit(uint64_t m, uint32_t r) {
    uint32_t pos = 0;
#pragma unroll
    for (uint32_t w = 32; w > 0; w >>= 1) {
        const uint32_t lo = uint32_t(__popcll(m & ((1ull << w) - 1ull)));
        if (r >= lo) {
            r -= lo;
            m >>= w;
            pos += w;
        }
    }
    return pos;
}

// Words of a cell blob: offsets (cnt + 1), level bounds (nl + 1), core refs, pad to even,
// entries (2 words each), pad to a multiple of 4.
__host__ __device__ __forceinline__ uint32_t blob_head_words(uint32_t cnt, uint32_t nl, uint32_t nrefs) {
    return ((cnt + 1) + (nl + 1) + nrefs + 1u) & ~1u;
}
__host__ __device__ __forceinline__ uint32_t blob_words(uint32_t cnt, uint32_t nl, uint32_t nrefs, uint32_t ne) {
    return (blob_head_words(cnt, nl, nrefs) + 2 * ne + 3u) & ~3u;
}

struct CellArgs {
    const uint32_t *items, *n_items, *cblob, *blob, *cell_off, *cell_ebase, *dcore, *uslot, *uval, *taus,
        *src_cell;
    const uint64_t *cmask;
    const uint4 *cmeta;
    uint32_t *dist_out;
    uint64_t *vmask;   // vertex output: lane masks by position (nullptr: edges only)
    uint64_t *out_keys;
    uint32_t *out_count;
    uint32_t out_cap, lane_base, lk, lg, num_cells;
};

// Cell workgroups have 256 or 512 threads (the cell_block knob); the item code reads blockDim.x.
constexpr uint32_t CELL_THREADS_MAX = 512;
// Isochrone edges found in a cell are first collected in LDS as candidate words and written
// out in bulk.  A word holds the internal head vertex i (12 bits; a cell has at most 4096
// vertices), the entry's offset k among i's entries (13 bits), the lane slot j (6 bits) and
// the direction (bit 31: the reverse arc).
constexpr uint32_t CAND_CAP = 512;
constexpr uint32_t CAND_K_MAX = 1u << 13;
__device__ __forceinline__ uint32_t cand_word(uint32_t i, uint32_t k, uint32_t j, bool rev) {
    return i | (k << 12) | (j << 25) | (uint32_t(rev) << 31);
}

// Bits of one vertex's first 32 entries, recorded while relaxing: tail in range, forward
// original arc, reverse original arc; `over` marks vertices with more entries.
struct CellBits {
    uint32_t in = 0, fwd = 0, rev = 0;
    bool over = false;
    __device__ __forceinline__ void see(uint32_t k, uint32_t x, bool tail_in) {
        if (k < 32) {
            if (tail_in) in |= 1u << k;
            if (x & FLAG_FWD) fwd |= 1u << k;
            if (x & FLAG_REV) rev |= 1u << k;
        } else {
            over = true;
        }
    }
};
// Relaxes internal vertex v's entries [e0, e1) for the thread's lane slot j into dv, recording
// the extraction bits.  Entries are taken four at a time: the four entry reads are issued,
// then the four label reads, so a vertex of up to four entries waits for two LDS round trips
// instead of two per entry.  Slots past e1 repeat entry e1 - 1 (harmless for the minimum) and
// record no bits.  The loop count is the same for the lanes of one vertex group only, so the
// loop is divergent across the wavefront like the one-entry loop it replaces.
template <class LOAD>
__device__ __forceinline__ void relax_cell_vertex(uint32_t e0, uint32_t e1, uint32_t &dv, CellBits &bits,
                                                  uint32_t tau, const uint32_t *s_lab, uint32_t lg, uint32_t j,
                                                  LOAD load) {
    for (uint32_t e = e0; e < e1; e += 4) {
        uint2 x[4];
        uint32_t lt[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) x[u] = load(min(e + u, e1 - 1));
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) lt[u] = s_lab[((x[u].x & LOCAL_MASK) << lg) + j];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            dv = min(dv, sat_add(lt[u], x[u].y));
            if (e + u < e1) bits.see(e + u - e0, x[u].x, lt[u] <= tau);
        }
    }
}

// Vertex output: the lanes of an item for which internal vertex p is in range (its label dv
// final), ORed over the G lane slots of the vertex (consecutive threads) into p's lane mask
// with one atomic per vertex (items of one cell hold different lanes).  Every thread of the
// wavefront must call it.
__device__ __forceinline__ void or_in_range(uint64_t *vmask, bool act, bool live, uint32_t p, uint32_t dv,
                                            uint32_t tau, uint32_t jj, uint32_t j, uint32_t lg) {
    uint64_t in = act && live && dv <= tau ? (1ull << jj) : 0ull;
    for (uint32_t o = 1; o < (1u << lg); o <<= 1) in |= (uint64_t)__shfl_xor((unsigned long long)in, (int)o);
    if (act && j == 0 && in) atomicOr((unsigned long long *)&vmask[p], (unsigned long long)in);
}

constexpr uint32_t CELL_BUF = 512;         // entries per LDS level buffer (two buffers)
constexpr uint32_t CELL_REGS = CELL_BUF / 256;   // entries per thread held for the next level (at most)

// LDS words of a cell workgroup: offsets and level bounds (padded to even), two level
// buffers of CELL_BUF entries, labels (cnt + refs rows of G lanes).
__host__ __device__ __forceinline__ uint32_t cell_lds_words(uint32_t cnt, uint32_t nl, uint32_t labels,
                                                            uint32_t lg) {
    return ((cnt + 1 + nl + 1 + 1u) & ~1u) + 4 * CELL_BUF + (labels << lg) + CAND_CAP + 4;
}

// Output key of a candidate: the rank of the forward (tail -> internal vertex i) or reverse
// arc of i's k-th entry, whose downward-entry index is the cell's first entry eb plus the
// entry's offset in the cell.  q is the rank of the work item's first lane among the cell's
// active lanes; the candidate's lane slot j is added to it.
__device__ __forceinline__ uint64_t cand_key(const CellArgs &A, uint32_t word, const uint32_t *s_off, uint32_t eb,
                                             uint64_t lanes, uint32_t q) {
    const uint32_t i = word & 0xFFFu, k = (word >> 12) & (CAND_K_MAX - 1u), j = (word >> 25) & 63u;
    const uint32_t lane = A.lane_base + nth_set_bit(lanes, q + j);
    return entry_key(lane, eb + s_off[i] + k, word >> 31);
}

// Wavefront-aggregated append of a candidate to the LDS list (count in ctl[0]); every lane of
// the wavefront must call it.  A candidate beyond the list's capacity is written out at once.
__device__ __forceinline__ void push_cand(bool pred, uint32_t word, uint32_t *s_cand, uint32_t *s_ctl,
                                          const CellArgs &A, const uint32_t *s_off, uint32_t eb, uint64_t lanes,
                                          uint32_t q) {
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    const uint32_t lane = __lane_id();
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if ((int)lane == leader) base = atomicAdd(&s_ctl[0], (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (pred) {
        const uint32_t k = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
        if (k < CAND_CAP) {
            s_cand[k] = word;
        } else {
            const uint64_t key = cand_key(A, word, s_off, eb, lanes, q);
            const uint32_t idx = atomicAdd(A.out_count, 1u);
            if (idx < A.out_cap) A.out_keys[idx] = key;
        }
    }
}

// Writes the first n listed candidates with one output reservation and empties the list.
// Called by every thread with the same n, read from ctl[0] between two barriers.
__device__ __forceinline__ void flush_cands(uint32_t n, uint32_t *s_cand, uint32_t *s_ctl, const CellArgs &A,
                                            const uint32_t *s_off, uint32_t eb, uint64_t lanes, uint32_t q) {
    const uint32_t tid = threadIdx.x;
    if (tid == 0) s_ctl[1] = atomicAdd(A.out_count, n);
    __syncthreads();
    const uint32_t base = s_ctl[1];
    for (uint32_t k = tid; k < n; k += blockDim.x) {
        const uint64_t key = cand_key(A, s_cand[k], s_off, eb, lanes, q);
        if (base + k < A.out_cap) A.out_keys[base + k] = key;
    }
    __syncthreads();
    if (tid == 0) s_ctl[0] = 0;
    __syncthreads();
}

// Isochrone edges at internal vertex i (label dv final) for the thread's lane slot j: its
// flagged entries whose tails lie on the other side of tau, from the bits recorded while
// relaxing; a vertex with more than 32 entries walks them again (ENT gives an entry, and
// s_lab the labels).  Candidates go to the LDS list.  Wavefront-uniform loops.
template <class ENT>
__device__ __forceinline__ void emit_cell_vertex(bool go, uint32_t i, uint32_t e0, uint32_t e1, uint32_t dv,
                                                 uint32_t tau, const CellBits &b, uint32_t j, uint32_t lg,
                                                 const uint32_t *s_lab, uint32_t *s_cand, uint32_t *s_ctl,
                                                 const CellArgs &A, const uint32_t *s_off, ENT ent, uint32_t eb,
                                                 uint64_t lanes, uint32_t q) {
    const bool vin = dv <= tau;
    const uint32_t str = go && !b.over ? (vin ? ~b.in : b.in) : 0u;
    uint32_t sf = str & b.fwd, sr = str & b.rev;
    while (__any((sf | sr) != 0)) {
        const bool hf = sf != 0, hr = sr != 0;
        const uint32_t kf = hf ? uint32_t(__ffs(sf) - 1) : 0u, kr = hr ? uint32_t(__ffs(sr) - 1) : 0u;
        sf &= sf - 1u;
        sr &= sr - 1u;
        push_cand(hf, cand_word(i, kf, j, false), s_cand, s_ctl, A, s_off, eb, lanes, q);
        push_cand(hr, cand_word(i, kr, j, true), s_cand, s_ctl, A, s_off, eb, lanes, q);
    }
    uint32_t e = go && b.over ? e0 : 0u, ee = go && b.over ? e1 : 0u;
    while (__any(e < ee)) {
        const bool have = e < ee;
        const uint2 x = have ? ent(e) : make_uint2(0u, 0u);
        const uint32_t lt = x.x & LOCAL_MASK;
        const bool st = have && (x.x & FLAGS) && ((s_lab[(lt << lg) + j] <= tau) != vin);
        push_cand(st && (x.x & FLAG_FWD), cand_word(i, e - e0, j, false), s_cand, s_ctl, A, s_off, eb, lanes, q);
        push_cand(st && (x.x & FLAG_REV), cand_word(i, e - e0, j, true), s_cand, s_ctl, A, s_off, eb, lanes, q);
        ++e;
    }
}

// End of level l of a work item: one barrier, after which every label of the level is final.
// The candidate list is written out after the last level, and earlier when it held more than
// a quarter of its capacity at the end of the previous level: thread 0 records the count after
// each level's barrier in one of two LDS words (alternating with the level's parity), and
// every thread decides on the word written a level before, so all decide alike without a
// second barrier.
__device__ __forceinline__ void level_end(uint32_t l, uint32_t nl, uint32_t *s_cand, uint32_t *s_ctl,
                                          const CellArgs &A, const uint32_t *s_off, uint32_t eb, uint64_t lanes,
                                          uint32_t q) {
    __syncthreads();
    if (l + 1 == nl) {
        const uint32_t n = s_ctl[0];   // no candidate is added after the last level
        if (n) flush_cands(min(n, CAND_CAP), s_cand, s_ctl, A, s_off, eb, lanes, q);
        return;
    }
    const uint32_t due = l ? s_ctl[2 + ((l - 1) & 1u)] : 0u;
    if (due > CAND_CAP / 4) {
        // every thread is between this level's barrier and the flush: the count is stable
        flush_cands(min(s_ctl[0], CAND_CAP), s_cand, s_ctl, A, s_off, eb, lanes, q);
        if (threadIdx.x == 0) s_ctl[2 + (l & 1u)] = 0;
    } else if (threadIdx.x == 0) {
        s_ctl[2 + (l & 1u)] = s_ctl[0];
    }
}

// One work item (an active cell and up to G = 1 << lg of the lanes for which it is active)
// on one workgroup, level pipeline variant.  Offsets, level bounds and labels live in LDS; the
// entries of level l+1 (contiguous in the blob) are loaded into registers while level l is
// relaxed, then written to the other LDS buffer.  Isochrone edges are extracted right after
// a vertex's label is final.  Slots of an item beyond its lane count repeat its first lane
// and neither write distances nor emit edges.
__device__ __forceinline__ void cell_item_pipelined(const CellArgs &A, uint32_t *smem, uint32_t it) {
    const uint32_t lk = A.lk;
    const uint32_t code = A.items[it];
    // code = cell << 8 | shift << 6 | index: the item has G >> shift lane slots
    const uint32_t c = code >> 8, lg = A.lg - ((code >> 6) & 3u);
    const uint32_t q = (code & 63u) << lg;   // rank of the item's first lane among the cell's
    const uint64_t lanes = A.cmask[c];
    const uint4 meta = A.cmeta[c];
    const uint32_t cnt = meta.x, nl = meta.y, nrefs = meta.z;
    const uint32_t cb = A.cell_off[c];
    const uint32_t *gblob = A.blob + A.cblob[c];
    const uint32_t *grefs = gblob + cnt + 1 + nl + 1;
    const uint2 *gent = reinterpret_cast<const uint2 *>(gblob + blob_head_words(cnt, nl, nrefs));
    uint32_t *s_off = smem;                                   // cnt + 1
    uint32_t *s_lvl = smem + cnt + 1;                         // nl + 1
    uint2 *s_buf = reinterpret_cast<uint2 *>(smem + ((cnt + 1 + nl + 1 + 1u) & ~1u));   // 2 * CELL_BUF
    uint32_t *s_lab = reinterpret_cast<uint32_t *>(s_buf + 2 * CELL_BUF);               // (cnt + nrefs) * G
    uint32_t *s_cand = s_lab + ((cnt + nrefs) << lg);                                   // CAND_CAP
    uint32_t *s_ctl = s_cand + CAND_CAP;                                                // count, base
    auto ent = [&](uint32_t e) { return gent[e]; };
    const uint32_t eb = A.cell_ebase[c];   // the cell's first downward entry
    const uint32_t tid = threadIdx.x;
    const uint32_t G = 1u << lg;
    const uint32_t j = tid & (G - 1);             // slot within the item
    const uint32_t rank = q + j;
    const bool live = rank < uint32_t(__popcll(lanes));
    const uint32_t jj = nth_set_bit(lanes, live ? rank : q);   // lane within the batch
    const uint32_t tau = A.taus[jj];
    const bool has_up = A.src_cell[jj] == c;
    const uint32_t T = blockDim.x, per_iter = T >> lg;
    const uint32_t wfirst = (tid & ~63u) >> lg;   // the first vertex slot of the thread's wavefront
    // touch the whole blob once so that the per-level loads below hit the L2 instead of HBM
    // (16-byte loads, up to eight per thread in flight; indices past the end repeat the last
    // vector); the vectors that hold the offsets and level bounds are stored to LDS, the
    // others are consumed by an empty asm statement.  Stores past the head land in the entry
    // buffer, which is filled after the barrier below.
    {
        const uint4 *g4 = reinterpret_cast<const uint4 *>(gblob);
        uint4 *s4 = reinterpret_cast<uint4 *>(smem);
        const uint32_t n4 = blob_words(cnt, nl, nrefs, meta.w) >> 2, last = n4 - 1;
        const uint32_t h4 = (cnt + 1 + nl + 1 + 3u) >> 2;
        for (uint32_t i = tid; i < n4; i += 8 * T) {
            const uint4 v0 = g4[i], v1 = g4[min(i + T, last)], v2 = g4[min(i + 2 * T, last)];
            const uint4 v3 = g4[min(i + 3 * T, last)], v4 = g4[min(i + 4 * T, last)];
            const uint4 v5 = g4[min(i + 5 * T, last)], v6 = g4[min(i + 6 * T, last)];
            const uint4 v7 = g4[min(i + 7 * T, last)];
            if (i < h4) s4[i] = v0;
            if (i + T < h4) s4[i + T] = v1;
            if (i + 2 * T < h4) s4[i + 2 * T] = v2;
            if (i + 3 * T < h4) s4[i + 3 * T] = v3;
            if (i + 4 * T < h4) s4[i + 4 * T] = v4;
            if (i + 5 * T < h4) s4[i + 5 * T] = v5;
            if (i + 6 * T < h4) s4[i + 6 * T] = v6;
            if (i + 7 * T < h4) s4[i + 7 * T] = v7;
            asm volatile("" ::"v"(v0.x), "v"(v1.x), "v"(v2.x), "v"(v3.x), "v"(v4.x), "v"(v5.x), "v"(v6.x),
                         "v"(v7.x));
        }
    }
    if (tid == 0) s_ctl[0] = s_ctl[2] = s_ctl[3] = 0;
    // labels: internal vertices start at INF, or at their upward labels for a lane whose source
    // lies in the cell.  An internal vertex's slot is first read at its own level (its tails lie on
    // earlier levels or in the core), so only such lanes fill theirs here; the others take INF there.
    if (has_up)
        for (uint32_t i = tid >> lg; i < cnt; i += per_iter) {
            uint32_t val = INF;
            uint32_t s = A.uslot[cb + i];
            if (s != NO_SLOT) val = A.uval[(s << lk) + jj];
            s_lab[(i << lg) + j] = val;
        }
    // ... referenced core vertices take their final core labels (loads issued four at a time)
    for (uint32_t r0 = tid >> lg; r0 < nrefs; r0 += 4 * per_iter) {
        uint32_t rr[4], vv[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            uint32_t r = r0 + u * per_iter;
            rr[u] = r < nrefs ? grefs[r] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            uint32_t r = r0 + u * per_iter;
            vv[u] = r < nrefs ? A.dcore[(rr[u] << lk) + jj] : INF;
        }
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            uint32_t r = r0 + u * per_iter;
            if (r < nrefs) s_lab[((cnt + r) << lg) + j] = vv[u];
        }
    }
    __syncthreads();
    // The leading levels hold a few vertices each: while a level fits the vertex slots of one
    // wavefront and the entries so far fit one buffer, wavefront 0 sweeps it alone (below).
    // Their entries go to buffer 0 in one round of loads, and the entries of the first level
    // after them (l0) to buffer 1, where the level pipeline starts.
    const uint32_t wslots = 64u >> lg, eb0 = s_off[s_lvl[0]];
    uint32_t l0 = 0;
    while (l0 < nl && s_lvl[l0 + 1] - s_lvl[l0] <= wslots && s_off[s_lvl[l0 + 1]] - eb0 <= CELL_BUF) ++l0;
    uint2 r[CELL_REGS];
    {
        const uint32_t n0 = s_off[s_lvl[l0]] - eb0;   // <= CELL_BUF
        const uint32_t eb1 = l0 < nl ? s_off[s_lvl[l0]] : eb0;
        const uint32_t n1 = l0 < nl ? min(s_off[s_lvl[l0 + 1]] - eb1, CELL_BUF) : 0u;
#pragma unroll
        for (uint32_t k = 0; k < CELL_REGS; ++k) {
            uint32_t idx = tid + k * T;
            if (k * T < CELL_BUF && idx < n0) s_buf[idx] = gent[eb0 + idx];
            if (k * T < CELL_BUF && idx < n1) s_buf[CELL_BUF + idx] = gent[eb1 + idx];
        }
    }
    __syncthreads();
    if (l0 > 0 && tid < 64) {
        // the wavefront's lanes see each other's label writes through the in-order LDS accesses
        // of one wavefront (a wavefront-scope fence between levels), not a workgroup barrier
        for (uint32_t l = 0; l < l0; ++l) {
            const uint32_t i = s_lvl[l] + (tid >> lg);
            const bool act = i < s_lvl[l + 1];
            const uint32_t e0 = act ? s_off[i] : 0, e1 = act ? s_off[i + 1] : 0;
            uint32_t dv = act && has_up ? s_lab[(i << lg) + j] : INF;
            CellBits bits;
            relax_cell_vertex(e0, e1, dv, bits, tau, s_lab, lg, j, [&](uint32_t e) { return s_buf[e - eb0]; });
            if (act) {
                s_lab[(i << lg) + j] = dv;
                if (A.dist_out && live) A.dist_out[(uint64_t(cb + i) << lk) + jj] = dv;
            }
            if (A.vmask) or_in_range(A.vmask, act, live, cb + i, dv, tau, jj, j, lg);
            emit_cell_vertex(act && live, i, e0, e1, dv, tau, bits, j, lg, s_lab, s_cand, s_ctl, A, s_off, ent, eb,
                             lanes, q);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (l0 == nl) {   // the whole cell fit one wavefront: write the candidates out
        __syncthreads();
        const uint32_t n = s_ctl[0];
        if (n) flush_cands(min(n, CAND_CAP), s_cand, s_ctl, A, s_off, eb, lanes, q);
        return;
    }
    if (l0) __syncthreads();
    for (uint32_t l = l0; l < nl; ++l) {
        const uint32_t par = (l - l0 + 1) & 1u;   // level l0 is in buffer 1
        const uint2 *cur = s_buf + par * CELL_BUF;
        uint2 *nxt = s_buf + (par ^ 1u) * CELL_BUF;
        const uint32_t a = s_lvl[l], bnd = s_lvl[l + 1];
        const uint32_t ebase = s_off[a];
        const bool in_buf = s_off[bnd] - ebase <= CELL_BUF;
        // prefetch the next level's entries into registers
        uint32_t n1 = 0, eb1 = 0;
        if (l + 1 < nl) {
            eb1 = s_off[bnd];
            n1 = min(s_off[s_lvl[l + 2]] - eb1, CELL_BUF);
#pragma unroll
            for (uint32_t k = 0; k < CELL_REGS; ++k) {
                uint32_t idx = tid + k * T;
                if (k * T < CELL_BUF && idx < n1) r[k] = gent[eb1 + idx];
            }
        }
        for (uint32_t base = a; base < bnd; base += per_iter) {
            // a wavefront with no vertex of the level left stops here (wavefront-uniform; the
            // loop body has no workgroup barrier), so small levels and narrow items do not cost
            // the issue slots of idle wavefronts
            if (base + wfirst >= bnd) break;
            uint32_t i = base + (tid >> lg);
            bool act = i < bnd;
            uint32_t e0 = act ? s_off[i] : 0, e1 = act ? s_off[i + 1] : 0;
            uint32_t dv = act && has_up ? s_lab[(i << lg) + j] : INF;
            CellBits bits;
            if (in_buf) {
                // the level's entries are all in the LDS buffer: no global load here, so the
                // next level's loads stay in flight
                relax_cell_vertex(e0, e1, dv, bits, tau, s_lab, lg, j,
                                  [&](uint32_t e) { return cur[e - ebase]; });
            } else {
                relax_cell_vertex(e0, e1, dv, bits, tau, s_lab, lg, j, [&](uint32_t e) {
                    const uint32_t le = e - ebase;
                    return le < CELL_BUF ? cur[le] : gent[e];
                });
            }
            if (act) {
                s_lab[(i << lg) + j] = dv;
                if (A.dist_out && live) A.dist_out[(uint64_t(cb + i) << lk) + jj] = dv;
            }
            if (A.vmask) or_in_range(A.vmask, act, live, cb + i, dv, tau, jj, j, lg);
            // isochrone edges at vertex i (its tails are on earlier levels or in the core) go to
            // the candidate list
            emit_cell_vertex(act && live, i, e0, e1, dv, tau, bits, j, lg, s_lab, s_cand, s_ctl, A, s_off, ent, eb,
                             lanes, q);
        }
        if (l + 1 < nl) {
#pragma unroll
            for (uint32_t k = 0; k < CELL_REGS; ++k) {
                uint32_t idx = tid + k * T;
                if (k * T < CELL_BUF && idx < n1) nxt[idx] = r[k];
            }
        }
        level_end(l, nl, s_cand, s_ctl, A, s_off, eb, lanes, q);
    }
}

// LDS words of the whole-cell variant: the blob itself, then the labels.
__host__ __device__ __forceinline__ uint32_t staged_lds_words(uint32_t words, uint32_t labels, uint32_t lg) {
    return words + (labels << lg) + CAND_CAP + 4;
}

// Same work item, results and extraction as cell_item_pipelined, but the whole blob (offsets, level
// bounds, core refs, entries) is copied into LDS once, with every load of a chunk issued
// before its stores, so that the level loop touches no global memory except where an
// isochrone edge is written: each level costs LDS accesses and one barrier.  The copy keeps up
// to eight 16-byte loads per thread in flight.
__device__ __forceinline__ void cell_item_staged(const CellArgs &A, uint32_t *smem, uint32_t it) {
    const uint32_t lk = A.lk;
    const uint32_t code = A.items[it];
    // code = cell << 8 | shift << 6 | index: the item has G >> shift lane slots
    const uint32_t c = code >> 8, lg = A.lg - ((code >> 6) & 3u);
    const uint32_t q = (code & 63u) << lg;   // rank of the item's first lane among the cell's
    const uint64_t lanes = A.cmask[c];
    const uint4 meta = A.cmeta[c];
    const uint32_t cnt = meta.x, nl = meta.y, nrefs = meta.z;
    const uint32_t cb = A.cell_off[c];
    const uint32_t *gblob = A.blob + A.cblob[c];
    const uint32_t words = blob_words(cnt, nl, nrefs, meta.w);
    const uint32_t *grefs = gblob + cnt + 1 + nl + 1;
    uint32_t *s_lab = smem + words;                           // (cnt + nrefs) * G
    uint32_t *s_cand = s_lab + ((cnt + nrefs) << lg);         // CAND_CAP
    uint32_t *s_ctl = s_cand + CAND_CAP;                      // count, base
    const uint32_t tid = threadIdx.x;
    const uint32_t G = 1u << lg;
    const uint32_t j = tid & (G - 1);
    const uint32_t rank = q + j;
    const bool live = rank < uint32_t(__popcll(lanes));
    const uint32_t jj = nth_set_bit(lanes, live ? rank : q);
    const uint32_t tau = A.taus[jj];
    const bool has_up = A.src_cell[jj] == c;
    const uint32_t per_iter = blockDim.x >> lg;
    // referenced core labels: loads issued before the blob copy is stored
    const uint32_t r0 = tid >> lg;
    uint32_t rv0 = INF, rv1 = INF;
    if (r0 < nrefs) rv0 = A.dcore[(grefs[r0] << lk) + jj];
    if (r0 + per_iter < nrefs) rv1 = A.dcore[(grefs[r0 + per_iter] << lk) + jj];
    {
        const uint4 *g4 = reinterpret_cast<const uint4 *>(gblob);
        uint4 *s4 = reinterpret_cast<uint4 *>(smem);
        const uint32_t n4 = words >> 2;
        const uint32_t T = blockDim.x;
        const uint32_t last = n4 - 1;   // a blob holds at least its offsets, so n4 >= 1
        for (uint32_t i = tid; i < n4; i += 8 * T) {
            // indices past the end read the last vector again (never stored): no branches
            const uint4 v0 = g4[i], v1 = g4[min(i + T, last)], v2 = g4[min(i + 2 * T, last)];
            const uint4 v3 = g4[min(i + 3 * T, last)], v4 = g4[min(i + 4 * T, last)];
            const uint4 v5 = g4[min(i + 5 * T, last)], v6 = g4[min(i + 6 * T, last)];
            const uint4 v7 = g4[min(i + 7 * T, last)];
            s4[i] = v0;
            if (i + T < n4) s4[i + T] = v1;
            if (i + 2 * T < n4) s4[i + 2 * T] = v2;
            if (i + 3 * T < n4) s4[i + 3 * T] = v3;
            if (i + 4 * T < n4) s4[i + 4 * T] = v4;
            if (i + 5 * T < n4) s4[i + 5 * T] = v5;
            if (i + 6 * T < n4) s4[i + 6 * T] = v6;
            if (i + 7 * T < n4) s4[i + 7 * T] = v7;
        }
    }
    if (r0 < nrefs) s_lab[((cnt + r0) << lg) + j] = rv0;
    if (r0 + per_iter < nrefs) s_lab[((cnt + r0 + per_iter) << lg) + j] = rv1;
    for (uint32_t r = r0 + 2 * per_iter; r < nrefs; r += per_iter)
        s_lab[((cnt + r) << lg) + j] = A.dcore[(grefs[r] << lk) + jj];
    if (tid == 0) s_ctl[0] = s_ctl[2] = s_ctl[3] = 0;
    // internal vertices start at INF; upward labels only in a source's cell
    for (uint32_t i = tid >> lg; i < cnt; i += per_iter) {
        uint32_t val = INF;
        if (has_up) {
            uint32_t s = A.uslot[cb + i];
            if (s != NO_SLOT) val = A.uval[(s << lk) + jj];
        }
        s_lab[(i << lg) + j] = val;
    }
    __syncthreads();
    const uint32_t *s_off = smem;
    const uint32_t *s_lvl = smem + cnt + 1;
    const uint2 *s_ent = reinterpret_cast<const uint2 *>(smem + blob_head_words(cnt, nl, nrefs));
    auto ent = [&](uint32_t e) { return s_ent[e]; };
    const uint32_t eb = A.cell_ebase[c];   // the cell's first downward entry
    // one vertex (slot i of the current level) for the thread's lane slot
    auto sweep_vertex = [&](uint32_t i, bool act) {
        uint32_t e0 = act ? s_off[i] : 0, e1 = act ? s_off[i + 1] : 0;
        uint32_t dv = act ? s_lab[(i << lg) + j] : INF;
        CellBits bits;
        // four entries at a time: their reads, then their tails' labels
        for (uint32_t e = e0; e < e1; e += 4) {
            uint2 x[4];
            uint32_t lt[4];
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) x[u] = e + u < e1 ? s_ent[e + u] : make_uint2(0u, INF);
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) lt[u] = e + u < e1 ? s_lab[((x[u].x & LOCAL_MASK) << lg) + j] : INF;
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                dv = min(dv, sat_add(lt[u], x[u].y));
                if (e + u < e1) bits.see(e + u - e0, x[u].x, lt[u] <= tau);
            }
        }
        if (act) {
            s_lab[(i << lg) + j] = dv;
            if (A.dist_out && live) A.dist_out[(uint64_t(cb + i) << lk) + jj] = dv;
        }
        if (A.vmask) or_in_range(A.vmask, act, live, cb + i, dv, tau, jj, j, lg);
        emit_cell_vertex(act && live, i, e0, e1, dv, tau, bits, j, lg, s_lab, s_cand, s_ctl, A, s_off, ent, eb,
                         lanes, q);
    };
    // The sweep starts with the top of the cell's hierarchy, where levels hold a few vertices:
    // while a level fits the vertex slots of one wavefront, wavefront 0 sweeps it alone, and its
    // lanes see each other's label writes through LDS ordering within a wavefront (a
    // wavefront-scope fence between levels) instead of a workgroup barrier.
    const uint32_t wslots = 64u >> lg;
    uint32_t l0 = 0;
    while (l0 < nl && s_lvl[l0 + 1] - s_lvl[l0] <= wslots) ++l0;
    if (tid < 64) {
        for (uint32_t l = 0; l < l0; ++l) {
            const uint32_t i = s_lvl[l] + (tid >> lg);
            sweep_vertex(i, i < s_lvl[l + 1]);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (l0 == nl) {   // the whole cell fit one wavefront: write the candidates out
        __syncthreads();
        const uint32_t n = s_ctl[0];
        if (n) flush_cands(min(n, CAND_CAP), s_cand, s_ctl, A, s_off, eb, lanes, q);
        return;
    }
    if (l0) __syncthreads();
    for (uint32_t l = l0; l < nl; ++l) {
        const uint32_t a = s_lvl[l], bnd = s_lvl[l + 1];
        for (uint32_t base = a; base < bnd; base += per_iter) {
            const uint32_t i = base + (tid >> lg);
            sweep_vertex(i, i < bnd);
        }
        level_end(l, nl, s_cand, s_ctl, A, s_off, eb, lanes, q);
    }
}

// The cell sweep: a grid of resident workgroups walks the work items.  XCD x (block index
// = x mod 8) takes the x-th eighth of the item list, so the items of one cell, which are
// consecutive, run on the same XCD and share its L2; its workgroups stride through that
// range.  No workgroup waits for another.  At least 6 wavefronts per SIMD (at most 80 VGPRs),
// so that three 512-thread workgroups fit a CU when the LDS of a work item allows it.
template <bool STAGED>
__global__ void __launch_bounds__(CELL_THREADS_MAX) __attribute__((amdgpu_waves_per_eu(6)))
k_cell_sweep(CellArgs A) {
    extern __shared__ uint32_t smem[];
    const uint32_t total = *A.n_items;
    const uint32_t rows = (total + 7u) >> 3;
    const uint32_t x = blockIdx.x & 7u, stride = gridDim.x >> 3;
    const uint32_t end = min(total, (x + 1u) * rows);
    for (uint32_t it = x * rows + (blockIdx.x >> 3); it < end; it += stride) {
        if (STAGED)
            cell_item_staged(A, smem, it);
        else
            cell_item_pipelined(A, smem, it);
        __syncthreads();   // the next item overwrites the LDS
    }
}

// ------------------------------------------------------------ cell sweep, one workgroup per cell
//
// One workgroup takes a whole active cell: it copies the cell's data into LDS once and sweeps
// it for all the queries that activate the cell, up to G of them at a time (a lane chunk), so
// a cell's data crosses HBM once per sweep and the level loop reads LDS only.  Within a chunk
// of W lanes, thread t serves lane slot t mod W of vertex slot t / W of the current level; the
// W slots of a vertex read the same entries and one LDS row of W labels per tail.  The levels
// that fit the vertex slots of one wavefront (the top of the cell's hierarchy) are swept by
// wavefront 0 alone, with wavefront-scope fences instead of workgroup barriers.  Vertices of
// the cell's last level are tails of no entry (every entry goes from an earlier level to a
// later one), so only the earlier levels' labels are stored.
//
// Cell data (one blob per cell, 16-byte aligned, a multiple of 4 words):
//   off[cnt + 1]   entry offsets of the internal vertices (relative to the cell's first entry)
//   lvl[nl + 1]    level starts, top level first; lvl[nl] = cnt
//   refs[nrefs]    the core positions the cell's entries read
//   (padding to an even word), then the entries, one word each in the packed form:
//     bits [0, LB) tail's row (internal vertex i < stored: i; core ref r: stored + r),
//     bit LB the forward original arc, bit LB + 1 the reverse one, bits [LB + 2, 32) the length
//     (below 2^(30 - LB) - 1; all ones for the dummy entry's infinite length),
//   or two words each in the wide form (row | FWD bit 31 | REV bit 30, length), used when a
//   length or a row index does not fit the packed word.
// stored = lvl[nl - 1]: the rows of every level but the last.

constexpr uint32_t C2_CAND = 1024;   // candidate words in LDS: C2_CAND / 2 output keys
constexpr uint32_t C2_CTL = 4;       // control words: candidate count, output base, two claims
constexpr uint32_t C2_THREADS = 512;

struct Cell2Args {
    const uint32_t *hdr, *counters, *blob, *dcore, *uslot, *uval, *taus, *src_cell;   // hdr: CELL_HDR words per cell
    uint32_t *claim;   // per-XCD claim counters (8 words, zero at launch)
    uint32_t *dist_out;
    uint64_t *vmask;
    uint64_t *out_keys;
    uint32_t *out_count;
    uint32_t out_cap, lane_base, lk, lgmax, lb;   // lb: row bits of a packed entry
    unsigned long long *dbg;                      // branch counters (nullptr: none)
};

__host__ __device__ __forceinline__ uint32_t c2_head_words(uint32_t cnt, uint32_t nl, uint32_t nrefs) {
    return ((cnt + 1) + (nl + 1) + nrefs + 1u) & ~1u;
}
__host__ __device__ __forceinline__ uint32_t c2_words(uint32_t cnt, uint32_t nl, uint32_t nrefs, uint32_t ne,
                                                      bool packed) {
    return (c2_head_words(cnt, nl, nrefs) + (packed ? ne : 2 * ne) + 3u) & ~3u;
}
// LDS words of a cell workgroup: control, candidates, the largest blob, label rows of W lanes.
__host__ __device__ __forceinline__ uint32_t c2_lds_words(uint32_t blob_words, uint32_t rows, uint32_t w) {
    return ((blob_words + 3u) & ~3u) + ((rows * w + 3u) & ~3u) + C2_CAND + C2_CTL;
}


// An entry decoded: tail row, length (INF for a dummy entry), forward / reverse original arc.
struct C2Ent {
    uint32_t row, w;
    bool fwd, rev;
};
template <bool PACKED>
__device__ __forceinline__ C2Ent c2_entry(const uint32_t *s_ent, uint32_t e, uint32_t lb) {
    C2Ent r;
    if (PACKED) {
        const uint32_t x = s_ent[e];
        r.row = x & ((1u << lb) - 1u);
        r.fwd = (x >> lb) & 1u;
        r.rev = (x >> (lb + 1)) & 1u;
        const uint32_t wc = x >> (lb + 2), wmax = 0xFFFFFFFFu >> (lb + 2);
        r.w = wc == wmax ? INF : wc;   // all ones: the dummy entry's infinite length
    } else {
        const uint2 x = reinterpret_cast<const uint2 *>(s_ent)[e];
        r.row = x.x & LOCAL_MASK;
        r.fwd = (x.x & FLAG_FWD) != 0;
        r.rev = (x.x & FLAG_REV) != 0;
        r.w = x.y;
    }
    return r;
}

// Appends a candidate's output key (lane, entry, direction) to the workgroup's LDS list, which
// outlives a cell, or writes it out at once when the list is full.
__device__ __forceinline__ void c2_push(const Cell2Args &A, uint64_t *s_cand, uint32_t *s_ctl, uint32_t lane,
                                        uint32_t entry, uint32_t rev) {
    const uint32_t k = atomicAdd(&s_ctl[0], 1u);
    if (k < C2_CAND / 2) {
        s_cand[k] = entry_key(lane, entry, rev);
    } else {
        if (A.dbg) atomicAdd(&A.dbg[0], 1ull);
        const uint32_t idx = atomicAdd(A.out_count, 1u);
        if (idx < A.out_cap) A.out_keys[idx] = entry_key(lane, entry, rev);
    }
}

// Writes the listed keys with one output reservation and empties the list.  Every thread calls
// it with the same n (read between two barriers); it ends with a barrier.
__device__ __forceinline__ void c2_flush(const Cell2Args &A, uint32_t n, const uint64_t *s_cand, uint32_t *s_ctl) {
    const uint32_t tid = threadIdx.x;
    if (tid == 0) s_ctl[1] = atomicAdd(A.out_count, n);
    __syncthreads();
    const uint32_t base = s_ctl[1];
    for (uint32_t k = tid; k < n; k += blockDim.x)
        if (base + k < A.out_cap) A.out_keys[base + k] = s_cand[k];
    __syncthreads();
    if (tid == 0) s_ctl[0] = 0;
    __syncthreads();
}

// One vertex i of the current level for one lane slot j of the chunk (a thread's work; the W
// slots of a vertex are consecutive threads, which read the same entries and the tail's row of
// W labels).  tau, live (a real lane), up (its source lies in the cell: the upward labels
// start the vertex's label), lane (the batch lane).
template <bool PACKED>
__device__ __forceinline__ void c2_vertex(const Cell2Args &A, bool act, uint32_t i, uint32_t j, uint32_t W, uint32_t lw,
                                          const uint32_t *s_off, const uint32_t *s_ent, uint32_t *s_lab,
                                          uint32_t stored, uint32_t tau, bool live, bool up, uint32_t lane,
                                          uint32_t cb, uint64_t *s_cand, uint32_t *s_ctl, uint32_t ebase,
                                          uint32_t lb) {
    uint32_t dv = INF, e0 = 0, e1 = 0;
    if (act) {
        if (up) {   // a source in the cell: its upward label (host search) starts the label
            const uint32_t sl = A.uslot[cb + i];
            if (sl != NO_SLOT) dv = A.uval[(sl << A.lk) + lane];
        }
        e0 = s_off[i];
        e1 = s_off[i + 1];
    }
    bool fin = false, fout = false;   // a flagged entry's tail in / out of range
    // four entries at a time: their words (read whether or not they belong to i: the reads stay
    // inside the workgroup's LDS), then the four tails' labels, then the minimum
    for (uint32_t e = e0; e < e1; e += 4) {
        uint32_t row[4], w[4], t[4];
        bool fl[4];
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
            const C2Ent x = c2_entry<PACKED>(s_ent, e + k, lb);
            const bool valid = e + k < e1;
            row[k] = valid ? x.row : 0u;
            w[k] = valid ? x.w : INF;
            fl[k] = valid && (x.fwd || x.rev);
        }
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) t[k] = s_lab[(row[k] << lw) + j];
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
            dv = min(dv, sat_add(t[k], w[k]));
            fin |= fl[k] && t[k] <= tau;
            fout |= fl[k] && t[k] > tau;
        }
    }
    const bool vin = dv <= tau;
    if (act) {
        if (i < stored) s_lab[(i << lw) + j] = dv;
        if (A.dist_out && live) A.dist_out[(uint64_t(cb + i) << A.lk) + lane] = dv;
    }
    if (A.vmask) {   // lanes in range, ORed over the vertex's W slots (consecutive threads)
        uint64_t m = act && live && vin ? (1ull << lane) : 0ull;
        for (uint32_t o = 1; o < W; o <<= 1) m |= (uint64_t)__shfl_xor((unsigned long long)m, (int)o);
        if (act && j == 0 && m) atomicOr((unsigned long long *)&A.vmask[cb + i], (unsigned long long)m);
    }
    // isochrone edges at i: in range, the flagged entries with tails out of range; out of range,
    // those with tails in range (a second walk, only where one exists)
    if (!(act && live && (vin ? fout : fin))) return;
    for (uint32_t e = e0; e < e1; ++e) {
        const C2Ent x = c2_entry<PACKED>(s_ent, e, lb);
        if (!(x.fwd || x.rev) || ((s_lab[(x.row << lw) + j] <= tau) == vin)) continue;
        if (x.fwd) c2_push(A, s_cand, s_ctl, A.lane_base + lane, ebase + e, 0u);
        if (x.rev) c2_push(A, s_cand, s_ctl, A.lane_base + lane, ebase + e, 1u);
    }
}

// A lane chunk of a staged cell: ranks [q0, q0 + W) of the cell's active lanes (W a power of
// two).  Thread t serves lane slot j = t mod W of vertex slot t / W; live (a real lane), lane
// (the batch lane), tau, up (its source lies in the cell: the upward labels start the vertex's
// label).  The label rows (W words each) follow the blob.
struct C2Lane {
    uint32_t W, lw, j, lane, tau;
    bool live, up;
};

__device__ __forceinline__ C2Lane c2_lane(const Cell2Args &A, uint32_t c, uint64_t lanes, uint32_t L, uint32_t q0,
                                          uint32_t W) {
    C2Lane r;
    r.W = W;
    r.lw = __builtin_ctz(W);
    r.j = threadIdx.x & (W - 1);
    const uint32_t rank = q0 + r.j;
    r.live = rank < L;
    r.lane = nth_set_bit(lanes, r.live ? rank : q0);
    r.tau = A.taus[r.lane];
    r.up = r.live && A.src_cell[r.lane] == c;
    return r;
}

// The referenced core vertices' final labels of the chunk's lanes into their LDS rows, one
// (ref, slot) pair per thread, four rows of a thread in flight before their stores; ends with a
// barrier.
__device__ __forceinline__ void c2_rows(const Cell2Args &A, const C2Lane &q, const uint32_t *s_refs, uint32_t nrefs,
                                        uint32_t *s_lab, uint32_t stored) {
    const uint32_t step = blockDim.x >> q.lw;
    for (uint32_t r = threadIdx.x >> q.lw; r < nrefs; r += 4 * step) {
        uint32_t v[4];
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
            const uint32_t x = r + k * step;
            v[k] = x < nrefs ? A.dcore[(s_refs[x] << A.lk) + q.lane] : 0u;
        }
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k)
            if (r + k * step < nrefs) s_lab[((stored + r + k * step) << q.lw) + q.j] = v[k];
    }
    __syncthreads();
}

// The chunk's levels.  The leading levels that fit wavefront 0 (64 / W vertices) are swept by
// it alone, with wavefront-scope fences between them; the other wavefronts join at the first
// wider level.
template <bool PACKED>
__device__ __forceinline__ void c2_levels(const Cell2Args &A, const C2Lane &q, uint32_t *s_ctl, uint64_t *s_cand,
                                          const uint32_t *blob, uint32_t *s_lab, uint32_t cnt, uint32_t nl,
                                          uint32_t nrefs, uint32_t stored, uint32_t cb, uint32_t ebase) {
    const uint32_t tid = threadIdx.x, T = blockDim.x;
    const uint32_t *s_off = blob, *s_lvl = blob + cnt + 1;
    const uint32_t *s_ent = blob + c2_head_words(cnt, nl, nrefs);
    const uint32_t wslots = 64u >> q.lw;   // vertex slots of one wavefront
    uint32_t l0 = 0;
    while (l0 < nl && s_lvl[l0 + 1] - s_lvl[l0] <= wslots) ++l0;
    const uint32_t per = T >> q.lw, wfirst = (tid & ~63u) >> q.lw;
    for (uint32_t l = tid < 64 ? 0u : l0; l < nl; ++l) {
        if (l == l0) __syncthreads();   // wavefront 0 done with the leading levels, the others waiting
        const uint32_t a = s_lvl[l], b = s_lvl[l + 1];
        if (A.dbg && tid == 0 && b - a > per) atomicAdd(&A.dbg[1], 1ull);
        for (uint32_t base = a; base < b; base += per) {
            if (base + wfirst >= b) break;   // whole wavefronts past the level's end
            const uint32_t i = base + (tid >> q.lw);
            c2_vertex<PACKED>(A, i < b, i, q.j, q.W, q.lw, s_off, s_ent, s_lab, stored, q.tau, q.live, q.up, q.lane,
                              cb, s_cand, s_ctl, ebase, A.lb);
        }
        if (l < l0) {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        } else {
            __syncthreads();
        }
    }
    if (l0 == nl) __syncthreads();
}

constexpr uint32_t C2_NONE = 0xFFFFFFFFu;   // no header record

// A cell's header, wavefront-uniform: the cell, its sizes (cnt, nl, nrefs, ne), active lanes,
// first vertex position, first entry index and blob offset.
struct C2Cell {
    uint32_t c, cnt, nl, nrefs, ne, cb, ebase, cblob;
    uint64_t lanes;
};

// The header record at list position p (none for C2_NONE), lane l < 10 of each wavefront
// holding its word l: a vector load, so that the barriers between its issue and its use (which
// wait for LDS and scalar loads) do not wait for it.
__device__ __forceinline__ uint32_t c2_head(const Cell2Args &A, uint32_t p) {
    const uint32_t l = threadIdx.x & 63u;
    return p != C2_NONE && l < 10u ? A.hdr[size_t(p) * CELL_HDR + l] : 0u;
}

__device__ __forceinline__ C2Cell c2_unpack(uint32_t h) {
    C2Cell r;
    r.c = __builtin_amdgcn_readlane(h, 0);
    r.cnt = __builtin_amdgcn_readlane(h, 1);
    r.nl = __builtin_amdgcn_readlane(h, 2);
    r.nrefs = __builtin_amdgcn_readlane(h, 3);
    r.ne = __builtin_amdgcn_readlane(h, 4);
    r.lanes = uint64_t(uint32_t(__builtin_amdgcn_readlane(h, 5))) |
              (uint64_t(uint32_t(__builtin_amdgcn_readlane(h, 6))) << 32);
    r.cb = __builtin_amdgcn_readlane(h, 7);
    r.ebase = __builtin_amdgcn_readlane(h, 8);
    r.cblob = __builtin_amdgcn_readlane(h, 9);
    return r;
}

// The first four rounds of a cell's blob (a round: one 16-byte word per thread), loaded ahead.
struct C2Pf {
    uint4 a, b, c, d;
};

// Issues the loads of the first four rounds of a cell's blob; an index past the blob reads its
// last word, so every load stays inside it.
template <bool PACKED>
__device__ __forceinline__ C2Pf c2_fetch(const Cell2Args &A, const C2Cell &h) {
    const uint4 *g4 = reinterpret_cast<const uint4 *>(A.blob + h.cblob);
    const uint32_t last = (c2_words(h.cnt, h.nl, h.nrefs, h.ne, PACKED) >> 2) - 1u;   // n4 >= 1
    const uint32_t t = threadIdx.x, T = blockDim.x;
    C2Pf v;
    v.a = g4[min(t, last)];
    v.b = g4[min(t + T, last)];
    v.c = g4[min(t + 2 * T, last)];
    v.d = g4[min(t + 3 * T, last)];
    return v;
}

// Stores the fetched rounds of the cell's blob into LDS and copies the rest (blobs of more than
// four rounds) directly, every load of a round before its stores.
template <bool PACKED>
__device__ __forceinline__ void c2_stage(const Cell2Args &A, const C2Cell &h, const C2Pf &v, uint32_t *smem) {
    const uint32_t tid = threadIdx.x, T = blockDim.x;
    const uint32_t n4 = c2_words(h.cnt, h.nl, h.nrefs, h.ne, PACKED) >> 2, last = n4 - 1;
    uint4 *s4 = reinterpret_cast<uint4 *>(smem);
    if (tid < n4) s4[tid] = v.a;
    if (tid + T < n4) s4[tid + T] = v.b;
    if (tid + 2 * T < n4) s4[tid + 2 * T] = v.c;
    if (tid + 3 * T < n4) s4[tid + 3 * T] = v.d;
    const uint4 *g4 = reinterpret_cast<const uint4 *>(A.blob + h.cblob);
    for (uint32_t i = tid + 4 * T; i < n4; i += 4 * T) {
        const uint4 v0 = g4[i], v1 = g4[min(i + T, last)], v2 = g4[min(i + 2 * T, last)];
        const uint4 v3 = g4[min(i + 3 * T, last)];
        s4[i] = v0;
        if (i + T < n4) s4[i + T] = v1;
        if (i + 2 * T < n4) s4[i + 2 * T] = v2;
        if (i + 3 * T < n4) s4[i + 3 * T] = v3;
    }
}

// The list position of claim k on the counter of XCD range (x + xs) mod 8; while that range is
// used up, the workgroup moves on to the next XCD's range (xs + 1) with a claim there.  Returns
// C2_NONE once all eight ranges are used up.  Every thread calls it with the same arguments.
__device__ __forceinline__ uint32_t c2_next(const Cell2Args &A, uint32_t *s_ctl, uint32_t x, uint32_t &xs,
                                            uint32_t rows, uint32_t total, uint32_t k) {
    for (;;) {
        const uint32_t lo = ((x + xs) & 7u) * rows, end = min(total, lo + rows);
        if (k < rows && lo + k < end) return lo + k;
        if (++xs == 8u) return C2_NONE;
        __syncthreads();   // every thread has read the previous claim
        if (threadIdx.x == 0) s_ctl[3] = atomicAdd(A.claim + ((x + xs) & 7u), 1u);
        __syncthreads();
        k = s_ctl[3];
    }
}

// The cell sweep over the active cells.  The active-cell list is cut into eight ranges, one per
// XCD (neighbouring cells share core rows in that XCD's L2).  The workgroups of XCD x (block
// index mod 8) claim cells one at a time from range x's counter, so that a workgroup given heavy
// cells takes fewer, then from the other XCDs' ranges in turn once range x is used up.  A
// workgroup works ahead: while it sweeps a cell, the header record of the next one is read with
// the first chunk's core rows, then that cell's blob is in flight to registers and the claim
// after it to thread 0.  A cell's lanes are swept in chunks of up to 2^lgmax lanes, the last one
// as narrow as its lanes allow.  No workgroup waits for another.
template <bool PACKED>
__global__ void __launch_bounds__(C2_THREADS) k_cell_chunks(Cell2Args A) {
    extern __shared__ uint32_t smem[];
    // LDS: control words (candidate count, output base, two claim words), the candidate keys,
    // then the current cell's blob and label rows
    uint32_t *s_ctl = smem;
    uint64_t *s_cand = reinterpret_cast<uint64_t *>(smem + C2_CTL);
    uint32_t *s_cell = smem + C2_CTL + C2_CAND;
    const uint32_t tid = threadIdx.x;
    const uint32_t total = A.counters[1];
    if (total == 0) return;
    const uint32_t rows = (total + 7u) >> 3;
    const uint32_t x = blockIdx.x & 7u;
    uint32_t xs = 0;   // claims come from range (x + xs) mod 8
    if (tid == 0) {
        s_ctl[0] = 0;
        s_ctl[2] = atomicAdd(A.claim + x, 1u);
    }
    __syncthreads();
    const uint32_t p0 = c2_next(A, s_ctl, x, xs, rows, total, s_ctl[2]);
    if (p0 != C2_NONE) {
        C2Cell h = c2_unpack(c2_head(A, p0));
        C2Pf v = c2_fetch<PACKED>(A, h);
        __syncthreads();   // every thread has read the first claim
        if (tid == 0) s_ctl[2] = atomicAdd(A.claim + ((x + xs) & 7u), 1u);
        __syncthreads();
        uint32_t pn = c2_next(A, s_ctl, x, xs, rows, total, s_ctl[2]);   // the next cell's position
        uint32_t hn = c2_head(A, pn);
        const uint32_t G = 1u << A.lgmax;
        for (;;) {
            c2_stage<PACKED>(A, h, v, s_cell);
            const bool more = pn != C2_NONE;
            C2Cell nxt = h;
            uint32_t q = 0;   // thread 0: the claim after the next cell
            __syncthreads();
            const uint32_t L = uint32_t(__popcll(h.lanes));
            const uint32_t words = c2_words(h.cnt, h.nl, h.nrefs, h.ne, PACKED);
            const uint32_t stored = h.nl ? s_cell[h.cnt + 1 + h.nl - 1] : 0u;
            const uint32_t *s_refs = s_cell + h.cnt + 1 + h.nl + 1;
            uint32_t *s_lab = s_cell + ((words + 3u) & ~3u);
            for (uint32_t q0 = 0; q0 < L; q0 += G) {
                const uint32_t rest = min(G, L - q0);
                uint32_t W = 1;
                while (W < rest) W <<= 1;   // the narrowest power of two that holds the chunk's lanes
                const C2Lane ql = c2_lane(A, h.c, h.lanes, L, q0, W);
                c2_rows(A, ql, s_refs, h.nrefs, s_lab, stored);
                if (q0 == 0 && more) {   // the rows were waited for, and with them the header record
                    nxt = c2_unpack(hn);
                    v = c2_fetch<PACKED>(A, nxt);
                    if (tid == 0) q = atomicAdd(A.claim + ((x + xs) & 7u), 1u);
                }
                c2_levels<PACKED>(A, ql, s_ctl, s_cand, s_cell, s_lab, h.cnt, h.nl, h.nrefs, stored, h.cb, h.ebase);
                // every thread passed the chunk's last barrier: the count is stable.  The list is
                // written out once half full, else after the workgroup's last cell.
                const uint32_t n = s_ctl[0];
                if (n > C2_CAND / 4) c2_flush(A, min(n, C2_CAND / 2), s_cand, s_ctl);
            }
            if (tid == 0) s_ctl[2] = q;
            __syncthreads();   // the claim is visible; the next cell overwrites the LDS
            if (!more) break;
            h = nxt;
            pn = c2_next(A, s_ctl, x, xs, rows, total, s_ctl[2]);
            hn = c2_head(A, pn);
        }
    }
    const uint32_t n = s_ctl[0];
    if (n) c2_flush(A, min(n, C2_CAND / 2), s_cand, s_ctl);
}

// Entry keys -> output keys: lane << rb | the rank of the entry's forward or reverse arc.
__global__ void k_rank_keys(uint64_t *__restrict__ keys, const uint32_t *__restrict__ count, uint32_t cap,
                            const uint2 *__restrict__ arc_rank, uint32_t rb) {
    const uint32_t n = min(*count, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint64_t k = keys[i];
        const uint2 r = arc_rank[uint32_t(k >> 1)];
        keys[i] = (uint64_t(uint32_t(k >> 33)) << rb) | ((k & 1u) ? r.y : r.x);
    }
}

// ----------------------------------------------------------------- host side

#define HIPCHK(x)                                                                   \
    do {                                                                            \
        hipError_t _e = (x);                                                        \
        if (_e != hipSuccess) {                                                     \
            set_error(std::string(#x) + ": " + hipGetErrorString(_e));              \
            return -3;                                                              \
        }                                                                           \
    } while (0)

static uint32_t ilog2(uint32_t x) {
    uint32_t r = 0;
    while ((1u << r) < x) ++r;
    return r;
}

template <class T>
static int dev_alloc_copy(T **dst, const T *src, size_t count, uint64_t &bytes) {
    size_t b = std::max<size_t>(16, count * sizeof(T));
    HIPCHK(hipMalloc((void **)dst, b));
    bytes += b;
    if (count) HIPCHK(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
    return 0;
}
template <class T>
static int dev_alloc_copy(T **dst, const std::vector<T> &src, uint64_t &bytes) {
    return dev_alloc_copy(dst, src.data(), src.size(), bytes);
}

void TargetSet::release() {
    if (device < 0) return;
    hipSetDevice(device);
    void *ptrs[] = {d_off, d_arc, d_rpos, d_row};
    for (void *p : ptrs) if (p) hipFree(p);
    *this = TargetSet();
}

// RPHAST target selection: a breadth-first search from the targets against the direction of
// the downward entries (from a vertex to the tails of its entries) collects every vertex with
// a downward path to a target; only these need labels.  The search does not continue inside
// the top table, whose labels all come from the table product.  The collected vertices below
// the table are grouped by level and laid out as rows after the table's, each with its entries
// of finite length re-pointed at rows.
int DevGraph::select_targets(const iso::Prep &P, const uint32_t *targets, uint32_t count, uint32_t tx,
                             uint32_t table_levels, TargetSet &T) {
    T = TargetSet();
    T.device = device;
    T.count = count;
    T.tx = tx;
    T.table_levels = table_levels;
    // position -> row (NO_SLOT: not collected yet); kept across selections, and only the
    // entries a selection touches are reset at its end
    std::vector<uint32_t> &row = sel_row;
    if (row.size() != P.n) row.assign(P.n, NO_SLOT);
    std::vector<uint32_t> found, stack;
    struct Reset {   // also on an exception: every marked position is in found or on the stack
        std::vector<uint32_t> &row, &found, &stack;
        ~Reset() {
            for (uint32_t p : found) row[p] = NO_SLOT;
            for (uint32_t p : stack) row[p] = NO_SLOT;
        }
    } reset{row, found, stack};
    for (uint32_t i = 0; i < count; ++i) {
        const uint32_t p = P.pos[targets[i]];
        if (p >= tx && row[p] == NO_SLOT) {
            row[p] = 0;
            stack.push_back(p);
        }
    }
    while (!stack.empty()) {
        const uint32_t p = stack.back();
        found.push_back(p);   // before the pop: a marked position is always in one of the two
        stack.pop_back();
        for (uint32_t e = P.down_off[p]; e < P.down_off[p + 1]; ++e) {
            const uint32_t u = P.down_arc[2 * uint64_t(e)] & TAIL_MASK;
            if (u >= tx && row[u] == NO_SLOT) {
                row[u] = 0;
                stack.push_back(u);
            }
        }
    }
    // group key: core level, then (after every core level) the cell-local level
    const uint32_t ncl = uint32_t(P.core_lvl.size() - 1);
    auto key = [&](uint32_t p) -> uint32_t {
        if (p < P.n_core)
            return uint32_t(std::upper_bound(P.core_lvl.begin(), P.core_lvl.end(), p) - P.core_lvl.begin()) - 1;
        const uint32_t c = P.cell_of[P.perm[p]];
        const auto b = P.cell_lvl.begin() + P.cell_lvl_ptr[c], e = P.cell_lvl.begin() + P.cell_lvl_ptr[c + 1];
        return ncl + uint32_t(std::upper_bound(b, e, p) - b) - 1;
    };
    std::vector<std::pair<uint32_t, uint32_t>> kp(found.size());
    for (size_t i = 0; i < found.size(); ++i) kp[i] = {key(found[i]), found[i]};
    std::sort(kp.begin(), kp.end());
    T.nr = uint32_t(kp.size());
    std::vector<uint32_t> rpos(T.nr), off(size_t(T.nr) + 1, 0);
    for (uint32_t i = 0; i < T.nr; ++i) {
        rpos[i] = kp[i].second;
        row[kp[i].second] = tx + i;
        if (i == 0 || kp[i].first != kp[i - 1].first) T.group.push_back(tx + i);
    }
    T.group.push_back(tx + T.nr);
    std::vector<uint2> arc;
    for (uint32_t i = 0; i < T.nr; ++i) {
        const uint32_t p = rpos[i];
        for (uint32_t e = P.down_off[p]; e < P.down_off[p + 1]; ++e) {
            const uint32_t u = P.down_arc[2 * uint64_t(e)] & TAIL_MASK, w = P.down_arc[2 * uint64_t(e) + 1];
            if (w == INF) continue;   // a dummy entry (reverse arc only) carries no path
            arc.push_back(make_uint2(u < tx ? u : row[u], w));
        }
        off[i + 1] = uint32_t(arc.size());
    }
    T.arcs = arc.size();
    std::vector<uint32_t> trow(count);
    for (uint32_t i = 0; i < count; ++i) {
        const uint32_t p = P.pos[targets[i]];
        trow[i] = p < tx ? p : row[p];
    }
    HIPCHK(hipSetDevice(device));
    int r;
    if ((r = dev_alloc_copy(&T.d_off, off, T.bytes))) return r;
    if ((r = dev_alloc_copy(&T.d_arc, arc, T.bytes))) return r;
    if ((r = dev_alloc_copy(&T.d_rpos, rpos, T.bytes))) return r;
    if ((r = dev_alloc_copy(&T.d_row, trow, T.bytes))) return r;
    return 0;
}

// Workgroups of a cell-sweep variant that fit one compute unit with `lds` bytes of LDS each
// (cached per variant and size).
int DevGraph::cell_occupancy(uint32_t variant, uint32_t threads, size_t lds, uint32_t &per_cu) {
    const uint64_t key = (uint64_t(variant) << 40) | (uint64_t(threads) << 24) | lds;
    std::lock_guard<std::mutex> lock(occ_mu);
    auto f = occ_cache.find(key);
    if (f != occ_cache.end()) {
        per_cu = f->second;
        return 0;
    }
    // variants: 0 level pipeline, 1 staged work item, 2 / 3 one workgroup per cell (wide / packed)
    const void *fn = variant == 0   ? (const void *)k_cell_sweep<false>
                     : variant == 1 ? (const void *)k_cell_sweep<true>
                     : variant == 2 ? (const void *)k_cell_chunks<false>
                                    : (const void *)k_cell_chunks<true>;
    int nb = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, int(threads), lds));
    per_cu = uint32_t(std::max(1, nb));
    occ_cache[key] = per_cu;
    return 0;
}

// Output keys of isochrone edges.  Every arc of the input is flagged on exactly one downward
// entry: forward (the entry's tail -> the entry's vertex) or reverse.  The arcs are ranked by
// (tail, head) over original ids (a counting sort by tail, then each tail's few heads sorted);
// an edge key is lane << rank_bits | rank, so sorted keys come out in (lane, tail, head) order
// with fewer bits than two vertex ids take, and decoding a key is one lookup in the rank's
// (tail, head) table.  Per entry the device keeps the ranks of its two arcs (INF: no arc).
int DevGraph::upload_arc_ranks(const iso::Prep &P) {
    const uint64_t E = P.down_off[n];
    std::vector<uint32_t> start(size_t(n) + 2, 0);
    for (uint32_t v = 0; v < n; ++v)
        for (uint64_t e = P.down_off[v]; e < P.down_off[v + 1]; ++e) {
            const uint32_t x = P.down_arc[2 * e], t = x & TAIL_MASK;
            if (x & FLAG_FWD) ++start[size_t(P.perm[t]) + 2];
            if (x & FLAG_REV) ++start[size_t(P.perm[v]) + 2];
        }
    for (size_t i = 2; i < start.size(); ++i) start[i] += start[i - 1];
    const uint64_t M = start[size_t(n) + 1];
    if (M >= INF || E >= INF) {
        set_error("too many arcs for 32-bit arc ranks");
        return -1;
    }
    // bucket by original tail: (head << 33 | entry << 1 | reverse), then sort each bucket
    std::vector<uint64_t> arcs(std::max<uint64_t>(1, M));
    for (uint32_t v = 0; v < n; ++v)
        for (uint64_t e = P.down_off[v]; e < P.down_off[v + 1]; ++e) {
            const uint32_t x = P.down_arc[2 * e], t = x & TAIL_MASK;
            const uint32_t ot = P.perm[t], ov = P.perm[v];
            if (x & FLAG_FWD) arcs[start[size_t(ot) + 1]++] = (uint64_t(ov) << 33) | (e << 1);
            if (x & FLAG_REV) arcs[start[size_t(ov) + 1]++] = (uint64_t(ot) << 33) | (e << 1) | 1u;
        }
    std::vector<uint2> rank(std::max<uint64_t>(1, E), make_uint2(INF, INF));
    std::vector<uint2> pair(std::max<uint64_t>(1, M));
    for (uint32_t u = 0; u < n; ++u) {
        const uint32_t a = start[u], b = start[size_t(u) + 1];
        std::sort(arcs.begin() + a, arcs.begin() + b);
        for (uint32_t r = a; r < b; ++r) {
            const uint64_t w = arcs[r];
            const uint64_t e = (w >> 1) & ((uint64_t(1) << 32) - 1u);
            if (w & 1u) rank[e].y = r;
            else rank[e].x = r;
            pair[r] = make_uint2(u, uint32_t(w >> 33));
        }
    }
    rank_bits = 1;
    while ((uint64_t(1) << rank_bits) < M) ++rank_bits;
    std::vector<uint32_t> ebase(std::max<uint32_t>(1, num_cells), 0);
    for (uint32_t c = 0; c < num_cells; ++c) ebase[c] = P.down_off[P.cell_off[c]];
    int r;
    if ((r = dev_alloc_copy(&d_arc_rank, rank, bytes))) return r;
    if ((r = dev_alloc_copy(&d_arc_pair, pair, bytes))) return r;
    if ((r = dev_alloc_copy(&d_cell_ebase, ebase, bytes))) return r;
    return 0;
}

// Cell data of k_cell_chunks (layout at c2_head_words): per cell its entry offsets, level
// starts, core refs and entries.  An entry's tail becomes a row index: internal vertex i ->
// i, core ref r -> stored + r, where stored is the first vertex of the cell's last level (no
// entry has its tail there: every entry goes from an earlier level to a later one).  The
// entries are packed into one word (row bits lb2, two flags, length) when every cell's rows
// and every finite length fit, else kept as two words.
int DevGraph::upload_cell_blobs2(const iso::Prep &P, const std::vector<std::vector<uint32_t>> &refs_of) {
    std::vector<uint32_t> stored(num_cells, 0);
    max_rows2 = 1;
    uint32_t wmax_seen = 0;
    for (uint32_t c = 0; c < num_cells; ++c) {
        const uint32_t b = P.cell_off[c], e = P.cell_off[c + 1];
        const uint32_t nl = P.cell_lvl_ptr[c + 1] - P.cell_lvl_ptr[c];
        stored[c] = nl ? P.cell_lvl[P.cell_lvl_ptr[c + 1] - 1] - b : 0u;
        max_rows2 = std::max(max_rows2, stored[c] + uint32_t(refs_of[c].size()));
        if (P.down_off[e] - P.down_off[b] >= (1u << 25)) {
            set_error("a cell has 2^25 or more downward entries");
            return -1;
        }
        for (uint64_t k = P.down_off[b]; k < P.down_off[e]; ++k) {
            const uint32_t t = P.down_arc[2 * k] & TAIL_MASK, w = P.down_arc[2 * k + 1];
            if (t >= b && t - b >= stored[c]) {
                set_error("a cell's last level holds the tail of a downward entry");
                return -1;
            }
            if (w != INF) wmax_seen = std::max(wmax_seen, w);
        }
    }
    lb2 = std::max<uint32_t>(1, ilog2(max_rows2));
    packed2 = lb2 <= 16 && uint64_t(wmax_seen) < (uint64_t(1) << (30 - lb2)) - 1;
    std::vector<uint32_t> cblob2(std::max<uint32_t>(1, num_cells), 0);
    uint64_t total = 0;
    max_blob2_words = 0;
    for (uint32_t c = 0; c < num_cells; ++c) {
        const uint32_t cnt = P.cell_off[c + 1] - P.cell_off[c], nl = P.cell_lvl_ptr[c + 1] - P.cell_lvl_ptr[c];
        const uint32_t ne = P.down_off[P.cell_off[c + 1]] - P.down_off[P.cell_off[c]];
        const uint32_t w = c2_words(cnt, nl, uint32_t(refs_of[c].size()), ne, packed2);
        cblob2[c] = uint32_t(total);
        total += w;
        max_blob2_words = std::max(max_blob2_words, w);
        if (total >= (uint64_t(1) << 32)) {
            set_error("cell data exceed 2^32 words");
            return -1;
        }
    }
    std::vector<uint32_t> blob(std::max<uint64_t>(4, total), 0);
    std::vector<uint32_t> ref_index(std::max<uint32_t>(1, n_core), 0);
    const uint32_t wcode_inf = packed2 ? (0xFFFFFFFFu >> (lb2 + 2)) : 0u;
    for (uint32_t c = 0; c < num_cells; ++c) {
        const uint32_t b = P.cell_off[c], e = P.cell_off[c + 1], cnt = e - b;
        const uint32_t nl = P.cell_lvl_ptr[c + 1] - P.cell_lvl_ptr[c];
        const auto &refs = refs_of[c];
        const uint32_t nr = uint32_t(refs.size());
        for (uint32_t r2 = 0; r2 < nr; ++r2) ref_index[refs[r2]] = r2;
        uint32_t *w = blob.data() + cblob2[c];
        const uint32_t base_e = P.down_off[b];
        for (uint32_t i = 0; i <= cnt; ++i) w[i] = P.down_off[b + i] - base_e;
        uint32_t *lv = w + cnt + 1;
        for (uint32_t l = 0; l < nl; ++l) lv[l] = P.cell_lvl[P.cell_lvl_ptr[c] + l] - b;
        lv[nl] = cnt;
        uint32_t *rf = lv + nl + 1;
        for (uint32_t r2 = 0; r2 < nr; ++r2) rf[r2] = refs[r2];
        uint32_t *en = w + c2_head_words(cnt, nl, nr);
        for (uint32_t k = 0; k < P.down_off[e] - base_e; ++k) {
            const uint32_t x = P.down_arc[2 * uint64_t(base_e + k)], t = x & TAIL_MASK;
            const uint32_t len = P.down_arc[2 * uint64_t(base_e + k) + 1];
            const uint32_t row = t >= b ? t - b : stored[c] + ref_index[t];
            if (packed2) {
                const uint32_t code = len == INF ? wcode_inf : len;
                en[k] = row | (((x & FLAG_FWD) ? 1u : 0u) << lb2) | (((x & FLAG_REV) ? 1u : 0u) << (lb2 + 1)) |
                        (code << (lb2 + 2));
            } else {
                en[2 * k] = row | (x & FLAGS);
                en[2 * k + 1] = len;
            }
        }
    }
    int r;
    if ((r = dev_alloc_copy(&d_blob2, blob, bytes))) return r;
    if ((r = dev_alloc_copy(&d_cblob2, cblob2, bytes))) return r;
    HIPCHK(hipFuncSetAttribute((const void *)k_cell_chunks<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(LDS_MAX)));
    HIPCHK(hipFuncSetAttribute((const void *)k_cell_chunks<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(LDS_MAX)));
    return 0;
}

int DevGraph::upload(const iso::Prep &P, int device_) {
    device = device_;
    HIPCHK(hipSetDevice(device));
    n = P.n;
    n_core = P.n_core;
    num_cells = P.num_cells;
    core_lvl = P.core_lvl;
    core_lvl_entries.resize(core_lvl.size());
    for (size_t i = 0; i < core_lvl.size(); ++i) core_lvl_entries[i] = P.down_off[core_lvl[i]];
    bytes = 0;
    int r;
    // the whole downward graph: the core levels read the core's part; the plain sweep's stream of
    // levels (k_plain_level64) reads the rest (the cell kernels use their blobs)
    if ((r = dev_alloc_copy(&d_down_off, P.down_off, bytes))) return r;
    if ((r = dev_alloc_copy((uint32_t **)&d_down_arc, P.down_arc.data(), 2 * size_t(P.down_off[n]), bytes)))
        return r;
    if (num_cells > 0) {
        // internal positions grouped by their level counted from the top of their cell: level l of
        // every cell is launch l of the plain sweep's stream.  A position whose label some
        // downward entry reads is marked in `readers`.
        uint32_t nl_max = 0;
        for (uint32_t c = 0; c < num_cells; ++c) nl_max = std::max(nl_max, P.cell_lvl_ptr[c + 1] - P.cell_lvl_ptr[c]);
        plvl_ptr.assign(nl_max + 1, 0);
        std::vector<uint32_t> lpos;
        lpos.reserve(n - n_core);
        for (uint32_t l = 0; l < nl_max; ++l) {
            for (uint32_t c = 0; c < num_cells; ++c) {
                const uint32_t lp = P.cell_lvl_ptr[c], nl = P.cell_lvl_ptr[c + 1] - lp;
                if (l >= nl) continue;
                const uint32_t a = P.cell_lvl[lp + l], b = l + 1 < nl ? P.cell_lvl[lp + l + 1] : P.cell_off[c + 1];
                for (uint32_t v = a; v < b; ++v) lpos.push_back(v);
            }
            plvl_ptr[l + 1] = uint32_t(lpos.size());
        }
        if (lpos.size() != size_t(n - n_core)) {
            set_error("cell levels do not cover the internal positions");
            return -1;
        }
        std::vector<uint32_t> readers((size_t(n) + 31) / 32, 0);
        for (uint64_t e = 0; e < P.down_off[n]; ++e) {
            const uint32_t t = P.down_arc[2 * e] & TAIL_MASK;
            readers[t >> 5] |= 1u << (t & 31);
        }
        plain_entries = P.down_off[n] - P.down_off[n_core];
        plain_written = 0;
        for (uint32_t v = n_core; v < n; ++v) plain_written += (readers[v >> 5] >> (v & 31)) & 1u;
        // the records of the stream, in list order
        std::vector<uint2> prec(std::max<size_t>(1, lpos.size() * PLAIN_REC), make_uint2(0u, INF));
        for (size_t i = 0; i < lpos.size(); ++i) {
            const uint32_t v = lpos[i], b0 = P.down_off[v], b1 = P.down_off[v + 1];
            uint2 *w = prec.data() + i * PLAIN_REC;
            w[0] = make_uint2(v, b0);
            w[1] = make_uint2(b1, (readers[v >> 5] >> (v & 31)) & 1u);
            for (uint32_t u = 0; u + 2 < PLAIN_REC && b0 + u < b1; ++u)
                w[u + 2] = make_uint2(P.down_arc[2 * (uint64_t(b0) + u)], P.down_arc[2 * (uint64_t(b0) + u) + 1]);
        }
        if ((r = dev_alloc_copy(&d_plvl_rec, prec, bytes))) return r;
    }
    {   // per core vertex its record: entry offsets, then its first CORE_REC - 1 entries
        std::vector<uint2> rec(std::max<size_t>(1, size_t(n_core) * CORE_REC), make_uint2(0u, INF));
        for (uint32_t v = 0; v < n_core; ++v) {
            uint2 *w = rec.data() + size_t(v) * CORE_REC;
            w[0] = make_uint2(P.down_off[v], P.down_off[v + 1]);
            for (uint32_t u = 0; u + 1 < CORE_REC && P.down_off[v] + u < P.down_off[v + 1]; ++u) {
                const uint64_t e = uint64_t(P.down_off[v]) + u;
                w[u + 1] = make_uint2(P.down_arc[2 * e], P.down_arc[2 * e + 1]);
            }
        }
        if ((r = dev_alloc_copy(&d_core_rec, rec, bytes))) return r;
    }
    if ((r = dev_alloc_copy(&d_pos, P.pos, bytes))) return r;
    if ((r = dev_alloc_copy(&d_core_cell, P.core_cell, bytes))) return r;
    if ((r = dev_alloc_copy(&d_core_ecc, P.core_ecc, bytes))) return r;
    // table of downward distances inside the top levels X = [0, TX), TX <= TABLE_MAX
    TX = 0;
    nlev_table = 0;
    for (size_t l = 0; l + 1 < P.core_lvl.size() && P.core_lvl[l + 1] <= TABLE_MAX; ++l) {
        TX = P.core_lvl[l + 1];
        nlev_table = uint32_t(l + 1);
    }
    if (TX > 0) {
        // F[y][x] = shortest path y -> x using only vertices of X and the hierarchy's arcs
        // among them (upward arcs and downward entries).  Every upward path that enters X stays
        // in X, and so does every downward path into a vertex of X, so with these distances
        // the host's upward search can stop at the first vertices of X it reaches.
        std::vector<uint32_t> xoff(TX + 1, 0), xhead, xw;
        {
            std::vector<std::vector<std::pair<uint32_t, uint32_t>>> adj(TX);
            for (uint32_t x = 0; x < TX; ++x) {
                for (uint32_t e = P.down_off[x]; e < P.down_off[x + 1]; ++e) {
                    uint32_t t2 = P.down_arc[2 * uint64_t(e)] & TAIL_MASK, w = P.down_arc[2 * uint64_t(e) + 1];
                    if (w != INF) adj[t2].push_back({x, w});
                }
                for (uint32_t e = P.up_off[x]; e < P.up_off[x + 1]; ++e) adj[x].push_back({P.up_head[e], P.up_w[e]});
            }
            for (uint32_t x = 0; x < TX; ++x) {
                xoff[x + 1] = xoff[x] + uint32_t(adj[x].size());
                for (auto &a : adj[x]) { xhead.push_back(a.first); xw.push_back(a.second); }
            }
        }
        std::vector<uint32_t> D(size_t(TX) * TX, INF);
        int T = iso::resolve_threads(0);
        std::vector<std::thread> pool;
        std::atomic<uint32_t> next{0};
        for (int t = 0; t < T; ++t)
            pool.emplace_back([&]() {
                std::vector<std::pair<uint32_t, uint32_t>> heap;
                auto cmp = [](const std::pair<uint32_t, uint32_t> &a, const std::pair<uint32_t, uint32_t> &b) {
                    return a.first > b.first;
                };
                for (;;) {
                    uint32_t y = next.fetch_add(1);
                    if (y >= TX) break;
                    uint32_t *row = D.data() + size_t(y) * TX;
                    row[y] = 0;
                    heap.assign(1, {0u, y});
                    while (!heap.empty()) {
                        std::pop_heap(heap.begin(), heap.end(), cmp);
                        auto [k, u] = heap.back();
                        heap.pop_back();
                        if (k != row[u]) continue;
                        for (uint32_t e = xoff[u]; e < xoff[u + 1]; ++e) {
                            uint32_t nd = iso::sat_add(k, xw[e]);
                            if (nd < row[xhead[e]]) {
                                row[xhead[e]] = nd;
                                heap.push_back({nd, xhead[e]});
                                std::push_heap(heap.begin(), heap.end(), cmp);
                            }
                        }
                    }
                }
            });
        for (auto &th : pool) th.join();
        if ((r = dev_alloc_copy(&d_table, D, bytes))) return r;
    }
    std::vector<uint32_t> co = P.cell_off;
    if (co.empty()) co.assign(1, n);
    if ((r = dev_alloc_copy(&d_cell_off, co, bytes))) return r;
    if ((r = dev_alloc_copy(&d_uncovered, P.uncovered, bytes))) return r;
    {
        // core positions of each cell, grouped by cell (read by the cell-mask kernel)
        std::vector<uint32_t> off(size_t(num_cells) + 1, 0), lst;
        for (uint32_t v = 0; v < n_core; ++v)
            if (P.core_cell[v] < num_cells) off[P.core_cell[v] + 1]++;
        for (uint32_t c = 0; c < num_cells; ++c) off[c + 1] += off[c];
        lst.resize(off[num_cells]);
        std::vector<uint32_t> at(off.begin(), off.end() - 1);
        for (uint32_t v = 0; v < n_core; ++v)
            if (P.core_cell[v] < num_cells) lst[at[P.core_cell[v]]++] = v;
        if ((r = dev_alloc_copy(&d_cell_core_off, off, bytes))) return r;
        if ((r = dev_alloc_copy(&d_cell_core, lst, bytes))) return r;
    }
    core_entries = P.down_off[n_core];

    // cell blobs: local entry offsets, local level bounds, sorted distinct core tails, and
    // entries whose tails are local indices (internal: 0..cnt-1, core ref r: cnt + r)
    cell_cnt.assign(num_cells, 0);
    cell_words.assign(num_cells, 0);
    cell_core_refs.assign(num_cells, 0);
    cell_entries.assign(num_cells, 0);
    std::vector<uint32_t> cblob(std::max<uint32_t>(1, num_cells), 0);
    std::vector<uint4> cmeta(std::max<uint32_t>(1, num_cells), make_uint4(0, 0, 0, 0));
    uint64_t total_words = 0;
    max_blob_words = 0;
    max_cell_labels = 0;
    std::vector<std::vector<uint32_t>> refs_of(num_cells);
    std::vector<uint32_t> ref_index(std::max<uint32_t>(1, n_core), 0);
    for (uint32_t c = 0; c < num_cells; ++c) {
        uint32_t b = P.cell_off[c], e = P.cell_off[c + 1];
        auto &refs = refs_of[c];
        for (uint64_t k = P.down_off[b]; k < P.down_off[e]; ++k) {
            uint32_t t = P.down_arc[2 * k] & TAIL_MASK;
            if (t < n_core) refs.push_back(t);
        }
        std::sort(refs.begin(), refs.end());
        refs.erase(std::unique(refs.begin(), refs.end()), refs.end());
        uint32_t cnt = e - b, nl = P.cell_lvl_ptr[c + 1] - P.cell_lvl_ptr[c], nr = uint32_t(refs.size());
        uint32_t ne = P.down_off[e] - P.down_off[b];
        if (cnt + nr > LOCAL_MASK) {
            set_error("a cell references too many vertices for 16-bit local indices");
            return -1;
        }
        for (uint32_t v = b; v < e; ++v)
            if (P.down_off[v + 1] - P.down_off[v] >= CAND_K_MAX) {
                set_error("a cell vertex has 8192 or more downward entries");
                return -1;
            }
        cell_cnt[c] = cnt;
        cell_core_refs[c] = nr;
        cell_entries[c] = ne;
        cell_words[c] = blob_words(cnt, nl, nr, ne);
        cblob[c] = uint32_t(total_words);
        cmeta[c] = make_uint4(cnt, nl, nr, ne);
        total_words += cell_words[c];
        if (total_words >= (uint64_t(1) << 32)) {
            set_error("cell blobs exceed 2^32 words");
            return -1;
        }
        max_blob_words = std::max(max_blob_words, cell_words[c]);
        max_cell_labels = std::max(max_cell_labels, cnt + nr);
        max_cell_cnt = std::max(max_cell_cnt, cnt);
    }
    std::vector<uint32_t> blob(std::max<uint64_t>(4, total_words), 0);
    for (uint32_t c = 0; c < num_cells; ++c) {
        uint32_t b = P.cell_off[c], e = P.cell_off[c + 1], cnt = e - b;
        uint32_t nl = P.cell_lvl_ptr[c + 1] - P.cell_lvl_ptr[c];
        const auto &refs = refs_of[c];
        uint32_t nr = uint32_t(refs.size());
        for (uint32_t r2 = 0; r2 < nr; ++r2) ref_index[refs[r2]] = r2;
        uint32_t *w = blob.data() + cblob[c];
        uint32_t base_e = P.down_off[b];
        for (uint32_t i = 0; i <= cnt; ++i) w[i] = P.down_off[b + i] - base_e;
        uint32_t *lv = w + cnt + 1;
        for (uint32_t l = 0; l < nl; ++l) lv[l] = P.cell_lvl[P.cell_lvl_ptr[c] + l] - b;
        lv[nl] = cnt;
        uint32_t *rf = lv + nl + 1;
        for (uint32_t r2 = 0; r2 < nr; ++r2) rf[r2] = refs[r2];
        uint32_t *en = w + blob_head_words(cnt, nl, nr);
        for (uint32_t k = 0; k < P.down_off[e] - base_e; ++k) {
            uint32_t x = P.down_arc[2 * uint64_t(base_e + k)], t = x & TAIL_MASK;
            uint32_t local = t >= b ? t - b : cnt + ref_index[t];
            en[2 * k] = local | (x & FLAGS);
            en[2 * k + 1] = P.down_arc[2 * uint64_t(base_e + k) + 1];
        }
    }
    if ((r = dev_alloc_copy(&d_blob, blob, bytes))) return r;
    if ((r = dev_alloc_copy(&d_cblob, cblob, bytes))) return r;
    if ((r = dev_alloc_copy(&d_cmeta, cmeta, bytes))) return r;
    blob.clear();
    blob.shrink_to_fit();
    if ((r = upload_cell_blobs2(P, refs_of))) return r;
    if ((r = upload_arc_ranks(P))) return r;
    max_cell_levels = 0;
    for (uint32_t c = 0; c < num_cells; ++c) max_cell_levels = std::max(max_cell_levels, uint32_t(cmeta[c].y));
    HIPCHK(hipFuncSetAttribute((const void *)k_cell_sweep<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(LDS_MAX)));
    HIPCHK(hipFuncSetAttribute((const void *)k_cell_sweep<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(LDS_MAX)));
    HIPCHK(hipDeviceGetAttribute(&num_cus, hipDeviceAttributeMultiprocessorCount, device));
    if ((r = main.create(device))) return r;
    return setup_fixed();
}

int SweepCtx::create(int device_) {
    device = device_;
    HIPCHK(hipSetDevice(device));
    HIPCHK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    for (auto &e : prof.ev) HIPCHK(hipEventCreate(&e));
    return 0;
}

void SweepCtx::release() {
    if (device < 0) return;
    hipSetDevice(device);
    if (stream) hipStreamSynchronize(stream);
    bufs.release();
    if (graph_exec) hipGraphExecDestroy(graph_exec);
    graph_exec = nullptr;
    xcap = 0;
    for (auto &e : prof.ev) if (e) hipEventDestroy(e);
    if (done) hipEventDestroy(done);
    if (stream) hipStreamDestroy(stream);
    stream = nullptr;
    done = nullptr;
    device = -1;
}

void DevGraph::release() {
    if (device < 0) return;
    main.release();
    if (aux_ready) aux.release();
    aux_ready = false;
    fixed.release();
    hipSetDevice(device);
    rot.release();
    poly.release();
    if (fixed_wait) hipEventDestroy(fixed_wait);
    fixed_wait = nullptr;
    hipSetDevice(device);
    void *ptrs[] = {d_down_off, d_down_arc, d_pos, d_core_cell, d_core_ecc, d_cell_off, d_uncovered,
                    d_cell_core_off, d_cell_core,
                    d_table, d_blob, d_cblob, d_cmeta, d_cell_ebase, d_arc_rank, d_arc_pair, d_blob2, d_cblob2,
                    d_plvl_rec, d_core_rec};
    for (void *p : ptrs) if (p) hipFree(p);
    (void)hipGetLastError();   // a failed free must not surface in another handle's next check
    device = -1;
}

void QueryBufs::release() {
    if (fixed) {   // carved from the static scratch: nothing to free but the staging block
        if (h_pinned) hipHostFree(h_pinned);
        *this = QueryBufs();
        return;
    }
    void *ptrs[] = {d_dcore, d_uval, d_uin, d_taus, d_src_cell, d_flags, d_list, d_counters, d_keys,
                    d_keys_sorted, d_sort_tmp, d_dist, d_xin, d_uslot, d_lane_off, d_vmask, d_cin, d_rlab, d_prof,
                    d_dbg};
    for (void *p : ptrs) if (p) hipFree(p);
    if (h_pinned) hipHostFree(h_pinned);
    *this = QueryBufs();
}

// Scratch memory of iso_query_batch_device_noalloc: a static device array, so that the entry
// point needs no allocation.  Each GPU the library runs on holds its own copy until the process
// ends.  Host code must not take the array's address directly (that is a host-side stand-in):
// scratch_setup asks the runtime for the device address of this GPU's copy, once per device,
// and every use goes through that address.
static __device__ __align__(256) uint8_t scratch[SCRATCH_BYTES];
static std::mutex scratch_mu;
static void *scratch_addr[256];

// Device address of the scratch array on `device` (which must be current).
static int scratch_setup(int device, void **addr) {
    if (device < 0 || device >= 256) {
        set_error("device ordinal out of range for the static scratch");
        return -1;
    }
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[device]) {
        void *ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) {
            set_error("hipGetSymbolAddress gave no address for the static scratch");
            return -3;
        }
        scratch_addr[device] = ptr;
    }
    *addr = scratch_addr[device];
    return 0;
}

// The sweep context of iso_query_batch_device_noalloc: its stream, events and a pinned staging
// block, made at load; its device buffers are carved from the static scratch per sweep.
int DevGraph::setup_fixed() {
    int r;
    if ((r = scratch_setup(device, &scratch_ptr))) return r;
    if ((r = fixed.create(device))) return r;
    fixed.bufs.fixed = true;
    HIPCHK(hipHostMalloc(&fixed.bufs.h_pinned, FIXED_STAGE_BYTES, hipHostMallocDefault));
    fixed.bufs.sz_pinned = FIXED_STAGE_BYTES;
    HIPCHK(hipEventCreateWithFlags(&fixed_wait, hipEventDisableTiming));
    return 0;
}

// Lays out the buffers of one sweep of K lanes with nu upward entries below the table and nx
// inside it in the static scratch, the edge keys taking what is left: *cap edges (at least
// min_cap, else ISO_ENOMEM).  Nothing is allocated.
int DevGraph::carve_fixed(uint32_t K, uint32_t nu, uint32_t nx, size_t min_cap, size_t &cap) {
    QueryBufs &B = fixed.bufs;
    uint8_t *base = static_cast<uint8_t *>(scratch_ptr);
    size_t off = 0;
    auto take = [&](void **p, size_t &sz, size_t bytes) {
        bytes = (std::max<size_t>(bytes, 256) + 255) & ~size_t(255);
        *p = off + bytes <= SCRATCH_BYTES ? base + off : nullptr;
        sz = bytes;
        off += bytes;
    };
    take((void **)&B.d_uslot, B.sz_uslot, size_t(n) * 4);
    take((void **)&B.d_dcore, B.sz_dcore, std::max<size_t>(1, size_t(n_core) * K) * 4);
    take((void **)&B.d_uval, B.sz_uval, size_t(std::max(8192u, nu)) * K * 4);
    take((void **)&B.d_uin, B.sz_uin, size_t(std::max(1u, nu)) * 3 * 4);
    fixed.xcap = std::max(1u, nx);
    take((void **)&B.d_xin, B.sz_xin, (size_t(K) + 1 + 2 * size_t(fixed.xcap)) * 4);
    take((void **)&B.d_taus, B.sz_taus, 2 * K * 4);
    take((void **)&B.d_flags, B.sz_flags, size_t(std::max(1u, n_core)) * 16);
    take((void **)&B.d_list, B.sz_list, size_t(std::max(1u, num_cells)) * (3 + MAX_LANES) * 4);
    take((void **)&B.d_counters, B.sz_counters, 64);
    take((void **)&B.d_lane_off, B.sz_lane_off, (MAX_LANES + 1) * 4);
    if (off > SCRATCH_BYTES) {
        set_error("a sweep of " + std::to_string(K) + " queries on this graph needs " + std::to_string(off >> 20) +
                  " MiB of buffers, more than the " + std::to_string(SCRATCH_BYTES >> 20) +
                  " MiB of static scratch (use fewer queries per sweep)");
        return -2;
    }
    // the rest: two key arrays and the radix sort's temporary storage for `cap` keys
    const size_t rest = SCRATCH_BYTES - off;
    size_t lo = 0, hi = rest / 16;
    auto need = [&](size_t c) {
        size_t tmp = 0;
        if (hipcub::DeviceRadixSort::SortKeys(nullptr, tmp, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                              int(std::min<size_t>(c, size_t(INT32_MAX))), 0, 64) != hipSuccess)
            tmp = c * 8 + (1 << 20);
        return 2 * ((c * 8 + 255) & ~size_t(255)) + ((tmp + 255) & ~size_t(255));
    };
    while (lo < hi) {   // the largest capacity that fits
        const size_t mid = (lo + hi + 1) / 2;
        if (need(mid) <= rest) lo = mid;
        else hi = mid - 1;
    }
    cap = std::min<size_t>(lo, INF - 1);
    if (cap < std::max<size_t>(1, min_cap)) {
        set_error("the isochrone edges of one sweep exceed the static scratch (" +
                  std::to_string(SCRATCH_BYTES >> 20) + " MiB)");
        return -2;
    }
    take((void **)&B.d_keys, B.sz_keys, cap * 8);
    take((void **)&B.d_keys_sorted, B.sz_keys_sorted, cap * 8);
    B.sz_sort_tmp = SCRATCH_BYTES - off;
    B.d_sort_tmp = base + off;
    return 0;
}

// grow-only allocation helper
static int ensure(bool fixed, void **p, size_t &have, size_t need) {
    if (need <= have && *p) return 0;
    if (fixed) {   // a buffer carved from the static scratch never grows
        set_error("the call needs more than the " + std::to_string(SCRATCH_BYTES >> 20) +
                  " MiB of static scratch memory");
        return -2;
    }
    if (*p) hipFree(*p);
    *p = nullptr;
    have = 0;
    size_t b = std::max<size_t>(need, 256);
    if (hipMalloc(p, b) != hipSuccess) {
        set_error("hipMalloc of " + std::to_string(b) + " bytes failed");
        return -2;
    }
    have = b;
    return 0;
}

size_t DevGraph::ctx_bytes(uint32_t k, size_t cap, size_t upward_entries, bool plain) const {
    uint32_t K = 1;
    while (K < k) K <<= 1;
    const size_t rows = plain && K == 64 && d_plvl_rec ? n : n_core;   // the stream of levels keeps every row
    // temporary storage of the radix sort over cap keys (the size query allocates nothing)
    size_t sort_tmp = 0;
    if (hipcub::DeviceRadixSort::SortKeys(nullptr, sort_tmp, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                          int(std::min<size_t>(cap, size_t(INT32_MAX))), 0, 64) != hipSuccess)
        sort_tmp = cap * 8 + (1 << 20);
    return rows * K * 4 + size_t(n) * 4 + upward_entries * (K + 3) * 4 + size_t(n_core) * 16 +
           size_t(num_cells) * (3 + MAX_LANES) * 4 + 2 * cap * 8 + sort_tmp + (1 << 20);
}

int DevGraph::run(SweepCtx &C, const RunArgs &A, RunResult &R) {
    int r = launch(C, A);
    if (r) return r;
    return finish(C, R);
}

int DevGraph::launch(SweepCtx &C, const RunArgs &A) {
    HIPCHK(hipSetDevice(device));
    const uint32_t K = A.k_pow2, lk = ilog2(K);
    if (A.core_dijkstra && (uint64_t(n_core) << lk) > 0xFFFFFF00ull) {
        set_error("core too large for the core-search mode at this batch width");
        return -2;
    }
    // upward labels: per-lane lists inside the table X (CSR over lanes), the others as
    // (position, lane, label) entries for the slot table
    std::vector<uint32_t> xptr(K + 1, 0), soff(K + 1, 0);
    for (uint32_t j = 0; j < A.xpos.size(); ++j) {
        xptr[j + 1] = uint32_t(A.xpos[j].size());
        soff[j + 1] = uint32_t(A.spos[j].size());
    }
    for (uint32_t j = 0; j < K; ++j) {
        xptr[j + 1] += xptr[j];
        soff[j + 1] += soff[j];
    }
    const uint32_t nu = soff[K], nx = xptr[K];
    QueryBufs &B = C.bufs;
    hipStream_t s = C.stream;
    int r;
    if (!B.d_uslot || A.fill_uslot) {   // the slot table is all NO_SLOT between sweeps
        if ((r = ensure(B.fixed, (void **)&B.d_uslot, B.sz_uslot, size_t(n) * 4))) return r;
        k_fill<<<dim3(2048), dim3(256), 0, s>>>(B.d_uslot, NO_SLOT, uint64_t(n));
    }
    // plain mode at 64 queries per sweep: the internal vertices as a stream of levels across all
    // cells, their label rows after the core's
    const bool pstream = A.plain_stream && A.mode_plain && K == 64 && A.core64 && num_cells > 0 && d_plvl_rec &&
                         !A.want_dist && !A.vbits && !A.vmask_only && !A.tg && !A.core_dijkstra && !B.fixed;
    size_t core_words = std::max<size_t>(1, size_t(pstream ? n : n_core) * K);
    if ((r = ensure(B.fixed, (void **)&B.d_dcore, B.sz_dcore, core_words * 4))) return r;
    if ((r = ensure(B.fixed, (void **)&B.d_uval, B.sz_uval, size_t(std::max(8192u, nu)) * K * 4))) return r;
    if ((r = ensure(B.fixed, (void **)&B.d_uin, B.sz_uin, size_t(std::max(1u, nu)) * 3 * 4))) return r;
    // table lists: ptr (K + 1) | positions (xcap) | labels (xcap), capacity kept across calls so
    // that the pointers in a captured graph stay valid
    if (C.xcap < nx || B.sz_xin < (size_t(K) + 1 + 2 * size_t(C.xcap)) * 4) {
        C.xcap = std::max<uint32_t>(std::max<uint32_t>(nx + nx / 2, 1024u * K), C.xcap);
        if ((r = ensure(B.fixed, (void **)&B.d_xin, B.sz_xin, (size_t(K) + 1 + 2 * size_t(C.xcap)) * 4))) return r;
    }
    const uint32_t xcap = C.xcap;
    if ((r = ensure(B.fixed, (void **)&B.d_taus, B.sz_taus, 2 * K * 4))) return r;
    // per core vertex: lanes in range, lanes whose range may leave the vertex's cell
    if ((r = ensure(B.fixed, (void **)&B.d_flags, B.sz_flags, size_t(std::max(1u, n_core)) * 16))) return r;
    if ((r = ensure(B.fixed, (void **)&B.d_list, B.sz_list, size_t(std::max(1u, num_cells)) * (3 + MAX_LANES) * 4)))
        return r;
    if ((r = ensure(B.fixed, (void **)&B.d_counters, B.sz_counters, 64))) return r;
    size_t cap = A.out_cap;
    if ((r = ensure(B.fixed, (void **)&B.d_keys, B.sz_keys, cap * 8))) return r;
    if ((r = ensure(B.fixed, (void **)&B.d_keys_sorted, B.sz_keys_sorted, cap * 8))) return r;
    if ((r = ensure(B.fixed, (void **)&B.d_lane_off, B.sz_lane_off, (MAX_LANES + 1) * 4))) return r;
    if (A.want_dist && (r = ensure(B.fixed, (void **)&B.d_dist, B.sz_dist, size_t(n) * K * 4))) return r;
    const bool vmode = A.vbits != nullptr || A.vmask_only;
    if (vmode) {
        if ((r = ensure(B.fixed, (void **)&B.d_vmask, B.sz_vmask, size_t(n) * 8))) return r;
        if ((r = ensure(B.fixed, (void **)&B.d_cin, B.sz_cin, size_t(std::max(1u, num_cells)) * 8))) return r;
    }
    // per-call host inputs staged in one pinned buffer: counters back, taus, source cells,
    // upward entries
    size_t stage = (16 + 2 * size_t(K) + 3 * size_t(nu) + (K + 1) + 2 * size_t(nx)) * 4;
    if (stage > B.sz_pinned && B.fixed) {
        set_error("the queries' upward labels exceed the staging block of the no-allocation entry point");
        return -2;
    }
    if (stage > B.sz_pinned) {
        HIPCHK(hipStreamSynchronize(s));
        if (B.h_pinned) hipHostFree(B.h_pinned);
        B.h_pinned = nullptr;
        size_t b = std::max<size_t>(stage * 2, 1 << 16);
        HIPCHK(hipHostMalloc(&B.h_pinned, b, hipHostMallocDefault));
        B.sz_pinned = b;
    }
    uint32_t *hp = (uint32_t *)B.h_pinned;
    C.h_counters = hp;
    hp[0] = hp[1] = hp[2] = hp[3] = 0;
    uint32_t *hin = hp + 16;
    std::copy(A.taus.begin(), A.taus.end(), hin);
    std::copy(A.src_cell.begin(), A.src_cell.end(), hin + K);
    uint32_t *hu = hin + 2 * K;
    uint32_t *hx = hu + 3 * size_t(nu);
    std::copy(xptr.begin(), xptr.end(), hx);
    for (uint32_t j = 0; j < A.xpos.size(); ++j) {
        std::copy(A.spos[j].begin(), A.spos[j].end(), hu + soff[j]);
        std::fill(hu + nu + soff[j], hu + nu + soff[j + 1], j);
        std::copy(A.sval[j].begin(), A.sval[j].end(), hu + 2 * size_t(nu) + soff[j]);
        std::copy(A.xpos[j].begin(), A.xpos[j].end(), hx + K + 1 + xptr[j]);
        std::copy(A.xval[j].begin(), A.xval[j].end(), hx + K + 1 + nx + xptr[j]);
    }
    uint32_t *d_taus = B.d_taus, *d_src = B.d_taus + K;
    HIPCHK(hipMemcpyAsync(d_taus, hin, 2 * K * 4, hipMemcpyHostToDevice, s));
    if (nu) HIPCHK(hipMemcpyAsync(B.d_uin, hu, size_t(nu) * 3 * 4, hipMemcpyHostToDevice, s));
    const uint32_t *d_xptr = B.d_xin, *d_xpos = B.d_xin + K + 1, *d_xval = B.d_xin + K + 1 + xcap;
    HIPCHK(hipMemcpyAsync(B.d_xin, hx, (size_t(K) + 1 + size_t(nx)) * 4, hipMemcpyHostToDevice, s));
    if (nx) HIPCHK(hipMemcpyAsync((void *)d_xval, hx + K + 1 + nx, size_t(nx) * 4, hipMemcpyHostToDevice, s));
    const uint32_t *d_upos = B.d_uin, *d_ulane = B.d_uin + nu, *d_ulab = B.d_uin + 2 * size_t(nu);
    // clear flags and counters with fill kernels (no memset nodes, so the sequence can be captured)
    k_fill<<<dim3(1), dim3(64), 0, s>>>(B.d_counters, 0u, 16);
    if (A.want_dist) k_fill<<<dim3(2048), dim3(256), 0, s>>>(B.d_dist, INF, uint64_t(n) * K);
    if (nu) {
        uint32_t g = (nu + 255) / 256;
        k_fill<<<dim3(std::min<uint32_t>(1024, (nu * K + 255) / 256)), dim3(256), 0, s>>>(B.d_uval, INF,
                                                                                          uint64_t(nu) * K);
        k_uset_claim<<<dim3(g), dim3(256), 0, s>>>(B.d_uslot, d_upos, nu);
        k_uset_write<<<dim3(g), dim3(256), 0, s>>>(B.d_uslot, d_upos, d_ulane, d_ulab, B.d_uval, nu, lk);
    }
    if (A.tg) {   // one-to-many: the table product, then the target set's level groups
        const TargetSet &T = *A.tg;
        const uint64_t rows = uint64_t(T.tx) + T.nr;
        if ((r = ensure(B.fixed, (void **)&B.d_rlab, B.sz_rlab, std::max<uint64_t>(1, rows) * K * 4))) return r;
        if (T.tx > 0) {
            k_fill<<<dim3(std::max<uint32_t>(1, std::min<uint32_t>(1024, (T.tx * K + 255) / 256))), dim3(256), 0,
                     s>>>(B.d_rlab, INF, uint64_t(T.tx) * K);
            const uint32_t tiles = (T.tx + 63) / 64;
            const uint32_t splits =
                std::max<uint32_t>(1, std::min<uint32_t>(64, 4096 / std::max<uint32_t>(1, tiles * K)));
            k_top_table<<<dim3(tiles * K * splits), dim3(64), 0, s>>>(d_table, T.tx, TX, d_xptr, d_xpos, d_xval,
                                                                       B.d_rlab, lk, tiles, splits);
        }
        for (size_t gi = 0; gi + 1 < T.group.size(); ++gi) {
            const uint32_t rb = T.group[gi], re = T.group[gi + 1];
            const uint64_t threads = uint64_t(re - rb) << lk;
            k_rphast_level<<<dim3(uint32_t((threads + 255) / 256)), dim3(256), 0, s>>>(
                T.d_off, T.d_arc, T.d_rpos, B.d_uslot, B.d_uval, B.d_rlab, T.tx, rb, re, lk);
        }
        if (T.count) {
            const uint64_t threads = uint64_t(A.lanes) * T.count;
            k_rphast_out<<<dim3(uint32_t((threads + 255) / 256)), dim3(256), 0, s>>>(B.d_rlab, T.d_row, T.count, lk,
                                                                                    A.lanes, A.tg_out);
        }
        HIPCHK(hipGetLastError());
        if (nu) k_uset_clear<<<dim3((nu + 255) / 256), dim3(256), 0, s>>>(B.d_uslot, d_upos, nu);
        HIPCHK(hipMemcpyAsync(C.h_counters, B.d_counters, 16, hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(C.done, s));
        C.pending = true;
        C.K = K;
        C.lk = lk;
        C.lg = 0;
        C.lanes = A.lanes;
        C.lane_base = A.lane_base;
        C.cap = cap;
        C.mode_plain = true;
        C.want_dist = false;
        C.vertex_mode = false;
        C.one_to_many = true;
        C.nlev = 0;
        C.top = 0;
        return 0;
    }
    uint64_t *vin = reinterpret_cast<uint64_t *>(B.d_flags), *vout = vin + n_core;
    // counters: edges emitted, active cells, work items, then (words 8-15) the cell sweep's
    // per-XCD claims; the list buffer holds the cells' lane masks, the active cells and the work
    // items or the cells' header records
    uint32_t *out_count = B.d_counters, *n_items = B.d_counters + 2;
    uint64_t *d_cmask = reinterpret_cast<uint64_t *>(B.d_list);
    uint32_t *d_clist = B.d_list + 2 * size_t(num_cells), *d_items = d_clist + num_cells;
    CoreArgs CA{d_down_off, d_down_arc, B.d_dcore, B.d_uslot, B.d_uval, d_core_cell, d_core_ecc, d_taus,
                vin, vout, B.d_keys, out_count, uint32_t(cap), A.lane_base, lk, nullptr};
    const bool prof_on = C.prof.on;
    // the core sweep (table and core levels, one launch per level) has only per-context kernel
    // arguments; with use_graph it is captured once per signature and replayed.  The cell
    // flags, the active cells and the cell sweep (three launches) follow it eagerly, so the
    // phase events of the profile sit between whole launches in both cases.
    const bool cd = A.core_dijkstra;
    // isoPHAST-CD's core part is two launches: no graph; the branch counters are not captured
    const bool use_graph = A.use_graph && !cd && !A.debug;
    GraphSig sig{K, A.mode_plain ? 1u : 0u, A.want_dist ? 1u : 0u, A.block | (A.core64 ? 1u << 31 : 0u),
                 uint32_t(A.cell_lds_bytes), xcap,
                 A.cell_stage, A.cell_block, A.table_x, A.table_levels, uint64_t(cap), {uint64_t(uintptr_t(B.d_dcore)), uint64_t(uintptr_t(B.d_uslot)),
                                 uint64_t(uintptr_t(B.d_uval)), uint64_t(uintptr_t(B.d_xin)),
                                 uint64_t(uintptr_t(B.d_keys)), uint64_t(uintptr_t(B.d_flags)),
                                 uint64_t(uintptr_t(B.d_counters)), uint64_t(uintptr_t(B.d_list)),
                                 uint64_t(uintptr_t(A.want_dist ? B.d_dist : nullptr)),
                                 uint64_t(uintptr_t(B.d_taus))}};
    // cell sweep plan: variant, lanes per work item (as many as fit the LDS budget), LDS per
    // workgroup and a grid of resident workgroups (no more than there can be items), a multiple of 8
    // one workgroup per cell (cell_stage 2) when a cell's data and one lane's rows fit the LDS,
    // else the per-item variants
    const bool chunks = A.cell_stage == 2 && size_t(c2_lds_words(max_blob2_words, max_rows2, 1)) * 4 <= LDS_MAX;
    bool staged = !chunks && A.cell_stage == 1 &&
                  size_t(staged_lds_words(max_blob_words, max_cell_labels, 0)) * 4 <= LDS_MAX;
    const uint32_t variant = chunks ? (packed2 ? 3u : 2u) : staged ? 1u : 0u;
    const uint32_t cell_threads = chunks ? C2_THREADS : A.cell_block;
    uint32_t cell_lg = 0, cell_grid = 8;
    size_t lds = 0;
    if (num_cells > 0) {
        auto lds_of = [&](uint32_t g) {
            if (chunks) return size_t(c2_lds_words(max_blob2_words, max_rows2, 1u << g)) * 4;
            return size_t(staged ? staged_lds_words(max_blob_words, max_cell_labels, g)
                                 : cell_lds_words(max_cell_cnt, max_cell_levels, max_cell_labels, g)) * 4;
        };
        cell_lg = lk;
        while (cell_lg > 0 && lds_of(cell_lg) > A.cell_lds_bytes) --cell_lg;
        lds = lds_of(cell_lg);
        if (lds > LDS_MAX) {
            set_error("a cell does not fit the LDS of one workgroup");
            return -2;
        }
        uint32_t per_cu = 0;
        if ((r = cell_occupancy(variant, cell_threads, lds, per_cu))) return r;
        if (A.cell_per_cu) per_cu = std::min(per_cu, A.cell_per_cu);
        uint64_t most = chunks ? uint64_t(num_cells) : uint64_t(num_cells) << (lk - cell_lg);
        uint64_t want = std::min<uint64_t>(uint64_t(per_cu) * uint64_t(std::max(1, num_cus)), most);
        cell_grid = uint32_t(std::max<uint64_t>(8, (want + 7) / 8 * 8));
    }
    unsigned long long *dbg = nullptr;
    if (A.debug) {   // summed over calls; cleared when first allocated and by iso_debug_enable
        if (!B.d_dbg) {
            if ((r = ensure(B.fixed, (void **)&B.d_dbg, B.sz_dbg, 8 * sizeof(uint64_t)))) return r;
            k_fill<<<dim3(1), dim3(64), 0, s>>>(reinterpret_cast<uint32_t *>(B.d_dbg), 0u, 16);
        }
        dbg = B.d_dbg;
    }
    CA.dbg = dbg;
    bool replay = use_graph && C.graph_exec && std::memcmp(&sig, &C.sig, sizeof sig) == 0;
    if (prof_on) HIPCHK(hipEventRecord(C.prof.ev[0], s));
    // core sweep: the table levels as one (min,+) product, then one launch per level (captured
    // once per signature and replayed with use_graph)
    size_t nlev = core_lvl.size() - 1;
    const uint32_t tx = A.table_x;
    size_t top = A.table_levels;
    const uint32_t lg = num_cells > 0 ? cell_lg : 0;
    if (cd) {
        // isoPHAST-CD: core labels from the host's core search, then flags and isochrone edges
        // of every core vertex in one pass (all labels are final)
        nlev = top = 0;
        if (n_core > 0) {
            const uint64_t words = uint64_t(n_core) << lk;
            k_core_from_slots<<<dim3(uint32_t(std::min<uint64_t>(4096, (words + 255) / 256))), dim3(256), 0, s>>>(
                B.d_uslot, B.d_uval, B.d_dcore, n_core, lk);
            const uint32_t entries = core_lvl_entries.back();
            uint32_t ls = level_ls(n_core, entries, K);
            while (ls > 0 && (uint64_t(n_core) << (lk + ls)) > 0xFFFFFF00ull) --ls;   // 32-bit thread ids
            k_top_finish<<<dim3(uint32_t(((uint64_t(n_core) << (lk + ls)) + 255) / 256)), dim3(256), 0, s>>>(
                CA, n_core, ls);
        }
    } else {
        if (tx > 0) {
            k_fill<<<dim3(std::max<uint32_t>(1, std::min<uint32_t>(1024, (tx * K + 255) / 256))), dim3(256), 0, s>>>(
                B.d_dcore, INF, uint64_t(tx) * K);
            uint32_t tiles = (tx + 63) / 64;
            // splits of each lane's upward list: enough wavefronts to cover the chip
            uint32_t splits = std::max<uint32_t>(1, std::min<uint32_t>(64, 4096 / std::max<uint32_t>(1, tiles * K)));
            k_top_table<<<dim3(tiles * K * splits), dim3(64), 0, s>>>(d_table, tx, TX, d_xptr, d_xpos, d_xval,
                                                                       B.d_dcore, lk, tiles, splits);
            {
                // sub-lanes per vertex from the mean entry count of the table vertices
                uint32_t deg = (core_lvl_entries[top] + tx - 1) / tx;
                uint32_t ls = 0;
                while ((1u << ls) < deg && (K << (ls + 1)) <= 64u) ++ls;
                k_top_finish<<<dim3(uint32_t(((uint64_t(tx) << (lk + ls)) + 255) / 256)), dim3(256), 0, s>>>(CA, tx, ls);
            }
        }
        if (prof_on) HIPCHK(hipEventRecord(C.prof.ev[6], s));
        if (replay) {
            HIPCHK(hipGraphLaunch(C.graph_exec, s));
        } else {
            if (use_graph) {
                if (C.graph_exec) hipGraphExecDestroy(C.graph_exec);
                C.graph_exec = nullptr;
                HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            }
            const uint32_t blk = A.block;
            for (size_t l = top; l < nlev; ++l) {
                uint32_t vb = core_lvl[l], ve = core_lvl[l + 1];
                if (K == 64 && A.core64) {   // one wavefront per vertex, 4 per workgroup
                    uint32_t grid = ((ve - vb + 3) / 4 + 7u) & ~7u;
                    k_core_level64<<<dim3(grid), dim3(256), 0, s>>>(CA, d_core_rec, vb, ve);
                    continue;
                }
                uint32_t ls = level_ls(ve - vb, core_lvl_entries[l + 1] - core_lvl_entries[l], K);
                uint64_t threads = uint64_t(ve - vb) << (lk + ls);
                uint32_t grid = uint32_t((threads + blk - 1) / blk);
                grid = (grid + 7u) & ~7u;   // a multiple of 8 (the block mapping assumes it)
                k_core_level<<<dim3(grid), dim3(blk), 0, s>>>(CA, ls, vb, ve);
            }
            if (use_graph) {
                hipGraph_t graph = nullptr;
                HIPCHK(hipStreamEndCapture(s, &graph));
                hipError_t ie = hipGraphInstantiate(&C.graph_exec, graph, nullptr, nullptr, 0);
                hipGraphDestroy(graph);
                if (ie != hipSuccess) {
                    C.graph_exec = nullptr;
                    set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
                    return -3;
                }
                C.sig = sig;
                HIPCHK(hipGraphLaunch(C.graph_exec, s));
            }
        }
        if (prof_on) HIPCHK(hipEventRecord(C.prof.ev[7], s));
    }
    if (prof_on) HIPCHK(hipEventRecord(C.prof.ev[1], s));
    if (vmode && n_core > 0)   // vertex output: lane masks of the core positions
        k_vmask_core<<<dim3(uint32_t(std::min<uint64_t>(65536, ((uint64_t(n_core) << lk) + 255) / 256))), dim3(256),
                       0, s>>>(B.d_dcore, d_taus, n_core, lk, B.d_vmask);
    if (num_cells > 0) {
        k_cell_masks<<<dim3((num_cells + 3) / 4), dim3(256), 0, s>>>(d_cell_core_off, d_cell_core, vin, vout,
                                                                      d_uncovered, d_cell_off, d_src, K, num_cells,
                                                                      A.mode_plain ? 1u : 0u, d_cmask,
                                                                      vmode ? B.d_cin : nullptr);
        // the one-workgroup-per-cell sweep reads header records where the per-item kernels read items
        const CellHdrSrc hsrc{d_cmeta, d_cell_off, d_cell_ebase, d_cblob2, chunks ? d_items : nullptr};
        k_active_cells<<<dim3((num_cells + 255) / 256), dim3(256), 0, s>>>(d_cmask, num_cells, cell_lg, d_clist,
                                                                          d_items, B.d_counters, hsrc);
        if (vmode)   // internal positions: the cells left out because they lie wholly in range
            k_vmask_cells<<<dim3((num_cells + 3) / 4), dim3(256), 0, s>>>(B.d_cin, d_cmask, d_cell_off, num_cells,
                                                                           B.d_vmask);
        if (prof_on) HIPCHK(hipEventRecord(C.prof.ev[2], s));
        if (pstream) {
            // a resident grid (every block starts at once: blocks stride through fixed shares of
            // the level), a multiple of 8
            if (!plain_per_cu) {
                int nb = 0;
                HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_plain_level64, 256, 0));
                plain_per_cu = uint32_t(std::max(1, nb));
            }
            const uint32_t pgrid = (uint32_t(std::max(1, num_cus)) * plain_per_cu + 7u) & ~7u;
            for (size_t l = 0; l + 1 < plvl_ptr.size(); ++l)
                if (plvl_ptr[l + 1] > plvl_ptr[l])
                    k_plain_level64<<<dim3(pgrid), dim3(256), 0, s>>>(CA, d_plvl_rec, plvl_ptr[l], plvl_ptr[l + 1]);
        } else if (chunks) {
            Cell2Args LA{d_items, B.d_counters, d_blob2, B.d_dcore, B.d_uslot, B.d_uval, d_taus, d_src,
                         B.d_counters + 8, A.want_dist ? B.d_dist : nullptr, vmode ? B.d_vmask : nullptr, B.d_keys,
                         out_count, uint32_t(cap), A.lane_base, lk, lg, lb2, dbg};
            if (packed2)
                k_cell_chunks<true><<<dim3(cell_grid), dim3(C2_THREADS), lds, s>>>(LA);
            else
                k_cell_chunks<false><<<dim3(cell_grid), dim3(C2_THREADS), lds, s>>>(LA);
        } else {
            CellArgs LA{d_items, n_items, d_cblob, d_blob, d_cell_off, d_cell_ebase, B.d_dcore, B.d_uslot, B.d_uval,
                        d_taus, d_src, d_cmask, d_cmeta, A.want_dist ? B.d_dist : nullptr,
                        vmode ? B.d_vmask : nullptr, B.d_keys, out_count, uint32_t(cap), A.lane_base, lk, lg,
                        num_cells};
            if (staged)
                k_cell_sweep<true><<<dim3(cell_grid), dim3(A.cell_block), lds, s>>>(LA);
            else
                k_cell_sweep<false><<<dim3(cell_grid), dim3(A.cell_block), lds, s>>>(LA);
        }
    } else if (prof_on) {
        HIPCHK(hipEventRecord(C.prof.ev[2], s));
    }
    if (prof_on) HIPCHK(hipEventRecord(C.prof.ev[3], s));
    if (prof_on && num_cells > 0 && !pstream) {   // after the last phase event: not part of any phase's time
        if ((r = ensure(B.fixed, (void **)&B.d_prof, B.sz_prof, 8 * sizeof(uint64_t)))) return r;
        if (!C.prof.acc_ready) {
            k_fill<<<dim3(1), dim3(64), 0, s>>>(reinterpret_cast<uint32_t *>(B.d_prof), 0u, 16);   // 8 sums
            C.prof.acc_ready = true;
        }
        k_prof_cells<<<dim3(64), dim3(256), 0, s>>>(d_clist, B.d_counters, d_cmask, d_cmeta,
                                                   reinterpret_cast<unsigned long long *>(B.d_prof),
                                                   chunks ? (packed2 ? 2u : 1u) : 0u, cell_lg);
    }
    if (A.vbits) {   // lane masks by position -> one bitmap row per lane over the original ids
        const uint32_t W = (n + 63) / 64;
        k_vmask_out<<<dim3((n + 255) / 256), dim3(256), 0, s>>>(B.d_vmask, d_pos, n, W, A.lanes, A.vbits);
    }
    if (!vmode && cap > 0)   // entry keys -> (lane, arc rank) keys for the sort
        k_rank_keys<<<dim3(uint32_t(std::min<size_t>(1024, (cap + 255) / 256))), dim3(256), 0, s>>>(
            B.d_keys, out_count, uint32_t(cap), d_arc_rank, rank_bits);
    HIPCHK(hipGetLastError());
    if (nu) k_uset_clear<<<dim3((nu + 255) / 256), dim3(256), 0, s>>>(B.d_uslot, d_upos, nu);
    HIPCHK(hipMemcpyAsync(C.h_counters, B.d_counters, 16, hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(C.done, s));
    C.pending = true;
    C.K = K;
    C.lk = lk;
    C.lg = lg;
    C.cell_variant = variant;
    C.levels_timed = !cd && n_core > 0;
    C.pstream = pstream;
    C.plain_launches = 0;
    if (pstream)
        for (size_t l = 0; l + 1 < plvl_ptr.size(); ++l) C.plain_launches += plvl_ptr[l + 1] > plvl_ptr[l];
    C.lanes = A.lanes;
    C.lane_base = A.lane_base;
    C.cap = cap;
    C.mode_plain = A.mode_plain;
    C.want_dist = A.want_dist;
    C.vertex_mode = vmode;
    C.one_to_many = false;
    C.nlev = uint32_t(nlev);
    C.top = uint32_t(top);
    return 0;
}

// Radix sort of a finished sweep's keys into d_keys_sorted (the lane above the arc rank, so
// the order is lane, tail, head); records the profile's sort-start event.
int DevGraph::sort_keys(SweepCtx &C, uint32_t cnt_all) {
    QueryBufs &B = C.bufs;
    hipStream_t s = C.stream;
    int end_bit = int(rank_bits) + int(ilog2(std::max<uint32_t>(1, C.lane_base + C.K)));
    if (end_bit > 64) end_bit = 64;
    size_t tmp = 0;
    int r;
    HIPCHK(hipcub::DeviceRadixSort::SortKeys(nullptr, tmp, (const uint64_t *)B.d_keys, B.d_keys_sorted,
                                             int(cnt_all), 0, end_bit, s));
    if ((r = ensure(B.fixed, (void **)&B.d_sort_tmp, B.sz_sort_tmp, tmp))) return r;
    if (C.prof.on) HIPCHK(hipEventRecord(C.prof.ev[4], s));
    HIPCHK(hipcub::DeviceRadixSort::SortKeys(B.d_sort_tmp, tmp, (const uint64_t *)B.d_keys, B.d_keys_sorted,
                                             int(cnt_all), 0, end_bit, s));
    return 0;
}

int DevGraph::finish(SweepCtx &C, RunResult &R) {
    if (!C.pending) {
        set_error("finish without a launched sweep");
        return -7;
    }
    C.pending = false;
    HIPCHK(hipSetDevice(device));
    HIPCHK(hipEventSynchronize(C.done));
    if (C.one_to_many) {   // the distances are written; no edges, no phase profile
        R = RunResult();
        return 0;
    }
    QueryBufs &B = C.bufs;
    hipStream_t s = C.stream;
    const uint32_t K = C.K;
    const uint32_t cnt_all = C.h_counters[0], n_active = C.h_counters[1];
    R.count = cnt_all;
    R.active_cells = C.mode_plain ? 0 : n_active;
    R.overflow = cnt_all > C.cap;
    if (C.want_dist) {
        R.dcore.resize(size_t(n_core) * K);
        R.dist.resize(size_t(n) * K);
        HIPCHK(hipMemcpy(R.dcore.data(), B.d_dcore, R.dcore.size() * 4, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(R.dist.data(), B.d_dist, R.dist.size() * 4, hipMemcpyDeviceToHost));
        R.active_list.resize(C.mode_plain ? 0 : n_active);
        if (!R.active_list.empty())
            HIPCHK(hipMemcpy(R.active_list.data(), B.d_list + 2 * size_t(num_cells), R.active_list.size() * 4,
                             hipMemcpyDeviceToHost));
    }
    Profile &prof = C.prof;
    if (prof.on) {
        float ms = 0;
        prof.calls++;
        HIPCHK(hipEventElapsedTime(&ms, prof.ev[0], prof.ev[1]));
        prof.core_ms += ms;
        prof.core_launches += (C.top > 0 ? 3 : 0) + (C.nlev - C.top);
        prof.core_entries += core_entries;
        // offsets + entries + cell ids and eccentricities + k labels written and read back once
        prof.core_bytes += 4ull * (n_core + 1) + 8ull * core_entries + 8ull * n_core + uint64_t(K) * 8ull * n_core;
        if (C.levels_timed) {   // the level launches below the table (k_core_level)
            HIPCHK(hipEventElapsedTime(&ms, prof.ev[6], prof.ev[7]));
            prof.level_ms += ms;
            prof.level_launches += C.nlev - C.top;
            const uint64_t nv = n_core - core_lvl[C.top], ne = core_entries - core_lvl_entries[C.top];
            prof.level_bytes += 4ull * (nv + 1) + 8ull * ne + 8ull * nv + uint64_t(K) * 8ull * nv;
        }
        if (num_cells > 0) {
            HIPCHK(hipEventElapsedTime(&ms, prof.ev[1], prof.ev[2]));
            prof.active_ms += ms;
            HIPCHK(hipEventElapsedTime(&ms, prof.ev[2], prof.ev[3]));
            prof.cell_ms += ms;
            if (C.pstream) {
                // the stream of levels: every internal vertex for every lane.  Bytes: its list
                // entry, offsets and slot; its entries; per lane each entry's tail label read and
                // the label written back where an entry reads it
                const uint64_t ni = n - n_core, ne = plain_entries, nlv = C.plain_launches;
                prof.cell_launches += nlv;
                prof.cell_bytes += 12ull * ni + 4ull * nlv + 8ull * ne + 4ull * K * (ne + plain_written);
                prof.cell_bytes_survey += 4ull * (ni + 1) + 8ull * ne + 8ull * ni * C.lanes;
                prof.cells_swept += num_cells;
                prof.cell_lanes += uint64_t(num_cells) * C.lanes;
                prof.cell_vertices += ni;
                prof.cell_entries += ne;
            } else {
                prof.cell_launches++;
                // the per-cell counts, work items and bytes are summed on the device (k_prof_cells)
            }
        }
    }
    if (C.vertex_mode) {   // the vertex bitmaps are written; the edge keys are not used
        R.overflow = false;
        R.count = 0;
        return 0;
    }
    if (R.overflow) return 0;   // caller grows the buffer and launches again
    const auto tr0 = std::chrono::steady_clock::now();
    if (R.dev_dst) {
        // device destination: lanes [0, dev_lanes) of this sweep go to dev_pairs[dev_base ...) and
        // their starts (plus dev_base) to dev_off[0 .. dev_lanes]; nothing is copied to the host
        if (R.dev_overflow || uint64_t(R.dev_base) + cnt_all > std::min<uint64_t>(R.dev_cap, INF - 1)) {
            R.dev_overflow = true;
            R.t_result_ms = 0;
            return 0;
        }
        k_fill<<<dim3(1), dim3(128), 0, s>>>(R.dev_off, R.dev_base + cnt_all, uint64_t(R.dev_lanes) + 1);
        if (cnt_all) {
            int r = sort_keys(C, cnt_all);
            if (r) return r;
            k_decode<<<dim3((cnt_all + 255) / 256), dim3(256), 0, s>>>(
                B.d_keys_sorted, cnt_all, reinterpret_cast<uint2 *>(R.dev_pairs) + R.dev_base, R.dev_off,
                R.dev_base, d_arc_pair, rank_bits);
            if (prof.on) HIPCHK(hipEventRecord(prof.ev[5], s));
        }
        HIPCHK(hipStreamSynchronize(s));
        if (prof.on && cnt_all) {
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, prof.ev[4], prof.ev[5]));
            prof.sort_ms += ms;
        }
        R.t_result_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tr0).count();
        return 0;
    }
    // sort the keys (lane, then arc rank: tail, then head), decode them into (tail, head)
    // pairs and lane starts on the device, copy both back
    R.lane_off.assign(size_t(K) + 1, 0);
    if (cnt_all) {
        int r = sort_keys(C, cnt_all);
        if (r) return r;
        k_fill<<<dim3(1), dim3(128), 0, s>>>(B.d_lane_off, cnt_all, uint64_t(K) + 1);
        // the pairs overwrite the unsorted keys (same size)
        k_decode<<<dim3((cnt_all + 255) / 256), dim3(256), 0, s>>>(B.d_keys_sorted, cnt_all,
                                                                    reinterpret_cast<uint2 *>(B.d_keys),
                                                                    B.d_lane_off, 0u, d_arc_pair, rank_bits);
        if (prof.on) HIPCHK(hipEventRecord(prof.ev[5], s));
        uint32_t *dst = nullptr;
        if (R.sink) {
            dst = R.sink(cnt_all);
        } else {
            R.edges.resize(size_t(cnt_all) * 2);
            dst = R.edges.data();
        }
        if (!dst) {
            HIPCHK(hipStreamSynchronize(s));
            set_error("out of host memory for the result");
            return -2;   // ISO_ENOMEM
        }
        HIPCHK(hipMemcpyAsync(dst, B.d_keys, size_t(cnt_all) * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(R.lane_off.data(), B.d_lane_off, (size_t(K) + 1) * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (prof.on) {
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, prof.ev[4], prof.ev[5]));
            prof.sort_ms += ms;
        }
    }
    R.t_result_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tr0).count();
    return 0;
}

}  // namespace isodev
