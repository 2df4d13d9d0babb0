// sweep.hip - HIP kernels (gfx950) of the isochrone query and their launch sequence.
//
// Query = upward CH search on the host (Section 2, PHAST upward phase), then on
// the device:
//   1. core sweep: the core block of the sweep order, level by level from the
//      top, each vertex taking min(upward label, tail label + length) over its
//      incoming downward arcs (Section 2, PHAST scanning phase; Section 5,
//      isoPHAST-CP second phase).  Every core vertex also sets its cell's flags
//      i (label <= tau) and o (label + ecc > tau) - the relaxed rule of the
//      parallel-query paragraph of Section 6 - and tests the flagged original
//      arcs at it for isochrone edges (Section 5, output during the sweep).
//   2. active cells: i and (o or uncovered), plus the source's cell (Section 4
//      definition of an active cell; Section 5 source-cell case).
//   3. cell sweep: one workgroup per active cell (cells are independent,
//      Section 5 parallelisation), internal labels kept in LDS, levels
//      separated by workgroup barriers, isochrone edges extracted from LDS.
// In the plain mode step 2 selects every cell (a PHAST one-to-all sweep).
//
// k queries share one sweep: labels are stored k-interleaved (row of k uint32
// per vertex), thread t serves vertex t / k, lane t % k.  Isochrone edges are
// appended with one atomic per wavefront (ballot + popcount), as 64-bit keys
// lane << 58 | tail << 29 | head, then radix-sorted, which orders them by
// query and then by (tail, head).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cstdint>
#include <cstdio>

#include "device.h"

namespace isodev {

constexpr uint32_t INF = 0xFFFFFFFFu;
constexpr uint32_t TAIL_MASK = 0x3FFFFFFFu;
constexpr uint32_t FLAG_FWD = 0x80000000u;
constexpr uint32_t FLAG_REV = 0x40000000u;
constexpr uint32_t NO_SLOT = 0xFFFFFFFFu;
constexpr uint32_t NO_CELL = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) {
    uint32_t s = a + b;
    return s < a ? INF : s;
}

__device__ __forceinline__ uint64_t edge_key(uint32_t lane, uint32_t tail, uint32_t head) {
    return (uint64_t(lane) << 58) | (uint64_t(tail) << 29) | uint64_t(head);
}

// Wavefront-aggregated append; every lane of the wavefront must call it.
__device__ __forceinline__ void emit_wave(bool pred, uint64_t key, uint64_t *__restrict__ out,
                                          uint32_t *__restrict__ counter, uint32_t cap) {
    uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    uint32_t lane = __lane_id();
    int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if ((int)lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (pred) {
        uint32_t idx = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
        if (idx < cap) out[idx] = key;
    }
}

__global__ void k_fill(uint32_t *__restrict__ p, uint32_t value, uint64_t count) {
    uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (; i < count; i += stride) p[i] = value;
}

__global__ void k_uslot_set(uint32_t *__restrict__ uslot, const uint32_t *__restrict__ upos, uint32_t nu,
                            uint32_t clear) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nu) uslot[upos[i]] = clear ? NO_SLOT : i;
}

// One level of the core block: positions [vbeg, vend), k lanes (k = 1 << lk).
__global__ void __launch_bounds__(256)
k_core_level(const uint32_t *__restrict__ down_off, const uint2 *__restrict__ down_arc,
             uint32_t *__restrict__ dcore, const uint32_t *__restrict__ uslot,
             const uint32_t *__restrict__ uval, const uint32_t *__restrict__ perm,
             const uint32_t *__restrict__ core_cell, const uint32_t *__restrict__ core_ecc,
             const uint32_t *__restrict__ taus, uint32_t *__restrict__ fl_in,
             uint32_t *__restrict__ fl_out, uint32_t flag_words, uint64_t *__restrict__ out_keys,
             uint32_t *__restrict__ out_count, uint32_t out_cap, uint32_t lane_base, uint32_t lk,
             uint32_t vbeg, uint32_t vend) {
    const uint32_t K = 1u << lk;
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t v = vbeg + (t >> lk);
    uint32_t j = t & (K - 1);
    bool act = v < vend;
    uint32_t tau = taus[j];
    uint32_t dv = INF, beg = 0, end = 0;
    if (act) {
        uint32_t s = uslot[v];
        if (s != NO_SLOT) dv = uval[(s << lk) + j];
        beg = down_off[v];
        end = down_off[v + 1];
        for (uint32_t e = beg; e < end; ++e) {
            uint2 a = down_arc[e];
            uint32_t tl = a.x & TAIL_MASK;
            dv = min(dv, sat_add(dcore[(tl << lk) + j], a.y));
        }
        dcore[(v << lk) + j] = dv;
        uint32_t c = core_cell[v];
        if (c != NO_CELL) {
            uint32_t bit = 1u << (c & 31u);
            uint32_t w = j * flag_words + (c >> 5);
            if (dv <= tau && !(fl_in[w] & bit)) atomicOr(&fl_in[w], bit);
            if (sat_add(dv, core_ecc[v]) > tau && !(fl_out[w] & bit)) atomicOr(&fl_out[w], bit);
        }
    }
    // isochrone edges at v: every tail is on a higher level, so its label is final
    bool vin = dv <= tau;
    uint32_t ov = act ? perm[v] : 0;
    uint32_t e = beg;
    while (__any(e < end)) {
        bool have = e < end;
        uint2 a = have ? down_arc[e] : make_uint2(0u, 0u);
        uint32_t tl = a.x & TAIL_MASK;
        bool cand = have && (a.x & (FLAG_FWD | FLAG_REV));
        bool st = cand && ((dcore[(tl << lk) + j] <= tau) != vin);
        uint32_t ot = st ? perm[tl] : 0u;
        emit_wave(st && (a.x & FLAG_FWD), edge_key(lane_base + j, ot, ov), out_keys, out_count, out_cap);
        emit_wave(st && (a.x & FLAG_REV), edge_key(lane_base + j, ov, ot), out_keys, out_count, out_cap);
        ++e;
    }
}

// Active cells of every lane; plain mode passes all_cells = 1.
__global__ void k_active_cells(const uint32_t *__restrict__ fl_in, const uint32_t *__restrict__ fl_out,
                               uint32_t flag_words, const uint8_t *__restrict__ uncovered,
                               const uint32_t *__restrict__ cell_off, const uint32_t *__restrict__ src_cell,
                               uint32_t k, uint32_t num_cells, uint32_t all_cells,
                               uint32_t *__restrict__ list, uint32_t *__restrict__ list_len) {
    uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    bool act = false;
    if (c < num_cells && cell_off[c + 1] > cell_off[c]) {
        if (all_cells) {
            act = true;
        } else {
            uint32_t bit = 1u << (c & 31u);
            for (uint32_t j = 0; j < k && !act; ++j) {
                uint32_t w = j * flag_words + (c >> 5);
                bool i_ = fl_in[w] & bit, o_ = fl_out[w] & bit;
                act = (i_ && (o_ || uncovered[c])) || src_cell[j] == c;
            }
        }
    }
    uint64_t mask = __ballot(act);
    if (mask == 0) return;
    uint32_t lane = __lane_id();
    int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if ((int)lane == leader) base = atomicAdd(list_len, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (act) list[base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull))] = c;
}

// One workgroup per (active cell, lane group).  G = 1 << lg lanes per workgroup out of
// K = 1 << lk; LDS holds the cell's internal labels as rows of G.
__global__ void __launch_bounds__(256)
k_cell_sweep(const uint32_t *__restrict__ list, const uint32_t *__restrict__ list_len,
             const uint32_t *__restrict__ cell_off, const uint32_t *__restrict__ cell_lvl_ptr,
             const uint32_t *__restrict__ cell_lvl, const uint32_t *__restrict__ down_off,
             const uint2 *__restrict__ down_arc, const uint32_t *__restrict__ dcore,
             const uint32_t *__restrict__ uslot, const uint32_t *__restrict__ uval,
             const uint32_t *__restrict__ perm, const uint32_t *__restrict__ taus,
             const uint32_t *__restrict__ src_cell, uint32_t *__restrict__ dist_out,
             uint64_t *__restrict__ out_keys, uint32_t *__restrict__ out_count, uint32_t out_cap,
             uint32_t lane_base, uint32_t lk, uint32_t lg) {
    extern __shared__ uint32_t lab[];
    const uint32_t K = 1u << lk, G = 1u << lg, groups = K >> lg;
    uint32_t item = blockIdx.x / groups;
    uint32_t grp = blockIdx.x - item * groups;
    if (item >= *list_len) return;
    uint32_t c = list[item];
    uint32_t cb = cell_off[c], ce = cell_off[c + 1], cnt = ce - cb;
    uint32_t j = threadIdx.x & (G - 1);         // lane within the group
    uint32_t jj = (grp << lg) + j;              // lane within the batch
    uint32_t tau = taus[jj];
    bool has_up = false;
    for (uint32_t q = 0; q < G; ++q) has_up |= src_cell[(grp << lg) + q] == c;
    const uint32_t per_iter = blockDim.x >> lg;   // vertices per block iteration
    // initial labels: upward-search labels exist only inside a source's cell
    for (uint32_t i = threadIdx.x >> lg; i < cnt; i += per_iter) {
        uint32_t val = INF;
        if (has_up) {
            uint32_t s = uslot[cb + i];
            if (s != NO_SLOT) val = uval[(s << lk) + jj];
        }
        lab[(i << lg) + j] = val;
    }
    __syncthreads();
    uint32_t lb = cell_lvl_ptr[c], le = cell_lvl_ptr[c + 1];
    for (uint32_t l = lb; l < le; ++l) {
        uint32_t a0 = cell_lvl[l], a1 = (l + 1 < le) ? cell_lvl[l + 1] : ce;
        for (uint32_t v = a0 + (threadIdx.x >> lg); v < a1; v += per_iter) {
            uint32_t li = v - cb;
            uint32_t dv = lab[(li << lg) + j];
            uint32_t eb = down_off[v], ee = down_off[v + 1];
            for (uint32_t e = eb; e < ee; ++e) {
                uint2 a = down_arc[e];
                uint32_t tl = a.x & TAIL_MASK;
                uint32_t dt = tl >= cb ? lab[((tl - cb) << lg) + j] : dcore[(tl << lk) + jj];
                dv = min(dv, sat_add(dt, a.y));
            }
            lab[(li << lg) + j] = dv;
        }
        __syncthreads();
    }
    // isochrone edges inside the cell (all labels final); loop bound is uniform per workgroup
    for (uint32_t base = 0; base < cnt; base += per_iter) {
        uint32_t li = base + (threadIdx.x >> lg);
        bool act = li < cnt;
        uint32_t v = cb + li;
        uint32_t dv = act ? lab[(li << lg) + j] : INF;
        if (act && dist_out) dist_out[(uint64_t(v) << lk) + jj] = dv;
        bool vin = dv <= tau;
        uint32_t e = act ? down_off[v] : 0, ee = act ? down_off[v + 1] : 0;
        uint32_t ov = act ? perm[v] : 0;
        while (__any(e < ee)) {
            bool have = e < ee;
            uint2 a = have ? down_arc[e] : make_uint2(0u, 0u);
            uint32_t tl = a.x & TAIL_MASK;
            bool cand = have && (a.x & (FLAG_FWD | FLAG_REV));
            uint32_t dt = INF;
            if (cand) dt = tl >= cb ? lab[((tl - cb) << lg) + j] : dcore[(tl << lk) + jj];
            bool st = cand && ((dt <= tau) != vin);
            uint32_t ot = st ? perm[tl] : 0u;
            emit_wave(st && (a.x & FLAG_FWD), edge_key(lane_base + jj, ot, ov), out_keys, out_count, out_cap);
            emit_wave(st && (a.x & FLAG_REV), edge_key(lane_base + jj, ov, ot), out_keys, out_count, out_cap);
            ++e;
        }
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
static int dev_alloc_copy(T **dst, const std::vector<T> &src, uint64_t &bytes) {
    size_t b = std::max<size_t>(sizeof(T), src.size() * sizeof(T));
    HIPCHK(hipMalloc((void **)dst, b));
    bytes += b;
    if (!src.empty()) HIPCHK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return 0;
}

int DevGraph::upload(const iso::Prep &P, int device_) {
    device = device_;
    HIPCHK(hipSetDevice(device));
    HIPCHK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    n = P.n;
    n_core = P.n_core;
    num_cells = P.num_cells;
    max_internal = P.max_cell_internal;
    core_lvl = P.core_lvl;
    bytes = 0;
    int r;
    if ((r = dev_alloc_copy(&d_down_off, P.down_off, bytes))) return r;
    std::vector<uint32_t> arcs = P.down_arc;
    if ((r = dev_alloc_copy((uint32_t **)&d_down_arc, arcs, bytes))) return r;
    if ((r = dev_alloc_copy(&d_perm, P.perm, bytes))) return r;
    if ((r = dev_alloc_copy(&d_core_cell, P.core_cell, bytes))) return r;
    if ((r = dev_alloc_copy(&d_core_ecc, P.core_ecc, bytes))) return r;
    std::vector<uint32_t> co = P.cell_off, clp = P.cell_lvl_ptr, cl = P.cell_lvl;
    if (co.empty()) co.assign(1, n);
    if (clp.empty()) clp.assign(1, 0);
    if ((r = dev_alloc_copy(&d_cell_off, co, bytes))) return r;
    if ((r = dev_alloc_copy(&d_cell_lvl_ptr, clp, bytes))) return r;
    if ((r = dev_alloc_copy(&d_cell_lvl, cl, bytes))) return r;
    if ((r = dev_alloc_copy(&d_uncovered, P.uncovered, bytes))) return r;
    std::vector<uint32_t> slots(n, NO_SLOT);
    if ((r = dev_alloc_copy(&d_uslot, slots, bytes))) return r;
    // sizes for the algorithmic byte accounting of the profile
    core_entries = P.down_off[n_core];
    cell_cnt.assign(num_cells, 0);
    cell_levels.assign(num_cells, 0);
    cell_core_refs.assign(num_cells, 0);
    cell_entries.assign(num_cells, 0);
    std::vector<uint32_t> mark(std::max<uint32_t>(1, n_core), 0xFFFFFFFFu);
    for (uint32_t c = 0; c < num_cells; ++c) {
        uint32_t b = P.cell_off[c], e = P.cell_off[c + 1];
        cell_cnt[c] = e - b;
        cell_levels[c] = P.cell_lvl_ptr[c + 1] - P.cell_lvl_ptr[c];
        cell_entries[c] = uint64_t(P.down_off[e]) - P.down_off[b];
        uint32_t refs = 0;
        for (uint64_t k = P.down_off[b]; k < P.down_off[e]; ++k) {
            uint32_t t = P.down_arc[2 * k] & TAIL_MASK;
            if (t < n_core && mark[t] != c) { mark[t] = c; ++refs; }
        }
        cell_core_refs[c] = refs;
    }
    for (auto &e : prof.ev) HIPCHK(hipEventCreate(&e));
    return 0;
}

void DevGraph::release() {
    if (device < 0) return;
    hipSetDevice(device);
    void *ptrs[] = {d_down_off, d_down_arc, d_perm, d_core_cell, d_core_ecc, d_cell_off, d_cell_lvl_ptr,
                    d_cell_lvl, d_uncovered, d_uslot};
    for (void *p : ptrs) if (p) hipFree(p);
    bufs.release();
    for (auto &e : prof.ev) if (e) hipEventDestroy(e);
    if (stream) hipStreamDestroy(stream);
    stream = nullptr;
    device = -1;
}

void QueryBufs::release() {
    void *ptrs[] = {d_dcore, d_uval, d_upos, d_taus, d_src_cell, d_flags, d_list, d_counters, d_keys,
                    d_keys_sorted, d_sort_tmp, d_dist};
    for (void *p : ptrs) if (p) hipFree(p);
    if (h_pinned) hipHostFree(h_pinned);
    *this = QueryBufs();
}

// grow-only allocation helper
static int ensure(void **p, size_t &have, size_t need) {
    if (need <= have && *p) return 0;
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

int DevGraph::run(const RunArgs &A, RunResult &R) {
    HIPCHK(hipSetDevice(device));
    const uint32_t K = A.k_pow2, lk = ilog2(K);
    const uint32_t nu = uint32_t(A.upos.size());
    const uint32_t flag_words = std::max<uint32_t>(1, (num_cells + 31) / 32);
    QueryBufs &B = bufs;
    int r;
    size_t core_words = std::max<size_t>(1, size_t(n_core) * K);
    if ((r = ensure((void **)&B.d_dcore, B.sz_dcore, core_words * 4))) return r;
    if ((r = ensure((void **)&B.d_uval, B.sz_uval, size_t(std::max(1u, nu)) * K * 4))) return r;
    if ((r = ensure((void **)&B.d_upos, B.sz_upos, size_t(std::max(1u, nu)) * 4))) return r;
    if ((r = ensure((void **)&B.d_taus, B.sz_taus, K * 4))) return r;
    if ((r = ensure((void **)&B.d_src_cell, B.sz_src_cell, K * 4))) return r;
    if ((r = ensure((void **)&B.d_flags, B.sz_flags, size_t(2) * flag_words * K * 4))) return r;
    if ((r = ensure((void **)&B.d_list, B.sz_list, size_t(std::max(1u, num_cells)) * 4))) return r;
    if ((r = ensure((void **)&B.d_counters, B.sz_counters, 64))) return r;
    size_t cap = A.out_cap;
    if ((r = ensure((void **)&B.d_keys, B.sz_keys, cap * 8))) return r;
    if ((r = ensure((void **)&B.d_keys_sorted, B.sz_keys_sorted, cap * 8))) return r;
    if (A.want_dist && (r = ensure((void **)&B.d_dist, B.sz_dist, size_t(n) * K * 4))) return r;
    // staging of the per-call host inputs in one pinned buffer
    size_t stage = (size_t(nu) * K + nu + 2 * K) * 4;
    if (stage > B.sz_pinned) {
        if (B.h_pinned) hipHostFree(B.h_pinned);
        B.h_pinned = nullptr;
        size_t b = std::max<size_t>(stage * 2, 1 << 16);
        HIPCHK(hipHostMalloc(&B.h_pinned, b, hipHostMallocDefault));
        B.sz_pinned = b;
    }
    uint32_t *hp = (uint32_t *)B.h_pinned;
    uint32_t *h_uval = hp, *h_upos = hp + size_t(nu) * K, *h_taus = h_upos + nu, *h_src = h_taus + K;
    std::copy(A.uval.begin(), A.uval.end(), h_uval);
    std::copy(A.upos.begin(), A.upos.end(), h_upos);
    std::copy(A.taus.begin(), A.taus.end(), h_taus);
    std::copy(A.src_cell.begin(), A.src_cell.end(), h_src);
    hipStream_t s = stream;
    if (nu) {
        HIPCHK(hipMemcpyAsync(B.d_uval, h_uval, size_t(nu) * K * 4, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(B.d_upos, h_upos, size_t(nu) * 4, hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipMemcpyAsync(B.d_taus, h_taus, K * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(B.d_src_cell, h_src, K * 4, hipMemcpyHostToDevice, s));
    // clear flags and counters with a fill kernel (no memset nodes, so the sequence can be captured)
    k_fill<<<dim3(64), dim3(256), 0, s>>>(B.d_flags, 0u, uint64_t(2) * flag_words * K);
    k_fill<<<dim3(1), dim3(64), 0, s>>>(B.d_counters, 0u, 16);
    if (A.want_dist) k_fill<<<dim3(2048), dim3(256), 0, s>>>(B.d_dist, INF, uint64_t(n) * K);
    if (nu) k_uslot_set<<<dim3((nu + 255) / 256), dim3(256), 0, s>>>(d_uslot, B.d_upos, nu, 0);
    uint32_t *fl_in = B.d_flags, *fl_out = B.d_flags + size_t(flag_words) * K;
    uint32_t *out_count = B.d_counters, *list_len = B.d_counters + 1;
    const bool prof_on = prof.on;
    if (prof_on) HIPCHK(hipEventRecord(prof.ev[0], s));
    // core levels, top first
    const uint32_t blk = 256;
    for (size_t l = 0; l + 1 < core_lvl.size(); ++l) {
        uint32_t vb = core_lvl[l], ve = core_lvl[l + 1];
        uint64_t threads = uint64_t(ve - vb) << lk;
        uint32_t grid = uint32_t((threads + blk - 1) / blk);
        k_core_level<<<dim3(grid), dim3(blk), 0, s>>>(d_down_off, d_down_arc, B.d_dcore, d_uslot, B.d_uval,
                                                      d_perm, d_core_cell, d_core_ecc, B.d_taus, fl_in, fl_out,
                                                      flag_words, B.d_keys, out_count, uint32_t(cap),
                                                      A.lane_base, lk, vb, ve);
    }
    if (prof_on) HIPCHK(hipEventRecord(prof.ev[1], s));
    if (num_cells > 0) {
        k_active_cells<<<dim3((num_cells + 255) / 256), dim3(256), 0, s>>>(
            fl_in, fl_out, flag_words, d_uncovered, d_cell_off, B.d_src_cell, A.lanes, num_cells,
            A.mode_plain ? 1u : 0u, B.d_list, list_len);
        // lanes per workgroup: as many as fit the LDS budget
        uint32_t lg = lk;
        while (lg > 0 && (size_t(max_internal) << lg) * 4 > size_t(LDS_BUDGET)) --lg;
        size_t lds = std::max<size_t>(4, (size_t(max_internal) << lg) * 4);
        if (lds > 65536) HIPCHK(hipFuncSetAttribute((const void *)k_cell_sweep,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
        uint32_t groups = K >> lg;
        if (prof_on) HIPCHK(hipEventRecord(prof.ev[2], s));
        k_cell_sweep<<<dim3(num_cells * groups), dim3(256), lds, s>>>(
            B.d_list, list_len, d_cell_off, d_cell_lvl_ptr, d_cell_lvl, d_down_off, d_down_arc, B.d_dcore,
            d_uslot, B.d_uval, d_perm, B.d_taus, B.d_src_cell, A.want_dist ? B.d_dist : nullptr, B.d_keys,
            out_count, uint32_t(cap), A.lane_base, lk, lg);
    }
    if (prof_on) HIPCHK(hipEventRecord(prof.ev[3], s));
    HIPCHK(hipGetLastError());
    if (nu) k_uslot_set<<<dim3((nu + 255) / 256), dim3(256), 0, s>>>(d_uslot, B.d_upos, nu, 1);
    uint32_t counters[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(counters, B.d_counters, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    R.count = counters[0];
    R.active_cells = A.mode_plain ? 0 : counters[1];
    R.overflow = counters[0] > cap;
    if (A.want_dist) {
        R.dcore.resize(size_t(n_core) * K);
        R.dist.resize(size_t(n) * K);
        HIPCHK(hipMemcpy(R.dcore.data(), B.d_dcore, R.dcore.size() * 4, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(R.dist.data(), B.d_dist, R.dist.size() * 4, hipMemcpyDeviceToHost));
        R.active_list.resize(A.mode_plain ? 0 : counters[1]);
        if (!R.active_list.empty())
            HIPCHK(hipMemcpy(R.active_list.data(), B.d_list, R.active_list.size() * 4, hipMemcpyDeviceToHost));
    }
    if (prof_on) {
        float ms = 0;
        prof.calls++;
        HIPCHK(hipEventElapsedTime(&ms, prof.ev[0], prof.ev[1]));
        prof.core_ms += ms;
        prof.core_launches += core_lvl.size() - 1;
        prof.core_entries += core_entries;
        prof.core_bytes += 4ull * (n_core + 1) + 8ull * core_entries + 12ull * n_core +
                           uint64_t(K) * 8ull * n_core;
        if (num_cells > 0) {
            HIPCHK(hipEventElapsedTime(&ms, prof.ev[1], prof.ev[2]));
            prof.active_ms += ms;
            HIPCHK(hipEventElapsedTime(&ms, prof.ev[2], prof.ev[3]));
            prof.cell_ms += ms;
            prof.cell_launches++;
            std::vector<uint32_t> lst;
            if (A.mode_plain) {
                for (uint32_t c = 0; c < num_cells; ++c) if (cell_cnt[c]) lst.push_back(c);
            } else {
                lst.resize(counters[1]);
                if (!lst.empty())
                    HIPCHK(hipMemcpy(lst.data(), B.d_list, lst.size() * 4, hipMemcpyDeviceToHost));
            }
            for (uint32_t c : lst) {
                prof.cells_swept++;
                prof.cell_vertices += cell_cnt[c];
                prof.cell_entries += cell_entries[c];
                prof.cell_bytes += 4ull * (cell_cnt[c] + 1) + 8ull * cell_entries[c] + 4ull * (cell_levels[c] + 3) +
                                   uint64_t(K) * 4ull * cell_core_refs[c];
            }
        }
    }
    if (R.overflow) return 0;   // caller grows the buffer and repeats
    // sort keys: lane bits above 58, then tail, then head
    uint32_t cnt = counters[0];
    R.keys.resize(cnt);
    if (cnt) {
        int end_bit = 58 + int(ilog2(std::max<uint32_t>(1, A.lane_base + K)));
        if (end_bit > 64) end_bit = 64;
        size_t tmp = 0;
        HIPCHK(hipcub::DeviceRadixSort::SortKeys(nullptr, tmp, (const uint64_t *)B.d_keys, B.d_keys_sorted,
                                                 int(cnt), 0, end_bit, s));
        if ((r = ensure((void **)&B.d_sort_tmp, B.sz_sort_tmp, tmp))) return r;
        if (prof_on) HIPCHK(hipEventRecord(prof.ev[4], s));
        HIPCHK(hipcub::DeviceRadixSort::SortKeys(B.d_sort_tmp, tmp, (const uint64_t *)B.d_keys,
                                                 B.d_keys_sorted, int(cnt), 0, end_bit, s));
        if (prof_on) HIPCHK(hipEventRecord(prof.ev[5], s));
        HIPCHK(hipMemcpyAsync(R.keys.data(), B.d_keys_sorted, size_t(cnt) * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (prof_on) {
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, prof.ev[4], prof.ev[5]));
            prof.sort_ms += ms;
        }
    }
    return 0;
}

}  // namespace isodev
