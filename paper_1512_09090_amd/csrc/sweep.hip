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
//      The top levels, where the hierarchy narrows to a chain, run in one
//      workgroup with labels and arcs in LDS; the rest runs one launch per level.
//   2. active cells: i and (o or uncovered), plus the source's cell (Section 4
//      definition of an active cell; Section 5 source-cell case).
//   3. cell sweep: one workgroup per active cell (cells are independent,
//      Section 5 parallelisation).  The cell's downward arcs, level bounds and
//      referenced core labels are staged in LDS first, then its levels run
//      between workgroup barriers and isochrone edges are extracted from LDS.
// In the plain mode step 2 selects every cell (a PHAST one-to-all sweep).
//
// k queries share one sweep: labels are stored k-interleaved (row of k uint32
// per vertex).  In the core kernels a group of S*k lanes serves one vertex:
// k lanes (one per query) times S sub-lanes that split the vertex's arc list,
// combined by a shuffle-xor minimum.  Isochrone edges are appended with one
// atomic per wavefront (ballot + popcount) as 64-bit keys
// lane << 58 | tail << 29 | head, then radix-sorted (query, tail, head).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstdint>
#include <cstdio>

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

// Flags of core vertex v in its cell for lane j (relaxed rule: d <= tau sets i, d + ecc > tau sets o).
__device__ __forceinline__ void set_cell_flags(uint32_t c, uint32_t ecc, uint32_t dv, uint32_t tau, uint32_t j,
                                               uint32_t flag_words, uint32_t *__restrict__ fl_in,
                                               uint32_t *__restrict__ fl_out) {
    if (c == NO_CELL) return;
    uint32_t bit = 1u << (c & 31u);
    uint32_t w = j * flag_words + (c >> 5);
    if (dv <= tau && !(fl_in[w] & bit)) atomicOr(&fl_in[w], bit);
    if (sat_add(dv, ecc) > tau && !(fl_out[w] & bit)) atomicOr(&fl_out[w], bit);
}

struct CoreArgs {
    const uint32_t *down_off;
    const uint2 *down_arc;
    uint32_t *dcore;
    const uint32_t *uslot, *uval, *perm, *core_cell, *core_ecc, *taus;
    uint32_t *fl_in, *fl_out;
    uint32_t flag_words;
    uint64_t *out_keys;
    uint32_t *out_count;
    uint32_t out_cap, lane_base, lk;
};

// One core vertex v for lane j, sub-lane `sub` of S (= 1 << ls): partial minimum over
// entries beg+sub, beg+sub+S, ...; LAB(tail) gives the tail's label for lane j.  The
// partial minima are combined across the S sub-lanes (lanes K, 2K, ... apart).  Returns
// the final label; any_in / any_out record whether a flagged entry of this sub-lane has
// its tail in / out of range (only then can it straddle).
template <class ARC, class LAB>
__device__ __forceinline__ uint32_t relax_group(ARC arc, LAB lab, uint32_t beg, uint32_t end, uint32_t sub,
                                                uint32_t S, uint32_t K, uint32_t init, uint32_t tau,
                                                bool &any_in, bool &any_out) {
    uint32_t m = INF;
    uint32_t e = beg + sub;
    for (; e + S < end; e += 2 * S) {
        uint2 a0 = arc(e), a1 = arc(e + S);
        uint32_t l0 = lab(a0.x & TAIL_MASK), l1 = lab(a1.x & TAIL_MASK);
        m = min(m, min(sat_add(l0, a0.y), sat_add(l1, a1.y)));
        if (a0.x & FLAGS) { if (l0 <= tau) any_in = true; else any_out = true; }
        if (a1.x & FLAGS) { if (l1 <= tau) any_in = true; else any_out = true; }
    }
    if (e < end) {
        uint2 a0 = arc(e);
        uint32_t l0 = lab(a0.x & TAIL_MASK);
        m = min(m, sat_add(l0, a0.y));
        if (a0.x & FLAGS) { if (l0 <= tau) any_in = true; else any_out = true; }
    }
    for (uint32_t o = K; o < K * S; o <<= 1) m = min(m, (uint32_t)__shfl_xor((int)m, (int)o));
    return min(init, m);
}

// Isochrone edges at core vertex v (label dv final): only sub-lanes that saw a possible
// straddle walk their entries again.  Wavefront-uniform loop (emit_wave inside).
template <class ARC, class LAB>
__device__ __forceinline__ void extract_group(ARC arc, LAB lab, const CoreArgs &A, bool act, uint32_t v,
                                              uint32_t beg, uint32_t end, uint32_t sub, uint32_t S,
                                              uint32_t j, uint32_t dv, uint32_t tau, bool any_in, bool any_out) {
    bool vin = dv <= tau;
    bool need = act && (vin ? any_out : any_in);
    uint32_t e = need ? beg + sub : 0, stop = need ? end : 0;
    uint32_t ov = need ? A.perm[v] : 0u;
    while (__any(e < stop)) {
        bool have = e < stop;
        uint2 a = have ? arc(e) : make_uint2(0u, 0u);
        uint32_t tl = a.x & TAIL_MASK;
        bool st = have && (a.x & FLAGS) && ((lab(tl) <= tau) != vin);
        uint32_t ot = st ? A.perm[tl] : 0u;
        emit_wave(st && (a.x & FLAG_FWD), edge_key(A.lane_base + j, ot, ov), A.out_keys, A.out_count, A.out_cap);
        emit_wave(st && (a.x & FLAG_REV), edge_key(A.lane_base + j, ov, ot), A.out_keys, A.out_count, A.out_cap);
        e += S;
    }
}

// Top of the core: positions [0, T), levels given by top_lvl[0..nl] (top first), one
// workgroup, labels (T rows of K) and the arcs of these vertices in LDS.
__global__ void __launch_bounds__(1024)
k_core_top(CoreArgs A, const uint32_t *__restrict__ top_lvl, uint32_t nl, uint32_t T, uint32_t ET) {
    extern __shared__ uint32_t smem[];
    const uint32_t lk = A.lk, K = 1u << lk;
    uint2 *s_arc = reinterpret_cast<uint2 *>(smem);                 // ET entries
    uint32_t *s_off = smem + 2 * ET;                                  // T + 1 offsets
    uint32_t *s_lab = s_off + T + 1;                                  // T * K labels
    for (uint32_t i = threadIdx.x; i < ET; i += blockDim.x) s_arc[i] = A.down_arc[i];
    for (uint32_t i = threadIdx.x; i <= T; i += blockDim.x) s_off[i] = A.down_off[i];
    for (uint32_t i = threadIdx.x; i < (T << lk); i += blockDim.x) {
        uint32_t v = i >> lk, j = i & (K - 1);
        uint32_t s = A.uslot[v];
        s_lab[i] = s != NO_SLOT ? A.uval[(s << lk) + j] : INF;
    }
    __syncthreads();
    auto arc = [&](uint32_t e) { return s_arc[e]; };
    for (uint32_t l = 0; l < nl; ++l) {
        uint32_t a = top_lvl[l], b = top_lvl[l + 1];
        // sub-lanes per vertex: enough to cover the level's mean in-degree, within one wavefront
        uint32_t deg = (s_off[b] - s_off[a] + (b - a) - 1) / (b - a);
        uint32_t ls = 0;
        while ((1u << ls) < deg && (K << (ls + 1)) <= 64u) ++ls;
        const uint32_t S = 1u << ls, lgs = lk + ls;
        const uint32_t per_pass = blockDim.x >> lgs;
        for (uint32_t vb = a; vb < b; vb += per_pass) {
            uint32_t v = vb + (threadIdx.x >> lgs);
            uint32_t j = threadIdx.x & (K - 1), sub = (threadIdx.x >> lk) & (S - 1);
            bool act = v < b;
            uint32_t tau = A.taus[j];
            uint32_t beg = act ? s_off[v] : 0, end = act ? s_off[v + 1] : 0;
            auto lab = [&](uint32_t t) { return s_lab[(t << lk) + j]; };
            bool any_in = false, any_out = false;
            uint32_t dv = relax_group(arc, lab, beg, end, sub, S, K, act ? s_lab[(v << lk) + j] : INF, tau,
                                      any_in, any_out);
            if (act && sub == 0) {
                s_lab[(v << lk) + j] = dv;
                set_cell_flags(A.core_cell[v], A.core_ecc[v], dv, tau, j, A.flag_words, A.fl_in, A.fl_out);
            }
            extract_group(arc, lab, A, act, v, beg, end, sub, S, j, dv, tau, any_in, any_out);
        }
        __syncthreads();
    }
    for (uint32_t i = threadIdx.x; i < (T << lk); i += blockDim.x) A.dcore[i] = s_lab[i];
}

// One core level: positions [vbeg, vend); S = 1 << ls sub-lanes per (vertex, lane).
__global__ void __launch_bounds__(256)
k_core_level(CoreArgs A, uint32_t ls, uint32_t vbeg, uint32_t vend) {
    const uint32_t lk = A.lk, K = 1u << lk, S = 1u << ls, lgs = lk + ls;
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t v = vbeg + (t >> lgs);
    uint32_t j = t & (K - 1), sub = (t >> lk) & (S - 1);
    bool act = v < vend;
    uint32_t tau = A.taus[j];
    uint32_t init = INF, beg = 0, end = 0;
    if (act) {
        uint32_t s = A.uslot[v];
        if (s != NO_SLOT) init = A.uval[(s << lk) + j];
        beg = A.down_off[v];
        end = A.down_off[v + 1];
    }
    const uint2 *__restrict__ darc = A.down_arc;
    const uint32_t *__restrict__ dc = A.dcore;
    auto arc = [&](uint32_t e) { return darc[e]; };
    auto lab = [&](uint32_t tl) { return dc[(tl << lk) + j]; };
    bool any_in = false, any_out = false;
    uint32_t dv = relax_group(arc, lab, beg, end, sub, S, K, init, tau, any_in, any_out);
    if (act && sub == 0) {
        A.dcore[(v << lk) + j] = dv;
        set_cell_flags(A.core_cell[v], A.core_ecc[v], dv, tau, j, A.flag_words, A.fl_in, A.fl_out);
    }
    extract_group(arc, lab, A, act, v, beg, end, sub, S, j, dv, tau, any_in, any_out);
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

// Words of a cell blob: offsets (cnt + 1), level bounds (nl + 1), core refs, pad to even,
// entries (2 words each), pad to a multiple of 4.
__host__ __device__ __forceinline__ uint32_t blob_head_words(uint32_t cnt, uint32_t nl, uint32_t nrefs) {
    return ((cnt + 1) + (nl + 1) + nrefs + 1u) & ~1u;
}
__host__ __device__ __forceinline__ uint32_t blob_words(uint32_t cnt, uint32_t nl, uint32_t nrefs, uint32_t ne) {
    return (blob_head_words(cnt, nl, nrefs) + 2 * ne + 3u) & ~3u;
}

struct CellArgs {
    const uint32_t *list, *list_len, *cblob, *blob, *cell_off, *dcore, *uslot, *uval, *perm, *taus,
        *src_cell;
    const uint4 *cmeta;
    uint32_t *dist_out;
    uint64_t *out_keys;
    uint32_t *out_count;
    uint32_t out_cap, lane_base, lk, lg;
};

// One workgroup per (active cell, group of G = 1 << lg lanes).  STAGED: the blob is copied
// to LDS; otherwise it is read from global memory (cells larger than the LDS budget).
template <bool STAGED>
__global__ void __launch_bounds__(256) k_cell_sweep(CellArgs A, uint32_t lab_offset_words) {
    extern __shared__ uint32_t smem[];
    const uint32_t lk = A.lk, lg = A.lg, K = 1u << lk, G = 1u << lg, groups = K >> lg;
    uint32_t item = blockIdx.x / groups;
    uint32_t grp = blockIdx.x - item * groups;
    if (item >= *A.list_len) return;
    const uint32_t c = A.list[item];
    const uint4 meta = A.cmeta[c];
    const uint32_t cnt = meta.x, nl = meta.y, nrefs = meta.z, ne = meta.w;
    const uint32_t cb = A.cell_off[c];
    const uint32_t words = blob_words(cnt, nl, nrefs, ne), head = blob_head_words(cnt, nl, nrefs);
    const uint32_t *gblob = A.blob + A.cblob[c];
    const uint32_t *blob;
    if (STAGED) {
        const uint4 *src = reinterpret_cast<const uint4 *>(gblob);
        uint4 *dst = reinterpret_cast<uint4 *>(smem);
        for (uint32_t i = threadIdx.x; i < (words >> 2); i += blockDim.x) dst[i] = src[i];
        blob = smem;
    } else {
        blob = gblob;
    }
    uint32_t *lab = smem + lab_offset_words;      // (cnt + nrefs) rows of G labels
    const uint32_t *off = blob, *lvl = blob + cnt + 1, *refs = lvl + nl + 1;
    const uint2 *ent = reinterpret_cast<const uint2 *>(blob + head);
    const uint32_t j = threadIdx.x & (G - 1);     // lane within the group
    const uint32_t jj = (grp << lg) + j;          // lane within the batch
    const uint32_t tau = A.taus[jj];
    bool has_up = false;
    for (uint32_t q = 0; q < G; ++q) has_up |= A.src_cell[(grp << lg) + q] == c;
    const uint32_t per_iter = blockDim.x >> lg;
    if (STAGED) __syncthreads();
    // labels: internal vertices start at INF (upward labels only in a source's cell),
    // referenced core vertices take their final core labels
    for (uint32_t i = threadIdx.x >> lg; i < cnt + nrefs; i += per_iter) {
        uint32_t val = INF;
        if (i < cnt) {
            if (has_up) {
                uint32_t s = A.uslot[cb + i];
                if (s != NO_SLOT) val = A.uval[(s << lk) + jj];
            }
        } else {
            val = A.dcore[(refs[i - cnt] << lk) + jj];
        }
        lab[(i << lg) + j] = val;
    }
    __syncthreads();
    for (uint32_t l = 0; l < nl; ++l) {
        uint32_t a = lvl[l], b = lvl[l + 1];
        for (uint32_t i = a + (threadIdx.x >> lg); i < b; i += per_iter) {
            uint32_t dv = lab[(i << lg) + j];
            for (uint32_t e = off[i]; e < off[i + 1]; ++e) {
                uint2 x = ent[e];
                dv = min(dv, sat_add(lab[((x.x & LOCAL_MASK) << lg) + j], x.y));
            }
            lab[(i << lg) + j] = dv;
        }
        __syncthreads();
    }
    // isochrone edges inside the cell; the loop bound is uniform per workgroup
    for (uint32_t base = 0; base < cnt; base += per_iter) {
        uint32_t i = base + (threadIdx.x >> lg);
        bool act = i < cnt;
        uint32_t dv = act ? lab[(i << lg) + j] : INF;
        if (act && A.dist_out) A.dist_out[(uint64_t(cb + i) << lk) + jj] = dv;
        bool vin = dv <= tau;
        uint32_t e = act ? off[i] : 0, ee = act ? off[i + 1] : 0;
        uint32_t ov = 0;
        bool ov_loaded = false;
        while (__any(e < ee)) {
            bool have = e < ee;
            uint2 x = have ? ent[e] : make_uint2(0u, 0u);
            uint32_t lt = x.x & LOCAL_MASK;
            bool st = have && (x.x & FLAGS) && ((lab[(lt << lg) + j] <= tau) != vin);
            uint32_t ot = 0;
            if (st) {
                if (!ov_loaded) { ov = A.perm[cb + i]; ov_loaded = true; }
                ot = A.perm[lt < cnt ? cb + lt : refs[lt - cnt]];
            }
            emit_wave(st && (x.x & FLAG_FWD), edge_key(A.lane_base + jj, ot, ov), A.out_keys, A.out_count, A.out_cap);
            emit_wave(st && (x.x & FLAG_REV), edge_key(A.lane_base + jj, ov, ot), A.out_keys, A.out_count, A.out_cap);
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

int DevGraph::upload(const iso::Prep &P, int device_) {
    device = device_;
    HIPCHK(hipSetDevice(device));
    HIPCHK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    n = P.n;
    n_core = P.n_core;
    num_cells = P.num_cells;
    core_lvl = P.core_lvl;
    core_lvl_entries.resize(core_lvl.size());
    for (size_t i = 0; i < core_lvl.size(); ++i) core_lvl_entries[i] = P.down_off[core_lvl[i]];
    bytes = 0;
    int r;
    // the core part of the downward graph (cells use their blobs)
    std::vector<uint32_t> coff(P.down_off.begin(), P.down_off.begin() + n_core + 1);
    if ((r = dev_alloc_copy(&d_down_off, coff, bytes))) return r;
    if ((r = dev_alloc_copy((uint32_t **)&d_down_arc, P.down_arc.data(), 2 * size_t(P.down_off[n_core]), bytes)))
        return r;
    if ((r = dev_alloc_copy(&d_perm, P.perm, bytes))) return r;
    if ((r = dev_alloc_copy(&d_core_cell, P.core_cell, bytes))) return r;
    if ((r = dev_alloc_copy(&d_core_ecc, P.core_ecc, bytes))) return r;
    if ((r = dev_alloc_copy(&d_top_lvl, P.core_lvl, bytes))) return r;
    std::vector<uint32_t> co = P.cell_off;
    if (co.empty()) co.assign(1, n);
    if ((r = dev_alloc_copy(&d_cell_off, co, bytes))) return r;
    if ((r = dev_alloc_copy(&d_uncovered, P.uncovered, bytes))) return r;
    std::vector<uint32_t> slots(n, NO_SLOT);
    if ((r = dev_alloc_copy(&d_uslot, slots, bytes))) return r;
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
    for (auto &e : prof.ev) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipFuncSetAttribute((const void *)k_cell_sweep<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(LDS_MAX)));
    HIPCHK(hipFuncSetAttribute((const void *)k_cell_sweep<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(LDS_MAX)));
    HIPCHK(hipFuncSetAttribute((const void *)k_core_top, hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(LDS_MAX)));
    return 0;
}

void DevGraph::release() {
    if (device < 0) return;
    hipSetDevice(device);
    void *ptrs[] = {d_down_off, d_down_arc, d_perm, d_core_cell, d_core_ecc, d_cell_off, d_uncovered,
                    d_uslot, d_top_lvl, d_blob, d_cblob, d_cmeta};
    for (void *p : ptrs) if (p) hipFree(p);
    bufs.release();
    for (auto &e : prof.ev) if (e) hipEventDestroy(e);
    if (stream) hipStreamDestroy(stream);
    stream = nullptr;
    device = -1;
}

void QueryBufs::release() {
    void *ptrs[] = {d_dcore, d_uval, d_uin, d_taus, d_src_cell, d_flags, d_list, d_counters, d_keys,
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
    if ((r = ensure((void **)&B.d_uin, B.sz_uin, size_t(std::max(1u, nu)) * 3 * 4))) return r;
    if ((r = ensure((void **)&B.d_taus, B.sz_taus, 2 * K * 4))) return r;
    if ((r = ensure((void **)&B.d_flags, B.sz_flags, size_t(2) * flag_words * K * 4))) return r;
    if ((r = ensure((void **)&B.d_list, B.sz_list, size_t(std::max(1u, num_cells)) * 4))) return r;
    if ((r = ensure((void **)&B.d_counters, B.sz_counters, 64))) return r;
    size_t cap = A.out_cap;
    if ((r = ensure((void **)&B.d_keys, B.sz_keys, cap * 8))) return r;
    if ((r = ensure((void **)&B.d_keys_sorted, B.sz_keys_sorted, cap * 8))) return r;
    if (A.want_dist && (r = ensure((void **)&B.d_dist, B.sz_dist, size_t(n) * K * 4))) return r;
    // per-call host inputs staged in one pinned buffer: taus, source cells, upward entries
    size_t stage = (2 * size_t(K) + 3 * size_t(nu)) * 4;
    if (stage > B.sz_pinned) {
        if (B.h_pinned) hipHostFree(B.h_pinned);
        B.h_pinned = nullptr;
        size_t b = std::max<size_t>(stage * 2, 1 << 16);
        HIPCHK(hipHostMalloc(&B.h_pinned, b, hipHostMallocDefault));
        B.sz_pinned = b;
    }
    uint32_t *hp = (uint32_t *)B.h_pinned;
    std::copy(A.taus.begin(), A.taus.end(), hp);
    std::copy(A.src_cell.begin(), A.src_cell.end(), hp + K);
    uint32_t *hu = hp + 2 * K;
    std::copy(A.upos.begin(), A.upos.end(), hu);
    std::copy(A.ulane.begin(), A.ulane.end(), hu + nu);
    std::copy(A.uval.begin(), A.uval.end(), hu + 2 * size_t(nu));
    hipStream_t s = stream;
    uint32_t *d_taus = B.d_taus, *d_src = B.d_taus + K;
    HIPCHK(hipMemcpyAsync(d_taus, hp, 2 * K * 4, hipMemcpyHostToDevice, s));
    if (nu) HIPCHK(hipMemcpyAsync(B.d_uin, hu, size_t(nu) * 3 * 4, hipMemcpyHostToDevice, s));
    const uint32_t *d_upos = B.d_uin, *d_ulane = B.d_uin + nu, *d_ulab = B.d_uin + 2 * size_t(nu);
    // clear flags and counters with fill kernels (no memset nodes, so the sequence can be captured)
    k_fill<<<dim3(64), dim3(256), 0, s>>>(B.d_flags, 0u, uint64_t(2) * flag_words * K);
    k_fill<<<dim3(1), dim3(64), 0, s>>>(B.d_counters, 0u, 16);
    if (A.want_dist) k_fill<<<dim3(2048), dim3(256), 0, s>>>(B.d_dist, INF, uint64_t(n) * K);
    if (nu) {
        uint32_t g = (nu + 255) / 256;
        k_fill<<<dim3(std::min<uint32_t>(1024, (nu * K + 255) / 256)), dim3(256), 0, s>>>(B.d_uval, INF,
                                                                                          uint64_t(nu) * K);
        k_uset_claim<<<dim3(g), dim3(256), 0, s>>>(d_uslot, d_upos, nu);
        k_uset_write<<<dim3(g), dim3(256), 0, s>>>(d_uslot, d_upos, d_ulane, d_ulab, B.d_uval, nu, lk);
    }
    uint32_t *fl_in = B.d_flags, *fl_out = B.d_flags + size_t(flag_words) * K;
    uint32_t *out_count = B.d_counters, *list_len = B.d_counters + 1;
    CoreArgs CA{d_down_off, d_down_arc, B.d_dcore, d_uslot, B.d_uval, d_perm, d_core_cell, d_core_ecc,
                d_taus, fl_in, fl_out, flag_words, B.d_keys, out_count, uint32_t(cap), A.lane_base, lk};
    const bool prof_on = prof.on;
    if (prof_on) HIPCHK(hipEventRecord(prof.ev[0], s));
    // core sweep: the top levels in one LDS-resident workgroup, then one launch per level
    size_t nlev = core_lvl.size() - 1;
    size_t top = 0;
    while (top < nlev) {
        size_t T = core_lvl[top + 1], ET = core_lvl_entries[top + 1];
        size_t need = (2 * ET + (T + 1) + (T << lk)) * 4;
        if (need > TOP_LDS_BUDGET) break;
        // stop where levels become wide enough for a grid of workgroups
        if (core_lvl[top + 1] - core_lvl[top] > 4096) break;
        ++top;
    }
    if (top > 0) {
        uint32_t T = core_lvl[top], ET = core_lvl_entries[top];
        size_t lds = (2 * size_t(ET) + (T + 1) + (size_t(T) << lk)) * 4;
        k_core_top<<<dim3(1), dim3(1024), lds, s>>>(CA, d_top_lvl, uint32_t(top), T, ET);
    }
    const uint32_t blk = 256;
    for (size_t l = top; l < nlev; ++l) {
        uint32_t vb = core_lvl[l], ve = core_lvl[l + 1];
        uint32_t deg = (core_lvl_entries[l + 1] - core_lvl_entries[l] + (ve - vb) - 1) / (ve - vb);
        uint32_t ls = 0;
        while ((1u << ls) < deg && (K << (ls + 1)) <= 64u && (ls + 1) <= 3) ++ls;
        uint64_t threads = uint64_t(ve - vb) << (lk + ls);
        uint32_t grid = uint32_t((threads + blk - 1) / blk);
        k_core_level<<<dim3(grid), dim3(blk), 0, s>>>(CA, ls, vb, ve);
    }
    if (prof_on) HIPCHK(hipEventRecord(prof.ev[1], s));
    uint32_t lg = 0;
    if (num_cells > 0) {
        k_active_cells<<<dim3((num_cells + 255) / 256), dim3(256), 0, s>>>(
            fl_in, fl_out, flag_words, d_uncovered, d_cell_off, d_src, A.lanes, num_cells,
            A.mode_plain ? 1u : 0u, B.d_list, list_len);
        // lanes per workgroup: as many as fit the LDS budget next to the staged blob
        size_t blob_bytes = size_t(max_blob_words) * 4;
        bool staged = blob_bytes + size_t(max_cell_labels) * 4 <= LDS_MAX;
        size_t fixed = staged ? blob_bytes : 0;
        lg = lk;
        while (lg > 0 && fixed + (size_t(max_cell_labels) << lg) * 4 > CELL_LDS_BUDGET) --lg;
        size_t lds = fixed + (size_t(max_cell_labels) << lg) * 4;
        if (lds > LDS_MAX) {
            set_error("a cell does not fit the LDS of one workgroup");
            return -2;
        }
        uint32_t groups = K >> lg;
        CellArgs LA{B.d_list, list_len, d_cblob, d_blob, d_cell_off, B.d_dcore, d_uslot, B.d_uval, d_perm,
                    d_taus, d_src, d_cmeta, A.want_dist ? B.d_dist : nullptr, B.d_keys, out_count,
                    uint32_t(cap), A.lane_base, lk, lg};
        if (prof_on) HIPCHK(hipEventRecord(prof.ev[2], s));
        if (staged)
            k_cell_sweep<true><<<dim3(num_cells * groups), dim3(256), lds, s>>>(LA, max_blob_words);
        else
            k_cell_sweep<false><<<dim3(num_cells * groups), dim3(256), lds, s>>>(LA, 0);
    } else if (prof_on) {
        HIPCHK(hipEventRecord(prof.ev[2], s));
    }
    if (prof_on) HIPCHK(hipEventRecord(prof.ev[3], s));
    HIPCHK(hipGetLastError());
    if (nu) k_uset_clear<<<dim3((nu + 255) / 256), dim3(256), 0, s>>>(d_uslot, d_upos, nu);
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
        prof.core_launches += (top > 0 ? 1 : 0) + (nlev - top);
        prof.core_entries += core_entries;
        // offsets + entries + cell ids and eccentricities + k labels written and read back once
        prof.core_bytes += 4ull * (n_core + 1) + 8ull * core_entries + 8ull * n_core + uint64_t(K) * 8ull * n_core;
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
            const uint64_t groups = K >> lg;
            for (uint32_t c : lst) {
                prof.cells_swept++;
                prof.cell_vertices += cell_cnt[c];
                prof.cell_entries += cell_entries[c];
                // each lane group streams the cell's blob once; each lane reads its core refs once
                prof.cell_bytes += groups * 4ull * cell_words[c] + uint64_t(K) * 4ull * cell_core_refs[c];
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
