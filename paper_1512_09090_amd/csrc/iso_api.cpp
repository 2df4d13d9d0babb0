// iso_api.cpp - the C ABI (include/iso.h): loading, the host upward search,
// batching of queries into device sweeps, decoding of the sorted edge keys.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <unordered_map>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "api_internal.h"

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

namespace {

struct BusyGuard {
    iso_graph *g;
    bool ok;
    explicit BusyGuard(iso_graph *g_) : g(g_) {
        bool f = false;
        ok = g->busy.compare_exchange_strong(f, true);
    }
    ~BusyGuard() { if (ok) g->busy.store(false); }
};

int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

uint32_t pow2_at_least(uint32_t x) {
    uint32_t k = 1;
    while (k < x) k <<= 1;
    return k;
}

}  // namespace

void build_run_args(iso_graph *g, const uint32_t *src, const uint32_t *tau, uint32_t lanes, bool plain,
                    bool want_dist, isodev::RunArgs &A, uint32_t *settled, bool core_dijkstra) {
    const iso::Prep &P = g->P;
    A = isodev::RunArgs();
    A.block = g->tuning.block;
    A.cell_lds_bytes = size_t(g->tuning.cell_lds_kb) * 1024;
    A.use_graph = g->tuning.use_graph;
    A.cell_stage = g->tuning.cell_stage;
    A.cell_block = g->tuning.cell_block ? g->tuning.cell_block : (pow2_at_least(lanes) >= 32 ? 512u : 256u);
    A.lanes = lanes;
    A.k_pow2 = pow2_at_least(lanes);
    A.mode_plain = plain;
    A.want_dist = want_dist;
    A.debug = g->debug;
    A.core64 = g->tuning.core_mode == 0;
    A.plain_stream = g->tuning.plain_sweep == 0;
    const uint32_t K = A.k_pow2;
    A.taus.assign(K, 0u);   // padding lanes: every label INF > 0, so they activate no cell and emit nothing
    A.src_cell.assign(K, iso::NO_CELL);
    // upward searches on the graph's worker pool; each worker also splits its lanes' labels into
    // the top-table part and the rest
    A.xpos.assign(lanes, {});
    A.xval.assign(lanes, {});
    A.spos.assign(lanes, {});
    A.sval.assign(lanes, {});
    A.core_dijkstra = core_dijkstra;
    if (core_dijkstra) {   // isoPHAST-CD: the core graph and one search workspace per worker
        if (!g->coreg) {
            auto cg = std::make_unique<CoreGraph>();
            cg->build(P);
            g->coreg = std::move(cg);
        }
        if (g->cdj.size() < g->up.size()) {
            g->cdj.resize(g->up.size());
            g->cd_out.resize(g->up.size());
        }
    }
    {
        std::atomic<uint32_t> next{0};
        if (core_dijkstra) {
            A.table_x = A.table_levels = 0;
        } else {
            g->D.table_cut(g->tuning.table_max, A.table_x, A.table_levels);
        }
        // the upward searches stop at the table's vertices, or (isoPHAST-CD) at the core
        const uint32_t TX = core_dijkstra ? P.n_core : A.table_x;
        const std::function<void(int)> work = [&](int w) {
            std::vector<std::pair<uint32_t, uint32_t>> &U = g->up_out[w];
            std::vector<std::pair<uint32_t, uint32_t>> seeds;
            for (;;) {
                uint32_t j = next.fetch_add(1);
                if (j >= lanes) break;
                uint32_t st = g->up[w].run(g->upg, P.pos[src[j]], U, TX, g->tuning.stall ? &P : nullptr);
                if (settled) settled[j] = st;
                auto &xp = A.xpos[j], &xv = A.xval[j], &sp = A.spos[j], &sv = A.sval[j];
                sp.reserve(U.size());
                sv.reserve(U.size());
                if (core_dijkstra) {
                    // internal vertices of the source's cell keep their upward labels; the core
                    // vertices reached seed the core search, whose settled labels join them
                    seeds.clear();
                    for (const auto &pr : U) {
                        if (pr.first < TX) {
                            seeds.push_back(pr);
                        } else {
                            sp.push_back(pr.first);
                            sv.push_back(pr.second);
                        }
                    }
                    g->cdj[w].run(*g->coreg, seeds, tau[j], g->cd_out[w]);
                    for (const auto &pr : g->cd_out[w]) {
                        sp.push_back(pr.first);
                        sv.push_back(pr.second);
                    }
                    continue;
                }
                for (const auto &pr : U) {
                    if (pr.first < TX) {
                        xp.push_back(pr.first);
                        xv.push_back(pr.second);
                    } else {
                        sp.push_back(pr.first);
                        sv.push_back(pr.second);
                    }
                }
            }
        };
        g->pool->run(int(lanes), work);
    }
    for (uint32_t j = 0; j < lanes; ++j) {
        A.taus[j] = tau[j];
        A.src_cell[j] = P.num_cells ? P.cell_of[src[j]] : iso::NO_CELL;
    }
}

void split_edges(const uint32_t *pairs, const std::vector<uint32_t> &lane_off, uint32_t lanes,
                 std::vector<EdgeBuf> &out) {
    out.clear();
    out.resize(lanes);
    for (uint32_t j = 0; j < lanes; ++j) {
        const size_t a = lane_off[j], b = lane_off[j + 1];
        EdgeBuf &e = out[j];
        e.p = (iso_edge *)std::malloc(std::max<size_t>(1, b - a) * sizeof(iso_edge));
        if (!e.p) throw std::bad_alloc();
        e.n = b - a;
        if (b > a) std::memcpy(e.p, pairs + 2 * a, (b - a) * sizeof(iso_edge));
    }
}

namespace {
struct PinnedPool {
    std::mutex mu;
    std::unordered_map<void *, size_t> owned;      // every block of the pool -> capacity
    std::multimap<size_t, void *> idle;            // blocks not handed out, by capacity
    size_t idle_bytes = 0;
    static constexpr size_t KEEP = size_t(1) << 30;   // idle pinned memory kept for reuse
};
PinnedPool &pool() {
    static PinnedPool *P = new PinnedPool();   // never destroyed: blocks may outlive static teardown
    return *P;
}
}  // namespace

void *pinned_get(size_t bytes, size_t &cap) {
    PinnedPool &P = pool();
    {
        std::lock_guard<std::mutex> lk(P.mu);
        auto it = P.idle.lower_bound(bytes);
        if (it != P.idle.end() && it->first <= 4 * std::max<size_t>(bytes, 1 << 20)) {
            cap = it->first;
            void *p = it->second;
            P.idle_bytes -= it->first;
            P.idle.erase(it);
            return p;
        }
    }
    size_t c = size_t(1) << 20;
    while (c < bytes) c <<= 1;
    void *p = nullptr;
    if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess || !p) return nullptr;
    std::lock_guard<std::mutex> lk(P.mu);
    P.owned[p] = c;
    cap = c;
    return p;
}

bool pinned_put(void *p) {
    PinnedPool &P = pool();
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.owned.find(p);
    if (it == P.owned.end()) return false;
    P.idle.emplace(it->second, p);
    P.idle_bytes += it->second;
    while (P.idle_bytes > PinnedPool::KEEP && !P.idle.empty()) {   // drop the largest idle blocks
        auto last = std::prev(P.idle.end());
        P.idle_bytes -= last->first;
        P.owned.erase(last->second);
        hipHostFree(last->second);
        P.idle.erase(last);
    }
    return true;
}

int api_fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

namespace {

// Run `lanes` queries (<= 64) through one device sweep of the graph's own context.
int run_lanes(iso_graph *g, const uint32_t *src, const uint32_t *tau, uint32_t lanes, bool plain,
              bool want_dist, isodev::RunResult &R) {
    isodev::RunArgs A;
    std::vector<uint32_t> settled(lanes, 0);
    double t0 = now_ms();
    build_run_args(g, src, tau, lanes, plain, want_dist, A, settled.data());
    double t1 = now_ms();
    for (int attempt = 0; attempt < 8; ++attempt) {
        A.out_cap = g->out_cap;
        int r = g->D.run(g->D.main, A, R);
        if (r) return r;
        if (!R.overflow) break;
        g->out_cap = std::max<size_t>(g->out_cap * 2, size_t(R.count) + (size_t(R.count) >> 3));
        g->resweeps++;
    }
    if (R.overflow) return fail(ISO_ENOMEM, "edge buffer overflow");
    double t2 = now_ms();
    g->last.lanes += lanes;
    g->last.active_cells += R.active_cells;
    for (uint32_t j = 0; j < lanes; ++j) g->last.upward_settled += settled[j];
    g->last.t_upward_ms += t1 - t0;
    g->last.t_device_ms += t2 - t1 - R.t_result_ms;
    g->last.t_sort_ms += R.t_result_ms;
    return ISO_OK;
}

int check_query(iso_graph *g, uint32_t s, uint32_t tau, int mode) {
    if (!g) return fail(ISO_EINVAL, "graph handle is NULL");
    if (s >= g->P.n) return fail(ISO_EINVAL, "source out of range");
    if (tau > ISO_TAU_MAX) return fail(ISO_EINVAL, "tau must be <= 2^32 - 2");
    if (mode != ISO_MODE_PLAIN && mode != ISO_MODE_CELLS && mode != ISO_MODE_CD) return fail(ISO_EINVAL, "unknown mode");
    if (mode != ISO_MODE_PLAIN && g->P.num_cells == 0) return fail(ISO_EINVAL, "cells mode needs a partition");
    if (!g->on_device) return fail(ISO_EDEVICE, "graph was loaded without a device");
    return ISO_OK;
}

}  // namespace

extern "C" {

const char *iso_last_error(void) { return g_err.c_str(); }

void iso_free(void *p) {
    if (p && !pinned_put(p)) std::free(p);
}

int iso_load_graph(const iso_graph_desc *d, iso_graph **out) {
    if (!d || !out) return fail(ISO_EINVAL, "NULL argument");
    *out = nullptr;
    if (d->n == 0 || d->n > iso::TAIL_MASK) return fail(ISO_EINVAL, "n must be in [1, 2^30)");
    if (d->m && (!d->tail || !d->head || !d->weight)) return fail(ISO_EINVAL, "arc arrays are NULL");
    uint32_t maxc = d->max_cell_size ? d->max_cell_size : 2048;
    if (maxc > 4096) return fail(ISO_EINVAL, "max_cell_size must be <= 4096");
    for (uint64_t e = 0; e < d->m; ++e) {
        if (d->tail[e] >= d->n || d->head[e] >= d->n) return fail(ISO_EINVAL, "arc endpoint out of range");
        if (d->weight[e] == ISO_INF) return fail(ISO_EINVAL, "arc weight 2^32-1 is reserved");
    }
    if (d->cell_of) {
        if (d->num_cells == 0) return fail(ISO_EINVAL, "cell_of given with num_cells = 0");
        for (uint32_t v = 0; v < d->n; ++v)
            if (d->cell_of[v] >= d->num_cells) return fail(ISO_EINVAL, "cell id out of range");
    }
    iso_graph *g = new (std::nothrow) iso_graph();
    if (!g) return fail(ISO_ENOMEM, "out of host memory");
    try {
        g->threads = iso::resolve_threads(d->threads);
        iso::ArcList A;
        iso::simplify_arcs(d->n, d->m, d->tail, d->head, d->weight, A);
        std::vector<uint32_t> cell_of;
        uint32_t num_cells = 0;
        if (d->cell_of) {
            cell_of.assign(d->cell_of, d->cell_of + d->n);
            num_cells = d->num_cells;
        } else if (d->num_cells > 0) {
            if (d->xy) {
                iso::partition_bisect(d->n, d->xy, d->num_cells, cell_of);
                num_cells = d->num_cells;
            } else {
                iso::partition_bfs(A, maxc, cell_of, num_cells);
            }
        }
        if (num_cells > isodev::MAX_CELLS) {
            delete g;
            return fail(ISO_EINVAL, "more than 2^24 cells");
        }
        if (num_cells) {
            std::vector<uint32_t> sz(num_cells, 0);
            for (uint32_t c : cell_of) sz[c]++;
            for (uint32_t c = 0; c < num_cells; ++c)
                if (sz[c] > maxc) {
                    delete g;
                    return fail(ISO_EINVAL, "a cell exceeds max_cell_size (use more cells)");
                }
        }
        uint64_t h = iso::hash_input(A, cell_of, num_cells);
        bool loaded = false;
        if (d->prep_path && *d->prep_path) {
            iso::LoadStatus st = iso::load_prep(d->prep_path, g->P, h);
            if (st == iso::LOAD_CORRUPT) {
                delete g;
                return fail(ISO_EFORMAT, std::string("corrupt or truncated preprocessed file ") + d->prep_path);
            }
            loaded = st == iso::LOAD_OK;
            if (!loaded) g->P = iso::Prep();
        }
        if (!loaded) {
            iso::PrepOptions o;
            o.num_cells = num_cells;
            o.max_cell_size = maxc;
            o.threads = g->threads;
            o.verbose = d->verbose;
            iso::build_prep(A, cell_of, num_cells, o, g->P);
            if (d->prep_path && *d->prep_path && !iso::save_prep(d->prep_path, g->P, h)) {
                delete g;
                return fail(ISO_EFORMAT, std::string("cannot write ") + d->prep_path);
            }
        } else {
            g->P.seconds = 0.0;
        }
        if (uint64_t(g->P.n_core) * isodev::MAX_LANES >= (uint64_t(1) << 32)) {
            delete g;
            return fail(ISO_EINVAL, "core too large for 64 interleaved lanes");
        }
        g->upg.build(g->P);
        if (!g->upg.dag_ok) {
            delete g;
            return fail(ISO_EFORMAT, "upward arcs must lead to smaller sweep positions");
        }
        {
            // one upward-search workspace per worker; a sweep has at most 64 searches
            const int W = std::min<int>(g->threads, int(isodev::MAX_LANES));
            g->up.resize(W);
            for (auto &u : g->up) u.init(g->P.n);
            g->up_out.resize(W);
            g->pool = std::make_unique<WorkerPool>(W);
        }
        if (d->xy) g->xy.assign(d->xy, d->xy + 2 * size_t(d->n));
        g->out_cap = std::max<size_t>(1 << 16, std::min<size_t>(g->P.m / 4 + 1024, size_t(1) << 24));
        if (d->device >= 0) {
            int r = g->D.upload(g->P, d->device);
            if (r) {
                g->D.release();
                delete g;
                return r;
            }
            g->on_device = true;
        }
    } catch (const std::bad_alloc &) {
        delete g;
        return fail(ISO_ENOMEM, "out of host memory during preprocessing");
    }
    *out = g;
    return ISO_OK;
}

void iso_free_graph(iso_graph *g) {
    if (!g) return;
    if (g->vbits_dev || g->tdist_dev) {
        hipSetDevice(g->D.device);
        if (g->vbits_dev) hipFree(g->vbits_dev);
        if (g->tdist_dev) hipFree(g->tdist_dev);
    }
    g->D.release();
    delete g;
}

int iso_graph_get_info(const iso_graph *g, iso_graph_info *info) {
    if (!g || !info) return fail(ISO_EINVAL, "NULL argument");
    const iso::Prep &P = g->P;
    info->n = P.n;
    info->n_core = P.n_core;
    info->num_cells = P.num_cells;
    info->core_levels = P.core_lvl.empty() ? 0 : uint32_t(P.core_lvl.size() - 1);
    info->max_cell_levels = P.max_cell_levels;
    info->max_cell_internal = P.max_cell_internal;
    info->m = P.m;
    info->down_arcs = P.down_off.empty() ? 0 : P.down_off[P.n];
    info->up_arcs = P.up_off.empty() ? 0 : P.up_off[P.n];
    info->shortcuts = P.shortcuts;
    info->device_bytes = g->D.bytes;
    info->prep_seconds = P.seconds;
    info->host_threads = uint32_t(g->threads);
    info->top_table = g->D.TX;
    return ISO_OK;
}

// k queries in sweeps of up to lanes_per_launch lanes.  With more than one sweep, two sweep
// contexts alternate: the host upward searches of sweep i overlap the device work of sweeps
// i - 1 and i - 2; then sweep i - 2's edges are collected and sweep i is launched on its
// context.  (Phase timings of the profile then include the device time that sweeps share.)
// With `dev` set the edges stay on the device instead (iso_query_batch_device): sweep i decodes its
// lanes into dev->pairs after the edges of the sweeps before it and writes their starts to
// dev->off; a sweep that would pass dev->cap is counted but not written, and the call then
// reports ISO_ESPACE with the exact total.
struct DevOut {
    uint32_t *pairs, *off;
    uint64_t cap;
    hipStream_t caller;   // the sweep streams wait for the work queued on it before the call
    uint64_t total = 0;
    bool over = false;
};

// Makes the sweep contexts' streams wait for the work queued so far on `caller`.
static int wait_for_caller(isodev::DevGraph &D, hipStream_t caller, bool aux) {
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return fail(ISO_EDEVICE, "hipEventCreate failed");
    bool ok = hipEventRecord(ev, caller) == hipSuccess && hipStreamWaitEvent(D.main.stream, ev, 0) == hipSuccess &&
              (!aux || hipStreamWaitEvent(D.aux.stream, ev, 0) == hipSuccess);
    hipEventDestroy(ev);
    return ok ? ISO_OK : fail(ISO_EDEVICE, "waiting for the caller's stream failed");
}

static int query_many(iso_graph *g, size_t k, const uint32_t *src, const uint32_t *tau, int mode,
                      iso_edge **edges, size_t *offsets, DevOut *dev = nullptr) {
    double t0 = now_ms();
    g->last = iso_query_stats{};
    const uint32_t per = std::max<uint32_t>(1, std::min<uint32_t>(g->tuning.lanes_per_launch, isodev::MAX_LANES));
    const size_t nsweeps = (k + per - 1) / per;
    isodev::DevGraph &D = g->D;
    const bool overlap = nsweeps > 1;
    if (overlap && !D.aux_ready) {
        if (D.aux.create(D.device)) return fail(ISO_EDEVICE, "creating the second sweep context failed");
        D.aux.prof.on = D.main.prof.on;
        D.aux_ready = true;
    }
    if (dev) {
        int r = wait_for_caller(D, dev->caller, overlap);
        if (r) return r;
    }
    // every sweep's edges are copied from the device straight into the result buffer, a
    // pinned pool block (grown by moving to a larger block when a later sweep needs room)
    EdgeBuf out;
    out.pinned = true;
    size_t cap = 0;
    if (offsets) offsets[0] = 0;
    if (!dev && nsweeps > 1 && g->edges_per_query > 0) {
        // a block for the expected result at once (the last multi-sweep call's edges per query and
        // an eighth more): growing from a small block copies the result several times over
        const size_t want = size_t(g->edges_per_query * double(k) * 1.125) + 1024;
        size_t got = 0;
        out.p = (iso_edge *)pinned_get(want * sizeof(iso_edge), got);
        cap = out.p ? got / sizeof(iso_edge) : 0;
    }
    struct Sweep {
        isodev::RunArgs A;
        isodev::SweepCtx *C = nullptr;
        size_t b = 0;
        uint32_t lanes = 0;
        std::vector<uint32_t> settled;
    };
    auto collect = [&](Sweep &W) -> int {
        isodev::RunResult R;
        if (dev) {
            R.dev_dst = true;
            R.dev_pairs = dev->pairs;
            R.dev_overflow = dev->over;   // past the capacity already: count only
            R.dev_off = dev->off + W.b;
            R.dev_cap = dev->cap;
            R.dev_base = uint32_t(dev->total);
            R.dev_lanes = W.lanes;
        }
        R.sink = [&](size_t n) -> uint32_t * {
            if (out.n + n > cap) {
                size_t want = std::max(out.n + n, cap + cap / 2), got = 0;
                iso_edge *p = (iso_edge *)pinned_get(want * sizeof(iso_edge), got);
                if (!p) return nullptr;
                if (out.n) std::memcpy(p, out.p, out.n * sizeof(iso_edge));
                if (out.p) pinned_put(out.p);
                out.p = p;
                cap = got / sizeof(iso_edge);
            }
            return reinterpret_cast<uint32_t *>(out.p + out.n);
        };
        const double tw = now_ms();
        int r = D.finish(*W.C, R);
        for (int attempt = 0; !r && R.overflow && attempt < 8; ++attempt) {   // grow the edge buffer, sweep again
            g->out_cap = std::max<size_t>(g->out_cap * 2, size_t(R.count) + (size_t(R.count) >> 3));
            g->resweeps++;
            W.A.out_cap = g->out_cap;
            r = D.launch(*W.C, W.A);
            if (!r) r = D.finish(*W.C, R);
        }
        if (r) return r;
        if (R.overflow) return fail(ISO_ENOMEM, "edge buffer overflow");
        if (dev) {
            dev->over = R.dev_overflow;
            dev->total += R.count;
            if (dev->total >= iso::INF) return fail(ISO_ESPACE, "more than 2^32 - 2 edges in one call");
        } else {
            for (uint32_t j = 0; j < W.lanes; ++j) offsets[W.b + j + 1] = out.n + R.lane_off[j + 1];
        }
        out.n += R.count;
        g->last.lanes += W.lanes;
        g->last.active_cells += R.active_cells;
        for (uint32_t s : W.settled) g->last.upward_settled += s;
        g->last.t_device_ms += now_ms() - tw - R.t_result_ms;
        g->last.t_sort_ms += R.t_result_ms;
        return ISO_OK;
    };
    // Sweeps in flight, oldest first: sweep i runs on context i mod nctx, whose previous sweep
    // (i - nctx) is collected only after sweep i's upward searches, so that those overlap the
    // device work of the sweeps before it.
    isodev::SweepCtx *ctxs[2] = {&D.main, &D.aux};
    const size_t nctx = overlap ? 2 : 1;
    std::deque<std::unique_ptr<Sweep>> inflight;
    auto drain = [&]() {   // leave every launched sweep's context idle after an error
        while (!inflight.empty()) {
            isodev::RunResult R;
            D.finish(*inflight.front()->C, R);
            inflight.pop_front();
        }
    };
    for (size_t i = 0; i < nsweeps; ++i) {
        auto W = std::make_unique<Sweep>();
        W->b = i * per;
        W->lanes = uint32_t(std::min<size_t>(per, k - W->b));
        W->C = ctxs[i % nctx];
        W->settled.assign(W->lanes, 0);
        const double tu = now_ms();
        build_run_args(g, src + W->b, tau + W->b, W->lanes, mode == ISO_MODE_PLAIN, false, W->A, W->settled.data(),
                       mode == ISO_MODE_CD);
        W->A.out_cap = g->out_cap;
        if (overlap)   // the sweeps share the GPU
            W->A.cell_per_cu = g->tuning.overlap_cells ? g->tuning.overlap_cells : isodev::OVERLAP_CELL_PER_CU;
        g->last.t_upward_ms += now_ms() - tu;
        if (inflight.size() == nctx) {   // frees W's context
            int r = collect(*inflight.front());
            inflight.pop_front();
            if (r) {
                drain();
                return r;
            }
        }
        int r = D.launch(*W->C, W->A);
        if (r) {
            drain();
            return r;
        }
        inflight.push_back(std::move(W));
    }
    while (!inflight.empty()) {
        int r = collect(*inflight.front());
        inflight.pop_front();
        if (r) {
            drain();
            return r;
        }
    }
    g->last.edges = out.n;
    if (!dev && nsweeps > 1) g->edges_per_query = double(out.n) / double(k);
    if (dev) {
        g->last.t_total_ms = now_ms() - t0;
        return dev->over ? fail(ISO_ESPACE, "device edge buffer holds " + std::to_string(dev->cap) +
                                                " pairs, the call found " + std::to_string(dev->total))
                         : ISO_OK;
    }
    if (!out.p) {   // no edges at all: a malloc'd placeholder
        out.pinned = false;
        if (!(out.p = (iso_edge *)std::malloc(sizeof(iso_edge))))
            return fail(ISO_ENOMEM, "out of host memory for the result");
    }
    *edges = out.release();
    g->last.t_total_ms = now_ms() - t0;
    return ISO_OK;
}

int iso_query(iso_graph *g, uint32_t source, uint32_t tau, int mode, iso_edge **edges, size_t *count) {
    if (edges) *edges = nullptr;
    if (!edges || !count) return fail(ISO_EINVAL, "NULL output pointer");
    int r = check_query(g, source, tau, mode);
    if (r) return r;
    BusyGuard guard(g);
    if (!guard.ok) return fail(ISO_EBUSY, "graph handle in use");
    size_t off[2];
    r = query_many(g, 1, &source, &tau, mode, edges, off);
    if (r) return r;
    *count = off[1];
    return ISO_OK;
}

int iso_query_batch(iso_graph *g, size_t k, const uint32_t *sources, const uint32_t *taus, int mode,
                    iso_edge **edges, size_t *offsets) {
    if (edges) *edges = nullptr;
    if (!edges || !offsets || (k && (!sources || !taus))) return fail(ISO_EINVAL, "NULL argument");
    if (!g) return fail(ISO_EINVAL, "graph handle is NULL");
    for (size_t j = 0; j < k; ++j) {
        int r = check_query(g, sources[j], taus[j], mode);
        if (r) return r;
    }
    if (k == 0) {
        offsets[0] = 0;
        *edges = (iso_edge *)std::malloc(sizeof(iso_edge));
        return *edges ? ISO_OK : fail(ISO_ENOMEM, "out of host memory");
    }
    BusyGuard guard(g);
    if (!guard.ok) return fail(ISO_EBUSY, "graph handle in use");
    return query_many(g, k, sources, taus, mode, edges, offsets);
}

// True if [p, p + bytes) lies inside one device allocation on `device`.
static bool device_range_ok(const void *p, size_t bytes, int device) {
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (at.type != hipMemoryTypeDevice || at.device != device) return false;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const uintptr_t b = uintptr_t(base), q = uintptr_t(p);
    return q >= b && bytes <= size && q - b <= size - bytes;
}

int iso_query_batch_device(iso_graph *g, size_t k, const uint32_t *sources, const uint32_t *taus, int mode,
                           uint32_t *pairs, uint64_t cap, uint32_t *offsets, uint64_t *total, void *stream) {
    if (total) *total = 0;
    if (!offsets || !total || (k && (!sources || !taus)) || (cap && !pairs))
        return fail(ISO_EINVAL, "NULL argument");
    if (!g) return fail(ISO_EINVAL, "graph handle is NULL");
    if (!g->on_device) return fail(ISO_EDEVICE, "graph was loaded without a device");
    for (size_t j = 0; j < k; ++j) {
        int r = check_query(g, sources[j], taus[j], mode);
        if (r) return r;
    }
    if (k >= iso::INF) return fail(ISO_EINVAL, "too many queries in one call");
    if (cap > (uint64_t(1) << 60)) return fail(ISO_EINVAL, "capacity out of range");
    if (hipSetDevice(g->D.device) != hipSuccess) return fail(ISO_EDEVICE, "hipSetDevice failed");
    if (!device_range_ok(offsets, (k + 1) * sizeof(uint32_t), g->D.device))
        return fail(ISO_EINVAL, "offsets is not k + 1 words of device memory on the graph's device");
    if (cap && !device_range_ok(pairs, cap * 2 * sizeof(uint32_t), g->D.device))
        return fail(ISO_EINVAL, "pairs is not cap pairs of device memory on the graph's device");
    BusyGuard guard(g);
    if (!guard.ok) return fail(ISO_EBUSY, "graph handle in use");
    DevOut dev{pairs, offsets, cap, (hipStream_t)stream};
    int r;
    if (k == 0) {
        isodev::SweepCtx &C = g->D.main;
        const uint32_t zero = 0;
        r = wait_for_caller(g->D, dev.caller, false);
        if (!r)
            r = hipMemcpyAsync(offsets, &zero, sizeof(uint32_t), hipMemcpyHostToDevice, C.stream) == hipSuccess &&
                        hipStreamSynchronize(C.stream) == hipSuccess
                    ? ISO_OK
                    : fail(ISO_EDEVICE, "writing the offsets failed");
    } else {
        r = query_many(g, k, sources, taus, mode, nullptr, nullptr, &dev);
    }
    *total = dev.total;
    return r;
}

// iso_query_batch_device without any allocation: one sweep at a time on the graph's fixed
// context, whose device buffers are carved from the static scratch for each sweep.
int iso_query_batch_device_noalloc(iso_graph *g, size_t k, const uint32_t *sources, const uint32_t *taus, int mode,
                                   uint32_t *pairs, uint64_t cap, uint32_t *offsets, uint64_t *total, void *stream) {
    if (total) *total = 0;
    if (!offsets || !total || (k && (!sources || !taus)) || (cap && !pairs))
        return fail(ISO_EINVAL, "NULL argument");
    if (!g) return fail(ISO_EINVAL, "graph handle is NULL");
    if (!g->on_device) return fail(ISO_EDEVICE, "graph was loaded without a device");
    for (size_t j = 0; j < k; ++j) {
        int r = check_query(g, sources[j], taus[j], mode);
        if (r) return r;
    }
    if (k >= iso::INF) return fail(ISO_EINVAL, "too many queries in one call");
    if (cap > (uint64_t(1) << 60)) return fail(ISO_EINVAL, "capacity out of range");
    if (hipSetDevice(g->D.device) != hipSuccess) return fail(ISO_EDEVICE, "hipSetDevice failed");
    if (!device_range_ok(offsets, (k + 1) * sizeof(uint32_t), g->D.device))
        return fail(ISO_EINVAL, "offsets is not k + 1 words of device memory on the graph's device");
    if (cap && !device_range_ok(pairs, cap * 2 * sizeof(uint32_t), g->D.device))
        return fail(ISO_EINVAL, "pairs is not cap pairs of device memory on the graph's device");
    BusyGuard guard(g);
    if (!guard.ok) return fail(ISO_EBUSY, "graph handle in use");
    isodev::DevGraph &D = g->D;
    isodev::SweepCtx &C = D.fixed;
    if (hipEventRecord(D.fixed_wait, (hipStream_t)stream) != hipSuccess ||
        hipStreamWaitEvent(C.stream, D.fixed_wait, 0) != hipSuccess)
        return fail(ISO_EDEVICE, "waiting for the caller's stream failed");
    g->last = iso_query_stats{};
    const double t0 = now_ms();
    if (k == 0) {
        const uint32_t zero = 0;
        if (hipMemcpyAsync(offsets, &zero, sizeof(uint32_t), hipMemcpyHostToDevice, C.stream) != hipSuccess ||
            hipStreamSynchronize(C.stream) != hipSuccess)
            return fail(ISO_EDEVICE, "writing the offsets failed");
        return ISO_OK;
    }
    const uint32_t per = std::max<uint32_t>(1, std::min<uint32_t>(g->tuning.lanes_per_launch, isodev::MAX_LANES));
    uint64_t done = 0;
    bool over = false;
    for (size_t b = 0; b < k; b += per) {
        const uint32_t lanes = uint32_t(std::min<size_t>(per, k - b));
        isodev::RunArgs A;
        const double tu = now_ms();
        build_run_args(g, sources + b, taus + b, lanes, mode == ISO_MODE_PLAIN, false, A, nullptr,
                       mode == ISO_MODE_CD);
        g->last.t_upward_ms += now_ms() - tu;
        A.use_graph = 0;
        A.debug = false;
        A.fill_uslot = b == 0;   // the scratch may hold another call's data
        uint32_t nu = 0, nx = 0;
        for (uint32_t j = 0; j < lanes; ++j) {
            nu += uint32_t(A.spos[j].size());
            nx += uint32_t(A.xpos[j].size());
        }
        size_t kcap = 0;
        int r = D.carve_fixed(A.k_pow2, nu, nx, 1, kcap);
        if (r) return r == -2 ? ISO_ENOMEM : r;
        A.out_cap = kcap;
        const double tw = now_ms();
        if ((r = D.launch(C, A))) {
            if (C.pending) {
                isodev::RunResult R0;
                D.finish(C, R0);
            }
            return r == -2 ? ISO_ENOMEM : r;
        }
        isodev::RunResult R;
        R.dev_dst = true;
        R.dev_pairs = pairs;
        R.dev_overflow = over;
        R.dev_off = offsets + b;
        R.dev_cap = cap;
        R.dev_base = uint32_t(done);
        R.dev_lanes = lanes;
        if ((r = D.finish(C, R))) return r == -2 ? ISO_ENOMEM : r;
        if (R.overflow)
            return fail(ISO_ENOMEM, "the isochrone edges of one sweep exceed the static scratch; use fewer "
                                    "queries per sweep");
        over = R.dev_overflow;
        done += R.count;
        if (done >= iso::INF) return fail(ISO_ESPACE, "more than 2^32 - 2 edges in one call");
        g->last.lanes += lanes;
        g->last.active_cells += R.active_cells;
        g->last.t_device_ms += now_ms() - tw - R.t_result_ms;
        g->last.t_sort_ms += R.t_result_ms;
    }
    *total = done;
    g->last.edges = done;
    g->last.t_total_ms = now_ms() - t0;
    return over ? fail(ISO_ESPACE, "device edge buffer holds " + std::to_string(cap) + " pairs, the call found " +
                                       std::to_string(done))
                : ISO_OK;
}

// One sweep of k <= 64 queries whose output is the vertices in range: bitmap rows of
// ceil(n / 64) words per query at `bits` (device), or with bits NULL only the lane masks by
// position in the sweep context (the polygon output).  With `wait` set, the caller's queued
// work is waited for first.
static int vertices_sweep(iso_graph *g, size_t k, const uint32_t *src, const uint32_t *tau, int mode,
                          uint64_t *bits, bool wait, hipStream_t caller) {
    const double t0 = now_ms();
    g->last = iso_query_stats{};
    isodev::RunArgs A;
    std::vector<uint32_t> settled(k, 0);
    build_run_args(g, src, tau, uint32_t(k), mode == ISO_MODE_PLAIN, false, A, settled.data(), mode == ISO_MODE_CD);
    A.out_cap = g->out_cap;
    A.vbits = bits;
    A.vmask_only = bits == nullptr;
    const double t1 = now_ms();
    if (wait) {
        int r = wait_for_caller(g->D, caller, false);
        if (r) return r;
    }
    isodev::RunResult R;
    int r = g->D.run(g->D.main, A, R);
    if (r) return r;
    g->last.lanes = uint32_t(k);
    g->last.active_cells = R.active_cells;
    for (uint32_t x : settled) g->last.upward_settled += x;
    g->last.t_upward_ms = t1 - t0;
    g->last.t_device_ms = now_ms() - t1;
    g->last.t_total_ms = now_ms() - t0;
    return ISO_OK;
}

int iso_query_batch_vertices_device(iso_graph *g, size_t k, const uint32_t *sources, const uint32_t *taus,
                                    int mode, uint64_t *bits, void *stream) {
    if (!bits || !sources || !taus) return fail(ISO_EINVAL, "NULL argument");
    if (!g) return fail(ISO_EINVAL, "graph handle is NULL");
    if (!g->on_device) return fail(ISO_EDEVICE, "graph was loaded without a device");
    if (k < 1 || k > isodev::MAX_LANES) return fail(ISO_EINVAL, "k must be in [1, 64]");
    for (size_t j = 0; j < k; ++j) {
        int r = check_query(g, sources[j], taus[j], mode);
        if (r) return r;
    }
    if (hipSetDevice(g->D.device) != hipSuccess) return fail(ISO_EDEVICE, "hipSetDevice failed");
    const size_t W = (size_t(g->P.n) + 63) / 64;
    if (!device_range_ok(bits, k * W * sizeof(uint64_t), g->D.device))
        return fail(ISO_EINVAL, "bits is not k * ceil(n / 64) words of device memory on the graph's device");
    BusyGuard guard(g);
    if (!guard.ok) return fail(ISO_EBUSY, "graph handle in use");
    return vertices_sweep(g, k, sources, taus, mode, bits, true, (hipStream_t)stream);
}

int iso_query_vertices(iso_graph *g, uint32_t source, uint32_t tau, int mode, uint32_t **vertices, size_t *count) {
    if (vertices) *vertices = nullptr;
    if (!vertices || !count) return fail(ISO_EINVAL, "NULL output pointer");
    int r = check_query(g, source, tau, mode);
    if (r) return r;
    if (!g->on_device) return fail(ISO_EDEVICE, "graph was loaded without a device");
    BusyGuard guard(g);
    if (!guard.ok) return fail(ISO_EBUSY, "graph handle in use");
    if (hipSetDevice(g->D.device) != hipSuccess) return fail(ISO_EDEVICE, "hipSetDevice failed");
    const size_t W = (size_t(g->P.n) + 63) / 64;
    if (!g->vbits_dev && hipMalloc((void **)&g->vbits_dev, W * sizeof(uint64_t)) != hipSuccess) {
        g->vbits_dev = nullptr;
        return fail(ISO_ENOMEM, "device allocation of the vertex bitmap failed");
    }
    if ((r = vertices_sweep(g, 1, &source, &tau, mode, g->vbits_dev, false, nullptr))) return r;
    std::vector<uint64_t> h(W);
    if (hipMemcpy(h.data(), g->vbits_dev, W * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(ISO_EDEVICE, "copying the vertex bitmap failed");
    size_t cnt = 0;
    for (uint64_t w : h) cnt += size_t(__builtin_popcountll(w));
    uint32_t *out = (uint32_t *)std::malloc(std::max<size_t>(1, cnt) * sizeof(uint32_t));
    if (!out) return fail(ISO_ENOMEM, "out of host memory for the result");
    size_t k = 0;
    for (size_t i = 0; i < W; ++i)
        for (uint64_t w = h[i]; w; w &= w - 1) out[k++] = uint32_t(i * 64 + size_t(__builtin_ctzll(w)));
    *vertices = out;
    *count = cnt;
    return ISO_OK;
}

int iso_query_polygon_batch(iso_graph *g, size_t k, const uint32_t *sources, const uint32_t *taus, int mode,
                            iso_edge **darts, size_t *dart_off, uint64_t **cycles, size_t *cycle_off) {
    if (darts) *darts = nullptr;
    if (cycles) *cycles = nullptr;
    if (!darts || !dart_off || !cycles || !cycle_off || !sources || !taus) return fail(ISO_EINVAL, "NULL argument");
    if (!g) return fail(ISO_EINVAL, "graph handle is NULL");
    if (!g->on_device) return fail(ISO_EDEVICE, "graph was loaded without a device");
    if (k < 1 || k > isodev::MAX_LANES) return fail(ISO_EINVAL, "k must be in [1, 64]");
    for (size_t j = 0; j < k; ++j) {
        int r = check_query(g, sources[j], taus[j], mode);
        if (r) return r;
    }
    if (g->xy.empty()) return fail(ISO_ESTATE, "polygons need the vertex coordinates (desc.xy at load)");
    BusyGuard guard(g);
    if (!guard.ok) return fail(ISO_EBUSY, "graph handle in use");
    if (hipSetDevice(g->D.device) != hipSuccess) return fail(ISO_EDEVICE, "hipSetDevice failed");
    int r;
    if (!g->D.rot.ready) {
        try {
            if ((r = g->D.upload_rotation(g->P, g->xy.data(), g->threads))) return fail(r, iso_last_error());
        } catch (const std::bad_alloc &) {
            return fail(ISO_ENOMEM, "out of host memory building the rotation system");
        }
    }
    if ((r = vertices_sweep(g, k, sources, taus, mode, nullptr, false, nullptr))) return r;
    const double t0 = now_ms();
    isodev::PolyResult PR;
    try {
        if ((r = g->D.polygons(g->D.main, uint32_t(k), PR))) return fail(r, iso_last_error());
    } catch (const std::bad_alloc &) {
        return fail(ISO_ENOMEM, "out of host memory for the polygons");
    }
    const size_t nd = PR.loff[k], nc = PR.lcyc[k];
    iso_edge *d = (iso_edge *)std::malloc(std::max<size_t>(1, nd) * sizeof(iso_edge));
    uint64_t *c = (uint64_t *)std::malloc((nc + 1) * sizeof(uint64_t));
    if (!d || !c) {
        std::free(d);
        std::free(c);
        return fail(ISO_ENOMEM, "out of host memory for the result");
    }
    if (nd) std::memcpy(d, PR.darts.data(), nd * sizeof(iso_edge));
    for (size_t i = 0; i < nc; ++i) c[i] = PR.cyc[i];
    c[nc] = nd;
    for (size_t j = 0; j <= k; ++j) {
        dart_off[j] = PR.loff[j];
        cycle_off[j] = PR.lcyc[j];
    }
    *darts = d;
    *cycles = c;
    g->last.edges = nd;
    g->last.t_sort_ms = now_ms() - t0;
    g->last.t_total_ms += g->last.t_sort_ms;
    return ISO_OK;
}

int iso_query_polygon(iso_graph *g, uint32_t source, uint32_t tau, int mode, iso_edge **darts, size_t *count,
                      uint64_t **cycles, size_t *ncycles) {
    if (darts) *darts = nullptr;
    if (cycles) *cycles = nullptr;
    if (!count || !ncycles) return fail(ISO_EINVAL, "NULL output pointer");
    size_t doff[2], coff[2];
    int r = iso_query_polygon_batch(g, 1, &source, &tau, mode, darts, doff, cycles, coff);
    if (r) return r;
    *count = doff[1];
    *ncycles = coff[1];
    return ISO_OK;
}

int iso_targets_select(iso_graph *g, const uint32_t *targets, size_t count, iso_targets **out) {
    if (out) *out = nullptr;
    if (!g || !out || (count && !targets)) return fail(ISO_EINVAL, "NULL argument");
    if (!g->on_device) return fail(ISO_EDEVICE, "graph was loaded without a device");
    if (count >= (size_t(1) << 31)) return fail(ISO_EINVAL, "too many targets");
    for (size_t i = 0; i < count; ++i)
        if (targets[i] >= g->P.n) return fail(ISO_EINVAL, "target out of range");
    BusyGuard guard(g);
    if (!guard.ok) return fail(ISO_EBUSY, "graph handle in use");
    const double t0 = now_ms();
    std::unique_ptr<iso_targets> t(new iso_targets());
    t->g = g;
    uint32_t tx = 0, levels = 0;
    g->D.table_cut(g->tuning.table_max, tx, levels);
    int r = 0;
    try {
        r = g->D.select_targets(g->P, targets, uint32_t(count), tx, levels, t->T);
    } catch (const std::bad_alloc &) {
        r = ISO_ENOMEM;
    }
    if (r) {
        t->T.release();
        return r == ISO_ENOMEM ? fail(ISO_ENOMEM, "out of memory selecting the targets") : r;
    }
    t->select_ms = now_ms() - t0;
    *out = t.release();
    return ISO_OK;
}

// Sweeps of up to lanes_per_launch sources against a target set, distances into `dist`
// (device, k * count words).
static int targets_sweeps(iso_graph *g, const iso_targets *t, size_t k, const uint32_t *src, uint32_t *dist) {
    const double t0 = now_ms();
    g->last = iso_query_stats{};
    const size_t per = std::max<uint32_t>(1, std::min<uint32_t>(g->tuning.lanes_per_launch, isodev::MAX_LANES));
    std::vector<uint32_t> zero(per, 0u), settled(per, 0u);
    for (size_t b = 0; b < k; b += per) {
        const uint32_t lanes = uint32_t(std::min(per, k - b));
        isodev::RunArgs A;
        const double tu = now_ms();
        build_run_args(g, src + b, zero.data(), lanes, true, false, A, settled.data());
        g->last.t_upward_ms += now_ms() - tu;
        if (A.table_x != t->T.tx)
            return fail(ISO_ESTATE, "the top table prefix changed since the targets were selected; select again");
        A.out_cap = g->out_cap;
        A.tg = &t->T;
        A.tg_out = dist + b * t->T.count;
        isodev::RunResult R;
        int r = g->D.run(g->D.main, A, R);
        if (r) return r;
        g->last.lanes += lanes;
        for (uint32_t j = 0; j < lanes; ++j) g->last.upward_settled += settled[j];
    }
    g->last.t_total_ms = now_ms() - t0;
    g->last.t_device_ms = g->last.t_total_ms - g->last.t_upward_ms;
    return ISO_OK;
}

static int targets_check(iso_graph *g, const iso_targets *t, size_t k, const uint32_t *sources) {
    if (!g || !t || (k && !sources)) return fail(ISO_EINVAL, "NULL argument");
    if (t->g != g) return fail(ISO_EINVAL, "target set of another graph");
    if (!g->on_device) return fail(ISO_EDEVICE, "graph was loaded without a device");
    for (size_t j = 0; j < k; ++j)
        if (sources[j] >= g->P.n) return fail(ISO_EINVAL, "source out of range");
    return ISO_OK;
}

int iso_targets_query_device(iso_graph *g, const iso_targets *t, size_t k, const uint32_t *sources, uint32_t *dist,
                             void *stream) {
    int r = targets_check(g, t, k, sources);
    if (r) return r;
    const size_t words = k * size_t(t->T.count);
    if (words == 0) return ISO_OK;
    if (!dist) return fail(ISO_EINVAL, "NULL argument");
    if (hipSetDevice(g->D.device) != hipSuccess) return fail(ISO_EDEVICE, "hipSetDevice failed");
    if (!device_range_ok(dist, words * sizeof(uint32_t), g->D.device))
        return fail(ISO_EINVAL, "dist is not k * count words of device memory on the graph's device");
    BusyGuard guard(g);
    if (!guard.ok) return fail(ISO_EBUSY, "graph handle in use");
    if ((r = wait_for_caller(g->D, (hipStream_t)stream, false))) return r;
    return targets_sweeps(g, t, k, sources, dist);
}

int iso_targets_query(iso_graph *g, const iso_targets *t, size_t k, const uint32_t *sources, uint32_t *dist) {
    int r = targets_check(g, t, k, sources);
    if (r) return r;
    const size_t words = k * size_t(t->T.count);
    if (words == 0) return ISO_OK;
    if (!dist) return fail(ISO_EINVAL, "NULL argument");
    BusyGuard guard(g);
    if (!guard.ok) return fail(ISO_EBUSY, "graph handle in use");
    if (hipSetDevice(g->D.device) != hipSuccess) return fail(ISO_EDEVICE, "hipSetDevice failed");
    if (g->tdist_cap < words) {
        if (g->tdist_dev) hipFree(g->tdist_dev);
        g->tdist_dev = nullptr;
        g->tdist_cap = 0;
        if (hipMalloc((void **)&g->tdist_dev, words * sizeof(uint32_t)) != hipSuccess) {
            g->tdist_dev = nullptr;
            return fail(ISO_ENOMEM, "device allocation of the distances failed");
        }
        g->tdist_cap = words;
    }
    if ((r = targets_sweeps(g, t, k, sources, g->tdist_dev))) return r;
    if (hipMemcpy(dist, g->tdist_dev, words * sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(ISO_EDEVICE, "copying the distances failed");
    return ISO_OK;
}

int iso_targets_get_info(const iso_targets *t, uint64_t *vertices, uint64_t *arcs, uint32_t *groups,
                         double *select_ms) {
    if (!t) return fail(ISO_EINVAL, "NULL argument");
    if (vertices) *vertices = t->T.nr;
    if (arcs) *arcs = t->T.arcs;
    if (groups) *groups = t->T.group.empty() ? 0u : uint32_t(t->T.group.size() - 1);
    if (select_ms) *select_ms = t->select_ms;
    return ISO_OK;
}

void iso_targets_free(iso_targets *t) {
    if (!t) return;
    t->T.release();
    delete t;
}

int iso_query_distances(iso_graph *g, uint32_t source, uint32_t tau, int mode, uint32_t *dist,
                        uint8_t *swept) {
    if (!dist) return fail(ISO_EINVAL, "NULL output pointer");
    int r = check_query(g, source, tau, mode);
    if (r) return r;
    if (mode == ISO_MODE_CD) return fail(ISO_EINVAL, "the core-search mode leaves core labels above tau unset");
    BusyGuard guard(g);
    if (!guard.ok) return fail(ISO_EBUSY, "graph handle in use");
    g->last = iso_query_stats{};
    isodev::RunResult R;
    r = run_lanes(g, &source, &tau, 1, mode == ISO_MODE_PLAIN, true, R);
    if (r) return r;
    const iso::Prep &P = g->P;
    std::vector<uint8_t> sw(P.n, 0);
    for (uint32_t p = 0; p < P.n_core; ++p) sw[p] = 1;
    if (P.num_cells) {
        auto mark = [&](uint32_t c) { for (uint32_t p = P.cell_off[c]; p < P.cell_off[c + 1]; ++p) sw[p] = 1; };
        if (mode == ISO_MODE_PLAIN) for (uint32_t c = 0; c < P.num_cells; ++c) mark(c);
        else for (uint32_t c : R.active_list) mark(c);
    }
    for (uint32_t p = 0; p < P.n; ++p) {
        uint32_t v = P.perm[p];
        uint32_t val = !sw[p] ? iso::INF : (p < P.n_core ? R.dcore[p] : R.dist[p]);
        dist[v] = val;
        if (swept) swept[v] = sw[p];
    }
    return ISO_OK;
}

int iso_graph_get_layout(const iso_graph *g, iso_layout *L) {
    if (!g || !L) return fail(ISO_EINVAL, "NULL argument");
    const iso::Prep &P = g->P;
    L->perm = P.perm.data();
    L->cell_of = P.cell_of.data();
    L->down_off = P.down_off.data();
    L->down_arc = P.down_arc.data();
    L->up_off = P.up_off.data();
    L->up_head = P.up_head.data();
    L->up_w = P.up_w.data();
    L->core_lvl = P.core_lvl.data();
    L->core_lvl_len = uint32_t(P.core_lvl.size());
    L->cell_off = P.cell_off.data();
    L->cell_lvl_ptr = P.cell_lvl_ptr.data();
    L->cell_lvl = P.cell_lvl.data();
    L->cell_lvl_len = uint32_t(P.cell_lvl.size());
    L->core_cell = P.core_cell.data();
    L->core_ecc = P.core_ecc.data();
    L->uncovered = P.uncovered.data();
    return ISO_OK;
}

int iso_profile_enable(iso_graph *g, int enable) {
    if (!g) return fail(ISO_EINVAL, "NULL argument");
    if (!g->on_device) return fail(ISO_EDEVICE, "graph was loaded without a device");
    for (isodev::SweepCtx *C : {&g->D.main, &g->D.aux}) {   // aux: created with main's setting
        auto &P = C->prof;
        hipEvent_t ev[sizeof(P.ev) / sizeof(P.ev[0])];
        std::copy(std::begin(P.ev), std::end(P.ev), ev);
        P = isodev::Profile();
        std::copy(std::begin(ev), std::end(ev), P.ev);
        P.on = enable != 0;
    }
    return ISO_OK;
}

int iso_profile_read(const iso_graph *g, iso_profile *o) {
    if (!g || !o) return fail(ISO_EINVAL, "NULL argument");
    *o = iso_profile{};
    for (const isodev::SweepCtx *C : {&g->D.main, &g->D.aux}) {   // both sweep contexts of query calls
        const auto &P = C->prof;
        if (P.acc_ready && C->bufs.d_prof) {   // the cell-sweep sums kept on the device
            uint64_t acc[7] = {0, 0, 0, 0, 0, 0, 0};
            if (hipSetDevice(g->D.device) != hipSuccess ||
                hipMemcpy(acc, C->bufs.d_prof, sizeof acc, hipMemcpyDeviceToHost) != hipSuccess)
                return fail(ISO_EDEVICE, "reading the profile sums failed");
            o->cell_bytes += acc[0]; o->cells_swept += acc[1]; o->cell_lanes += acc[2];
            o->cell_vertices += acc[3]; o->cell_entries += acc[4];
            o->cell_bytes_survey += acc[5]; o->cell_items += acc[6];
        }
        o->core_ms += P.core_ms; o->active_ms += P.active_ms; o->cell_ms += P.cell_ms; o->sort_ms += P.sort_ms;
        o->core_launches += P.core_launches; o->cell_launches += P.cell_launches; o->calls += P.calls;
        o->core_bytes += P.core_bytes; o->cell_bytes += P.cell_bytes; o->cell_bytes_survey += P.cell_bytes_survey;
        o->core_entries += P.core_entries; o->cell_entries += P.cell_entries;
        o->cell_vertices += P.cell_vertices; o->cells_swept += P.cells_swept;
        o->cell_lanes += P.cell_lanes; o->cell_items += P.cell_items;
        o->level_ms += P.level_ms; o->level_launches += P.level_launches; o->level_bytes += P.level_bytes;
    }
    return ISO_OK;
}

int iso_debug_enable(iso_graph *g, int enable) {
    if (!g) return fail(ISO_EINVAL, "NULL argument");
    if (!g->on_device) return fail(ISO_EDEVICE, "graph was loaded without a device");
    BusyGuard guard(g);
    if (!guard.ok) return fail(ISO_EBUSY, "graph handle in use");
    g->debug = enable != 0;
    g->resweeps = 0;
    if (hipSetDevice(g->D.device) != hipSuccess) return fail(ISO_EDEVICE, "hipSetDevice failed");
    for (isodev::SweepCtx *C : {&g->D.main, &g->D.aux})
        if (C->bufs.d_dbg && hipMemset(C->bufs.d_dbg, 0, 8 * sizeof(uint64_t)) != hipSuccess)
            return fail(ISO_EDEVICE, "clearing the branch counters failed");
    return ISO_OK;
}

int iso_debug_read(iso_graph *g, uint64_t counts[8]) {
    if (!g || !counts) return fail(ISO_EINVAL, "NULL argument");
    std::fill(counts, counts + 8, uint64_t(0));
    if (hipSetDevice(g->D.device) != hipSuccess) return fail(ISO_EDEVICE, "hipSetDevice failed");
    for (isodev::SweepCtx *C : {&g->D.main, &g->D.aux}) {
        if (!C->bufs.d_dbg) continue;
        uint64_t v[8];
        if (hipMemcpy(v, C->bufs.d_dbg, sizeof v, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(ISO_EDEVICE, "reading the branch counters failed");
        for (int k = 0; k < 8; ++k) counts[k] += v[k];
    }
    counts[4] += g->resweeps;
    return ISO_OK;
}

int iso_last_query_stats(const iso_graph *g, iso_query_stats *s) {
    if (!g || !s) return fail(ISO_EINVAL, "NULL argument");
    *s = g->last;
    return ISO_OK;
}

int iso_set_tuning(iso_graph *g, const iso_tuning *t) {
    if (!g || !t) return fail(ISO_EINVAL, "NULL argument");
    if (t->lanes_per_launch < 1 || t->lanes_per_launch > isodev::MAX_LANES) return fail(ISO_EINVAL, "lanes_per_launch out of range");
    if (t->block < 64 || t->block > 1024 || t->block % 64) return fail(ISO_EINVAL, "block must be a multiple of 64 in [64, 1024]");
    if (t->cell_lds_kb < 16 || t->cell_lds_kb > 160) return fail(ISO_EINVAL, "cell_lds_kb must be in [16, 160]");
    if (t->use_graph > 1) return fail(ISO_EINVAL, "use_graph must be 0 or 1");
    if (t->cell_stage > 2) return fail(ISO_EINVAL, "cell_stage must be 0, 1 or 2");
    if (t->cell_block != 0 && t->cell_block != 256 && t->cell_block != 512)
        return fail(ISO_EINVAL, "cell_block must be 0, 256 or 512");
    if (t->table_max > isodev::TABLE_MAX) return fail(ISO_EINVAL, "table_max must be at most 16384");
    if (t->stall > 1) return fail(ISO_EINVAL, "stall must be 0 or 1");
    if (t->overlap_cells > 16) return fail(ISO_EINVAL, "overlap_cells must be at most 16");
    if (t->plain_sweep > 1) return fail(ISO_EINVAL, "plain_sweep must be 0 or 1");
    if (t->core_mode != 0 && t->core_mode != 2)
        return fail(ISO_EINVAL, "core_mode must be 0 or 2 (1, a single-launch core sweep with a grid "
                                "barrier, was removed)");
    g->tuning = *t;
    if (t->edge_cap) g->out_cap = std::max<size_t>(16, t->edge_cap);
    return ISO_OK;
}

int iso_get_tuning(const iso_graph *g, iso_tuning *t) {
    if (!g || !t) return fail(ISO_EINVAL, "NULL argument");
    *t = g->tuning;
    return ISO_OK;
}

}  // extern "C"
