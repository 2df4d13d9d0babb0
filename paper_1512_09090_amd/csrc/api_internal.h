// api_internal.h - internals shared by the C ABI (iso_api.cpp) and the serving loop
// (server.cpp): the graph handle, the host upward search, marshalling of queries into a
// device sweep.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <thread>
#include <mutex>
#include <memory>
#include <functional>
#include <condition_variable>
#include <cstdlib>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/iso.h"
#include "device.h"
#include "prep.h"

inline double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Upward CH search (Section 2: forward search on G-up; no stopping criterion, as in
// the first phase of PHAST and of isoPHAST-CP).  In the sweep layout every upward arc
// goes to a strictly smaller position (a higher level, or from a cell's internal
// vertex to the core), so the search space is a DAG in position order: visiting the
// reached vertices from the largest position down finalises each label before it is
// used, which gives exactly the labels of Dijkstra's algorithm on G-up without a
// priority queue.  Reached vertices are kept in a two-level bitmap (words, and a
// summary bit per non-zero word); labels live in a small open-addressing table,
// since the search space is a few thousand vertices.
struct UpwardGraph {
    static constexpr uint32_t INLINE = 4;   // arcs stored in the vertex's own 32-byte slot
    std::vector<uint64_t> inl;   // n * INLINE: head << 32 | length (length INF = empty)
    std::vector<uint32_t> off;   // n + 1: further arcs of each vertex in `more`
    std::vector<uint64_t> more;
    bool dag_ok = true;          // every arc goes to a smaller position
    void build(const iso::Prep &P) {
        inl.assign(size_t(P.n) * INLINE, uint64_t(iso::INF));
        off.assign(size_t(P.n) + 1, 0);
        for (uint32_t u = 0; u < P.n; ++u) {
            uint32_t d = P.up_off[u + 1] - P.up_off[u];
            off[u + 1] = off[u] + (d > INLINE ? d - INLINE : 0);
        }
        more.resize(off[P.n]);
        for (uint32_t u = 0; u < P.n; ++u)
            for (uint32_t e = P.up_off[u], k = 0; e < P.up_off[u + 1]; ++e, ++k) {
                uint64_t a = (uint64_t(P.up_head[e]) << 32) | P.up_w[e];
                if (k < INLINE) inl[size_t(u) * INLINE + k] = a;
                else more[off[u] + k - INLINE] = a;
                if (P.up_head[e] >= u) dag_ok = false;
            }
    }
};

struct UpwardSearch {
    static constexpr uint32_t EMPTY = 0xFFFFFFFFu;
    std::vector<uint32_t> key, val;   // open addressing, power-of-two capacity
    uint32_t mask = 0;
    std::vector<uint32_t> used;       // occupied slots (for clearing)
    std::vector<uint64_t> bits, sum;  // reached positions; summary bit per non-zero word

    void init(uint32_t n) {
        rehash(1u << 14);
        bits.assign((size_t(n) + 63) / 64, 0);
        sum.assign((bits.size() + 63) / 64, 0);
    }
    void rehash(uint32_t cap) {
        std::vector<std::pair<uint32_t, uint32_t>> keep;
        for (uint32_t s : used) keep.push_back({key[s], val[s]});
        key.assign(cap, EMPTY);
        val.assign(cap, iso::INF);
        mask = cap - 1;
        used.clear();
        for (auto &kv : keep) *slot(kv.first) = kv.second;
    }
    static uint32_t hash(uint32_t v) { return (v * 0x9E3779B1u) ^ (v >> 15); }
    uint32_t find(uint32_t v) const {   // label of v, INF if absent
        uint32_t h = hash(v) & mask;
        while (key[h] != EMPTY) {
            if (key[h] == v) return val[h];
            h = (h + 1) & mask;
        }
        return iso::INF;
    }
    uint32_t *slot(uint32_t v) {   // label slot of v (inserted with INF if absent)
        uint32_t h = hash(v) & mask;
        while (key[h] != EMPTY && key[h] != v) h = (h + 1) & mask;
        if (key[h] == EMPTY) {
            key[h] = v;
            used.push_back(h);
        }
        return &val[h];
    }
    void mark(const UpwardGraph &G, uint32_t x) {
        __builtin_prefetch(&G.inl[size_t(x) * UpwardGraph::INLINE]);
        size_t w = x >> 6;
        bits[w] |= 1ull << (x & 63);
        sum[w >> 6] |= 1ull << (w & 63);
    }

    // out: (position, label) pairs sorted by position; returns the number of reached vertices.
    // Vertices at positions below `stop` (the top-of-hierarchy table) are recorded but not
    // expanded: the table covers every path continuing inside that set.
    // With `down` given, stall-on-demand (a standard CH search pruning, Section 2): a vertex u
    // with a downward entry from a reached higher vertex v such that label(v) + length < label(u)
    // is neither recorded nor expanded.  Then d(s, u) < label(u), so u lies on the upward part of
    // no shortest up-down path, and the downward sweep gives u its distance through that entry.
    // label(v) may still fall later (positions are processed bottom-up), which only makes the
    // test more conservative.
    uint32_t run(const UpwardGraph &G, uint32_t src_pos, std::vector<std::pair<uint32_t, uint32_t>> &out,
                 uint32_t stop = 0, const iso::Prep *down = nullptr) {
        for (uint32_t s : used) { key[s] = EMPTY; val[s] = iso::INF; }
        used.clear();
        out.clear();
        *slot(src_pos) = 0;
        mark(G, src_pos);
        uint32_t settled = 0;
        // summary words from the source's down to 0; inside them, words and bits high to low
        for (int64_t si = int64_t(src_pos >> 12); si >= 0; --si) {
            while (sum[si]) {
                int wb = 63 - __builtin_clzll(sum[si]);
                size_t wi = size_t(si) * 64 + wb;
                while (bits[wi]) {
                    int b = 63 - __builtin_clzll(bits[wi]);
                    uint32_t u = uint32_t(wi * 64 + b);
                    bits[wi] &= ~(1ull << b);
                    uint32_t du = *slot(u);
                    ++settled;
                    if (down && du != 0) {
                        bool stalled = false;
                        for (uint32_t e = down->down_off[u]; e < down->down_off[u + 1] && !stalled; ++e) {
                            const uint32_t w = down->down_arc[2 * uint64_t(e) + 1];
                            if (w == iso::INF) continue;   // a dummy entry (reverse arc only)
                            const uint32_t dv = find(down->down_arc[2 * uint64_t(e)] & iso::TAIL_MASK);
                            stalled = dv != iso::INF && iso::sat_add(dv, w) < du;
                        }
                        if (stalled) continue;
                    }
                    out.push_back({u, du});
                    if (u < stop) continue;
                    auto relax = [&](uint64_t a) {
                        uint32_t x = uint32_t(a >> 32);
                        uint32_t nd = iso::sat_add(du, uint32_t(a));
                        if (used.size() * 2 >= key.size()) rehash(uint32_t(key.size()) * 2);
                        uint32_t *d = slot(x);
                        if (nd < *d) *d = nd;
                        mark(G, x);
                    };
                    const uint64_t *il = &G.inl[size_t(u) * UpwardGraph::INLINE];
                    for (uint32_t k = 0; k < UpwardGraph::INLINE && uint32_t(il[k]) != iso::INF; ++k) relax(il[k]);
                    for (uint32_t e = G.off[u]; e < G.off[u + 1]; ++e) relax(G.more[e]);
                }
                sum[si] &= ~(1ull << wb);
            }
        }
        std::reverse(out.begin(), out.end());   // ascending positions
        return settled;
    }
};

// isoPHAST-CD (Section 5): the core graph as out-arcs over core positions: the upward arcs of
// the core and its downward entries turned around (finite lengths only).  Together they are
// the contraction hierarchy of the core graph, which keeps every distance between core
// vertices, so a Dijkstra search on them gives the core distances.
struct CoreGraph {
    std::vector<uint32_t> off;   // n_core + 1
    std::vector<uint64_t> arc;   // head << 32 | length
    void build(const iso::Prep &P) {
        const uint32_t nc = P.n_core;
        off.assign(size_t(nc) + 1, 0);
        for (uint32_t x = 0; x < nc; ++x) off[x + 1] += P.up_off[x + 1] - P.up_off[x];
        for (uint32_t v = 0; v < nc; ++v)
            for (uint32_t e = P.down_off[v]; e < P.down_off[v + 1]; ++e)
                if (P.down_arc[2 * uint64_t(e) + 1] != iso::INF) off[(P.down_arc[2 * uint64_t(e)] & iso::TAIL_MASK) + 1]++;
        for (uint32_t x = 0; x < nc; ++x) off[x + 1] += off[x];
        arc.resize(off[nc]);
        std::vector<uint32_t> fill(off.begin(), off.end() - 1);
        for (uint32_t x = 0; x < nc; ++x)
            for (uint32_t e = P.up_off[x]; e < P.up_off[x + 1]; ++e)
                arc[fill[x]++] = (uint64_t(P.up_head[e]) << 32) | P.up_w[e];
        for (uint32_t v = 0; v < nc; ++v)
            for (uint32_t e = P.down_off[v]; e < P.down_off[v + 1]; ++e) {
                const uint32_t w = P.down_arc[2 * uint64_t(e) + 1];
                if (w == iso::INF) continue;   // a dummy entry (reverse arc only)
                const uint32_t u = P.down_arc[2 * uint64_t(e)] & iso::TAIL_MASK;
                arc[fill[u]++] = (uint64_t(v) << 32) | w;
            }
    }
};

// isoDijkstra on the core graph (stopping criterion of Section 3) from the core vertices an
// upward search reached, with their labels.  Returns the settled vertices (label <= tau, exact)
// as (position, label) pairs; the labels of the others are upper bounds or missing, which the
// query treats as out of range (Section 5).  Labels are stamped per call (no O(n_core) reset).
struct CoreDijkstra {
    std::vector<uint32_t> dist, stamp;
    std::vector<uint8_t> done;
    uint32_t epoch = 0;
    std::vector<std::pair<uint32_t, uint32_t>> heap;   // (label, position), a min-heap
    void run(const CoreGraph &G, const std::vector<std::pair<uint32_t, uint32_t>> &seeds, uint32_t tau,
             std::vector<std::pair<uint32_t, uint32_t>> &out) {
        const size_t nc = G.off.size() - 1;
        if (dist.size() != nc) {
            dist.assign(nc, iso::INF);
            stamp.assign(nc, 0);
            done.assign(nc, 0);
            epoch = 0;
        }
        if (++epoch == 0) {   // wrapped: clear the stamps once
            std::fill(stamp.begin(), stamp.end(), 0u);
            epoch = 1;
        }
        auto label = [&](uint32_t v) { return stamp[v] == epoch ? dist[v] : iso::INF; };
        auto cmp = [](const std::pair<uint32_t, uint32_t> &a, const std::pair<uint32_t, uint32_t> &b) {
            return a.first > b.first;
        };
        heap.clear();
        out.clear();
        for (const auto &sd : seeds)
            if (sd.second < label(sd.first)) {
                dist[sd.first] = sd.second;
                stamp[sd.first] = epoch;
                done[sd.first] = 0;
                heap.push_back({sd.second, sd.first});
            }
        std::make_heap(heap.begin(), heap.end(), cmp);
        while (!heap.empty() && heap.front().first <= tau) {
            std::pop_heap(heap.begin(), heap.end(), cmp);
            const auto [d, u] = heap.back();
            heap.pop_back();
            if (d != dist[u] || done[u]) continue;   // stale entry
            done[u] = 1;
            out.push_back({u, d});
            for (uint32_t e = G.off[u]; e < G.off[u + 1]; ++e) {
                const uint32_t x = uint32_t(G.arc[e] >> 32), nd = iso::sat_add(d, uint32_t(G.arc[e]));
                if (nd < label(x)) {
                    dist[x] = nd;
                    if (stamp[x] != epoch) done[x] = 0;
                    stamp[x] = epoch;
                    heap.push_back({nd, x});
                    std::push_heap(heap.begin(), heap.end(), cmp);
                }
            }
        }
    }
};

// Persistent host worker threads: run(use, f) calls f(w) for w in [0, use) on the pool's
// threads (the caller is worker 0) and returns when every call has returned.  One run at a
// time (a graph is used by one call, or by its server, at a time).
class WorkerPool {
public:
    explicit WorkerPool(int n) : n_(std::max(1, n)) {
        for (int w = 1; w < n_; ++w) th_.emplace_back([this, w] { loop(w); });
    }
    ~WorkerPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    int size() const { return n_; }
    void run(int use, const std::function<void(int)> &f) {
        use = std::max(1, std::min(use, n_));
        if (use > 1) {
            std::lock_guard<std::mutex> lk(mu_);
            job_ = &f;
            want_ = use;
            busy_ = use - 1;
            ++gen_;
        }
        if (use > 1) cv_.notify_all();
        f(0);
        if (use > 1) {
            std::unique_lock<std::mutex> lk(mu_);
            done_.wait(lk, [&] { return busy_ == 0; });
            job_ = nullptr;
        }
    }

private:
    void loop(int w) {
        uint64_t seen = 0;
        for (;;) {
            const std::function<void(int)> *job = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                if (w >= want_) continue;
                job = job_;
            }
            (*job)(w);
            std::lock_guard<std::mutex> lk(mu_);
            if (--busy_ == 0) done_.notify_one();
        }
    }
    int n_;
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_;
    const std::function<void(int)> *job_ = nullptr;
    uint64_t gen_ = 0;
    int want_ = 0, busy_ = 0;
    bool stop_ = false;
};

struct iso_graph {
    iso::Prep P;
    isodev::DevGraph D;
    bool on_device = false;
    int threads = 1;
    std::atomic<bool> busy{false};
    iso_query_stats last{};
    iso_tuning tuning{64, 256, 64, 1, 0, 2, 0, 0, 1, 0, 0, 0};   // defaults (include/iso.h)
    UpwardGraph upg;                // packed upward graph
    std::vector<UpwardSearch> up;   // one workspace per host thread
    std::unique_ptr<WorkerPool> pool;   // runs the upward searches of a sweep
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> up_out;   // one search result buffer per worker
    size_t out_cap = 1 << 20;
    double edges_per_query = 0;      // of the last multi-sweep host-result call (sizes the next result block)
    bool debug = false;              // count rare kernel branches (iso_debug_enable)
    uint64_t resweeps = 0;           // sweeps run again with a larger edge buffer
    uint64_t *vbits_dev = nullptr;   // device bitmap of iso_query_vertices (ceil(n / 64) words)
    std::vector<double> xy;          // vertex coordinates given at load (the polygon output's embedding)
    std::unique_ptr<CoreGraph> coreg;         // isoPHAST-CD: core graph (built on first use)
    std::vector<CoreDijkstra> cdj;            // one workspace per host thread
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> cd_out;   // per worker: settled core labels
    uint32_t *tdist_dev = nullptr;   // device distances of iso_targets_query
    size_t tdist_cap = 0;            // its capacity in words
};

struct iso_targets {
    iso_graph *g = nullptr;
    isodev::TargetSet T;
    double select_ms = 0;
};


// Upward searches of `lanes` queries (up to g->threads host threads) and the device inputs
// of one sweep.  settled (optional, lanes entries) receives the upward search sizes.
void build_run_args(iso_graph *g, const uint32_t *src, const uint32_t *tau, uint32_t lanes, bool plain,
                    bool want_dist, isodev::RunArgs &A, uint32_t *settled, bool core_dijkstra = false);
// Process-wide pool of pinned host blocks for results (device copies into pinned memory run
// at full link speed).  pinned_get returns a block of at least `bytes` (its capacity in cap)
// or nullptr; pinned_put takes a block back and returns false for pointers it does not own.
// iso_free hands every pointer to pinned_put first, then to free().
void *pinned_get(size_t bytes, size_t &cap);
bool pinned_put(void *p);

// An edge array released to the caller, who frees it with iso_free: malloc'd, or a pinned
// pool block.
struct EdgeBuf {
    iso_edge *p = nullptr;
    size_t n = 0;
    bool pinned = false;
    EdgeBuf() = default;
    EdgeBuf(const EdgeBuf &) = delete;
    EdgeBuf &operator=(const EdgeBuf &) = delete;
    EdgeBuf(EdgeBuf &&o) noexcept : p(o.p), n(o.n), pinned(o.pinned) { o.p = nullptr; o.n = 0; }
    EdgeBuf &operator=(EdgeBuf &&o) noexcept {
        if (this != &o) {
            drop();
            p = o.p; n = o.n; pinned = o.pinned;
            o.p = nullptr; o.n = 0;
        }
        return *this;
    }
    ~EdgeBuf() { drop(); }
    void drop() {
        if (p && !(pinned && pinned_put(p))) std::free(p);
        p = nullptr;
    }
    iso_edge *release() { iso_edge *r = p; p = nullptr; n = 0; return r; }
};
// The edges of one sweep ((tail, head) pairs, lane starts) -> one malloc'd array per lane;
// throws std::bad_alloc when host memory runs out.
void split_edges(const uint32_t *pairs, const std::vector<uint32_t> &lane_off, uint32_t lanes,
                 std::vector<EdgeBuf> &out);
int api_fail(int code, const std::string &msg);
