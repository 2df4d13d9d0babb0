// prep.cpp - partition, contraction hierarchy, sweep layout, eccentricities.
// See prep.h for what is built and which part of the paper each step follows.
#include "prep.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <thread>
#include <cstdlib>
#include <sched.h>

namespace iso {

// Default thread count: the CPUs this process may run on (affinity mask), capped by a cgroup
// CPU quota when one is set.
int resolve_threads(int t) {
    if (t > 0) return t;
    unsigned h = std::thread::hardware_concurrency();
    int n = h ? int(h) : 1;
    cpu_set_t set;
    if (sched_getaffinity(0, sizeof set, &set) == 0) n = std::max(1, CPU_COUNT(&set));
    if (FILE *f = std::fopen("/sys/fs/cgroup/cpu.max", "r")) {
        char quota[32] = {0};
        long period = 0;
        if (std::fscanf(f, "%31s %ld", quota, &period) == 2 && std::strcmp(quota, "max") != 0 && period > 0) {
            long q = std::atol(quota);
            if (q > 0) n = std::min<long>(n, std::max<long>(1, (q + period - 1) / period));
        }
        std::fclose(f);
    }
    return n;
}

// Run f(i, tid) for i in [0, n) on `threads` threads with dynamic chunking.
template <class F>
static void parallel_for(size_t n, int threads, size_t chunk, F f) {
    if (n == 0) return;
    threads = std::max(1, std::min<int>(threads, int((n + chunk - 1) / chunk)));
    std::atomic<size_t> next{0};
    auto worker = [&](int tid) {
        for (;;) {
            size_t b = next.fetch_add(chunk);
            if (b >= n) break;
            size_t e = std::min(n, b + chunk);
            for (size_t i = b; i < e; ++i) f(i, tid);
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < threads; ++t) pool.emplace_back(worker, t);
    worker(0);
    for (auto &th : pool) th.join();
}

static double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------ arc list

void simplify_arcs(uint32_t n, uint64_t m, const uint32_t *tail, const uint32_t *head,
                   const uint32_t *w, ArcList &out) {
    std::vector<uint64_t> off(uint64_t(n) + 1, 0);
    for (uint64_t e = 0; e < m; ++e) off[tail[e] + 1]++;
    for (uint32_t v = 0; v < n; ++v) off[v + 1] += off[v];
    std::vector<uint64_t> fill(off.begin(), off.end() - 1);
    std::vector<std::pair<uint32_t, uint32_t>> hw(m);
    for (uint64_t e = 0; e < m; ++e) hw[fill[tail[e]]++] = {head[e], w[e]};
    // per tail: sort by (head, weight), keep the first (minimum) of each head, drop self-loops
    std::vector<uint64_t> keep_cnt(n, 0);
    int T = resolve_threads(0);
    parallel_for(n, T, 4096, [&](size_t v, int) {
        auto b = hw.begin() + off[v], e = hw.begin() + off[v + 1];
        std::sort(b, e);
        uint64_t k = 0;
        for (auto it = b; it != e; ++it) {
            if (it->first == v) continue;
            if (k > 0 && (b + (k - 1))->first == it->first) continue;
            *(b + k) = *it;
            ++k;
        }
        keep_cnt[v] = k;
    });
    uint64_t total = 0;
    for (uint32_t v = 0; v < n; ++v) total += keep_cnt[v];
    out.n = n;
    out.tail.resize(total);
    out.head.resize(total);
    out.w.resize(total);
    uint64_t o = 0;
    for (uint32_t v = 0; v < n; ++v) {
        for (uint64_t i = 0; i < keep_cnt[v]; ++i) {
            out.tail[o] = v;
            out.head[o] = hw[off[v] + i].first;
            out.w[o] = hw[off[v] + i].second;
            ++o;
        }
    }
}

// ------------------------------------------------------------ partition

// Recursive coordinate bisection: split along the longer side of the bounding
// box at the size-proportional quantile until the requested cell count.
static void bisect_rec(std::vector<uint32_t> &ids, size_t lo, size_t hi, uint32_t cells,
                       uint32_t first_cell, const double *xy, std::vector<uint32_t> &cell_of,
                       int depth_threads) {
    if (cells <= 1 || hi - lo <= 1) {
        for (size_t i = lo; i < hi; ++i) cell_of[ids[i]] = first_cell;
        return;
    }
    double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
    for (size_t i = lo; i < hi; ++i) {
        double x = xy[2 * size_t(ids[i])], y = xy[2 * size_t(ids[i]) + 1];
        x0 = std::min(x0, x); x1 = std::max(x1, x);
        y0 = std::min(y0, y); y1 = std::max(y1, y);
    }
    int axis = (x1 - x0) >= (y1 - y0) ? 0 : 1;
    uint32_t cl = cells / 2, cr = cells - cl;
    size_t mid = lo + size_t((hi - lo) * uint64_t(cl) / cells);
    std::nth_element(ids.begin() + lo, ids.begin() + mid, ids.begin() + hi,
                     [&](uint32_t a, uint32_t b) {
                         double ka = xy[2 * size_t(a) + axis], kb = xy[2 * size_t(b) + axis];
                         return ka < kb || (ka == kb && a < b);
                     });
    if (depth_threads > 1) {
        std::thread th(bisect_rec, std::ref(ids), lo, mid, cl, first_cell, xy, std::ref(cell_of),
                       depth_threads / 2);
        bisect_rec(ids, mid, hi, cr, first_cell + cl, xy, cell_of, depth_threads - depth_threads / 2);
        th.join();
    } else {
        bisect_rec(ids, lo, mid, cl, first_cell, xy, cell_of, 1);
        bisect_rec(ids, mid, hi, cr, first_cell + cl, xy, cell_of, 1);
    }
}

void partition_bisect(uint32_t n, const double *xy, uint32_t num_cells, std::vector<uint32_t> &cell_of) {
    cell_of.assign(n, 0);
    std::vector<uint32_t> ids(n);
    std::iota(ids.begin(), ids.end(), 0u);
    bisect_rec(ids, 0, n, std::max<uint32_t>(1, num_cells), 0, xy, cell_of, resolve_threads(0));
}

void partition_bfs(const ArcList &g, uint32_t max_cell_size, std::vector<uint32_t> &cell_of,
                   uint32_t &num_cells) {
    uint32_t n = g.n;
    std::vector<uint64_t> off(uint64_t(n) + 1, 0);
    for (size_t e = 0; e < g.tail.size(); ++e) { off[g.tail[e] + 1]++; off[g.head[e] + 1]++; }
    for (uint32_t v = 0; v < n; ++v) off[v + 1] += off[v];
    std::vector<uint32_t> nb(off[n]);
    std::vector<uint64_t> f(off.begin(), off.end() - 1);
    for (size_t e = 0; e < g.tail.size(); ++e) { nb[f[g.tail[e]]++] = g.head[e]; nb[f[g.head[e]]++] = g.tail[e]; }
    cell_of.assign(n, NO_CELL);
    uint32_t c = 0;
    std::vector<uint32_t> queue;
    for (uint32_t s = 0; s < n; ++s) {
        if (cell_of[s] != NO_CELL) continue;
        queue.clear();
        queue.push_back(s);
        cell_of[s] = c;
        // grow in BFS order up to max_cell_size vertices
        uint32_t size = 1;
        for (size_t qi = 0; qi < queue.size(); ++qi) {
            uint32_t v = queue[qi];
            for (uint64_t e = off[v]; e < off[v + 1] && size < max_cell_size; ++e) {
                uint32_t x = nb[e];
                if (cell_of[x] != NO_CELL) continue;
                cell_of[x] = c;
                queue.push_back(x);
                ++size;
            }
        }
        ++c;
    }
    num_cells = c;
}

// ------------------------------------------------------------ contraction

namespace {

constexpr uint32_t ORIG_OUT = 1;   // original arc v -> x
constexpr uint32_t ORIG_IN = 2;    // original arc x -> v

struct Adj {
    uint32_t x;      // neighbour
    uint32_t wout;   // length of v -> x in E u E+ (INF if none)
    uint32_t win;    // length of x -> v in E u E+ (INF if none)
    uint32_t flags;  // ORIG_OUT | ORIG_IN
};

enum : uint8_t { REMAIN = 0, FIXED = 1, CONTRACTING = 2, DONE = 3 };

struct DynGraph {
    std::vector<std::vector<Adj>> adj;
    std::vector<uint32_t> level;
    std::vector<uint8_t> state;
    std::vector<std::atomic<uint8_t>> *locks = nullptr;   // only for multi-threaded contraction
};

struct Witness {
    std::vector<uint32_t> dist, stamp;
    uint32_t epoch = 0;
    std::vector<std::pair<uint32_t, uint32_t>> heap;   // (key, vertex), min-heap via std::*_heap
    void init(size_t n) { dist.assign(n, INF); stamp.assign(n, 0); epoch = 0; }
    void next() {
        if (++epoch == 0) { std::fill(stamp.begin(), stamp.end(), 0u); epoch = 1; }
        heap.clear();
    }
    uint32_t get(uint32_t v) const { return stamp[v] == epoch ? dist[v] : INF; }
    void set(uint32_t v, uint32_t d) { stamp[v] = epoch; dist[v] = d; }
};

// Dijkstra from u over remaining arcs, never entering `avoid` or vertices that are
// contracted / being contracted; stops at key > bound or after `limit` settles.
static void witness_search(const DynGraph &G, Witness &W, uint32_t u, uint32_t avoid, uint32_t bound,
                           uint32_t limit) {
    W.next();
    W.set(u, 0);
    auto cmp = [](const std::pair<uint32_t, uint32_t> &a, const std::pair<uint32_t, uint32_t> &b) {
        return a.first > b.first;
    };
    W.heap.push_back({0, u});
    uint32_t settled = 0;
    while (!W.heap.empty()) {
        std::pop_heap(W.heap.begin(), W.heap.end(), cmp);
        auto [k, x] = W.heap.back();
        W.heap.pop_back();
        if (k != W.get(x)) continue;
        if (k > bound || ++settled > limit) break;
        for (const Adj &a : G.adj[x]) {
            if (a.wout == INF || a.x == avoid) continue;
            uint8_t st = G.state[a.x];
            if (st == CONTRACTING || st == DONE) continue;
            uint32_t nd = sat_add(k, a.wout);
            if (nd < W.get(a.x)) {
                W.set(a.x, nd);
                W.heap.push_back({nd, a.x});
                std::push_heap(W.heap.begin(), W.heap.end(), cmp);
            }
        }
    }
}

struct Shortcut { uint32_t from, to, w; };

// Shortcuts needed to contract v (witness searches with the given settle limit).
static void find_shortcuts(const DynGraph &G, Witness &W, uint32_t v, uint32_t limit,
                           std::vector<Shortcut> &out) {
    out.clear();
    const auto &A = G.adj[v];
    for (const Adj &in : A) {
        if (in.win == INF) continue;
        uint32_t u = in.x;
        uint32_t bound = 0;
        bool any = false;
        for (const Adj &o : A) {
            if (o.wout == INF || o.x == u) continue;
            uint32_t L = sat_add(in.win, o.wout);
            if (L == INF) continue;              // a path of length >= INF reaches nothing
            bound = std::max(bound, L);
            any = true;
        }
        if (!any) continue;
        witness_search(G, W, u, v, bound, limit);
        for (const Adj &o : A) {
            if (o.wout == INF || o.x == u) continue;
            uint32_t L = sat_add(in.win, o.wout);
            if (L == INF) continue;
            if (W.get(o.x) > L) out.push_back({u, o.x, L});
        }
    }
}

static inline void lock(DynGraph &G, uint32_t v) {
    if (!G.locks) return;
    auto &l = (*G.locks)[v];
    uint8_t z = 0;
    while (!l.compare_exchange_weak(z, 1, std::memory_order_acquire)) { z = 0; std::this_thread::yield(); }
}
static inline void unlock(DynGraph &G, uint32_t v) {
    if (G.locks) (*G.locks)[v].store(0, std::memory_order_release);
}

// Add or shorten arc from -> to (both adjacency sides).
static void add_arc(DynGraph &G, uint32_t from, uint32_t to, uint32_t w) {
    lock(G, from);
    {
        auto &A = G.adj[from];
        bool found = false;
        for (Adj &a : A) if (a.x == to) { a.wout = std::min(a.wout, w); found = true; break; }
        if (!found) A.push_back({to, w, INF, 0});
    }
    unlock(G, from);
    lock(G, to);
    {
        auto &A = G.adj[to];
        bool found = false;
        for (Adj &a : A) if (a.x == from) { a.win = std::min(a.win, w); found = true; break; }
        if (!found) A.push_back({from, INF, w, 0});
    }
    unlock(G, to);
}

static void remove_neighbor(DynGraph &G, uint32_t x, uint32_t v, uint32_t v_level) {
    lock(G, x);
    auto &A = G.adj[x];
    for (size_t i = 0; i < A.size(); ++i)
        if (A[i].x == v) { A[i] = A.back(); A.pop_back(); break; }
    G.level[x] = std::max(G.level[x], v_level + 1);
    unlock(G, x);
}

static inline uint64_t mix(uint64_t x) {
    x ^= x >> 33; x *= 0xff51afd7ed558ccdULL; x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL; x ^= x >> 33;
    return x;
}

struct ContractParams {
    uint32_t sim_limit = 60;      // settles per witness search when estimating priorities
    uint32_t limit = 400;         // settles per witness search when contracting
    int threads = 1;
    uint64_t max_quot = 0;        // > 0: vertices whose (1000 * added / removed arcs) exceeds this are not
                                  // contracted; contraction stops when no other vertex is left
};

// Contract every REMAIN vertex of G in rounds of independent sets of local priority
// minima.  on_contract(v, adj_at_contraction) is called once per vertex (possibly
// concurrently); afterwards G.level holds final levels.
template <class OnContract>
static void contract_all(DynGraph &G, const ContractParams &P, OnContract on_contract,
                         uint64_t &shortcut_count, int verbose, const char *tag) {
    size_t n = G.adj.size();
    std::vector<uint64_t> prio(n, 0), quot(n, 0);
    std::vector<uint8_t> dirty(n, 1);
    std::vector<uint32_t> remaining;
    for (uint32_t v = 0; v < n; ++v) if (G.state[v] == REMAIN) remaining.push_back(v);
    int T = std::max(1, P.threads);
    std::vector<Witness> W(T);
    for (auto &w : W) w.init(n);
    std::vector<std::vector<Shortcut>> tmp(T);
    std::vector<uint32_t> contracted_nb(n, 0);
    std::vector<uint8_t> sel(n, 0);
    std::vector<std::vector<Shortcut>> sc_of;   // per selected vertex
    uint64_t added = 0;
    size_t round = 0;
    double t0 = now_s();
    double tp[4] = {0, 0, 0, 0};
    while (!remaining.empty()) {
        double ta = now_s();
        // 1. priorities of vertices whose neighbourhood changed
        parallel_for(remaining.size(), T, 256, [&](size_t i, int tid) {
            uint32_t v = remaining[i];
            if (!dirty[v]) return;
            dirty[v] = 0;
            find_shortcuts(G, W[tid], v, P.sim_limit, tmp[tid]);
            uint64_t removed = 0;
            for (const Adj &a : G.adj[v]) removed += (a.wout != INF) + (a.win != INF);
            uint64_t addq = removed ? (1000ull * tmp[tid].size()) / removed : 1000ull * tmp[tid].size();
            quot[v] = addq;
            prio[v] = 1000ull * G.level[v] + addq + 100ull * contracted_nb[v];
        });
        double tb = now_s();
        // 2. independent set of local minima (ties broken by a hash of the id)
        std::vector<uint32_t> chosen;
        std::mutex mu;
        auto eligible = [&](uint32_t v) { return P.max_quot == 0 || quot[v] <= P.max_quot; };
        parallel_for(remaining.size(), T, 1024, [&](size_t i, int) {
            uint32_t v = remaining[i];
            if (!eligible(v)) { sel[v] = 0; return; }
            uint64_t hv = mix(v);
            for (const Adj &a : G.adj[v]) {
                if (G.state[a.x] != REMAIN || !eligible(a.x)) continue;
                uint64_t hx = mix(a.x);
                if (prio[a.x] < prio[v] || (prio[a.x] == prio[v] && (hx < hv || (hx == hv && a.x < v)))) {
                    sel[v] = 0;
                    return;
                }
            }
            sel[v] = 1;
        });
        for (uint32_t v : remaining) if (sel[v]) { chosen.push_back(v); G.state[v] = CONTRACTING; }
        if (chosen.empty()) break;   // only ineligible vertices are left (bounded contraction)
        double tc = now_s();
        // 3. shortcuts of the chosen vertices (witnesses avoid every vertex being contracted)
        sc_of.assign(chosen.size(), {});
        parallel_for(chosen.size(), T, 16, [&](size_t i, int tid) {
            uint32_t v = chosen[i];
            find_shortcuts(G, W[tid], v, P.limit, sc_of[i]);
            on_contract(v, G.adj[v], G.level[v]);
        });
        double td = now_s();
        // 4. remove the chosen vertices from their neighbours and insert shortcuts
        parallel_for(chosen.size(), T, 16, [&](size_t i, int) {
            uint32_t v = chosen[i];
            for (const Adj &a : G.adj[v]) {
                remove_neighbor(G, a.x, v, G.level[v]);
            }
            for (const Shortcut &s : sc_of[i]) add_arc(G, s.from, s.to, s.w);
        });
        for (size_t i = 0; i < chosen.size(); ++i) {
            uint32_t v = chosen[i];
            added += sc_of[i].size();
            for (const Adj &a : G.adj[v]) { dirty[a.x] = 1; contracted_nb[a.x]++; }
            G.state[v] = DONE;
            G.adj[v].clear();
            G.adj[v].shrink_to_fit();
            sel[v] = 0;
        }
        size_t k = 0;
        for (uint32_t v : remaining) if (G.state[v] == REMAIN) remaining[k++] = v;
        remaining.resize(k);
        ++round;
        double te = now_s();
        tp[0] += tb - ta; tp[1] += tc - tb; tp[2] += td - tc; tp[3] += te - td;
        if (verbose && (round % 20 == 0 || remaining.empty()))
            std::fprintf(stderr, "[prep] %s round %zu: %zu left, %llu shortcuts, %.1fs (prio %.1f sel %.1f sc %.1f apply %.1f)\n", tag, round,
                         remaining.size(), (unsigned long long)added, now_s() - t0, tp[0], tp[1], tp[2], tp[3]);
    }
    shortcut_count += added;
}

}  // namespace

// ------------------------------------------------------------ build

static void build_prep_impl(const ArcList &g, const std::vector<uint32_t> &cell_of_in, uint32_t num_cells,
                            const PrepOptions &opt, Prep &P) {
    double t_start = now_s();
    const uint32_t n = g.n;
    const uint64_t m = g.tail.size();
    const int T = resolve_threads(opt.threads);
    const bool part = !cell_of_in.empty() && num_cells > 0;
    P = Prep();
    P.n = n;
    P.m = m;
    P.num_cells = part ? num_cells : 0;
    P.cell_of = part ? cell_of_in : std::vector<uint32_t>(n, NO_CELL);
    const auto &cell_of = P.cell_of;

    // original graph: out-CSR (arcs are sorted by tail) and in-CSR
    std::vector<uint64_t> out_off(uint64_t(n) + 1, 0), in_off(uint64_t(n) + 1, 0);
    for (uint64_t e = 0; e < m; ++e) { out_off[g.tail[e] + 1]++; in_off[g.head[e] + 1]++; }
    for (uint32_t v = 0; v < n; ++v) { out_off[v + 1] += out_off[v]; in_off[v + 1] += in_off[v]; }
    std::vector<uint32_t> in_tail(m), in_w(m);
    {
        std::vector<uint64_t> f(in_off.begin(), in_off.end() - 1);
        for (uint64_t e = 0; e < m; ++e) { uint64_t k = f[g.head[e]]++; in_tail[k] = g.tail[e]; in_w[k] = g.w[e]; }
    }

    // core = boundary vertices of the partition (every vertex without a partition), plus the
    // internal vertices the bounded cell contraction leaves uncontracted
    std::vector<uint8_t> is_core(n, part ? 0 : 1);
    if (part) {
        parallel_for(n, T, 8192, [&](size_t v, int) {
            for (uint64_t e = out_off[v]; e < out_off[v + 1]; ++e)
                if (cell_of[g.head[e]] != cell_of[v]) { is_core[v] = 1; return; }
            for (uint64_t e = in_off[v]; e < in_off[v + 1]; ++e)
                if (cell_of[in_tail[e]] != cell_of[v]) { is_core[v] = 1; return; }
        });
    }
    const std::vector<uint8_t> is_boundary = is_core;

    // symmetric adjacency entries of the original graph for vertex v restricted by `pred`
    auto orig_adj = [&](uint32_t v, auto pred, auto map, std::vector<Adj> &outv) {
        outv.clear();
        uint64_t a = out_off[v], ae = out_off[v + 1], b = in_off[v], be = in_off[v + 1];
        // both lists are sorted by neighbour id
        while (a < ae || b < be) {
            uint32_t xa = a < ae ? g.head[a] : INF, xb = b < be ? in_tail[b] : INF;
            uint32_t x = std::min(xa, xb);
            Adj r{0, INF, INF, 0};
            if (xa == x) { r.wout = g.w[a]; r.flags |= ORIG_OUT; ++a; }
            if (xb == x) { r.win = in_w[b]; r.flags |= ORIG_IN; ++b; }
            if (pred(x)) { r.x = map(x); outv.push_back(r); }
        }
    };

    // contraction records: adjacency (original ids) of each vertex when it was contracted
    std::vector<std::vector<Adj>> rec(n);
    std::vector<uint32_t> level(n, 0);
    uint64_t shortcuts = 0;

    // ---- phase 1: contract the internal vertices of every cell (cell-induced subgraphs)
    std::vector<uint32_t> cell_ptr, cell_verts;
    std::vector<std::vector<Adj>> core_seed;   // residual adjacency of core vertices (original ids)
    if (part) {
        cell_ptr.assign(num_cells + 1, 0);
        for (uint32_t v = 0; v < n; ++v) cell_ptr[cell_of[v] + 1]++;
        for (uint32_t c = 0; c < num_cells; ++c) cell_ptr[c + 1] += cell_ptr[c];
        cell_verts.resize(n);
        {
            std::vector<uint32_t> f(cell_ptr.begin(), cell_ptr.end() - 1);
            for (uint32_t v = 0; v < n; ++v) cell_verts[f[cell_of[v]]++] = v;
        }
        std::vector<uint32_t> local_id(n);
        for (uint32_t c = 0; c < num_cells; ++c)
            for (uint32_t i = cell_ptr[c]; i < cell_ptr[c + 1]; ++i) local_id[cell_verts[i]] = i - cell_ptr[c];
        core_seed.resize(n);
        std::atomic<uint64_t> sc_total{0};
        std::atomic<uint32_t> cells_done{0};
        double t1 = now_s();
        parallel_for(num_cells, T, 4, [&](size_t c, int) {
            uint32_t b = cell_ptr[c], e = cell_ptr[c + 1], nc = e - b;
            if (nc == 0) return;
            DynGraph G;
            G.adj.resize(nc);
            G.level.assign(nc, 0);
            G.state.assign(nc, REMAIN);
            std::vector<Adj> tmpv;
            for (uint32_t i = 0; i < nc; ++i) {
                uint32_t v = cell_verts[b + i];
                orig_adj(v, [&](uint32_t x) { return cell_of[x] == c; },
                         [&](uint32_t x) { return local_id[x]; }, G.adj[i]);
                if (is_boundary[v]) G.state[i] = FIXED;
            }
            ContractParams cp;
            cp.threads = 1;
            cp.sim_limit = 20;
            cp.limit = 1000;
            cp.max_quot = opt.cell_max_quot;
            uint64_t sc = 0;
            contract_all(
                G, cp,
                [&](uint32_t lv, const std::vector<Adj> &A, uint32_t lvl) {
                    uint32_t v = cell_verts[b + lv];
                    auto &R = rec[v];
                    R = A;
                    for (Adj &a : R) a.x = cell_verts[b + a.x];
                    level[v] = lvl;
                },
                sc, 0, "cell");
            sc_total += sc;
            for (uint32_t i = 0; i < nc; ++i) {
                uint32_t v = cell_verts[b + i];
                if (G.state[i] == REMAIN) is_core[v] = 1;    // left uncontracted: joins the core
                if (!is_core[v]) continue;
                level[v] = G.level[i];
                auto &S = core_seed[v];
                S = G.adj[i];
                for (Adj &a : S) a.x = cell_verts[b + a.x];
            }
            uint32_t d = ++cells_done;
            if (opt.verbose && (d % 2048 == 0 || d == num_cells))
                std::fprintf(stderr, "[prep] cells contracted %u/%u (%.1fs)\n", d, num_cells, now_s() - t1);
        });
        shortcuts += sc_total.load();
    }

    // ---- phase 2: contract the core
    std::vector<uint32_t> core_ids;
    for (uint32_t v = 0; v < n; ++v) if (is_core[v]) core_ids.push_back(v);
    const uint32_t nc = uint32_t(core_ids.size());
    {
        std::vector<uint32_t> cid(n, INF);
        for (uint32_t i = 0; i < nc; ++i) cid[core_ids[i]] = i;
        DynGraph G;
        G.adj.resize(nc);
        G.level.assign(nc, 0);
        G.state.assign(nc, REMAIN);
        std::vector<std::atomic<uint8_t>> locks(nc);
        for (auto &l : locks) l.store(0);
        G.locks = &locks;
        parallel_for(nc, T, 1024, [&](size_t i, int) {
            uint32_t v = core_ids[i];
            G.level[i] = level[v];
            auto &A = G.adj[i];
            if (part) {
                // residual cell adjacency (within-cell arcs and shortcuts between boundary vertices)
                A = core_seed[v];
                for (Adj &a : A) a.x = cid[a.x];
                // cut arcs (original arcs to other cells)
                std::vector<Adj> cut;
                orig_adj(v, [&](uint32_t x) { return cell_of[x] != cell_of[v]; },
                         [&](uint32_t x) { return cid[x]; }, cut);
                A.insert(A.end(), cut.begin(), cut.end());
                core_seed[v].clear();
                core_seed[v].shrink_to_fit();
            } else {
                orig_adj(v, [](uint32_t) { return true; }, [&](uint32_t x) { return cid[x]; }, A);
            }
        });
        ContractParams cp;
        cp.threads = T;
        cp.sim_limit = 10;
        cp.limit = 500;
        contract_all(
            G, cp,
            [&](uint32_t ci, const std::vector<Adj> &A, uint32_t lvl) {
                uint32_t v = core_ids[ci];
                auto &R = rec[v];
                R = A;
                for (Adj &a : R) a.x = core_ids[a.x];
                level[v] = lvl;
            },
            shortcuts, opt.verbose, "core");
    }
    P.shortcuts = shortcuts;

    // ---- layout: core by (level desc, cell, id); then cells, internal by (level desc, id)
    std::vector<uint32_t> core_order = core_ids;
    std::sort(core_order.begin(), core_order.end(), [&](uint32_t a, uint32_t b) {
        if (level[a] != level[b]) return level[a] > level[b];
        if (cell_of[a] != cell_of[b]) return cell_of[a] < cell_of[b];
        return a < b;
    });
    P.n_core = nc;
    P.perm.resize(n);
    P.pos.resize(n);
    std::copy(core_order.begin(), core_order.end(), P.perm.begin());
    P.core_lvl.clear();
    for (uint32_t i = 0; i < nc; ++i)
        if (i == 0 || level[core_order[i]] != level[core_order[i - 1]]) P.core_lvl.push_back(i);
    P.core_lvl.push_back(nc);
    if (part) {
        P.cell_off.assign(num_cells + 1, 0);
        P.cell_lvl_ptr.assign(num_cells + 1, 0);
        uint32_t p = nc;
        std::vector<uint32_t> tmp;
        for (uint32_t c = 0; c < num_cells; ++c) {
            P.cell_off[c] = p;
            P.cell_lvl_ptr[c] = uint32_t(P.cell_lvl.size());
            tmp.clear();
            for (uint32_t i = cell_ptr[c]; i < cell_ptr[c + 1]; ++i)
                if (!is_core[cell_verts[i]]) tmp.push_back(cell_verts[i]);
            std::sort(tmp.begin(), tmp.end(), [&](uint32_t a, uint32_t b) {
                return level[a] != level[b] ? level[a] > level[b] : a < b;
            });
            for (size_t i = 0; i < tmp.size(); ++i) {
                if (i == 0 || level[tmp[i]] != level[tmp[i - 1]]) P.cell_lvl.push_back(p);
                P.perm[p++] = tmp[i];
            }
            P.max_cell_internal = std::max<uint32_t>(P.max_cell_internal, uint32_t(tmp.size()));
            P.max_cell_levels = std::max<uint32_t>(P.max_cell_levels,
                                                   uint32_t(P.cell_lvl.size()) - P.cell_lvl_ptr[c]);
        }
        P.cell_off[num_cells] = p;
        P.cell_lvl_ptr[num_cells] = uint32_t(P.cell_lvl.size());
    }
    for (uint32_t p = 0; p < n; ++p) P.pos[P.perm[p]] = p;

    // ---- downward graph (CSR by head position) and upward graph (CSR by tail position)
    P.down_off.assign(uint64_t(n) + 1, 0);
    P.up_off.assign(uint64_t(n) + 1, 0);
    parallel_for(n, T, 8192, [&](size_t p, int) {
        uint32_t v = P.perm[p], dn = 0, up = 0;
        for (const Adj &a : rec[v]) {
            if (a.win != INF || (a.flags & ORIG_OUT)) ++dn;
            if (a.wout != INF) ++up;
        }
        P.down_off[p + 1] = dn;
        P.up_off[p + 1] = up;
    });
    for (uint32_t p = 0; p < n; ++p) { P.down_off[p + 1] += P.down_off[p]; P.up_off[p + 1] += P.up_off[p]; }
    P.down_arc.resize(2 * uint64_t(P.down_off[n]));
    P.up_head.resize(P.up_off[n]);
    P.up_w.resize(P.up_off[n]);
    parallel_for(n, T, 8192, [&](size_t p, int) {
        uint32_t v = P.perm[p];
        std::vector<std::pair<uint32_t, uint32_t>> dn, up;
        for (const Adj &a : rec[v]) {
            uint32_t tp = P.pos[a.x];
            if (a.win != INF || (a.flags & ORIG_OUT)) {
                uint32_t f = ((a.flags & ORIG_IN) ? FLAG_FWD : 0u) | ((a.flags & ORIG_OUT) ? FLAG_REV : 0u);
                dn.push_back({tp | f, a.win});
            }
            if (a.wout != INF) up.push_back({tp, a.wout});
        }
        std::sort(dn.begin(), dn.end(), [](auto &x, auto &y) { return (x.first & TAIL_MASK) < (y.first & TAIL_MASK); });
        std::sort(up.begin(), up.end());
        uint64_t o = P.down_off[p];
        for (auto &d : dn) { P.down_arc[2 * o] = d.first; P.down_arc[2 * o + 1] = d.second; ++o; }
        uint64_t u = P.up_off[p];
        for (auto &d : up) { P.up_head[u] = d.first; P.up_w[u] = d.second; ++u; }
    });
    rec.clear();
    rec.shrink_to_fit();

    // ---- eccentricities of core vertices within their cell, uncovered cells
    P.core_cell.assign(nc, NO_CELL);
    P.core_ecc.assign(nc, INF);
    P.uncovered.assign(P.num_cells, 0);
    if (part) {
        for (uint32_t i = 0; i < nc; ++i) P.core_cell[i] = cell_of[P.perm[i]];
        std::vector<uint32_t> local_id(n);
        for (uint32_t c = 0; c < num_cells; ++c)
            for (uint32_t i = cell_ptr[c]; i < cell_ptr[c + 1]; ++i) local_id[cell_verts[i]] = i - cell_ptr[c];
        parallel_for(num_cells, T, 8, [&](size_t c, int) {
            uint32_t b = cell_ptr[c], nc_ = cell_ptr[c + 1] - b;
            if (nc_ == 0) return;
            // local out-CSR of the cell-induced subgraph
            std::vector<uint32_t> lo(nc_ + 1, 0), lh, lw;
            for (uint32_t i = 0; i < nc_; ++i) {
                uint32_t v = cell_verts[b + i];
                for (uint64_t e = out_off[v]; e < out_off[v + 1]; ++e)
                    if (cell_of[g.head[e]] == c) { lh.push_back(local_id[g.head[e]]); lw.push_back(g.w[e]); }
                lo[i + 1] = uint32_t(lh.size());
            }
            std::vector<uint64_t> dist(nc_);
            std::vector<uint8_t> covered(nc_, 0);
            std::vector<std::pair<uint64_t, uint32_t>> heap;
            auto cmp = [](const std::pair<uint64_t, uint32_t> &x, const std::pair<uint64_t, uint32_t> &y) {
                return x.first > y.first;
            };
            // ecc for every core vertex; coverage counts only what boundary vertices reach
            for (uint32_t i = 0; i < nc_; ++i) {
                uint32_t v = cell_verts[b + i];
                if (!is_core[v]) continue;
                const bool from_boundary = is_boundary[v];
                std::fill(dist.begin(), dist.end(), UINT64_MAX);
                dist[i] = 0;
                heap.assign(1, {0, i});
                uint64_t ecc = 0;
                while (!heap.empty()) {
                    std::pop_heap(heap.begin(), heap.end(), cmp);
                    auto [k, x] = heap.back();
                    heap.pop_back();
                    if (k != dist[x]) continue;
                    ecc = std::max(ecc, k);
                    if (from_boundary) covered[x] = 1;
                    for (uint32_t e = lo[x]; e < lo[x + 1]; ++e) {
                        uint64_t nd = k + lw[e];
                        if (nd < dist[lh[e]]) { dist[lh[e]] = nd; heap.push_back({nd, lh[e]}); std::push_heap(heap.begin(), heap.end(), cmp); }
                    }
                }
                P.core_ecc[P.pos[v]] = ecc >= INF ? INF : uint32_t(ecc);
            }
            for (uint32_t i = 0; i < nc_; ++i) if (!covered[i]) { P.uncovered[c] = 1; break; }
        });
    }
    P.seconds = now_s() - t_start;
    if (opt.verbose)
        std::fprintf(stderr, "[prep] done: n=%u core=%u cells=%u core_levels=%zu down=%u up=%u shortcuts=%llu (%.1fs)\n",
                     n, nc, P.num_cells, P.core_lvl.size() - 1, P.down_off[n], P.up_off[n],
                     (unsigned long long)P.shortcuts, P.seconds);
}

// Vertex order with locality (breadth-first over the undirected graph, or cell
// by cell and breadth-first inside each cell), so that neighbours are close in
// memory during contraction.  Returns new -> old.
static std::vector<uint32_t> locality_order(const ArcList &g, const std::vector<uint32_t> &cell_of,
                                            uint32_t num_cells) {
    uint32_t n = g.n;
    std::vector<uint64_t> off(uint64_t(n) + 1, 0);
    for (size_t e = 0; e < g.tail.size(); ++e) { off[g.tail[e] + 1]++; off[g.head[e] + 1]++; }
    for (uint32_t v = 0; v < n; ++v) off[v + 1] += off[v];
    std::vector<uint32_t> nb(off[n]);
    {
        std::vector<uint64_t> f(off.begin(), off.end() - 1);
        for (size_t e = 0; e < g.tail.size(); ++e) { nb[f[g.tail[e]]++] = g.head[e]; nb[f[g.head[e]]++] = g.tail[e]; }
    }
    std::vector<uint32_t> order;
    order.reserve(n);
    std::vector<uint8_t> seen(n, 0);
    auto bfs_from = [&](uint32_t s, auto same) {
        size_t q = order.size();
        order.push_back(s);
        seen[s] = 1;
        for (; q < order.size(); ++q) {
            uint32_t v = order[q];
            for (uint64_t e = off[v]; e < off[v + 1]; ++e) {
                uint32_t x = nb[e];
                if (!seen[x] && same(x, v)) { seen[x] = 1; order.push_back(x); }
            }
        }
    };
    if (!cell_of.empty() && num_cells > 0) {
        std::vector<uint32_t> cptr(num_cells + 1, 0), cv(n);
        for (uint32_t v = 0; v < n; ++v) cptr[cell_of[v] + 1]++;
        for (uint32_t c = 0; c < num_cells; ++c) cptr[c + 1] += cptr[c];
        {
            std::vector<uint32_t> f(cptr.begin(), cptr.end() - 1);
            for (uint32_t v = 0; v < n; ++v) cv[f[cell_of[v]]++] = v;
        }
        for (uint32_t c = 0; c < num_cells; ++c)
            for (uint32_t i = cptr[c]; i < cptr[c + 1]; ++i)
                if (!seen[cv[i]]) bfs_from(cv[i], [&](uint32_t x, uint32_t v) { return cell_of[x] == cell_of[v]; });
    } else {
        for (uint32_t v = 0; v < n; ++v)
            if (!seen[v]) bfs_from(v, [](uint32_t, uint32_t) { return true; });
    }
    return order;
}

void build_prep(const ArcList &g, const std::vector<uint32_t> &cell_of, uint32_t num_cells,
                const PrepOptions &opt, Prep &P) {
    const uint32_t n = g.n;
    std::vector<uint32_t> n2o = locality_order(g, cell_of, num_cells);
    std::vector<uint32_t> o2n(n);
    for (uint32_t i = 0; i < n; ++i) o2n[n2o[i]] = i;
    ArcList h;
    {
        std::vector<uint32_t> tt(g.tail.size()), hh(g.tail.size());
        for (size_t e = 0; e < g.tail.size(); ++e) { tt[e] = o2n[g.tail[e]]; hh[e] = o2n[g.head[e]]; }
        simplify_arcs(n, tt.size(), tt.data(), hh.data(), g.w.data(), h);   // re-sorts by the new ids
    }
    std::vector<uint32_t> c2;
    if (!cell_of.empty()) {
        c2.resize(n);
        for (uint32_t i = 0; i < n; ++i) c2[i] = cell_of[n2o[i]];
    }
    build_prep_impl(h, c2, num_cells, opt, P);
    for (uint32_t p = 0; p < n; ++p) P.perm[p] = n2o[P.perm[p]];
    for (uint32_t p = 0; p < n; ++p) P.pos[P.perm[p]] = p;
    P.cell_of = cell_of.empty() ? std::vector<uint32_t>(n, NO_CELL) : cell_of;
}

// ------------------------------------------------------------ file I/O

namespace {
constexpr uint64_t MAGIC = 0x31504552504F5349ULL;   // "ISOPREP1"
constexpr uint32_t VERSION = 1;

struct Fnv {
    uint64_t h = 1469598103934665603ULL;
    void add(const void *p, size_t n) {
        const uint8_t *b = static_cast<const uint8_t *>(p);
        for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ULL; }
    }
};

template <class T> void put_vec(FILE *f, Fnv &h, const std::vector<T> &v) {
    uint64_t k = v.size();
    std::fwrite(&k, 8, 1, f);
    h.add(&k, 8);
    if (k) { std::fwrite(v.data(), sizeof(T), k, f); h.add(v.data(), sizeof(T) * k); }
}
template <class T> bool get_vec(FILE *f, Fnv &h, std::vector<T> &v) {
    uint64_t k;
    if (std::fread(&k, 8, 1, f) != 1) return false;
    h.add(&k, 8);
    if (k > (uint64_t(1) << 36)) return false;
    v.resize(k);
    if (k && std::fread(v.data(), sizeof(T), k, f) != k) return false;
    if (k) h.add(v.data(), sizeof(T) * k);
    return true;
}
}  // namespace

uint64_t hash_input(const ArcList &g, const std::vector<uint32_t> &cell_of, uint32_t num_cells) {
    Fnv h;
    h.add(&g.n, 4);
    uint64_t m = g.tail.size();
    h.add(&m, 8);
    // sample-free full hash of the arrays (linear in m, cheap next to preprocessing)
    if (m) { h.add(g.tail.data(), 4 * m); h.add(g.head.data(), 4 * m); h.add(g.w.data(), 4 * m); }
    h.add(&num_cells, 4);
    if (!cell_of.empty()) h.add(cell_of.data(), 4 * cell_of.size());
    return h.h;
}

bool save_prep(const std::string &path, const Prep &p, uint64_t input_hash) {
    std::string tmp = path + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    Fnv h;
    std::fwrite(&MAGIC, 8, 1, f);
    std::fwrite(&VERSION, 4, 1, f);
    std::fwrite(&input_hash, 8, 1, f);
    uint32_t hdr[6] = {p.n, p.n_core, p.num_cells, p.max_cell_internal, p.max_cell_levels, 0};
    std::fwrite(hdr, 4, 6, f);
    std::fwrite(&p.m, 8, 1, f);
    std::fwrite(&p.shortcuts, 8, 1, f);
    h.add(hdr, sizeof hdr);
    put_vec(f, h, p.perm); put_vec(f, h, p.pos); put_vec(f, h, p.cell_of);
    put_vec(f, h, p.down_off); put_vec(f, h, p.down_arc);
    put_vec(f, h, p.up_off); put_vec(f, h, p.up_head); put_vec(f, h, p.up_w);
    put_vec(f, h, p.core_lvl); put_vec(f, h, p.cell_off); put_vec(f, h, p.cell_lvl_ptr);
    put_vec(f, h, p.cell_lvl); put_vec(f, h, p.core_cell); put_vec(f, h, p.core_ecc);
    put_vec(f, h, p.uncovered);
    std::fwrite(&h.h, 8, 1, f);
    bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path.c_str()) == 0;
}

LoadStatus load_prep(const std::string &path, Prep &p, uint64_t input_hash) {
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) return LOAD_MISSING;
    Fnv h;
    uint64_t magic = 0, ih = 0, stored = 0;
    uint32_t ver = 0, hdr[6];
    bool ok = std::fread(&magic, 8, 1, f) == 1 && magic == MAGIC && std::fread(&ver, 4, 1, f) == 1 &&
              ver == VERSION && std::fread(&ih, 8, 1, f) == 1;
    if (ok && ih != input_hash) {
        std::fclose(f);
        return LOAD_OTHER_INPUT;
    }
    ok = ok && std::fread(hdr, 4, 6, f) == 6 && std::fread(&p.m, 8, 1, f) == 1 &&
         std::fread(&p.shortcuts, 8, 1, f) == 1;
    if (ok) {
        h.add(hdr, sizeof hdr);
        p.n = hdr[0]; p.n_core = hdr[1]; p.num_cells = hdr[2]; p.max_cell_internal = hdr[3]; p.max_cell_levels = hdr[4];
        ok = get_vec(f, h, p.perm) && get_vec(f, h, p.pos) && get_vec(f, h, p.cell_of) &&
             get_vec(f, h, p.down_off) && get_vec(f, h, p.down_arc) && get_vec(f, h, p.up_off) &&
             get_vec(f, h, p.up_head) && get_vec(f, h, p.up_w) && get_vec(f, h, p.core_lvl) &&
             get_vec(f, h, p.cell_off) && get_vec(f, h, p.cell_lvl_ptr) && get_vec(f, h, p.cell_lvl) &&
             get_vec(f, h, p.core_cell) && get_vec(f, h, p.core_ecc) && get_vec(f, h, p.uncovered) &&
             std::fread(&stored, 8, 1, f) == 1 && stored == h.h;
    }
    std::fclose(f);
    if (ok) {
        // structural sanity so that a well-formed but inconsistent file cannot drive the kernels out of bounds
        ok = p.perm.size() == p.n && p.pos.size() == p.n && p.down_off.size() == uint64_t(p.n) + 1 &&
             p.up_off.size() == uint64_t(p.n) + 1 && p.down_arc.size() == 2 * uint64_t(p.down_off[p.n]) &&
             p.up_head.size() == p.up_off[p.n] && p.core_cell.size() == p.n_core &&
             p.core_ecc.size() == p.n_core && !p.core_lvl.empty() && p.core_lvl.back() == p.n_core &&
             p.uncovered.size() == p.num_cells &&
             (p.num_cells == 0 || (p.cell_off.size() == p.num_cells + 1 && p.cell_off.back() == p.n &&
                                   p.cell_lvl_ptr.size() == p.num_cells + 1));
        // every index the kernels derive from the file must stay inside its array
        for (uint32_t v = 0; ok && v < p.n; ++v) ok = p.down_off[v] <= p.down_off[v + 1];
        for (size_t i = 0; ok && i + 1 < p.core_lvl.size(); ++i) ok = p.core_lvl[i] < p.core_lvl[i + 1];
        if (ok && p.num_cells) {
            ok = p.cell_off[0] == p.n_core;
            for (uint32_t c = 0; ok && c < p.num_cells; ++c)
                ok = p.cell_off[c] <= p.cell_off[c + 1] && p.cell_lvl_ptr[c] <= p.cell_lvl_ptr[c + 1] &&
                     p.cell_lvl_ptr[c + 1] <= p.cell_lvl.size() &&
                     p.cell_off[c + 1] - p.cell_off[c] <= p.max_cell_internal;
            for (uint32_t c = 0; ok && c < p.num_cells; ++c)
                for (uint32_t l = p.cell_lvl_ptr[c]; ok && l < p.cell_lvl_ptr[c + 1]; ++l)
                    ok = p.cell_lvl[l] >= p.cell_off[c] && p.cell_lvl[l] < p.cell_off[c + 1];
            for (uint32_t i = 0; ok && i < p.n_core; ++i) ok = p.core_cell[i] < p.num_cells;
        } else if (ok) {
            ok = p.n_core == p.n;
        }
        for (uint32_t c = 0; ok && c < p.num_cells; ++c)
            for (uint32_t v = p.cell_off[c]; ok && v < p.cell_off[c + 1]; ++v)
                for (uint32_t e = p.down_off[v]; ok && e < p.down_off[v + 1]; ++e) {
                    uint32_t t = p.down_arc[2 * uint64_t(e)] & TAIL_MASK;
                    ok = t < p.n_core || (t >= p.cell_off[c] && t < v);
                }
        for (uint32_t v = 0; ok && v < p.n_core; ++v)
            for (uint32_t e = p.down_off[v]; ok && e < p.down_off[v + 1]; ++e)
                ok = (p.down_arc[2 * uint64_t(e)] & TAIL_MASK) < v;
        for (uint32_t v = 0; ok && v < p.n; ++v)
            for (uint32_t e = p.up_off[v]; ok && e < p.up_off[v + 1]; ++e) ok = p.up_head[e] < v;
        for (uint32_t v = 0; ok && v < p.n; ++v) ok = p.perm[v] < p.n && p.pos[p.perm[v]] == v;
    }
    return ok ? LOAD_OK : LOAD_CORRUPT;
}

}  // namespace iso
