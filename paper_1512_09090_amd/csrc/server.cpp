// server.cpp - serving loop with continuous batching (include/iso.h, iso_server_*).
//
// Two threads per server.  The launcher waits for queued requests and a free sweep
// context, takes up to lanes_cap requests (oldest first), runs their upward searches and
// launches the sweep asynchronously on the context's stream; it then immediately looks
// for the next batch, so upward searches of batch b+1 and the device work of batch b (and
// of other contexts' batches) overlap.  The completer waits for in-flight sweeps in
// launch order, sorts and copies back the edges, hands each request its result and
// returns the context.
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "api_internal.h"

namespace {

struct Request {
    uint32_t source = 0, tau = 0;
    double t_submit = 0, t_launch = 0, t_done = 0;
    uint32_t batch_lanes = 0;
    bool done = false;
    int status = ISO_OK;
    EdgeBuf edges;
};

struct InFlight {
    isodev::SweepCtx *ctx;
    std::vector<uint64_t> tickets;
    isodev::RunArgs args;
};

}  // namespace

struct iso_server {
    iso_graph *g = nullptr;
    iso_server_config cfg{};
    uint32_t lanes_cap = 64;
    size_t ctx_bytes = 0;
    std::vector<std::unique_ptr<isodev::SweepCtx>> ctxs;
    std::vector<isodev::SweepCtx *> free_ctx;
    std::deque<uint64_t> queue;
    std::deque<InFlight> inflight;
    std::unordered_map<uint64_t, Request> reqs;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread launcher, completer;
    uint64_t next_ticket = 1, submitted = 0, completed = 0, sweeps = 0, lanes_total = 0, regrown = 0;
    size_t out_cap = 1 << 20;   // edge-key capacity of a sweep; guarded by mu (grown by the completer)
    bool accepting = false, stopping = false, launcher_done = false, stopped = false;
};

namespace {

void fail_batch(iso_server *s, const std::vector<uint64_t> &tickets, int code) {
    std::lock_guard<std::mutex> lk(s->mu);
    double t = now_ms();
    for (uint64_t tk : tickets) {
        auto it = s->reqs.find(tk);
        if (it == s->reqs.end()) continue;
        it->second.done = true;
        it->second.status = code;
        it->second.t_done = t;
        s->completed++;
    }
    s->cv_done.notify_all();
}

void launcher_loop(iso_server *s) {
    iso_graph *g = s->g;
    hipSetDevice(g->D.device);
    for (;;) {
        std::vector<uint64_t> tickets;
        std::vector<uint32_t> src, tau;
        isodev::SweepCtx *ctx = nullptr;
        size_t cap = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return (s->stopping && s->queue.empty()) || (!s->queue.empty() && !s->free_ctx.empty()); });
            if (s->queue.empty()) break;   // stopping and drained
            ctx = s->free_ctx.back();
            s->free_ctx.pop_back();
            double t = now_ms();
            while (!s->queue.empty() && tickets.size() < s->lanes_cap) {
                uint64_t tk = s->queue.front();
                s->queue.pop_front();
                Request &r = s->reqs[tk];
                r.t_launch = t;
                tickets.push_back(tk);
                src.push_back(r.source);
                tau.push_back(r.tau);
            }
            for (uint64_t tk : tickets) s->reqs[tk].batch_lanes = uint32_t(tickets.size());
            cap = s->out_cap;   // written by the completer when a sweep overflows
        }
        InFlight f;
        f.ctx = ctx;
        f.tickets = tickets;
        build_run_args(g, src.data(), tau.data(), uint32_t(src.size()), s->cfg.mode == ISO_MODE_PLAIN, false,
                       f.args, nullptr, s->cfg.mode == ISO_MODE_CD);
        f.args.out_cap = cap;
        int r = g->D.launch(*ctx, f.args);
        if (r) {
            fail_batch(s, tickets, r);
            std::lock_guard<std::mutex> lk(s->mu);
            s->free_ctx.push_back(ctx);
            s->cv_work.notify_all();
            continue;
        }
        std::lock_guard<std::mutex> lk(s->mu);
        s->inflight.push_back(std::move(f));
        s->sweeps++;
        s->lanes_total += tickets.size();
        s->cv_done.notify_all();
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->launcher_done = true;
    s->cv_done.notify_all();
}

void completer_loop(iso_server *s) {
    iso_graph *g = s->g;
    hipSetDevice(g->D.device);
    for (;;) {
        InFlight f;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_done.wait(lk, [&] { return !s->inflight.empty() || s->launcher_done; });
            if (s->inflight.empty()) break;   // launcher finished and nothing in flight
            f = std::move(s->inflight.front());
            s->inflight.pop_front();
        }
        isodev::RunResult R;
        EdgeBuf batch;   // the sweep's edges, copied from the device into a pinned pool block
        batch.pinned = true;
        R.sink = [&](size_t n) -> uint32_t * {
            size_t cap = 0;
            batch.drop();
            batch.p = (iso_edge *)pinned_get(n * sizeof(iso_edge), cap);
            return reinterpret_cast<uint32_t *>(batch.p);
        };
        int r = g->D.finish(*f.ctx, R);
        for (int attempt = 0; !r && R.overflow && attempt < 8; ++attempt) {
            // grow the edge buffer and sweep again, as long as every context still fits the
            // device budget with the larger buffer (otherwise the batch fails with ISO_ENOMEM)
            size_t cap = 0;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                cap = std::max<size_t>(std::max(s->out_cap, f.args.out_cap * 2),
                                       size_t(R.count) + (size_t(R.count) >> 3));
                const size_t need = g->D.ctx_bytes(s->lanes_cap, cap, size_t(s->lanes_cap) * 4096,
                                                   s->cfg.mode == ISO_MODE_PLAIN && g->tuning.plain_sweep == 0);
                if (s->cfg.device_budget && need * s->ctxs.size() > s->cfg.device_budget) {
                    r = api_fail(ISO_ENOMEM, "the edge buffer this sweep needs exceeds the device budget");
                    break;
                }
                s->out_cap = cap;
                s->ctx_bytes = std::max(s->ctx_bytes, need);
                s->regrown++;
            }
            f.args.out_cap = cap;
            r = g->D.launch(*f.ctx, f.args);
            if (!r) r = g->D.finish(*f.ctx, R);
        }
        if (!r && R.overflow) r = api_fail(ISO_ENOMEM, "edge buffer overflow");
        if (r) {
            fail_batch(s, f.tickets, r);
        } else {
            std::vector<EdgeBuf> per;
            try {
                split_edges(reinterpret_cast<const uint32_t *>(batch.p), R.lane_off, uint32_t(f.tickets.size()),
                            per);
            } catch (const std::bad_alloc &) {
                fail_batch(s, f.tickets, api_fail(ISO_ENOMEM, "out of host memory for the results"));
                std::lock_guard<std::mutex> lk(s->mu);
                s->free_ctx.push_back(f.ctx);
                s->cv_work.notify_all();
                continue;
            }
            std::lock_guard<std::mutex> lk(s->mu);
            double t = now_ms();
            for (size_t j = 0; j < f.tickets.size(); ++j) {
                Request &q = s->reqs[f.tickets[j]];
                q.edges = std::move(per[j]);
                q.done = true;
                q.status = ISO_OK;
                q.t_done = t;
                s->completed++;
            }
            s->cv_done.notify_all();
        }
        std::lock_guard<std::mutex> lk(s->mu);
        s->free_ctx.push_back(f.ctx);
        s->cv_work.notify_all();
    }
}

}  // namespace

extern "C" {

int iso_server_start(iso_graph *g, const iso_server_config *cfg, iso_server **out) {
    if (!g || !cfg || !out) return api_fail(ISO_EINVAL, "NULL argument");
    *out = nullptr;
    if (!g->on_device) return api_fail(ISO_EDEVICE, "graph was loaded without a device");
    if (cfg->mode != ISO_MODE_PLAIN && cfg->mode != ISO_MODE_CELLS && cfg->mode != ISO_MODE_CD)
        return api_fail(ISO_EINVAL, "unknown mode");
    if (cfg->mode != ISO_MODE_PLAIN && g->P.num_cells == 0) return api_fail(ISO_EINVAL, "cells mode needs a partition");
    uint32_t lanes = cfg->max_lanes ? cfg->max_lanes : 64;
    uint32_t inflight = cfg->max_inflight ? cfg->max_inflight : 2;
    if (lanes > isodev::MAX_LANES || inflight > 4) return api_fail(ISO_EINVAL, "max_lanes <= 64, max_inflight <= 4");
    bool f = false;
    if (!g->busy.compare_exchange_strong(f, true)) return api_fail(ISO_EBUSY, "graph handle in use");
    auto *s = new (std::nothrow) iso_server();
    if (!s) {
        g->busy.store(false);
        return api_fail(ISO_ENOMEM, "out of host memory");
    }
    s->g = g;
    s->cfg = *cfg;
    s->cfg.max_lanes = lanes;
    s->cfg.max_inflight = inflight;
    s->out_cap = g->out_cap;
    // admission by device memory: fewer contexts first, then fewer lanes per sweep
    const size_t upward_per_lane = 4096;
    const bool stream = cfg->mode == ISO_MODE_PLAIN && g->tuning.plain_sweep == 0;
    auto need = [&](uint32_t k) { return g->D.ctx_bytes(k, s->out_cap, size_t(k) * upward_per_lane, stream); };
    uint32_t ctxs = inflight;
    if (cfg->device_budget) {
        while (ctxs > 1 && need(lanes) * ctxs > cfg->device_budget) --ctxs;
        while (lanes > 1 && need(lanes) > cfg->device_budget) lanes = (lanes + 1) / 2;
        if (need(lanes) > cfg->device_budget) {
            delete s;
            g->busy.store(false);
            return api_fail(ISO_ENOMEM, "device_budget cannot hold one sweep of one query");
        }
    }
    s->lanes_cap = lanes;
    s->ctx_bytes = need(lanes);
    for (uint32_t i = 0; i < ctxs; ++i) {
        s->ctxs.emplace_back(new isodev::SweepCtx());
        int r = s->ctxs.back()->create(g->D.device);
        if (r) {
            for (auto &c : s->ctxs) c->release();
            delete s;
            g->busy.store(false);
            return r;
        }
        s->free_ctx.push_back(s->ctxs.back().get());
    }
    s->accepting = true;
    s->launcher = std::thread(launcher_loop, s);
    s->completer = std::thread(completer_loop, s);
    *out = s;
    return ISO_OK;
}

int iso_server_submit(iso_server *s, uint32_t source, uint32_t tau, uint64_t *ticket) {
    if (!s || !ticket) return api_fail(ISO_EINVAL, "NULL argument");
    if (source >= s->g->P.n) return api_fail(ISO_EINVAL, "source out of range");
    if (tau > ISO_TAU_MAX) return api_fail(ISO_EINVAL, "tau must be <= 2^32 - 2");
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->accepting) return api_fail(ISO_ESTATE, "server stopped");
    uint64_t tk = s->next_ticket++;
    Request &r = s->reqs[tk];
    r.source = source;
    r.tau = tau;
    r.t_submit = now_ms();
    s->queue.push_back(tk);
    s->submitted++;
    *ticket = tk;
    s->cv_work.notify_one();
    return ISO_OK;
}

int iso_server_wait(iso_server *s, uint64_t ticket, int timeout_ms, iso_edge **edges, size_t *count,
                    iso_request_stats *stats) {
    if (edges) *edges = nullptr;
    if (!s || !edges || !count) return api_fail(ISO_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return api_fail(ISO_EINVAL, "unknown ticket");
    auto ready = [&] { return s->reqs[ticket].done; };
    if (timeout_ms < 0) {
        s->cv_done.wait(lk, ready);
    } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
        return api_fail(ISO_EAGAIN, "not ready");
    }
    Request q = std::move(s->reqs[ticket]);
    s->reqs.erase(ticket);
    lk.unlock();
    if (stats) {
        stats->t_queue_ms = q.t_launch - q.t_submit;
        stats->t_total_ms = q.t_done - q.t_submit;
        stats->batch_lanes = q.batch_lanes;
    }
    if (q.status != ISO_OK) return q.status;
    *count = q.edges.n;
    *edges = q.edges.release();
    return ISO_OK;
}

int iso_server_get_stats(iso_server *s, iso_server_stats *o) {
    if (!s || !o) return api_fail(ISO_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    o->submitted = s->submitted;
    o->completed = s->completed;
    o->sweeps = s->sweeps;
    o->lanes_total = s->lanes_total;
    o->contexts = uint32_t(s->ctxs.size());
    o->lanes_cap = s->lanes_cap;
    o->queue_depth = uint32_t(s->queue.size());
    o->inflight = uint32_t(s->inflight.size());
    o->ctx_bytes = s->ctx_bytes;
    o->regrown = s->regrown;
    return ISO_OK;
}

int iso_server_stop(iso_server *s) {
    if (!s) return api_fail(ISO_EINVAL, "NULL argument");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopped) return ISO_OK;
        s->accepting = false;
        s->stopping = true;
        s->cv_work.notify_all();
    }
    s->launcher.join();
    s->completer.join();
    for (auto &c : s->ctxs) c->release();
    s->ctxs.clear();
    s->free_ctx.clear();
    s->g->out_cap = std::max(s->g->out_cap, s->out_cap);
    s->g->busy.store(false);
    s->stopped = true;
    return ISO_OK;
}

void iso_server_free(iso_server *s) {
    if (!s) return;
    iso_server_stop(s);
    delete s;
}

}  // extern "C"
