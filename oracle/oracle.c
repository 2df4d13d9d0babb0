/*
 * oracle.c - plain, slow, obviously correct CPU reference for isochrone queries.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; it reads the original arc list
 * (original vertex ids) and nothing the GPU path produces.
 *
 * What it computes (Baum, Buchhold, Dibbelt, Wagner: "Fast Computation of
 * Isochrones in Road Networks"):
 *   - Section 2, Dijkstra's algorithm: labels d(.), a priority queue, settle the
 *     minimum, scan its outgoing arcs.
 *   - Section 3, problem statement: v is in range iff d(s,v) <= tau; the output
 *     is the set of arcs (u,v) in E with exactly one endpoint in range
 *     ("isochrone edges").
 *   - Section 3, isoDijkstra: Dijkstra with the stopping criterion "minimum key
 *     exceeds tau", incoming arcs of settled vertices pushed with key infinity,
 *     and a final sweep over the vertices left in the queue.
 *
 * Arithmetic: 64-bit unsigned keys, no clamping, so sums of uint32 weights never
 * overflow for graphs below 2^32 vertices.  "Unreachable" is ORC_INF.
 * Parity status: every exported function is pinned by the CPU test suite
 * (brute-force Bellman-Ford, scipy's Dijkstra, the uniform-grid closed form,
 * the special limits tau = 0 / tau = d(s,v) / tau >= max distance, invariants).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_INF UINT64_MAX

typedef struct {
    uint32_t n;
    uint64_t m;
    /* outgoing arcs grouped by tail, incoming arcs grouped by head (original ids) */
    uint64_t *out_off; uint32_t *out_head; uint32_t *out_w;
    uint64_t *in_off;  uint32_t *in_tail;  uint32_t *in_w;
} orc_graph;

typedef struct { uint64_t key; uint32_t v; } orc_item;

/* per-call scratch; epoch stamps avoid an O(n) reset between queries */
typedef struct {
    uint32_t n;
    uint64_t *dist;       /* valid where stamp == epoch */
    uint32_t *stamp;
    uint32_t *done;       /* settled iff done == epoch */
    uint32_t *mark;       /* auxiliary per-query mark (queued / swept) */
    uint32_t epoch;
    orc_item *heap; uint64_t heap_len, heap_cap;
    uint32_t *order; uint64_t order_len;   /* settled vertices in settle order */
} orc_ws;

/* ------------------------------------------------------------------ graph */

orc_graph *orc_graph_new(uint32_t n, uint64_t m, const uint32_t *tail,
                         const uint32_t *head, const uint32_t *w)
{
    orc_graph *g = calloc(1, sizeof *g);
    if (!g) return NULL;
    g->n = n; g->m = m;
    g->out_off = calloc((size_t)n + 1, sizeof(uint64_t));
    g->in_off  = calloc((size_t)n + 1, sizeof(uint64_t));
    g->out_head = malloc((m ? m : 1) * sizeof(uint32_t));
    g->out_w    = malloc((m ? m : 1) * sizeof(uint32_t));
    g->in_tail  = malloc((m ? m : 1) * sizeof(uint32_t));
    g->in_w     = malloc((m ? m : 1) * sizeof(uint32_t));
    if (!g->out_off || !g->in_off || !g->out_head || !g->out_w || !g->in_tail || !g->in_w)
        return NULL;
    for (uint64_t e = 0; e < m; ++e) {
        g->out_off[tail[e] + 1]++;
        g->in_off[head[e] + 1]++;
    }
    for (uint32_t v = 0; v < n; ++v) {
        g->out_off[v + 1] += g->out_off[v];
        g->in_off[v + 1] += g->in_off[v];
    }
    uint64_t *fo = malloc(((size_t)n + 1) * sizeof(uint64_t));
    uint64_t *fi = malloc(((size_t)n + 1) * sizeof(uint64_t));
    memcpy(fo, g->out_off, ((size_t)n + 1) * sizeof(uint64_t));
    memcpy(fi, g->in_off, ((size_t)n + 1) * sizeof(uint64_t));
    for (uint64_t e = 0; e < m; ++e) {
        uint64_t a = fo[tail[e]]++;
        g->out_head[a] = head[e]; g->out_w[a] = w[e];
        uint64_t b = fi[head[e]]++;
        g->in_tail[b] = tail[e]; g->in_w[b] = w[e];
    }
    free(fo); free(fi);
    return g;
}

void orc_graph_free(orc_graph *g)
{
    if (!g) return;
    free(g->out_off); free(g->out_head); free(g->out_w);
    free(g->in_off); free(g->in_tail); free(g->in_w);
    free(g);
}

/* -------------------------------------------------------------- workspace */

orc_ws *orc_ws_new(uint32_t n)
{
    orc_ws *ws = calloc(1, sizeof *ws);
    if (!ws) return NULL;
    ws->n = n;
    ws->dist = malloc(((size_t)n + 1) * sizeof(uint64_t));
    ws->stamp = calloc((size_t)n + 1, sizeof(uint32_t));
    ws->done = calloc((size_t)n + 1, sizeof(uint32_t));
    ws->mark = calloc((size_t)n + 1, sizeof(uint32_t));
    ws->order = malloc(((size_t)n + 1) * sizeof(uint32_t));
    ws->heap_cap = 1024;
    ws->heap = malloc(ws->heap_cap * sizeof(orc_item));
    return ws;
}

void orc_ws_free(orc_ws *ws)
{
    if (!ws) return;
    free(ws->dist); free(ws->stamp); free(ws->done); free(ws->mark);
    free(ws->order); free(ws->heap); free(ws);
}

static void new_epoch(orc_ws *ws)
{
    ws->epoch++;
    if (ws->epoch == 0) {               /* wrapped: clear stamps once */
        memset(ws->stamp, 0, ((size_t)ws->n + 1) * sizeof(uint32_t));
        memset(ws->done, 0, ((size_t)ws->n + 1) * sizeof(uint32_t));
        memset(ws->mark, 0, ((size_t)ws->n + 1) * sizeof(uint32_t));
        ws->epoch = 1;
    }
    ws->heap_len = 0;
    ws->order_len = 0;
}

static uint64_t get_dist(const orc_ws *ws, uint32_t v)
{
    return ws->stamp[v] == ws->epoch ? ws->dist[v] : ORC_INF;
}

static void set_dist(orc_ws *ws, uint32_t v, uint64_t d)
{
    ws->stamp[v] = ws->epoch;
    ws->dist[v] = d;
}

static int is_settled(const orc_ws *ws, uint32_t v) { return ws->done[v] == ws->epoch; }

/* binary min-heap on key; stale entries are skipped when popped (lazy deletion) */
static void heap_push(orc_ws *ws, uint64_t key, uint32_t v)
{
    if (ws->heap_len == ws->heap_cap) {
        ws->heap_cap *= 2;
        ws->heap = realloc(ws->heap, ws->heap_cap * sizeof(orc_item));
    }
    uint64_t i = ws->heap_len++;
    while (i > 0) {
        uint64_t p = (i - 1) / 2;
        if (ws->heap[p].key <= key) break;
        ws->heap[i] = ws->heap[p];
        i = p;
    }
    ws->heap[i].key = key;
    ws->heap[i].v = v;
}

static orc_item heap_pop(orc_ws *ws)
{
    orc_item top = ws->heap[0];
    orc_item last = ws->heap[--ws->heap_len];
    uint64_t i = 0, len = ws->heap_len;
    for (;;) {
        uint64_t c = 2 * i + 1;
        if (c >= len) break;
        if (c + 1 < len && ws->heap[c + 1].key < ws->heap[c].key) c++;
        if (ws->heap[c].key >= last.key) break;
        ws->heap[i] = ws->heap[c];
        i = c;
    }
    if (len > 0) ws->heap[i] = last;
    return top;
}

/* ---------------------------------------------------- Dijkstra (Section 2) */

/*
 * Dijkstra from s that stops once the minimum key exceeds tau (the stopping
 * criterion of Section 3).  tau = ORC_INF runs to exhaustion.  Afterwards the
 * settled vertices are exactly those with d(s,v) <= tau, and their labels are
 * final.  Returns the number of settled vertices.
 */
static uint64_t bounded_dijkstra(const orc_graph *g, orc_ws *ws, uint32_t s, uint64_t tau)
{
    new_epoch(ws);
    set_dist(ws, s, 0);
    heap_push(ws, 0, s);
    while (ws->heap_len > 0) {
        if (ws->heap[0].key > tau) break;              /* stopping criterion */
        orc_item it = heap_pop(ws);
        uint32_t u = it.v;
        if (is_settled(ws, u) || it.key != get_dist(ws, u)) continue;   /* stale */
        ws->done[u] = ws->epoch;
        ws->order[ws->order_len++] = u;
        for (uint64_t e = g->out_off[u]; e < g->out_off[u + 1]; ++e) {
            uint32_t v = g->out_head[e];
            uint64_t nd = it.key + g->out_w[e];
            if (nd < get_dist(ws, v)) {
                set_dist(ws, v, nd);
                heap_push(ws, nd, v);
            }
        }
    }
    return ws->order_len;
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* sort (tail << 32 | head) keys and drop duplicates (parallel arcs); returns the new count */
static uint64_t sort_unique(uint64_t *keys, uint64_t cnt)
{
    if (cnt == 0) return 0;
    qsort(keys, cnt, sizeof(uint64_t), cmp_u64);
    uint64_t k = 1;
    for (uint64_t i = 1; i < cnt; ++i)
        if (keys[i] != keys[k - 1]) keys[k++] = keys[i];
    return k;
}

static uint64_t *push_key(uint64_t *buf, uint64_t *cnt, uint64_t *cap, uint32_t t, uint32_t h)
{
    if (*cnt == *cap) {
        *cap = *cap ? 2 * *cap : 1024;
        buf = realloc(buf, *cap * sizeof(uint64_t));
    }
    buf[(*cnt)++] = ((uint64_t)t << 32) | h;
    return buf;
}

/*
 * Isochrone query by the plain definition.
 * Distances: bounded Dijkstra.  Output: every arc with exactly one endpoint in
 * range (Section 3), found locally: for each settled (in-range) u, its outgoing
 * arcs to unsettled heads and its incoming arcs from unsettled tails.  A
 * straddling arc has exactly one in-range endpoint, so it is found exactly once
 * (up to parallel arcs, removed by the final sort-unique).
 *
 * dist_out (optional, n entries): d(s,v) for settled v, ORC_INF otherwise.
 * *edges_out: malloc'ed array of (tail << 32 | head) keys, sorted, unique;
 * release with orc_free.  Returns the number of settled vertices.
 */
uint64_t orc_isochrone(const orc_graph *g, orc_ws *ws, uint32_t s, uint64_t tau,
                       uint64_t *dist_out, uint64_t **edges_out, uint64_t *n_edges)
{
    uint64_t settled = bounded_dijkstra(g, ws, s, tau);
    uint64_t *buf = NULL, cnt = 0, cap = 0;
    for (uint64_t i = 0; i < ws->order_len; ++i) {
        uint32_t u = ws->order[i];
        for (uint64_t e = g->out_off[u]; e < g->out_off[u + 1]; ++e)
            if (!is_settled(ws, g->out_head[e]))
                buf = push_key(buf, &cnt, &cap, u, g->out_head[e]);
        for (uint64_t e = g->in_off[u]; e < g->in_off[u + 1]; ++e)
            if (!is_settled(ws, g->in_tail[e]))
                buf = push_key(buf, &cnt, &cap, g->in_tail[e], u);
    }
    *n_edges = sort_unique(buf, cnt);
    *edges_out = buf;
    if (dist_out)
        for (uint32_t v = 0; v < g->n; ++v)
            dist_out[v] = is_settled(ws, v) ? ws->dist[v] : ORC_INF;
    return settled;
}

/*
 * All distances d(s,.) (Dijkstra run to exhaustion).  ORC_INF marks vertices
 * that s cannot reach.  Returns the number of reachable vertices.
 */
uint64_t orc_distances(const orc_graph *g, orc_ws *ws, uint32_t s, uint64_t *dist_out)
{
    uint64_t settled = bounded_dijkstra(g, ws, s, ORC_INF);
    for (uint32_t v = 0; v < g->n; ++v)
        dist_out[v] = is_settled(ws, v) ? ws->dist[v] : ORC_INF;
    return settled;
}

/*
 * The problem statement of Section 3 applied literally to given distances:
 * scan every arc (u,v) and keep it iff exactly one of d(u) <= tau, d(v) <= tau
 * holds.  Output as in orc_isochrone.
 */
void orc_edges_by_definition(const orc_graph *g, const uint64_t *dist, uint64_t tau,
                             uint64_t **edges_out, uint64_t *n_edges)
{
    uint64_t *buf = NULL, cnt = 0, cap = 0;
    for (uint32_t u = 0; u < g->n; ++u) {
        int u_in = dist[u] <= tau;
        for (uint64_t e = g->out_off[u]; e < g->out_off[u + 1]; ++e) {
            int v_in = dist[g->out_head[e]] <= tau;
            if (u_in != v_in) buf = push_key(buf, &cnt, &cap, u, g->out_head[e]);
        }
    }
    *n_edges = sort_unique(buf, cnt);
    *edges_out = buf;
}

/*
 * The vertices in range (Section 3): v with d(s,v) <= tau, i.e. exactly the
 * vertices the bounded Dijkstra settles, in increasing id.  *verts_out:
 * malloc'ed, release with orc_free.  Returns their number.
 */
static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

uint64_t orc_in_range(const orc_graph *g, orc_ws *ws, uint32_t s, uint64_t tau, uint32_t **verts_out)
{
    uint64_t settled = bounded_dijkstra(g, ws, s, tau);
    uint32_t *buf = malloc((settled ? settled : 1) * sizeof(uint32_t));
    for (uint64_t i = 0; i < settled; ++i) buf[i] = ws->order[i];
    qsort(buf, settled, sizeof(uint32_t), cmp_u32);
    *verts_out = buf;
    return settled;
}

/* ------------------------------------------------- isoDijkstra (Section 3) */

/*
 * The paper's basic approach.  Dijkstra with the stopping criterion; when a
 * vertex u is settled its incoming arcs (v,u) are also scanned and every tail v
 * whose label is still infinite is put into the queue with key infinity.  When
 * the search stops, every vertex still in the queue is out of range; each one's
 * incoming arcs from in-range tails and outgoing arcs to in-range heads are
 * reported.  (The text names the incoming side; the outgoing side is what the
 * infinity-key insertions exist for, so both are swept.)
 * Returns the number of settled vertices.
 */
uint64_t orc_iso_dijkstra(const orc_graph *g, orc_ws *ws, uint32_t s, uint64_t tau,
                          uint64_t **edges_out, uint64_t *n_edges)
{
    new_epoch(ws);
    set_dist(ws, s, 0);
    heap_push(ws, 0, s);
    ws->mark[s] = ws->epoch;                        /* mark = "has been queued" */
    /* tau must be below ORC_INF, so key-infinity entries are never settled */
    while (ws->heap_len > 0 && ws->heap[0].key <= tau && ws->heap[0].key != ORC_INF) {
        orc_item it = heap_pop(ws);
        uint32_t u = it.v;
        if (is_settled(ws, u) || it.key != get_dist(ws, u)) continue;
        ws->done[u] = ws->epoch;
        ws->order[ws->order_len++] = u;
        for (uint64_t e = g->out_off[u]; e < g->out_off[u + 1]; ++e) {
            uint32_t v = g->out_head[e];
            uint64_t nd = it.key + g->out_w[e];
            if (nd < get_dist(ws, v)) {
                set_dist(ws, v, nd);
                heap_push(ws, nd, v);
                ws->mark[v] = ws->epoch;
            }
        }
        for (uint64_t e = g->in_off[u]; e < g->in_off[u + 1]; ++e) {
            uint32_t v = g->in_tail[e];
            if (get_dist(ws, v) == ORC_INF && ws->mark[v] != ws->epoch) {
                heap_push(ws, ORC_INF, v);          /* key infinity */
                ws->mark[v] = ws->epoch;
            }
        }
    }
    uint64_t *buf = NULL, cnt = 0, cap = 0;
    /* sweep over the vertices left in the queue (each handled once) */
    for (uint64_t i = 0; i < ws->heap_len; ++i) {
        uint32_t v = ws->heap[i].v;
        if (is_settled(ws, v) || ws->mark[v] != ws->epoch) continue;
        ws->mark[v] = ws->epoch - 1;                /* swept; epoch >= 1 so this differs */
        for (uint64_t e = g->in_off[v]; e < g->in_off[v + 1]; ++e)
            if (is_settled(ws, g->in_tail[e]))
                buf = push_key(buf, &cnt, &cap, g->in_tail[e], v);
        for (uint64_t e = g->out_off[v]; e < g->out_off[v + 1]; ++e)
            if (is_settled(ws, g->out_head[e]))
                buf = push_key(buf, &cnt, &cap, v, g->out_head[e]);
    }
    *n_edges = sort_unique(buf, cnt);
    *edges_out = buf;
    return ws->order_len;
}

/* ---------------------------------------------------------------- polygon */
/*
 * The isochrone polygon (Section 7: traverse the faces of a planar embedding
 * along the border of the region in range, switching to the twin face at every
 * isochrone edge), written out plainly:
 *   - the graph is taken undirected (u and v are neighbours if either arc
 *     exists), each vertex's neighbours ordered counterclockwise by the angle
 *     atan2(dy, dx) of the straight segment to them (ties, which a planar
 *     embedding does not have, by id);
 *   - a boundary dart is an ordered pair (u, v) of neighbours with u in range
 *     and v not;
 *   - from a boundary dart, walk the face on its left (from dart (a, b) the walk
 *     goes on to (b, c), c the neighbour of b next clockwise from a) until a
 *     dart (p, q) leads from out of range into range; the next boundary dart is
 *     its twin (q, p), and the walk goes on in the twin's face;
 *   - these successors form cycles; each cycle is listed from its smallest dart
 *     (by (u, v)), the cycles in the order of their smallest darts.
 * in_range: n bytes, nonzero for vertices in range.  Output: *darts_out holds
 * the darts as (u << 32 | v) in cycle order, *cyc_out the start of every cycle
 * plus the end (ncycles + 1 words); returns the number of darts.  Returns
 * UINT64_MAX if a face walk exceeds every dart of the graph (not planar).
 */
#include <math.h>

typedef struct { uint32_t v; double a; } orc_nb;

static int cmp_nb(const void *x, const void *y)
{
    const orc_nb *p = x, *q = y;
    if (p->a < q->a) return -1;
    if (p->a > q->a) return 1;
    return p->v < q->v ? -1 : (p->v > q->v);
}

/* index of w in the neighbour list of v (present by construction) */
static uint64_t nb_index(const uint64_t *off, const orc_nb *nb, uint32_t v, uint32_t w)
{
    for (uint64_t k = off[v]; k < off[v + 1]; ++k)
        if (nb[k].v == w) return k;
    return UINT64_MAX;
}

uint64_t orc_polygon(const orc_graph *g, const double *xy, const uint8_t *in_range,
                     uint64_t **darts_out, uint64_t **cyc_out, uint64_t *ncyc_out)
{
    uint32_t n = g->n;
    /* undirected neighbour lists: both directions of every arc, self-loops dropped */
    uint64_t *off = calloc((size_t)n + 1, sizeof(uint64_t));
    for (uint32_t u = 0; u < n; ++u)
        for (uint64_t e = g->out_off[u]; e < g->out_off[u + 1]; ++e)
            if (g->out_head[e] != u) { off[u + 1]++; off[g->out_head[e] + 1]++; }
    for (uint32_t v = 0; v < n; ++v) off[v + 1] += off[v];
    orc_nb *nb = malloc((off[n] ? off[n] : 1) * sizeof(orc_nb));
    uint64_t *fill = malloc(((size_t)n + 1) * sizeof(uint64_t));
    memcpy(fill, off, ((size_t)n + 1) * sizeof(uint64_t));
    for (uint32_t u = 0; u < n; ++u)
        for (uint64_t e = g->out_off[u]; e < g->out_off[u + 1]; ++e) {
            uint32_t v = g->out_head[e];
            if (v == u) continue;
            nb[fill[u]++].v = v;
            nb[fill[v]++].v = u;
        }
    /* sort by id, drop duplicates, then sort counterclockwise */
    uint64_t *noff = calloc((size_t)n + 1, sizeof(uint64_t));
    uint64_t w = 0;
    for (uint32_t u = 0; u < n; ++u) {
        uint64_t b = off[u], e = off[u + 1];
        for (uint64_t k = b; k < e; ++k) nb[k].a = (double)nb[k].v;
        qsort(nb + b, e - b, sizeof(orc_nb), cmp_nb);
        uint64_t start = w;
        for (uint64_t k = b; k < e; ++k)
            if (k == b || nb[k].v != nb[k - 1].v) nb[w++] = nb[k];
        for (uint64_t k = start; k < w; ++k) {
            uint32_t v = nb[k].v;
            nb[k].a = atan2(xy[2 * (size_t)v + 1] - xy[2 * (size_t)u + 1], xy[2 * (size_t)v] - xy[2 * (size_t)u]);
        }
        qsort(nb + start, w - start, sizeof(orc_nb), cmp_nb);
        noff[u + 1] = w;
    }
    free(off);
    off = noff;
    /* boundary darts, sorted by (u, v) */
    uint64_t nd = 0;
    for (uint32_t u = 0; u < n; ++u)
        if (in_range[u])
            for (uint64_t k = off[u]; k < off[u + 1]; ++k)
                if (!in_range[nb[k].v]) nd++;
    uint64_t *darts = malloc((nd ? nd : 1) * sizeof(uint64_t));
    uint64_t *next = malloc((nd ? nd : 1) * sizeof(uint64_t));
    uint8_t *seen = calloc(nd ? nd : 1, 1);
    nd = 0;
    for (uint32_t u = 0; u < n; ++u)
        if (in_range[u])
            for (uint64_t k = off[u]; k < off[u + 1]; ++k)
                if (!in_range[nb[k].v]) darts[nd++] = ((uint64_t)u << 32) | nb[k].v;
    qsort(darts, nd, sizeof(uint64_t), cmp_u64);
    uint64_t limit = 2 * off[n] + 2, bad = 0;
    for (uint64_t i = 0; i < nd && !bad; ++i) {
        uint32_t a = (uint32_t)(darts[i] >> 32), b = (uint32_t)darts[i];
        uint64_t steps = 0;
        for (;;) {
            /* from (a, b): c is the neighbour of b next clockwise from a */
            uint64_t ka = nb_index(off, nb, b, a);
            uint64_t kc = ka == off[b] ? off[b + 1] - 1 : ka - 1;
            uint32_t c = nb[kc].v;
            a = b;
            b = c;
            if (!in_range[a] && in_range[b]) break;   /* (a, b) enters the region: its twin leaves it */
            if (++steps > limit) { bad = 1; break; }
        }
        uint64_t key = ((uint64_t)b << 32) | a, lo = 0, hi = nd;   /* twin (b, a) */
        while (lo < hi) {
            uint64_t mid = (lo + hi) / 2;
            if (darts[mid] < key) lo = mid + 1; else hi = mid;
        }
        if (lo == nd || darts[lo] != key) { bad = 1; break; }   /* not a boundary dart: no planar embedding */
        next[i] = lo;
    }
    uint64_t *outd = malloc((nd ? nd : 1) * sizeof(uint64_t));
    uint64_t *cyc = malloc((nd + 1) * sizeof(uint64_t));
    uint64_t no = 0, nc = 0;
    for (uint64_t i = 0; i < nd && !bad; ++i) {
        if (seen[i]) continue;
        cyc[nc++] = no;
        for (uint64_t j = i; !seen[j]; j = next[j]) {   /* i is the smallest dart of its cycle */
            seen[j] = 1;
            outd[no++] = darts[j];
        }
    }
    cyc[nc] = no;
    free(off); free(nb); free(fill); free(darts); free(next); free(seen);
    if (bad) { free(outd); free(cyc); return UINT64_MAX; }
    *darts_out = outd;
    *cyc_out = cyc;
    *ncyc_out = nc;
    return no;
}

void orc_free(void *p) { free(p); }
