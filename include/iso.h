/*
 * iso.h - C ABI of the MI355X isochrone library (libiso.so).
 *
 * Operation (Baum, Buchhold, Dibbelt, Wagner, "Fast Computation of Isochrones
 * in Road Networks"):
 *   Section 3 (problem statement): given a directed graph G = (V, E) with
 *   non-negative arc lengths, a source s and a limit tau, a vertex v is in
 *   range iff d(s, v) <= tau; the answer is the set of isochrone edges, the
 *   arcs (u, v) in E with exactly one endpoint in range.
 *   Section 2 (CH, PHAST) and Section 5 (isoPHAST): the library answers it with
 *   an upward contraction-hierarchy search from s followed by a level-ordered
 *   downward sweep over the hierarchy - over every vertex (ISO_MODE_PLAIN) or
 *   over the core and the active cells of a single-level partition only
 *   (ISO_MODE_CELLS, the isoPHAST-CP query with the relaxed cell-flag rule
 *   that Section 5 gives for parallel queries) - with isochrone edges
 *   extracted during the sweep.
 *
 * Arithmetic is exact uint32: weights are in [0, 2^32 - 2]; ISO_INF =
 * 2^32 - 1 marks "unreachable"; path lengths saturate at ISO_INF, so a
 * reported distance is min(d(s, v), ISO_INF); tau must be <= 2^32 - 2, so
 * saturation never changes which vertices are in range.
 *
 * Conventions for every entry point:
 *   - Return value: ISO_OK (0) or a negative iso_status.  No call throws or
 *     aborts across the ABI.  On error nothing is written to outputs except
 *     that *edges is set to NULL; the graph handle stays usable.
 *     iso_last_error() gives a thread-local message for the last failure.
 *   - Vertex ids are the caller's original ids 0..n-1.
 *   - Pointers named h_* / plain arrays are host memory; the library never
 *     keeps a caller pointer after a call returns (inputs are copied).
 *   - Arrays returned through iso_edge** are allocated by the library (host
 *     memory) and released with iso_free().
 *   - One iso_graph may be used by one thread at a time (ISO_EBUSY if a call
 *     overlaps another on the same handle); distinct handles are independent.
 */
#ifndef ISO_H
#define ISO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ISO_INF 0xFFFFFFFFu
#define ISO_TAU_MAX 0xFFFFFFFEu

typedef enum {
    ISO_OK = 0,
    ISO_EINVAL = -1,    /* bad argument: NULL pointer, source >= n, tau > ISO_TAU_MAX, weight == ISO_INF, ... */
    ISO_ENOMEM = -2,    /* host or device allocation failed, or a configured memory budget was exceeded */
    ISO_EDEVICE = -3,   /* a HIP runtime call or kernel launch failed */
    ISO_EFORMAT = -4,   /* preprocessed file missing fields, wrong version or checksum mismatch */
    ISO_EBUSY = -6,     /* the handle is in use by another call */
    ISO_ESTATE = -7,    /* call not valid in the current state (e.g. server stopped) */
    ISO_EAGAIN = -8,    /* result not ready within the given timeout */
    ISO_ESPACE = -9     /* a caller-supplied output buffer is too small; the size needed is returned */
} iso_status;

typedef enum {
    ISO_MODE_PLAIN = 0, /* sweep every vertex (PHAST one-to-all, Section 2) */
    ISO_MODE_CELLS = 1, /* sweep the core, then the active cells only (isoPHAST-CP, Section 5) */
    ISO_MODE_CD = 2     /* isoPHAST-CD (Section 5): the core labels come from an isoDijkstra search on
                           the host over the core graph, stopped at tau, instead of a sweep of the
                           core; the active cells and their sweeps are those of ISO_MODE_CELLS, and so
                           is the answer.  Needs a partition.  Suited to small limits: its cost grows
                           with the core vertices in range, the core sweep's with the whole core.
                           Not for iso_query_distances (core labels above tau are left unset). */
} iso_mode;

typedef struct iso_graph iso_graph;

/* An isochrone edge: an arc (tail, head) of the input graph, original ids. */
typedef struct {
    uint32_t tail;
    uint32_t head;
} iso_edge;

/*
 * Input description for iso_load_graph.  All arrays are caller-owned host
 * memory and are copied; self-loops are dropped and parallel arcs merged to
 * their minimum weight (the answer is keyed on (tail, head), Section 3).
 */
typedef struct {
    uint32_t n;                 /* |V| (>= 1, < 2^30: a downward entry holds its tail's sweep position in
                                   30 bits beside two flag bits) */
    uint64_t m;                 /* |E| (number of entries in tail/head/weight) */
    const uint32_t *tail;       /* m tails, < n */
    const uint32_t *head;       /* m heads, < n */
    const uint32_t *weight;     /* m lengths, each <= 2^32 - 2 */
    const double *xy;           /* optional, 2n coordinates (x0, y0, x1, y1, ...): the partitioner's input
                                   (with num_cells and no cell_of) and the embedding of the polygon output
                                   (copied and kept with the graph) */
    const uint32_t *cell_of;    /* optional explicit single-level partition: a cell id < num_cells per vertex */
    uint32_t num_cells;         /* cells of the single-level partition (Section 5), at most 2^24; 0 = no
                                   partition: the hierarchy is a plain CH and only ISO_MODE_PLAIN is
                                   available */
    uint32_t max_cell_size;     /* upper bound on vertices per cell (0 = 2048); at most 4096 */
    const char *prep_path;      /* optional: if the file exists and matches the input it is loaded instead
                                   of preprocessing; otherwise the preprocessed data is written there */
    int device;                 /* HIP device ordinal; -1 = host-only preprocessing (queries fail with ISO_EDEVICE) */
    int threads;                /* host threads for preprocessing and upward searches (0 = the CPUs the
                                   process may run on, capped by a cgroup CPU quota) */
    int verbose;                /* 1 = progress lines on stderr during preprocessing */
} iso_graph_desc;

/* Sizes of a loaded graph (for reporting and tests). */
typedef struct {
    uint32_t n, n_core, num_cells, core_levels, max_cell_levels, max_cell_internal;
    uint64_t m;                 /* arcs after merging parallel arcs and dropping self-loops */
    uint64_t down_arcs;         /* entries of the downward graph incl. dummy entries (Section 5) */
    uint64_t up_arcs;           /* arcs of the upward graph */
    uint64_t shortcuts;         /* arcs added by contraction */
    uint64_t device_bytes;      /* resident device memory of the graph */
    double prep_seconds;        /* partition + contraction + layout (0 when loaded from a file) */
    uint32_t host_threads;      /* host threads for preprocessing; the upward searches use up to 64 */
    uint32_t top_table;         /* core positions in the top distance table (TX) */
} iso_graph_info;

/* Per-call counters of the last query on a handle (phase times in ms). */
typedef struct {
    uint32_t lanes;             /* queries in the call */
    uint32_t active_cells;      /* summed over lanes (cells swept) */
    uint64_t swept_vertices;    /* vertices whose label was computed, summed over lanes */
    uint64_t edges;             /* isochrone edges returned, summed over lanes */
    uint64_t upward_settled;    /* vertices settled by the upward searches, summed over lanes */
    double t_upward_ms;         /* host upward searches and staging of the device inputs */
    double t_device_ms;         /* device sweep, waited for on the host */
    double t_sort_ms;           /* device sort and decode of the edges, copy to host memory */
    double t_total_ms;
} iso_query_stats;

/* Preprocess (or load) a graph and make it resident on the device. */
int iso_load_graph(const iso_graph_desc *desc, iso_graph **out);
void iso_free_graph(iso_graph *g);
int iso_graph_get_info(const iso_graph *g, iso_graph_info *info);

/*
 * One isochrone query (Section 3).  *edges receives count arcs sorted by
 * (tail, head) without duplicates; release with iso_free.  mode selects the
 * full sweep, the cell-restricted sweep or the core search (iso_mode); all
 * return the same set.
 */
int iso_query(iso_graph *g, uint32_t source, uint32_t tau, int mode,
              iso_edge **edges, size_t *count);

/*
 * k queries in one call, answered by one sweep over the hierarchy with k
 * distance labels per vertex.  offsets (caller-allocated, k + 1 entries)
 * receives the start of each query's edges in *edges; query j's result is
 * bit-identical to iso_query(sources[j], taus[j]).
 */
int iso_query_batch(iso_graph *g, size_t k, const uint32_t *sources, const uint32_t *taus,
                    int mode, iso_edge **edges, size_t *offsets);

/*
 * iso_query_batch with the result left in device memory (Section 3's edge set
 * per query, nothing copied to the host).  sources and taus are host arrays
 * (the upward searches run on the host).  pairs (capacity cap pairs) and
 * offsets (k + 1 words) are caller-owned device memory on the graph's device,
 * e.g. PyTorch allocations; each must lie inside one device allocation, else
 * ISO_EINVAL before any work.  On ISO_OK, query j's edges are the (tail, head)
 * pairs pairs[2 * offsets[j] ...] up to offsets[j + 1], sorted by (tail, head),
 * bit-identical to iso_query_batch, and *total = offsets[k].  If they do not
 * fit, the call returns ISO_ESPACE with *total set to the exact number needed
 * and the contents of pairs and offsets unspecified.  stream (a hipStream_t,
 * NULL = the null stream) is the caller's stream: work queued on it before the
 * call (e.g. the allocation or a previous use of the buffers) completes before
 * the library writes them.  The call returns after its device writes are
 * complete, so the buffers can be used on any stream.  At most 2^32 - 2 edges
 * per call.
 */
int iso_query_batch_device(iso_graph *g, size_t k, const uint32_t *sources, const uint32_t *taus,
                           int mode, uint32_t *pairs, uint64_t cap, uint32_t *offsets,
                           uint64_t *total, void *stream);

/*
 * iso_query_batch_device for callers that cannot allocate memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same arguments, checks, results
 * and errors, but the call makes no device or pinned-host allocation (no hipMalloc,
 * hipHostMalloc, hipFree, and no allocating library routine).  Its device buffers are carved
 * from a static scratch array of 64 MiB that every GPU the library runs on holds until the
 * process ends (the stream, events and a 4 MiB pinned staging block of this path are made when
 * the graph is loaded); host-side bookkeeping still uses the C++ heap.  The queries run one
 * sweep of up to lanes_per_launch (iso_tuning) at a time.  A sweep whose buffers (for k lanes
 * about n * 4 + n_core * k * 4 + n_core * 16 + num_cells * 268 bytes) or isochrone edges (16
 * bytes each plus the sort's temporary storage) do not fit the scratch fails with ISO_ENOMEM
 * and a message; use fewer queries per sweep.  Calls that overlap on one GPU share its scratch
 * and race: the caller must not run two of them at once on the same device, even on different
 * graphs.
 */
int iso_query_batch_device_noalloc(iso_graph *g, size_t k, const uint32_t *sources, const uint32_t *taus,
                                   int mode, uint32_t *pairs, uint64_t cap, uint32_t *offsets,
                                   uint64_t *total, void *stream);

/*
 * The other output that Section 3 says every approach can serve: the set of
 * vertices in range, d(s, v) <= tau, instead of the isochrone edges.  In
 * ISO_MODE_CELLS the internal vertices of a cell that is not swept for a
 * query are in range exactly when one of the cell's core vertices is (the
 * flag rule of Section 5 then guarantees d(u) + ecc(u) <= tau for all of
 * them), so they are output without being swept.
 *
 * iso_query_batch_vertices_device: k (1..64) queries in one sweep.  bits is
 * caller-owned device memory on the graph's device (e.g. a torch tensor)
 * holding k rows of W = ceil(n / 64) words, checked to lie inside one device
 * allocation (ISO_EINVAL before any work otherwise); bit (v mod 64) of word
 * bits[j * W + v / 64] is set iff original vertex v is in range of query j,
 * and every bit of the k rows is written.  stream as in
 * iso_query_batch_device; the call returns after the writes are complete.
 */
int iso_query_batch_vertices_device(iso_graph *g, size_t k, const uint32_t *sources,
                                    const uint32_t *taus, int mode, uint64_t *bits, void *stream);

/* The vertices in range of one query as sorted original ids (library-allocated,
 * release with iso_free); *count of them. */
int iso_query_vertices(iso_graph *g, uint32_t source, uint32_t tau, int mode,
                       uint32_t **vertices, size_t *count);

/*
 * Isochrone polygons (Section 7: the region in range outlined by traversing the faces of a
 * planar embedding, starting from the isochrone edges).  The embedding comes from the vertex
 * coordinates given at load (desc.xy; ISO_ESTATE without them): every pair of vertices
 * joined by an arc, in either direction, is one straight segment, and the neighbours of a
 * vertex are ordered counterclockwise by the angle atan2(dy, dx) of their segments (equal
 * angles by neighbour id).  A boundary dart is an ordered neighbour pair (u, v) with u in
 * range and v not (one per undirected isochrone edge).  From a boundary dart the face on its
 * left is walked - from (a, b) on to (b, c), c the neighbour of b next clockwise from a - up
 * to the first pair (p, q) with p out of range and q in range; the successor of the dart is
 * (q, p), again a boundary dart.  The successors form the polygon's cycles: on a plane
 * embedding one per component of the region's border, outer borders counterclockwise and
 * holes clockwise.  Each cycle is listed from its smallest dart by (tail, head), the cycles
 * in the order of those.  Where segments cross, the same rule still defines cycles (the
 * faces of the rotation system) and they are returned as such.
 *
 * iso_query_polygon_batch: k (1..64) queries in one sweep, modes as iso_query.  *darts
 * (library-allocated, iso_free) receives every lane's boundary darts in cycle order, lane j's
 * at [dart_off[j], dart_off[j + 1]) (dart_off: k + 1 entries, caller memory).  *cycles
 * (library-allocated, iso_free) receives the start of every cycle as an index into *darts,
 * then one more entry, the total dart count; lane j's cycles are c in
 * [cycle_off[j], cycle_off[j + 1]) (cycle_off: k + 1, caller memory), cycle c spanning darts
 * [cycles[c], cycles[c + 1]).  The first call on a graph builds the embedding on the host and
 * makes it resident (five words per dart, two darts per neighbour pair); ISO_EINVAL if a
 * coordinate is not finite.
 * iso_query_polygon: one query; *count darts and *ncycles cycles (*cycles has ncycles + 1
 * entries).
 */
int iso_query_polygon_batch(iso_graph *g, size_t k, const uint32_t *sources, const uint32_t *taus, int mode,
                            iso_edge **darts, size_t *dart_off, uint64_t **cycles, size_t *cycle_off);
int iso_query_polygon(iso_graph *g, uint32_t source, uint32_t tau, int mode, iso_edge **darts, size_t *count,
                      uint64_t **cycles, size_t *ncycles);

/*
 * One-to-many distances on the same hierarchy: RPHAST (Section 2), the
 * restricted PHAST the paper times in Table 1.  iso_targets_select runs the
 * target selection once: a search from the targets against the direction of
 * the downward arcs collects every vertex with a downward path to a target
 * (the restricted downward graph), which is uploaded grouped by level.  Each
 * query then runs the upward search and sweeps only those vertices (the top
 * table's vertices through the table product).  The selection depends on the
 * tuning's table_max at selection time; a later query with another table
 * prefix fails with ISO_ESTATE.  A target set must be freed before its graph.
 *
 * iso_targets_query: k >= 1 sources, dist (caller host memory, k * count
 * words) receives d(sources[j], targets[i]) at dist[j * count + i], ISO_INF
 * where a target is unreachable.  iso_targets_query_device: the same into
 * caller-owned device memory (checked to lie inside one device allocation),
 * waiting for the caller's stream first; it returns after the writes.
 */
typedef struct iso_targets iso_targets;
int iso_targets_select(iso_graph *g, const uint32_t *targets, size_t count, iso_targets **out);
int iso_targets_query(iso_graph *g, const iso_targets *t, size_t k, const uint32_t *sources,
                      uint32_t *dist);
int iso_targets_query_device(iso_graph *g, const iso_targets *t, size_t k, const uint32_t *sources,
                             uint32_t *dist, void *stream);
/* Size of the restricted graph: vertices below the top table, their entries, level groups, and
 * the host time of the selection (search, layout and upload) in ms. */
int iso_targets_get_info(const iso_targets *t, uint64_t *vertices, uint64_t *arcs, uint32_t *groups,
                         double *select_ms);
void iso_targets_free(iso_targets *t);

/*
 * Distance labels of one query (test hook).  dist (n entries, caller host
 * memory) receives min(d(s, v), ISO_INF) for every vertex the sweep labelled
 * (all vertices in ISO_MODE_PLAIN; core vertices and the vertices of active
 * cells in ISO_MODE_CELLS) and ISO_INF elsewhere; swept (optional, n bytes)
 * receives 1 for labelled vertices and 0 otherwise.  ISO_MODE_CD gives
 * ISO_EINVAL.
 */
int iso_query_distances(iso_graph *g, uint32_t source, uint32_t tau, int mode,
                        uint32_t *dist, uint8_t *swept);

/* Counters of the last query call on g. */
int iso_last_query_stats(const iso_graph *g, iso_query_stats *stats);

/*
 * Branch counters (test hook).  While enabled, the query calls on g count how often the rare
 * paths of the device sweep run, summed until the next iso_debug_enable (which clears them;
 * enabling also turns graph replay off for the core sweep):
 *   counts[0] an isochrone edge of a cell found the workgroup's edge list full and was written
 *             out on its own;
 *   counts[1] a level of a cell held more vertices than a cell workgroup has threads (the level
 *             was swept in several rounds);
 *   counts[2] a core vertex with more than 32 entries per thread had its entries walked again
 *             for a straddling entry;
 *   counts[3] an isochrone edge of a core level found the workgroup's key list full;
 *   counts[4] a sweep found more isochrone edges than the edge-key buffer held and was run again
 *             with a larger buffer (direct query calls);
 *   counts[5..7] reserved (0).
 * iso_debug_read: counts must hold 8 words.
 */
int iso_debug_enable(iso_graph *g, int enable);
int iso_debug_read(iso_graph *g, uint64_t counts[8]);

/*
 * Tuning knobs of the device sweep (the autotuner measures them; when never set:
 * lanes_per_launch 64, block 256, cell_lds_kb 64, use_graph 1, core_mode 0, cell_stage 2,
 * cell_block 0, table_max 0, stall 1, edge_cap 0, overlap_cells 0, plain_sweep 0).  lanes_per_launch: queries per sweep in
 * iso_query_batch (1..64); block: threads per workgroup of the core level
 * kernel (64..1024, multiple of 64); cell_lds_kb: LDS budget of one cell
 * workgroup in KiB (16..160), which sets how many queries' labels a cell
 * workgroup holds (more lanes per workgroup = fewer re-reads of the cell's
 * arcs, fewer resident workgroups per compute unit).
 */
typedef struct {
    uint32_t lanes_per_launch;
    uint32_t block;
    uint32_t cell_lds_kb;
    uint32_t use_graph;         /* 1 = capture the device sweep of a context once (per shape and buffers)
                                   into a hipGraph and replay it */
    uint32_t core_mode;         /* one launch per core level below the table; 0 = with 64 queries per sweep
                                   one wavefront per core vertex (its entries read once for the 64
                                   queries), else threads per (vertex, query, share of its entries);
                                   2 = the latter at every width.  Other values give ISO_EINVAL */
    uint32_t cell_stage;        /* 2 = one workgroup per active cell (default): the cell's data is copied
                                   into LDS once and swept for all the queries that activate the cell, in
                                   chunks of as many queries as cell_lds_kb holds label rows for (at most
                                   64), each thread serving one (vertex, query) slot; the workgroups claim
                                   the active cells one at a time (needs the largest cell's data and one
                                   query's labels to fit 160 KiB, else 0 is used); 0 = work items of a cell and up to G queries, a
                                   workgroup holds two levels' entries in LDS and loads the next level
                                   while relaxing the current one; 1 = work items as in 0, the item's
                                   whole cell data copied into LDS first (needs the largest cell's data
                                   plus one lane's labels to fit 160 KiB, else 0 is used); cell_lds_kb
                                   bounds the LDS in every variant, raised to the minimum it needs */
    uint32_t cell_block;        /* threads per cell workgroup of variants 0 and 1: 256 or 512; 0 = 512 for
                                   sweeps of 32 or more queries, else 256 (variant 2 uses 512) */
    uint32_t table_max;         /* level-merge threshold: the top core levels are merged into one (min,+)
                                   product with the distance table of their vertices while they hold at
                                   most this many vertices; the levels below get one launch each.  0 =
                                   16384; 1 = no table (every core level is its own launch and the upward
                                   search runs to its end); 2..16384, capped at the table built at load
                                   (iso_graph_info top_table) */
    uint32_t stall;             /* 1 = stall-on-demand in the upward search (Section 2, CH): a reached vertex
                                   with a shorter path through a downward arc from a reached higher vertex
                                   is neither expanded nor handed to the sweep (default); 0 = off.  The
                                   answer is the same either way */
    uint32_t edge_cap;          /* 0 = keep the edge-key buffer as it is; otherwise its capacity (in edges,
                                   at least 16) is reset to this value by iso_set_tuning.  A sweep that finds
                                   more isochrone edges than the buffer holds is run again with a larger
                                   buffer (for the serving loop, within its device budget), so this only
                                   moves memory against repeated sweeps; the answer is the same */
    uint32_t overlap_cells;     /* resident cell workgroups per compute unit while two sweeps of one call
                                   overlap on two streams (0 = 3; at most what fits, at most 16) */
    uint32_t plain_sweep;       /* ISO_MODE_PLAIN with 64 queries per sweep: 0 = the cells' internal vertices
                                   as one launch per level counted from the top of each cell, across all
                                   cells, one wavefront per vertex and the 64 queries' labels in device
                                   memory (default; needs 4 * 64 * n bytes per sweep context); 1 = cell by
                                   cell as in ISO_MODE_CELLS.  Other widths, the distance and vertex
                                   outputs use the latter.  The answer is the same */
} iso_tuning;
int iso_set_tuning(iso_graph *g, const iso_tuning *t);
int iso_get_tuning(const iso_graph *g, iso_tuning *t);

/*
 * Read-only view of the preprocessed hierarchy (host memory owned by the
 * library, valid until iso_free_graph).  Sweep positions number the vertices
 * in sweep order: the core block [0, n_core) by descending CH level (Section
 * 2, levels), then each cell's internal vertices by descending level.
 * Downward entries are grouped by head position; entry e is the pair
 * (down_arc[2e], down_arc[2e+1]) = (tail position | flags, length) with flag
 * bit 31 = original arc tail->head exists, bit 30 = original arc head->tail
 * exists (a length of ISO_INF marks the dummy entry of Section 5).  Works for
 * graphs loaded with device = -1 (host only).
 */
typedef struct {
    const uint32_t *perm;          /* n: position -> original id */
    const uint32_t *cell_of;       /* n: original id -> cell (all 2^32-1 without partition) */
    const uint32_t *down_off;      /* n + 1 */
    const uint32_t *down_arc;      /* 2 * down_off[n] */
    const uint32_t *up_off;        /* n + 1, upward arcs grouped by tail position */
    const uint32_t *up_head;       /* head positions */
    const uint32_t *up_w;          /* lengths */
    const uint32_t *core_lvl;      /* core_lvl_len entries: level i = [core_lvl[i], core_lvl[i+1]) */
    uint32_t core_lvl_len;
    const uint32_t *cell_off;      /* num_cells + 1: internal positions of each cell */
    const uint32_t *cell_lvl_ptr;  /* num_cells + 1 */
    const uint32_t *cell_lvl;      /* level start positions of every cell, top level first */
    uint32_t cell_lvl_len;
    const uint32_t *core_cell;     /* n_core: cell of each core position */
    const uint32_t *core_ecc;      /* n_core: eccentricity within the cell */
    const uint8_t *uncovered;      /* num_cells */
} iso_layout;
int iso_graph_get_layout(const iso_graph *g, iso_layout *layout);

/*
 * Device-side phase profile (for roofline reporting).  While enabled, each
 * query call records HIP events on the stream of each sweep around its device
 * phases (core sweep; cell flags and active cells; cell sweep; sort) and
 * accumulates their durations, launch counts and algorithmic HBM
 * bytes: the downward-graph entries and offsets the phase reads, the
 * per-lane label writes and reads it must make (core labels written once and
 * read once; cell-internal labels never leave LDS; each cell reads its
 * distinct core tails once), and the per-vertex cell ids and eccentricities
 * of the flag rule.  Enabling resets the accumulators.  Calls with more
 * than lanes_per_launch queries run consecutive sweeps on two streams, so
 * there a phase's duration includes device time shared with the other sweep.
 */
typedef struct {
    double core_ms, active_ms, cell_ms, sort_ms;        /* summed event durations */
    uint64_t core_launches, cell_launches, calls;       /* kernel launches; query sweeps */
    uint64_t core_bytes, cell_bytes;                    /* summed algorithmic bytes */
    uint64_t core_entries, cell_entries;                /* downward entries swept */
    uint64_t cell_vertices, cells_swept;                /* internal vertices and cells swept */
    uint64_t cell_lanes;        /* (cell, query) pairs swept: each cell counts its active lanes */
    uint64_t cell_items;        /* cell-sweep work items (a cell and up to G of its lanes) */
    uint64_t cell_bytes_survey; /* the cell sweep's bytes counted as a plain PHAST sweep moves them: offsets
                                   and 8-byte entries of the swept cells once, plus per (cell, query) every
                                   internal label written once and read back once (also those that stay
                                   in LDS) */
    double level_ms;            /* the core level launches below the top table alone (k_core_level) */
    uint64_t level_launches, level_bytes;   /* their launches and algorithmic bytes (as core_bytes) */
} iso_profile;
int iso_profile_enable(iso_graph *g, int enable);
int iso_profile_read(const iso_graph *g, iso_profile *out);

/*
 * Serving loop: continuous batching of isochrone queries on a resident graph.
 * Requests are queued by iso_server_submit and answered by device sweeps of up
 * to max_lanes queries each; whenever a sweep context is free, the queued
 * requests (oldest first) are taken into the next sweep, whose host upward
 * searches and device work overlap the sweeps already in flight on other
 * streams.  Contexts and lanes per sweep are admitted by device memory: a
 * context for k lanes needs about n_core*k*4 + n*4 bytes plus its edge and
 * label buffers; if device_budget cannot hold max_inflight contexts of
 * max_lanes lanes, fewer contexts and then fewer lanes are used
 * (ISO_ENOMEM if not even one lane fits).  Every result equals iso_query's
 * for the same (source, tau).  While a server runs on a graph, direct query
 * calls on that graph return ISO_EBUSY.  One server per graph.
 */
typedef struct iso_server iso_server;
typedef struct {
    uint32_t max_lanes;         /* queries per sweep, 1..64 (0 = 64) */
    uint32_t max_inflight;      /* sweeps in flight at once, 1..4 (0 = 2) */
    uint64_t device_budget;     /* device bytes for the sweep contexts (0 = no limit) */
    int mode;                   /* ISO_MODE_PLAIN, ISO_MODE_CELLS or ISO_MODE_CD */
} iso_server_config;
typedef struct {
    double t_queue_ms;          /* submit -> its sweep was launched */
    double t_total_ms;          /* submit -> result ready */
    uint32_t batch_lanes;       /* queries in the sweep that answered it */
} iso_request_stats;
typedef struct {
    uint64_t submitted, completed, sweeps, lanes_total;
    uint32_t contexts, lanes_cap, queue_depth, inflight;
    uint64_t ctx_bytes;         /* device bytes reserved per context (grows with the edge buffer) */
    uint64_t regrown;           /* sweeps run again with a larger edge buffer after an overflow */
} iso_server_stats;
int iso_server_start(iso_graph *g, const iso_server_config *cfg, iso_server **out);
/* Non-blocking; *ticket identifies the request.  ISO_ESTATE after iso_server_stop. */
int iso_server_submit(iso_server *s, uint32_t source, uint32_t tau, uint64_t *ticket);
/* Waits up to timeout_ms (< 0: forever) for a request; on ISO_OK *edges (release with
 * iso_free) holds its sorted edges and the request is forgotten; ISO_EAGAIN if not ready;
 * ISO_EINVAL for an unknown ticket; the request's own error code if its sweep failed. */
int iso_server_wait(iso_server *s, uint64_t ticket, int timeout_ms, iso_edge **edges, size_t *count,
                    iso_request_stats *stats);
int iso_server_get_stats(iso_server *s, iso_server_stats *out);
/* Stops admission, completes every submitted request (results stay collectable with
 * iso_server_wait), releases the sweep contexts and the graph. */
int iso_server_stop(iso_server *s);
void iso_server_free(iso_server *s);   /* stops if needed and frees the handle */

void iso_free(void *p);
const char *iso_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ISO_H */
