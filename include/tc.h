/*
 * tc.h — cover-edge triangle counting on AMD Instinct MI355X (gfx950).
 *
 * Method: Bader, Li, Du et al., "Cover Edge-Based Novel Triangle Counting"
 * (arXiv 2403.02997).
 *   - Section 2: simple undirected graph G = (V, E); a triangle is a set of three
 *     distinct pairwise-adjacent vertices; T = number of triangles.
 *   - Def. BFS-Edge and Lemma H-E / Theorem Gen-CES (Section 4.1): with L(v) the BFS
 *     level of v, the horizontal edges (L(u) == L(v)) cover every triangle.
 *   - Algorithm CETC-Seq and Theorem Correctness (Section 4.2): BFS restarted from every
 *     unvisited vertex; for every horizontal edge (u, v) with u < v and every
 *     w in N(u) ∩ N(v), count w when L(w) != L(u), or when L(w) == L(u) and v < w.
 *   - Algorithm CETC-SM (Section 4.4): the same count, edge-parallel; c1 = apexes on
 *     another level, c2 = apexes on the same level, T = c1 + c2 / 3.
 *
 * Graph format (all entry points): symmetric CSR of a simple graph.
 *   rowptr[n + 1] : uint32, rowptr[0] = 0, non-decreasing, rowptr[n] = m.
 *   colidx[m]     : uint32 neighbour IDs < n; each row strictly increasing; no self-loops;
 *                   v in N(u) iff u in N(v).
 *   m             : number of stored entries = 2 |E|.  Input edges = m / 2.
 * The arrays are DEVICE pointers on the current HIP device, owned by the caller and
 * never written by the library.  Validity is a precondition (a self-loop or duplicate
 * would be counted); tc_validate_csr checks it on the device.  The single-graph calls
 * return TC_ERR_INVALID_GRAPH when they meet an asymmetry between two vertices on the
 * same BFS level (their partner records would be inconsistent); other violations are
 * not detected.
 *
 * Roots: each BFS restarts from the smallest vertex ID of its component (the paper's
 * restart loop taken in ascending ID).  T does not depend on this choice; the levels,
 * cover-edge set and diagnostics do.
 *
 * Errors: every function returns a tc_status.  On error the outputs are left untouched.
 * All entry points are stream-ordered on `stream` (0 = the null stream).
 * Thread safety: calls on different streams may run concurrently; the library keeps no
 * mutable global state besides a per-device cache of the device properties and the
 * tuning set by tc_set_isect_params, tc_set_hub_params and tc_set_forward_threshold.
 *
 * Streams: on graphs of at least 2^22 stored entries, tc_count runs its wavefront-class
 * intersections and its hub count on a second stream that it creates for the call
 * (default priority), ordered after the work queued on `stream`, joined back into it and
 * destroyed before the call returns; everything else runs on `stream`.  The server's
 * worker threads keep to their own streams.
 */
#ifndef TC_H_
#define TC_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TC_OK = 0,
  TC_ERR_INVALID_ARG = -1,    /* null pointer where data is required, bad size      */
  TC_ERR_OUT_OF_MEMORY = -2,  /* device workspace allocation failed                 */
  TC_ERR_HIP = -3,            /* a HIP runtime call failed                          */
  TC_ERR_INVALID_GRAPH = -4,  /* a contract violation was found (see above)         */
  TC_ERR_TOO_LARGE = -5,      /* n >= 2^30 or m > 2^32 - 2^20                       */
  TC_ERR_INTERNAL = -6        /* an internal consistency check failed               */
} tc_status;

/* Statistics of one counting run (host struct, filled by tc_count_ex). */
typedef struct {
  uint64_t triangles;     /* T                                                     */
  uint64_t c1;            /* apexes on another level than the cover edge (CETC-SM) */
  uint64_t c2;            /* apexes on the same level, each triangle seen 3 times  */
  uint64_t cover_edges;   /* |S| = number of horizontal edges                      */
  uint64_t probes;        /* neighbour-list elements streamed by the intersection  */
  uint32_t depth;         /* largest BFS level                                     */
  uint32_t num_roots;     /* connected components (isolated vertices included)    */
  uint32_t bfs_levels_bottom_up; /* levels expanded bottom-up                      */
  uint32_t reserved;
  /* per intersection class (0 lane merge, 1 wavefront, 2 workgroup): elements read from
     the streamed partner lists, and elements of the staged lists N(x) */
  uint64_t class_streamed[3];
  uint64_t class_staged[3];
} tc_stats;

/*
 * tc_count — number of triangles of one graph (CETC-Seq result, CETC-SM data-parallel
 * form).  rowptr/colidx/n/m as above; `count` is a HOST pointer receiving T.
 * Allocates its device workspace stream-ordered on `stream`, frees it before returning,
 * and synchronises `stream`.  n == 0 or m == 0 gives T = 0 without a launch.
 * For cover edges staged as long lists, a same-level apex w <= max(u, v) can never
 * count, so those list entries are skipped: T = c1 + t2 is computed, c2 is not.
 * When the covering ratio |S| / |E| reaches the forward threshold (off by default; the
 * paper uses 0.7; see tc_set_forward_threshold) the count runs with every vertex on one
 * level instead (CETC-Seq-FE's switch to the forward algorithm).
 * Returns TC_ERR_INVALID_ARG for null pointers (when m > 0) or a null `count`,
 * TC_ERR_TOO_LARGE for n >= 2^30 or m > 2^32 - 2^20, TC_ERR_OUT_OF_MEMORY, TC_ERR_HIP.
 */
int tc_count(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n, uint64_t m,
             hipStream_t stream, uint64_t* count);

/*
 * tc_count_split — the two terms of the split form CETC-Seq-S (Section 4.3, Alg.
 * CETC-Seq-S) from tc_count's own pruned pass.  With the BFS levels, G0 is the
 * subgraph of the horizontal edges and G1 that of the other edges.  t0_t1 is a HOST
 * uint64[2]:
 *   t0_t1[0] = t0, the triangles whose three edges are all in G0 (all three vertices on
 *              one level; the paper counts them by forward hashing on G0);
 *   t0_t1[1] = t1, the triangles with an edge in G1 (the apex on another level; the
 *              paper counts them by hashed intersections in G1 over the edges of G0).
 * t0 + t1 = T.  The call runs exactly the kernels of tc_count (same classes, hub pass and
 * streams); every counted apex is tallied by the level of the streamed entry: an entry
 * of the partner's same-level range counts towards t0, one of its other-level range
 * towards t1.  Same arguments, workspace, blocking and errors as tc_count (a null t0_t1
 * is TC_ERR_INVALID_ARG); n == 0 or m == 0 gives {0, 0} without a launch.
 */
int tc_count_split(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n, uint64_t m,
                   hipStream_t stream, uint64_t* t0_t1);

/*
 * tc_count_ex — tc_count plus diagnostics.  `level_out` (DEVICE uint32[n], may be NULL)
 * receives the BFS level of every vertex; `stats` (HOST, may be NULL) the statistics
 * above.  `count` may be NULL when `stats` is given.  With `stats` every intersection
 * streams whole lists and tallies c1, c2 and t2, and the call fails with
 * TC_ERR_INTERNAL unless c2 = 3 t2; without `stats` it counts like tc_count.
 */
int tc_count_ex(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n, uint64_t m,
                hipStream_t stream, uint64_t* count, uint32_t* level_out, tc_stats* stats);

/*
 * tc_count_per_vertex — t(v) = number of triangles containing v, for every v
 * (Section 2: the vertex-based form of the count; sum of t(v) = 3 T).
 * `tri_out` is a DEVICE uint64[n] overwritten with t(v).  Blocking like tc_count.
 */
int tc_count_per_vertex(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n,
                        uint64_t m, hipStream_t stream, uint64_t* tri_out);

/*
 * tc_local_clustering — local clustering coefficient of every vertex from its triangle
 * count (Watts and Strogatz; Section 1 names clustering coefficients among the uses of
 * triangle counts): C(v) = 2 t(v) / (d(v) (d(v) - 1)), the fraction of v's neighbour
 * pairs that are adjacent, and C(v) = 0 when d(v) < 2.
 * rowptr is the graph's DEVICE uint32[n + 1] (read for the degrees only), tri the
 * DEVICE uint64[n] that tc_count_per_vertex wrote, cc_out a DEVICE double[n] that is
 * overwritten.  Computed in double with one correctly rounded division per vertex.
 * Stream-ordered on `stream`: returns after queueing one kernel, without synchronising,
 * so tri may come from a tc_count_per_vertex call on the same stream.  Nothing is
 * allocated.  Returns TC_OK at once for n = 0, TC_ERR_INVALID_ARG for null pointers,
 * TC_ERR_TOO_LARGE for n >= 2^30, TC_ERR_HIP if the launch fails.
 */
int tc_local_clustering(const uint32_t* rowptr, const uint64_t* tri, uint32_t n,
                        hipStream_t stream, double* cc_out);

/*
 * tc_count_batch — triangle counts of many independent graphs in one persistent launch:
 * one workgroup per graph at a time, larger graphs first, each running component roots,
 * BFS, level split, cover-edge selection and intersections without waiting for others.
 * Graph g owns rowptr_cat[row_off[g] .. row_off[g+1]) (its n_g + 1 local offsets,
 * starting at 0, so n_g = row_off[g+1] - row_off[g] - 1) and
 * colidx_cat[col_off[g] .. col_off[g+1]) (m_g = col_off[g+1] - col_off[g] entries,
 * equal to the graph's own rowptr[n_g], holding LOCAL IDs < n_g).
 * row_off / col_off are DEVICE int64[num_graphs + 1], non-decreasing, starting at 0,
 * with row_off[g+1] - row_off[g] >= 1 for every g.
 * total_rows = row_off[num_graphs] and total_cols = col_off[num_graphs] (passed by value
 * so the host never reads device memory).  counts is a DEVICE uint64[num_graphs]
 * receiving T_g.  `workspace` is a DEVICE buffer of at least
 * tc_count_batch_workspace_size(num_graphs, total_rows, total_cols) bytes owned by the
 * caller, or NULL to let the library allocate (and free) it stream-ordered on `stream`.
 * With a caller workspace the call allocates nothing, issues no memset, never
 * synchronises and reads no device data on the host, so it can be captured into a HIP
 * graph and replayed; a workspace must not be shared by calls that overlap in time.
 * Per graph: n_g < 2^30 and m_g <= 2^32 - 2^20 (precondition).  Returns
 * TC_ERR_INVALID_ARG (null pointers, workspace too small), TC_ERR_TOO_LARGE (total_rows or
 * total_cols > 2^32 - 2^20), TC_ERR_OUT_OF_MEMORY, TC_ERR_HIP.
 */
int tc_count_batch(const uint32_t* rowptr_cat, const uint32_t* colidx_cat,
                   const int64_t* row_off, const int64_t* col_off, uint32_t num_graphs,
                   uint64_t total_rows, uint64_t total_cols, void* workspace,
                   size_t workspace_bytes, hipStream_t stream, uint64_t* counts);

/* Bytes of device workspace tc_count_batch needs: 21 per row, 8 per stored entry, and a
   small header. */
size_t tc_count_batch_workspace_size(uint32_t num_graphs, uint64_t total_rows,
                                     uint64_t total_cols);

/*
 * tc_count_batch_noalloc — tc_count_batch for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops that forbid allocation, harnesses
 * that disallow hipMalloc).  Same arguments, meaning and results as tc_count_batch with
 * a caller workspace, but the workspace is a fixed array inside the library of
 * TC_NOALLOC_SCRATCH_BYTES bytes per device, held by every GPU the library runs on until
 * the process ends.  The call allocates nothing, issues no memset, never synchronises
 * and reads no device data on the host.  Its first call on a device looks up that
 * device's copy of the array (hipGetSymbolAddress).
 * All calls on one device share the array, which keeps the last call's contents: calls
 * that overlap in time on one device race and must be serialised by the caller (for
 * example by issuing them on one stream).  A batch whose
 * tc_count_batch_workspace_size(num_graphs, total_rows, total_cols) exceeds
 * TC_NOALLOC_SCRATCH_BYTES is refused with TC_ERR_TOO_LARGE before any launch.
 * Errors as tc_count_batch (TC_ERR_HIP also when the array's address cannot be found).
 */
#define TC_NOALLOC_SCRATCH_BYTES (64u << 20) /* 64 MiB per device */
int tc_count_batch_noalloc(const uint32_t* rowptr_cat, const uint32_t* colidx_cat,
                           const int64_t* row_off, const int64_t* col_off,
                           uint32_t num_graphs, uint64_t total_rows, uint64_t total_cols,
                           hipStream_t stream, uint64_t* counts);

/*
 * ---- continuous-batching server ----------------------------------------------------
 * A server counts a stream of independent graphs handed over as HOST CSR arrays (same
 * format as above).  Each request is routed at submission, by its stored entries, to one
 * of three paths: at most small_max_entries go to the batched path, which packs
 * everything queued, whenever its previous batch has completed, into one tc_count_batch
 * launch; larger requests run through tc_count, those below large_min_entries in
 * arrival order (medium path) and the rest smallest first (large path; one that has
 * waited 2 s since submission goes next), so that no request waits behind the upload of
 * a much larger one.  The paths' uploads overlap with each other and with the counting;
 * the counting runs one job at a time, the device going to the waiting path of smallest
 * jobs first (batched, medium, large) unless another has waited 0.5 s for it.  Each path
 * keeps one device buffer for its jobs, grown when a job needs more, so that a steady
 * stream of requests allocates nothing; the buffers are held against the HBM budget (a
 * path that must grow waits, in the order the paths asked, while the new size does not
 * fit beside the other paths' buffers, which they give back when idle or after their
 * current job).  A request's job starts (its admit time) once its path has its buffer;
 * queued requests hold no device memory.  Results equal tc_count's.  Each server drives
 * the device that is current at tc_serve_create with three host threads and three
 * non-blocking streams of default priority; its tc_count calls keep to those streams (no
 * second stream per call) and take their workspace from the path's buffer.
 */
typedef struct tc_server tc_server;

typedef struct {
  uint64_t hbm_budget_bytes;   /* device bytes admitted requests may hold; 0 = 80 % of the
                                  device memory free at creation                          */
  uint64_t small_max_entries;  /* requests with m <= this use the batched path; 0 = 2^18  */
  uint32_t batch_max_graphs;   /* requests per batched launch at most; 0 = 4096           */
  uint32_t reserved;           /* set to 0                                                */
  uint64_t batch_max_entries;  /* stored entries per batched launch at most (a single
                                  request above it still forms its own batch); 0 = 2^28  */
  uint64_t large_min_entries;  /* single-graph requests with m >= this use the large
                                  worker, the others the medium one; 0 = 2^25            */
} tc_serve_config;

typedef struct {
  uint64_t ticket;             /* as returned by tc_serve_submit                          */
  uint64_t triangles;          /* T (0 when status != TC_OK)                              */
  int32_t status;              /* TC_OK, or the error of its path; TC_ERR_OUT_OF_MEMORY
                                  when the request can never fit the budget               */
  uint32_t path;               /* 0 batched, 1 single-graph (medium), 3 single-graph
                                  (large), 2 rejected at submission                      */
  uint64_t input_edges;        /* m / 2                                                   */
  double submit_s, admit_s, count_s, done_s;
                               /* server clock, seconds since tc_serve_create: submitted,
                                  job started (memory reserved, upload begins), counting
                                  took the device, result ready                          */
} tc_serve_result;

typedef struct {
  uint64_t submitted, completed, rejected;
  uint64_t batches, singles;   /* launches of each path                                   */
  uint64_t queued;             /* submitted and not yet started                           */
  uint64_t in_flight;          /* submitted and not yet completed                         */
  uint64_t hbm_in_use, hbm_peak, hbm_budget;  /* bytes of the paths' buffers             */
  double busy_s[3];            /* seconds each path spent running jobs (start to result):
                                  batched, medium, large                                  */
  double device_s[3];          /* of which holding the device for counting                */
} tc_serve_stats;

/* Creates a server on the current device; `cfg` may be NULL (all defaults). */
int tc_serve_create(const tc_serve_config* cfg, tc_server** out);

/*
 * Queues one graph.  rowptr[n + 1] and colidx[m] are HOST arrays that must stay valid
 * and unchanged until this request's result has been returned by tc_serve_poll.  Writes
 * the request's ticket.  Returns TC_ERR_INVALID_ARG for null pointers,
 * TC_ERR_TOO_LARGE for n >= 2^30 or m > 2^32 - 2^20, TC_ERR_INVALID_GRAPH when
 * rowptr[0] != 0 or rowptr[n] != m; a request whose footprint exceeds the whole budget is
 * accepted and completes at once with TC_ERR_OUT_OF_MEMORY.  Before any kernel reads a
 * request the server checks that rowptr is non-decreasing and every ID is below n (on the
 * host for batched requests, on the device for the others); a request that fails
 * completes with TC_ERR_INVALID_GRAPH and costs the requests beside it nothing.  The
 * other properties of the format (sorted rows, symmetry, no self-loops) stay the
 * caller's precondition: breaking them gives a wrong count, never an access outside the
 * request's own arrays.
 */
int tc_serve_submit(tc_server* server, const uint32_t* rowptr, const uint32_t* colidx,
                    uint32_t n, uint64_t m, uint64_t* ticket);

/*
 * Device bytes a request of n vertices and m stored entries needs when its job runs
 * alone (its path's buffer: CSR, bounds flag or offsets, counting workspace), under the
 * current counting settings; a request above the budget is rejected at submission.
 * Returns TC_ERR_TOO_LARGE as tc_serve_submit would.
 */
int tc_serve_footprint(const tc_server* server, uint32_t n, uint64_t m, uint64_t* bytes);

/*
 * Moves up to `cap` completed results (completion order) into the HOST array `out`;
 * *got receives how many.  Waits up to timeout_ms for the first one (0 = do not wait,
 * negative = wait without limit).
 */
int tc_serve_poll(tc_server* server, tc_serve_result* out, uint32_t cap, uint32_t* got,
                  int32_t timeout_ms);

/* Counters of the server (HOST struct). */
int tc_serve_get_stats(tc_server* server, tc_serve_stats* stats);

/* Waits until every submitted request has completed, then stops the server's threads
   and frees it.  Results not yet polled are dropped. */
int tc_serve_destroy(tc_server* server);

/*
 * tc_validate_csr — checks the graph format contract on the device: rowptr[0] == 0,
 * non-decreasing, rowptr[n] == m, IDs < n, rows strictly increasing, no self-loops,
 * symmetric.  Returns TC_OK or TC_ERR_INVALID_GRAPH (or an argument/HIP error).
 * Synchronises `stream`.
 */
int tc_validate_csr(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n, uint64_t m,
                    hipStream_t stream);

/*
 * Intersection tuning (used by the autotuner).  The staged endpoint x of a cover edge
 * goes to the lane class when d(x) <= lane_max, to the wavefront class when
 * d(x) <= wave_max (<= 512), else to the workgroup class, which stages N(x) in chunks
 * of `chunk` (<= 16384; default 4096) entries and takes `seg` (<= 1024) partners per work item.  The setting
 * is process-wide; change it only while no count is running.  Out-of-range values give
 * TC_ERR_INVALID_ARG and leave the setting unchanged.
 */
int tc_set_isect_params(uint32_t lane_max, uint32_t wave_max, uint32_t chunk, uint32_t seg);
/* Current setting as {lane_max, wave_max, chunk, seg} into the HOST array out4[4]. */
int tc_get_isect_params(uint32_t* out4);

/*
 * Hub pass of tc_count (the apex test of CETC-Seq, Section 4.2, applied as the pruned
 * count, with its per-edge sum regrouped by partner; the result is the same T).  The
 * hubs are the vertices of the highest degree classes: as many whole classes as hold at
 * most max_hubs (<= 256) vertices together, each class at least the class of min_degree
 * (classes are four per octave of the degree).  The cover
 * edges staged under a hub are not intersected one by one: for each partner y the pass
 * streams y's other-level neighbours and its same-level neighbours above y once and looks
 * each one up in a per-vertex bit mask of the hubs whose pruned list holds it, masked
 * with the hubs that stage y.  The pass runs on graphs of at least 1024 * min_degree
 * stored entries (2^22 by default); max_hubs = 0 turns it off.  tc_count_ex and
 * tc_count_per_vertex never use it.  Default {256, 4096}; process-wide, change it only
 * while no count is running; max_hubs > 256 gives TC_ERR_INVALID_ARG.
 * Workspace of tc_count with the pass on: 64 bytes per vertex more, plus 8 bytes per
 * work item (at most n + m / 1024 items).
 */
int tc_set_hub_params(uint32_t max_hubs, uint32_t min_degree);

/*
 * tc_set_forward_threshold — the switch of CETC-Seq-FE (Section 4.3, Alg. CETC-Seq-FE).
 * After the BFS and the extraction, tc_count has the covering ratio c = |S| / |E|
 * (|E| = m / 2).  When c >= threshold it counts again with every vertex on one level:
 * every edge is then a cover edge and the apex rule keeps exactly the apexes above both
 * endpoints, so the same kernels run the ID-ordered forward algorithm (Alg. TC_forward
 * with the hashed intersections of Alg. TC_forward-hashed), which the paper picks for
 * graphs whose covering ratio leaves little to skip.  T is the same either way.
 * Default 2.0, i.e. off: in this implementation the pruned pass already skips what the
 * forward ordering skips, so the switch only adds its second extraction.  Pass 0.7 for
 * the paper's setting; a threshold above 1 never switches, 0 always does.
 * Only the counting call switches (tc_count, tc_count_ex without statistics, the
 * server's single-graph paths); statistics, per-vertex counts, tc_count_split and the
 * batch keep the BFS levels.  Set it while no count is running.  A negative or NaN
 * threshold gives TC_ERR_INVALID_ARG.
 */
int tc_set_forward_threshold(double threshold);
/* Current threshold. */
double tc_get_forward_threshold(void);
/* Current setting as {max_hubs, min_degree} into the HOST array out2[2]. */
int tc_get_hub_params(uint32_t* out2);

/*
 * tc_last_call_info — how the calling thread's last successful tc_count, tc_count_ex or
 * tc_count_per_vertex divided its work (diagnostics; all zero before the first such
 * call on this thread, and after a call on an empty graph).  HOST output.
 */
typedef struct {
  uint64_t cover_edges;     /* |S|                                                   */
  uint32_t lane_vertices;   /* staged vertices of the lane class                     */
  uint32_t wave_vertices;   /* staged vertices of the wavefront class                */
  uint32_t block_vertices;  /* staged vertices of the workgroup class                */
  uint32_t block_items;     /* workgroup-class work items                            */
  uint32_t hubs;            /* hubs of the hub pass (0: the pass did not run)        */
  uint32_t hub_items;       /* hub-pass work items                                   */
  uint32_t side_stream;     /* 1: the wavefront class and hub count ran on a second  */
                            /*    stream beside the workgroup class                  */
  uint32_t forward;         /* 1: c >= the forward threshold, so the count ran with  */
                            /*    every vertex on one level (the other fields then   */
                            /*    describe that run; cover_edges stays the BFS |S|)  */
} tc_call_info;
int tc_last_call_info(tc_call_info* out);

/*
 * Step timing (diagnostics).  While enabled, tc_count / tc_count_ex /
 * tc_count_per_vertex record HIP events on their stream at every step boundary and add
 * each step's elapsed milliseconds to a process-wide accumulator.  tc_profile_read copies
 * up to `cap` per-step totals into the HOST array ms_out, the number of profiled calls
 * into *calls, optionally resets, and returns the number of steps; tc_profile_step_name
 * names step i ("roots", "bfs", "extract", "plan", "isect_lane", "isect_block",
 * "isect_wave", "reduce").
 */
int tc_profile_enable(int on);
int tc_profile_read(double* ms_out, uint32_t cap, uint64_t* calls, int reset);
const char* tc_profile_step_name(int step);

/* Static description of a status code. */
const char* tc_status_string(int status);

/* Library version as major * 10000 + minor * 100 + patch. */
int tc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TC_H_ */
