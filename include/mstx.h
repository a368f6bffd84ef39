/*
 * mstx.h -- C ABI of the MI355X (gfx950) parallel Boruvka minimum spanning tree.
 *
 * Problem (Durbhakula, arXiv 2005.06913, Section 2.1): given an undirected
 * graph as an edge list (src[e], dst[e], w[e]), src and dst interchangeable,
 * find the minimum spanning tree M.  The paper assumes a connected graph with
 * distinct weights.  This library accepts any edge list:
 *   - equal weights are ordered by edge index: edge e precedes edge f iff
 *     (w[e], e) < (w[f], f), so the selected tree is unique;
 *   - self-loops and parallel edges are allowed (a self-loop is never taken);
 *   - a disconnected graph yields the minimum spanning forest and status
 *     MSTX_DISCONNECTED.
 *
 * Method (Sections 2.1 and 2.2.2): Boruvka rounds.  Each round every component
 * selects its lightest outgoing edge (64-bit atomic minimum on the packed key
 * (w << 32) | e; from round 1 on the low half is the edge's position in the
 * stably compacted edge stream, which orders edges exactly as e does),
 * components are united along the selected edges (each component's parent
 * becomes the component its lightest edge reaches; of two components that
 * chose each other the smaller id stays the root), parent pointers are
 * compressed, components are renumbered densely, and edges that
 * became internal are dropped (the paper's "covered" edges).  Rounds repeat
 * until no component has an outgoing edge.  When few components remain the
 * last round is a dense finish (contraction of the remaining graph to the
 * lightest edge between every pair of components, see mst_set_dense_limit).
 *
 * Conventions for every entry point below:
 *   - Array arguments are DEVICE pointers (hipMalloc / torch CUDA memory on
 *     the current HIP device) owned by the caller.  Inputs are never modified.
 *     The library keeps no caller pointer after a call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     All device work is ordered on it.  Calls are blocking: they synchronise
 *     `stream` before returning, because some errors are only known on the
 *     device.
 *   - Vertex ids are int32 in [0, n); edge counts are int64 with
 *     m <= 0xFFFFFFFF (the edge index must fit the key's low 32 bits).
 *   - A negative status means the outputs are unspecified.
 *   - Scratch memory (the workspace) is owned by the library, cached per
 *     (device, stream) and reused across calls: calls on the same stream are
 *     serialised by a mutex, calls on different streams run concurrently,
 *     each with its own workspace.  MSTX_WORKSPACE_LIMIT_BYTES (environment,
 *     bytes) caps one call's workspace; mst_workspace_release frees it.
 */
#ifndef MSTX_H
#define MSTX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes.  >= 0: outputs valid. */
#define MSTX_OK 0                  /* spanning tree found (or n <= 1)                 */
#define MSTX_DISCONNECTED 1        /* graph disconnected: outputs hold the forest     */
#define MSTX_ERR_INVALID_ARG (-1)  /* n < 0, m < 0, or NULL array with m > 0          */
#define MSTX_ERR_VERTEX_RANGE (-2) /* some src/dst id outside [0, n)                  */
#define MSTX_ERR_TOO_LARGE (-3)    /* m > 0xFFFFFFFF                                  */
#define MSTX_ERR_OUT_OF_MEMORY (-4)/* workspace allocation failed or over the limit   */
#define MSTX_ERR_DEVICE (-5)       /* a HIP call failed, or a round-count watchdog    */
#define MSTX_ERR_SCRATCH_LIMIT (-6)/* mst_solve_noalloc: graph over its fixed scratch */

/*
 * Minimum spanning tree of one graph (Section 2.1; parallel form after
 * Section 2.2.2).
 *   n                 number of vertices (>= 0)
 *   m                 number of edges (>= 0)
 *   src, dst          int32[m] edge end points, ids in [0, n)
 *   w                 uint32[m] edge weights
 *   out_in_mst        uint8[m], overwritten: 1 iff edge e is in the tree/forest
 *   out_total_weight  uint64[1], overwritten: sum of w over the marked edges
 * Returns MSTX_OK, MSTX_DISCONNECTED or a negative error.
 * Argument checks (INVALID_ARG, TOO_LARGE) happen on the host before any HIP
 * call.  VERTEX_RANGE is detected during the first edge scan.
 */
int mst_solve(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const uint32_t* w,
              uint8_t* out_in_mst, uint64_t* out_total_weight, void* stream);

/*
 * mst_solve for callers that cannot allocate memory: code that must not call
 * hipMalloc (a harness that forbids it, a tight serving loop that keeps its
 * memory fixed).  Same arguments, results, statuses and round statistics as
 * mst_solve; it allocates nothing, device or host (no hipMalloc, hipFree,
 * pinned memory, events or library allocations), so it does not use the
 * per-stream workspace or MSTX_WORKSPACE_LIMIT_BYTES.
 * Scratch: one fixed 256 MiB device array inside the library, a copy per
 * device, held from the library's first use on that device until the process
 * ends.  A graph fits if mst_workspace_bytes(n, m) plus 2 KB of round records
 * is at most 256 MiB (for example n = 2^20 with m = 2^22, or n = 2^18 with
 * m = 5 * 2^20); graphs that take the one-workgroup path (n <= 8192,
 * m <= 131072, see mst_set_small_limit) always fit.  A larger graph returns
 * MSTX_ERR_SCRATCH_LIMIT before any device work.
 * Every call on a device shares that device's scratch, which keeps the last
 * call's contents (each call initialises what it reads).  Calls on one device
 * are serialised by a lock in the library and each finishes its device work
 * before returning, so they never overlap on the scratch; two calls that
 * overlapped on one device would race.  The round records travel to the host
 * by a plain copy after each synchronisation (two rounds per
 * synchronisation), so a solve may take longer than mst_solve.
 */
int mst_solve_noalloc(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const uint32_t* w,
                      uint8_t* out_in_mst, uint64_t* out_total_weight, void* stream);

/*
 * mst_solve advanced round by round by the caller, for a server that admits
 * other work at Boruvka round boundaries (Section 2.1's while loop: each
 * round acts on every component independently, so other graphs' work can
 * run between two rounds of this one).  Same arguments, results and
 * statuses as mst_solve; the arrays must stay valid until mst_solve_end.
 *   mst_solve_begin    checks the arguments, enqueues round 0 on `stream`
 *                      and returns at once with *out_handle set (a graph that
 *                      needs no rounds, m = 0 or the one-workgroup path, is
 *                      solved before it returns).  At most one stepwise
 *                      solve per (device, stream) at a time (another returns
 *                      MSTX_ERR_INVALID_ARG); it has its own workspace, so
 *                      other calls on the stream may run while it is open.
 *                      Returns a status as mst_solve (negative: no handle).
 *   mst_solve_advance  non-blocking: takes the records of the rounds that
 *                      have finished and enqueues the next round (at most
 *                      two rounds are enqueued at any time); *out_done = 1
 *                      once the solve has ended.  Work enqueued on `stream`
 *                      between two calls runs after the rounds enqueued so
 *                      far.  Returns MSTX_OK or MSTX_ERR_INVALID_ARG.
 *   mst_solve_end      completes the solve (blocking), frees the handle and
 *                      returns the final status (as mst_solve).  The round
 *                      statistics (mst_last_round_stats) go to the thread
 *                      whose call finished the solve.
 * Per-launch profiling (mst_profile_enable) does not cover stepwise solves.
 */
typedef struct MstxSolve MstxSolve;
int mst_solve_begin(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const uint32_t* w,
                    uint8_t* out_in_mst, uint64_t* out_total_weight, void* stream, MstxSolve** out_handle);
int mst_solve_advance(MstxSolve* handle, int32_t* out_done);
/* The same as mst_solve_advance, but waits (on the host, on the round's
 * event) until the next round's record is there, takes that one record and
 * enqueues what follows it: one round per call, without polling. */
int mst_solve_wait_round(MstxSolve* handle, int32_t* out_done);
int mst_solve_end(MstxSolve* handle);

/*
 * Minimum spanning forests of many independent graphs in one call (the
 * disjoint union of graphs has the union of their forests as its forest, and
 * Boruvka rounds never merge components of different graphs).
 *   num_graphs        G >= 0
 *   vertex_offsets    HOST int64[G+1], nondecreasing, [0] = 0: graph g has
 *                     n_g = vertex_offsets[g+1] - vertex_offsets[g] vertices
 *   edge_offsets      HOST int64[G+1], nondecreasing, [0] = 0: graph g owns
 *                     edges [edge_offsets[g], edge_offsets[g+1]) of the arrays
 *   src, dst          int32[edge_offsets[G]], vertex ids LOCAL to the graph,
 *                     in [0, n_g)
 *   w                 uint32[edge_offsets[G]]
 *   out_in_mst        uint8[edge_offsets[G]], overwritten
 *   out_total_weight  uint64[G], overwritten: forest weight per graph
 *   out_status        int32[G], overwritten: per-graph MSTX_OK /
 *                     MSTX_DISCONNECTED / MSTX_ERR_VERTEX_RANGE (then the
 *                     graph's outputs are those of its in-range edges)
 * Ties break by the edge's position inside its graph, as in mst_solve, so
 * every graph's result equals mst_solve on that graph alone.  Graphs with at
 * most 8192 vertices and 2097152 edges are solved by one workgroup each (see
 * mst_set_mid_limit for larger ones); graphs with more edges, and graphs too
 * large for the one-workgroup paths, as parts of a disjoint union solved by
 * the round kernels.
 * Returns MSTX_OK when the call ran (see out_status per graph),
 * MSTX_ERR_INVALID_ARG (bad offsets or NULL arrays), MSTX_ERR_TOO_LARGE (a
 * graph with more than 0xFFFFFFFF edges), MSTX_ERR_OUT_OF_MEMORY or
 * MSTX_ERR_DEVICE.  Argument checks run on the host before any HIP call.
 */
int mst_solve_batched(int32_t num_graphs, const int64_t* vertex_offsets, const int64_t* edge_offsets,
                      const int32_t* src, const int32_t* dst, const uint32_t* w, uint8_t* out_in_mst,
                      uint64_t* out_total_weight, int32_t* out_status, void* stream);

/*
 * Repeated batched solves of one shape (Section 2.1 on each graph, as
 * mst_solve_batched): the batch's offsets are planned once and the solve is
 * captured as a HIP graph on the given device buffers; every
 * mst_batched_plan_run replays it on `stream` (asynchronously: the results
 * are there when the stream has reached that point).  Between runs the
 * caller may change the contents of src / dst / w, not the pointers, the
 * offsets or the library's limits (mst_set_mid_limit and the like are read
 * at creation).  Only batches whose every graph is solved by one workgroup
 * can be captured (under the default limits: at most 65536 vertices and 2^21
 * edges per graph); others return MSTX_ERR_INVALID_ARG -- use
 * mst_solve_batched for them.  Unlike mst_solve_batched, a run does not
 * synchronise and reports no call status: out_status holds every graph's.
 * The plan owns about mst_batched_workspace_bytes of device memory until
 * mst_batched_plan_destroy, which the caller calls when no run is in flight.
 * Creation allocates and captures (on an internal stream); runs allocate
 * nothing.  Errors: MSTX_ERR_INVALID_ARG, MSTX_ERR_VERTEX_RANGE is reported
 * per graph in out_status, MSTX_ERR_OUT_OF_MEMORY, MSTX_ERR_DEVICE.
 */
typedef struct MstxBatchPlan MstxBatchPlan;
int mst_batched_plan_create(int32_t num_graphs, const int64_t* vertex_offsets, const int64_t* edge_offsets,
                            const int32_t* src, const int32_t* dst, const uint32_t* w, uint8_t* out_in_mst,
                            uint64_t* out_total_weight, int32_t* out_status, void* stream, MstxBatchPlan** out_plan);
int mst_batched_plan_run(MstxBatchPlan* plan, void* stream);
int mst_batched_plan_destroy(MstxBatchPlan* plan);

/* Device workspace bytes of mst_solve_batched for these offsets (upper bound;
 * 0 for invalid offsets).  Pure host arithmetic. */
size_t mst_batched_workspace_bytes(int32_t num_graphs, const int64_t* vertex_offsets,
                                   const int64_t* edge_offsets);

/*
 * The first Boruvka step alone (Section 2.1, the edge loop): for every vertex
 * v, out_best[v] = min over non-loop edges e incident to v of the key
 * ((uint64)w[e] << 32) | e, or 0xFFFFFFFFFFFFFFFF when v has no such edge.
 *   out_best  uint64[n], overwritten.
 * Returns MSTX_OK or a negative error (VERTEX_RANGE as for mst_solve).
 */
int mst_select_min_edges(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                         const uint32_t* w, uint64_t* out_best, void* stream);

/*
 * The edge list of one graph given as a symmetric adjacency structure (CSR),
 * the input form the solve entry points take (Section 2.1's undirected graph,
 * each edge once): every arc u -> v with u < v becomes the edge (src = u,
 * dst = v, w = the arc's weight), in row-major arc order; the mirrored arcs
 * (u > v) and self-loops are dropped.  A batch is converted graph by graph
 * (ids stay local to the graph).
 *   n         vertices, >= 0
 *   nnz       arcs, >= 0
 *   row_ptr   DEVICE int64[n+1]: 0 = row_ptr[0] <= ... <= row_ptr[n] = nnz;
 *             the arcs of u are [row_ptr[u], row_ptr[u+1])
 *   col, w    DEVICE int32[nnz] (arc targets, in [0, n)), uint32[nnz]
 *   out_src, out_dst, out_w
 *             DEVICE int32 / int32 / uint32 [nnz] (an upper bound): the edges
 *             are written from the start, owned by the caller
 *   out_m     HOST int64: the number of edges written
 * Returns MSTX_OK; MSTX_ERR_INVALID_ARG (negative sizes, NULL arrays, or a
 * row_ptr not as above, checked on the device); MSTX_ERR_VERTEX_RANGE (a
 * column outside [0, n)); MSTX_ERR_TOO_LARGE (more than 0xFFFFFFFF edges);
 * MSTX_ERR_OUT_OF_MEMORY or MSTX_ERR_DEVICE.  After an error the outputs are
 * unspecified.  Blocks until the count is on the host.
 */
int mst_csr_to_edges(int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col, const uint32_t* w,
                     int32_t* out_src, int32_t* out_dst, uint32_t* out_w, int64_t* out_m, void* stream);

/*
 * Per-round statistics of the most recent mst_solve call made by the calling
 * thread.  For round r (0-based), out[3r+0] = components with at least one
 * outgoing edge candidate at the start of the round (all components in round
 * 0), out[3r+1] = live edges (ends in different components at the start of
 * the round), out[3r+2] = edges added to the tree in the round.
 *   out        host int64[3 * max_rounds]
 * Returns the number of rounds recorded (<= max_rounds), or
 * MSTX_ERR_INVALID_ARG if out is NULL with max_rounds > 0.
 */
int mst_last_round_stats(int64_t* out, int32_t max_rounds);

/*
 * Bytes of device workspace a call of mst_solve with (n, m) uses: an upper
 * bound, for admission control by memory budget.  Pure arithmetic, no HIP call.
 * Returns 0 for invalid (n, m).
 */
size_t mst_workspace_bytes(int32_t n, int64_t m);

/*
 * Per-kernel timing (profiling aid, off by default).  While enabled, each
 * kernel launch of mst_solve is bracketed by HIP events on the solve's
 * stream; after each solve the elapsed times, launch counts and algorithmic
 * bytes are accumulated per kernel (template instantiation, named as a
 * profiler lists it: "k_scan<mode, input, compact>", "k_bucket_min",
 * "k_slab_min", "k_dense_finish", "k_hook", "k_compress", "k_finalize",
 * "k_relabel").  Every
 * launch is counted, including launches that return at once (a minima mode
 * not chosen for the actual component count, the round enqueued after the
 * last one).  Algorithmic bytes are credited to the scan launch that did a
 * round's work: the edge stream read once (12 B per input edge, 16 B per
 * record), the previous round's label map read once (4 B per entry), the
 * minima initialised and written once (16 B per component) and the survivors
 * written once (16 B per record); a dense round writes its pair table once
 * (8 B per pair) instead of minima and survivors.
 *   mst_profile_enable: enable != 0 starts (and zeroes) the counters, 0 stops;
 *                       returns the previous state.
 *   mst_profile_read:   copies min(kinds, K) entries to host arrays; returns
 *                       the number K of kernels tracked or MSTX_ERR_INVALID_ARG.
 *   mst_profile_kernel_name: name of kernel i ("" if out of range).
 * Intended for benchmarking; the events add a little time per launch.
 */
int mst_profile_enable(int enable);
int mst_profile_read(double* out_ms, int64_t* out_launches, double* out_bytes, int32_t kinds);
const char* mst_profile_kernel_name(int kind);

/*
 * The same counters split by Boruvka round (Section 2.1's while loop; the
 * round a launch was enqueued for).  Row r of each host array holds K
 * entries (K = the kernel count mst_profile_read returns), kernel i at
 * [r * K + i], for rounds r < min(max_rounds, 41).  k_bucket_min launches
 * are credited with 16 B per live edge of their round (two 8-byte offers
 * read) plus 8 B per component (its minimum written).
 *   out_ms, out_launches, out_bytes  host arrays of max_rounds * K entries
 * Returns K, or MSTX_ERR_INVALID_ARG.
 */
int mst_profile_read_rounds(double* out_ms, int64_t* out_launches, double* out_bytes, int32_t max_rounds);

/*
 * Frees the workspace cached for (current device, stream), after the stream's
 * work has finished.  For memory-budgeted callers (a server that retires a
 * stream).  Must not run while another thread has a call in flight on the
 * same stream.  Returns MSTX_OK or MSTX_ERR_DEVICE.
 */
int mst_workspace_release(void* stream);

/*
 * Dense finish (a contraction of the graph that Section 2.1's cycle property
 * allows: of the edges joining two components only the lightest can be in the
 * tree).  When a round of mst_solve starts with at most `limit` components,
 * that round keeps the lightest edge of every component pair (a table of
 * limit * (limit - 1) / 2 keys in LDS) and one workgroup completes Boruvka on
 * that small complete graph; it is the last round.  The tree is the same; the
 * per-round statistics then end with that round, whose "edges added" is the
 * sum over the rounds it replaces.  limit is clamped to [0, 200] (0: off,
 * every round is a plain Boruvka round; the default is 200).  limit < 0 only
 * queries.  Returns the previous limit.  Process-wide; read at the start of
 * each call (mst_solve_batched's large graphs included).
 */
int32_t mst_set_dense_limit(int32_t limit);

/*
 * Small graphs (Section 2.1's rounds, one launch): mst_solve solves a graph
 * with at most `limit` vertices and at most 131072 edges with a single
 * workgroup that keeps every vertex's state in LDS and runs all rounds behind
 * workgroup barriers, instead of one kernel chain per round (the path
 * mst_solve_batched uses for its small graphs).  The tree and the round
 * statistics are the same (no dense finish on this path).  limit is clamped
 * to [0, 8192] (0: off; the default is 8192); limit < 0 only queries.
 * Returns the previous limit.  Process-wide; read at the start of each call.
 */
int32_t mst_set_small_limit(int32_t limit);

/*
 * Mid-size graphs of mst_solve_batched (Section 2.1's rounds, one workgroup
 * per graph): a graph with more than 8192 and at most `limit` vertices and at
 * most 2097152 edges is solved by one workgroup that keeps each vertex's
 * minimum key and a 2-byte union-find in LDS (10 bytes per vertex) and reads
 * the graph's edges once per round.  A graph with more than `limit` and at
 * most 65536 vertices (same edge bound) is first contracted by one workgroup
 * round by round (minima in LDS windows, components renumbered densely, the
 * edges rewritten as 16-bit pairs in the batched workspace) until at most
 * `limit` components are left, which are then solved the same way.  Larger
 * graphs, and all of them when this path is off, are solved as parts of a
 * disjoint union by the round kernels.  The results are the same.  limit is
 * clamped to [0, 16280] (at most 8192: off; the default is 16280); limit < 0
 * only queries.  Returns the previous limit.  Process-wide; read at the start
 * of each mst_solve_batched and mst_batched_workspace_bytes call.
 */
int32_t mst_set_mid_limit(int32_t limit);

/*
 * Late rounds (Section 2.2.2's union and find, one launch): when mst_solve's
 * bound on a round's component count is at most `limit`, the round's hook
 * (each component's parent is the component its lightest edge reaches; the
 * smaller of a mutual pair stays a root), pointer jumping, root count and
 * relabel run in one workgroup with the parent forest in LDS, instead of
 * four grid-wide kernels.  The tree, the labels and the round
 * statistics are the same.  limit is clamped to [0, 10240] (0: off; the
 * default is 10240); limit < 0 only queries.  Returns the previous limit.
 * Process-wide; read at the start of each call (mst_solve_batched's large
 * graphs included).
 */
int32_t mst_set_tail_limit(int32_t limit);

/*
 * Minima of large rounds (Section 2.1's edge loop): a round of mst_solve
 * whose bound on the component count is above the LDS range (20352) and at
 * most `limit` takes its per-component minima by sorting the edges' offers
 * into buckets of consecutive components, each bucket's minima taken in one
 * workgroup's LDS; a round above the limit takes them with filtered 64-bit
 * atomic minima in device memory (one per edge end).  The tree, the labels
 * and the round statistics are the same.  limit is clamped to
 * [0, 16760832] (0: never bucket mode; the default is 16760832, the largest
 * count the 1023 buckets of 16384 components cover); limit < 0 only queries.
 * Returns the previous limit.  Process-wide; read at the start of each call
 * (mst_solve_batched's large graphs and mst_select_min_edges included).
 */
int32_t mst_set_bucket_limit(int32_t limit);

/*
 * Occupancy of the LDS-mode edge scans (Section 2.1's edge loop with the
 * per-component minima in LDS): how many scan workgroups share a compute
 * unit.  0 (the default) chooses from the scan's LDS size (at most 4); 1..8
 * asks for that many, as far as 160 KB of LDS per compute unit holds them.
 * The results are the same for every value.  wg_per_cu < 0 only queries.
 * Returns the previous value.  Process-wide; read when each round is
 * enqueued.  A tuning knob (paper_2005_06913_amd/autotune.py sets it).
 */
int32_t mst_set_scan_occupancy(int32_t wg_per_cu);

/*
 * Sparse finish (the cycle property of Section 2.1's covered edges, applied
 * to component pairs): in a round r >= 1 of mst_solve whose previous round
 * had at most 16384 components, if at most `live_edges` live edges were left
 * two rounds before, the lightest edge of every pair of components is
 * collected and, when the pairs fit one workgroup (about 13,000 pairs at
 * few components, fewer as the count grows), the remaining Boruvka rounds
 * run on that small graph in one launch and the solve ends in that round.
 * Otherwise the round goes on as usual.  The tree and total are the same;
 * the round statistics then end with that round, whose edges added are the
 * sum of the remaining rounds'.  0 = never; the default is 2^20; limit < 0
 * only queries.  Returns the previous value.  Process-wide; read at the start
 * of each call.
 */
int32_t mst_set_sparse_limit(int32_t live_edges);

/* Static description of a status code. */
const char* mst_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* MSTX_H */
