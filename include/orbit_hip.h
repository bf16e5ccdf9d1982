/*
 * orbit_hip.h -- C ABI of liborbit_hip.so: exact per-vertex orbit counts of
 * all connected patterns with 2..5 vertices (orbits 0..72) on an AMD
 * Instinct MI355X (gfx950), computed by the EVOKE method of Pashanasangi and
 * Seshadhri ("Efficiently Counting Vertex Orbits of All 5-vertex Subgraphs,
 * by EVOKE").
 *
 * Pipeline (all steps run in the library's own HIP kernels):
 *   1. validate the CSR and compute degrees;
 *   2. orient the graph into a DAG by a degeneracy order (bucketed k-core
 *      peeling on the GPU; section "Preliminaries", degree-ordering
 *      paragraph, uses a degree order -- any total order gives the same
 *      counts, it only changes the work);
 *   3. enumerate directed triangles, 4-cycles, 4-/5-cliques, wedges,
 *      diamonds and directed 3-paths (Fig. 5vertex-basis; Theorem 4orbit;
 *      Theorem on 5-cycle/5-clique running time);
 *   4. combine them through the orbit equations (Lemma 4vertexorbit,
 *      Lemma 4edgeorbit, Theorem 5vertexorbit) into non-induced counts;
 *   5. convert to induced counts with the exact integer inverse of the
 *      transform of appendix "Conversion between Induced and Noninduced
 *      counts".
 *
 * Conventions shared by every entry point
 *   - Graph: simple undirected graph as a symmetric CSR.  row_ptr has n+1
 *     uint32 entries, row_ptr[0] == 0, row_ptr[n] == 2m; col_idx has 2m
 *     uint32 entries; each neighbour list strictly ascending; no self-loops;
 *     every edge stored in both directions; 2m < 2^32.  Isolated vertices
 *     are allowed.  The input is always validated; a malformed graph is
 *     rejected with an error code before any counting kernel runs.
 *   - Output: counts[u * K + o], uint64, K = orbit_num_orbits(k_max)
 *     (4 for k_max = 3, 15 for k_max = 4, 73 for k_max = 5).  Induced
 *     counts by default (the paper's problem statement asks for induced
 *     counts); ORB_NONINDUCED returns the non-induced counts DM(u, theta)
 *     of Definition unlabeled-match.  Values are exact modulo 2^64 (all
 *     arithmetic wraps; binomials are formed exactly before reduction).
 *   - Pointers: row_ptr, col_idx, counts and workspace are DEVICE pointers
 *     owned by the caller; the library never frees them.  `stream` is a
 *     hipStream_t (NULL = the null stream).
 *   - Errors: an int status, 0 on success, negative ORB_E_* otherwise; never
 *     throws across the ABI, never aborts.  On error the contents of counts
 *     are unspecified.
 *   - Synchronisation: the calls return after the work has finished on the
 *     stream (they read a few status words back from the device).
 *   - Thread safety: calls on different streams/devices may run concurrently;
 *     each call uses only its own workspace.
 */
#ifndef ORBIT_HIP_H
#define ORBIT_HIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define ORB_OK 0
#define ORB_E_INVALID_ARG (-1)  /* bad n/m/k_max/pointer/flags */
#define ORB_E_NOT_SORTED (-2)   /* a neighbour list is not ascending */
#define ORB_E_SELF_LOOP (-3)
#define ORB_E_DUPLICATE (-4)    /* an edge appears twice in a list */
#define ORB_E_ASYMMETRIC (-5)   /* (u,v) present but (v,u) missing */
#define ORB_E_OUT_OF_RANGE (-6) /* col_idx >= n, or row_ptr not monotone / not ending at 2m */
#define ORB_E_WORKSPACE (-7)    /* workspace too small: see *ws_required */
#define ORB_E_DEVICE (-8)       /* a HIP call failed */
#define ORB_E_INTERNAL (-9)     /* internal consistency check failed */
#define ORB_E_BATCH (-10)       /* batched input: graph offsets not 0..n and non-decreasing,
                                   or an edge joining two graphs */
#define ORB_E_TOO_LARGE (-11)   /* the count needs more memory than there is: more than the
                                   static buffer of orbit_count_noalloc
                                   (orbit_noalloc_capacity()), or, for orbit_count, a
                                   workspace larger than the device's free memory */

/* option flags */
#define ORB_NONINDUCED 0x1u /* return non-induced counts DM(u, theta) */
#define ORB_TIMING 0x2u     /* record per-phase times (orbit_last_phase_times) */
#define ORB_RELABEL 0x4u    /* count on a copy of the graph renumbered heaviest degree
                               class first (rows, maps and per-vertex data of the hubs
                               together: faster on graphs whose ids are unrelated to
                               degree); the counts come back under the caller's ids.  One
                               graph only (not batched), not with features_out/steps_out;
                               the workspace grows by about 8m + 40n bytes. */
#define ORB_ASYNC 0x10u      /* orbit_count_ex / orbit_count_edges: enqueue the whole count
                               on `stream` and return without any host synchronisation,
                               using the sizes orbit_prepare reported for this graph
                               (orb_opts.sizes, required); the peeling runs that many
                               launch groups and stops early on the device.  Sizes
                               that do not match the graph are detected on the device
                               and reported, with every other error, by
                               orbit_count_status.  Not with ORB_TIMING. */
#define ORB_SERIAL_GROUPS 0x8u /* k_max = 5: run the three independent orbit groups
                               (pair sweep, 5-cycles, second clique pass) one after
                               another on `stream` instead of running the last two on
                               a helper stream beside the pair sweep (section "Runtime
                               distribution and parallel speedup" runs these groups in
                               parallel) */

/* order in which the per-source kernels take their sources (the counts
 * are the same under every schedule; only the work balance changes) */
#define ORB_SCHED_ID 0u     /* ascending vertex id */
#define ORB_SCHED_STATIC 1u /* heaviest first by degree thresholds:
                               bins of 4*(log2(1+d) + log2(1+d+)) */
#define ORB_SCHED_MLP 2u    /* heaviest first by the cost model's prediction
                               (bins of 4 * predicted log2 steps) */

/* execution groups of the per-source kernels (counts are the same either way) */
#define ORB_GROUPS_AUTO 0u  /* waves when every source is light: per-source maps of
                               <= 4096 entries (graphs, or a batch's largest graph, of
                               <= 4096 vertices) and degeneracy < 64 */
#define ORB_GROUPS_WG 1u    /* a 256-thread workgroup per source */
#define ORB_GROUPS_WAVE 2u  /* a 64-lane wave per source, four sources per workgroup,
                               queue entries taken 16 at a time */

/* Data-dependent sizes of one graph's count, as orbit_prepare finds them:
 * the number of 32-round peeling launch groups, the triangle count, the
 * largest peel level (degeneracy - the out-degree bound) and, for batches,
 * the largest graph. */
typedef struct orb_sizes {
    uint64_t ntri;
    uint32_t peel_groups;
    uint32_t maxlevel;
    uint32_t gmax;
    uint32_t reserved;
} orb_sizes;

/* cost model: a 3 -> 32 -> 32 -> 1 fp32 ReLU network, parameters packed as
 * W1[32][3], b1[32], W2[32][32], b2[32], W3[32], b3 */
#define ORB_MLP_PARAMS 1217

typedef struct orb_opts {
    uint32_t flags;           /* ORB_* option bits */
    uint32_t num_wg;          /* persistent workgroups for the per-source kernels; 0 = default */
    uint32_t schedule;        /* ORB_SCHED_* */
    uint32_t groups;          /* ORB_GROUPS_*: who works on one source in the per-source
                                 kernels */
    const float *mlp_weights; /* device, ORB_MLP_PARAMS floats; needed by ORB_SCHED_MLP */
    float *features_out;      /* device, n*3 floats, nullable: per-vertex cost features
                                 (log2(1+d+(u)), log2(1+sum_{w in N+(u)} d+(w)), log2(1+d(u)))
                                 under the degeneracy orientation */
    uint64_t *steps_out;      /* device, n uint64, nullable: per-source loop iterations
                                 of the pair sweep and the 5-cycle kernel (the cost
                                 model's training target) */
    uint64_t *pass_cycles_out; /* device, 4 uint64, nullable (profiling): shader clock
                                  cycles summed over execution groups in the pair sweep's
                                  passes: wedges, wheel maps, pair terms, centre terms;
                                  accumulated (the caller zeroes them) */
    const orb_sizes *sizes;   /* host, needed by ORB_ASYNC: from orbit_prepare */
} orb_opts;

/* Number of output columns K for k_max (3, 4 or 5); 0 if k_max is invalid. */
int orbit_num_orbits(int k_max);

/* Minimal form: counts for every vertex, default options, null stream.
 * Allocates its workspace with hipMalloc and frees it before returning;
 * ORB_E_TOO_LARGE when that workspace exceeds the device's free memory.
 * m = number of undirected edges (col_idx has 2m entries). */
int orbit_count(const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n, uint64_t m,
                int k_max, uint64_t *counts);

/* Edge orbit counts of the 3- and 4-vertex patterns (Definition edge-orbit,
 * Fig. edge_orbits, computed by the equations of Lemma 4edgeorbit) together
 * with the vertex counts of orbit_count_ex: edge_counts (DEVICE, 2m x 12
 * uint64) receives, for every CSR slot s = (u, v),
 *   edge_counts[s * 12 + i] = E_i<u,v>,  i = 0..11,
 * the number of non-induced copies of the edge orbit's pattern in which
 * the edge (u,v) lies in edge orbit i with u in the endpoint vertex orbit of
 * larger index; for an edge orbit whose two endpoint orbits coincide (1, 3,
 * 5, 7, 10, 11) both slots of the edge hold the same count.  k_max must be
 * 4 or 5 (counts has K = 15 or 73 columns); the workspace is that of
 * orbit_count_ex with the same k_max (orbit_workspace_query).  Not with
 * ORB_RELABEL (ORB_E_INVALID_ARG).  Values wrap modulo 2^64 like the
 * vertex counts. */
int orbit_count_edges(const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n, uint64_t m,
                      int k_max, uint64_t *counts, uint64_t *edge_counts, void *workspace,
                      uint64_t ws_bytes, uint64_t *ws_required, void *stream,
                      const orb_opts *opts);

/* Number of patterns with 2..k_max vertices (3, 9 or 30); 0 if k_max is
 * invalid. */
int orbit_num_patterns(int k_max);

/* Global counts and VOC distributions of a count array (the paper's
 * experiments section, "VOC distributions", Figs. orb70CCD, orb17CCD and
 * H9CCD), asynchronous on `stream`.  counts: DEVICE, n x K uint64 as written
 * by the count calls (K = orbit_num_orbits(k_max)).  Outputs, DEVICE,
 * overwritten:
 *   orbit_sums[2o], [2o+1]: low and high 64 bits of sum_u counts[u][o];
 *   pattern_counts (nullable, 2 x orbit_num_patterns(k_max)): the number of
 *     induced copies of pattern H_h (low, high words): the sum of one of its
 *     orbits divided by the number of its vertices in that orbit;
 *   hist[o * 65 + b]: vertices whose count of orbit o has bit length b
 *     (b = 0: count 0; else 2^(b-1) <= count < 2^b), so the fraction of
 *     vertices with count >= 2^(b-1) -- the complementary cumulative
 *     distribution the paper plots -- is sum_{b' >= b} hist[o*65+b'] / n.
 * Sums are exact when every row is (counts modulo 2^64 otherwise; see the
 * overflow flags of orbit_count_ex).  For induced counts the sum over an
 * orbit of H_h is the same multiple of its size for every orbit of H_h. */
int orbit_voc_summary(const uint64_t *counts, uint32_t n, int k_max, uint64_t *orbit_sums,
                      uint64_t *pattern_counts, uint64_t *hist, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the count
 * of orbit_count_ex with default options, whose workspace is a static
 * device array of orbit_noalloc_capacity() bytes (64 MiB) that every GPU the
 * library runs on holds until the process ends.  Calls no hipMalloc or
 * hipFree and allocates through no library.  The caller passes the CSR and
 * counts (device pointers, as for orbit_count_ex); `stream` may be NULL.
 * Returns ORB_E_TOO_LARGE, before any kernel runs when n and m alone are
 * too large, else after the graph was validated and its triangles counted,
 * when the count does not fit (fewer persistent workgroups are used first).
 * All calls on one GPU share that GPU's array: calls that overlap on one
 * GPU (other threads, other streams) race and must be serialised by the
 * caller.  Like orbit_count_ex it returns after the stream has finished. */
int orbit_count_noalloc(const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n,
                        uint64_t m, int k_max, uint64_t *counts, void *stream);

/* Size in bytes of orbit_count_noalloc's static buffer (host only). */
uint64_t orbit_noalloc_capacity(void);

/* Validates the graph and finds the sizes its count depends on (this call
 * synchronises `stream`), for asynchronous counts (ORB_ASYNC): writes the
 * workspace size orbit_count_ex needs with these opts to *bytes and the
 * sizes to *sizes.  Allocates and frees a temporary workspace like
 * orbit_workspace_query. */
int orbit_prepare(const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n, uint64_t m,
                  int k_max, void *stream, const orb_opts *opts, uint64_t *bytes,
                  orb_sizes *sizes);

/* Status of the last count enqueued on `workspace` (one graph; the device
 * state is at its start): waits for `stream`, then returns ORB_OK or the
 * error the kernels recorded -- the status call of ORB_ASYNC counts. */
int orbit_count_status(const void *workspace, void *stream);

/* Workspace size that orbit_count_ex needs for this graph.  The size
 * depends on the number of triangles, so this call validates the graph,
 * orients it and counts triangles on the device (allocating and freeing
 * its own temporary memory) before returning the size in *bytes. */
int orbit_workspace_query(const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n,
                          uint64_t m, int k_max, void *stream, const orb_opts *opts,
                          uint64_t *bytes);

/* Full form: uses only the caller's workspace (device memory of ws_bytes
 * bytes, 256-byte aligned); allocates no device memory.  If the workspace
 * is too small it returns ORB_E_WORKSPACE and, when ws_required is not
 * NULL, stores the size it needs there.  opts may be NULL.
 *
 * overflow_flags (DEVICE, n bytes, nullable): the paper does not discuss
 * integer width; counts are exact modulo 2^64.  When given, byte u is set
 * to 1 when an upper bound of u's non-induced counts reaches 2^63, else 0,
 * so every row whose flag is 0 is exact (induced counts never exceed the
 * non-induced ones).  The bound, evaluated in fp64: a non-induced copy of a
 * k-vertex pattern at u is a connected k-vertex subgraph containing u; it
 * contains a spanning tree, and at most 2^(C(k,2)-k+1) such subgraphs share
 * one tree, while the number of k-vertex trees containing u is at most the
 * sum, over the rooted tree shapes with k vertices, of the homomorphism
 * counts into G with the root at u (nested neighbour-degree sums) divided
 * by the shape's root-fixing automorphisms.  Flagged rows still hold the
 * counts modulo 2^64. */
int orbit_count_ex(const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n, uint64_t m,
                   int k_max, uint64_t *counts, uint8_t *overflow_flags, void *workspace,
                   uint64_t ws_bytes, uint64_t *ws_required, void *stream,
                   const orb_opts *opts);

/* ---- many small graphs in one call.
 * The batch is the disjoint union of num_graphs graphs stored as one CSR
 * over global vertex ids: graph g owns vertices vptr[g] .. vptr[g+1]-1
 * (vptr: DEVICE array of num_graphs+1 uint64, vptr[0] = 0, non-decreasing,
 * vptr[num_graphs] = n; empty graphs allowed) and every edge joins two
 * vertices of the same graph (else ORB_E_BATCH).  The counts of graph g are
 * rows vptr[g] .. vptr[g+1]-1 of counts -- the counts of each graph on its
 * own, since every orbit lives inside one connected component.  The
 * per-source maps are indexed within the source's graph, so the scratch
 * scales with the largest graph instead of n.  Otherwise as orbit_count_ex. */
int orbit_count_batched(const uint64_t *vptr, uint32_t num_graphs, const uint32_t *row_ptr,
                        const uint32_t *col_idx, uint32_t n, uint64_t m, int k_max,
                        uint64_t *counts, void *workspace, uint64_t ws_bytes,
                        uint64_t *ws_required, void *stream, const orb_opts *opts);

/* Workspace size of orbit_count_batched (validates the batch on the device). */
int orbit_workspace_query_batched(const uint64_t *vptr, uint32_t num_graphs,
                                  const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n,
                                  uint64_t m, int k_max, void *stream, const orb_opts *opts,
                                  uint64_t *bytes);

/* Autotuner: runs the count (batched when vptr is not NULL, else one graph)
 * once per candidate workgroup count, execution group (workgroup or wave
 * per source) and schedule (id, static thresholds, and the cost model when
 * base->mlp_weights is set), timed with HIP events, and returns in *best
 * the options (base's flags, the fastest num_wg, groups and schedule) and
 * in *best_ms its GPU time.  Candidates whose workspace does
 * not fit ws_bytes are skipped.  counts receives the last run's counts. */
int orbit_autotune(const uint64_t *vptr, uint32_t num_graphs, const uint32_t *row_ptr,
                   const uint32_t *col_idx, uint32_t n, uint64_t m, int k_max, uint64_t *counts,
                   void *workspace, uint64_t ws_bytes, void *stream, const orb_opts *base,
                   const uint32_t *nwg_candidates, int num_candidates, orb_opts *best,
                   float *best_ms);

/* ---- plans: the whole count captured as one HIP graph.
 * orbit_plan_create runs the count once (validating the input and fixing
 * every data-dependent choice: peel launches, triangle count, degeneracy,
 * largest graph), then captures the same kernel sequence -- with nothing
 * read back to the host -- into a graph bound to these buffers.
 * orbit_plan_launch replays it on `stream` (asynchronous, no host sync): it
 * recounts the buffers it was built on, so the input must be unchanged
 * (the graph ends with a check that the sizes agree and records
 * ORB_E_INTERNAL otherwise; a changed input is not otherwise guarded).
 * orbit_plan_status waits for `stream` and returns the status of the last
 * replay.  vptr may be NULL (one graph).  ORB_TIMING, features_out and
 * steps_out are ignored.  The workspace must outlive the plan. */
typedef struct orb_plan orb_plan;
int orbit_plan_create(const uint64_t *vptr, uint32_t num_graphs, const uint32_t *row_ptr,
                      const uint32_t *col_idx, uint32_t n, uint64_t m, int k_max,
                      uint64_t *counts, void *workspace, uint64_t ws_bytes, void *stream,
                      const orb_opts *opts, orb_plan **plan);
int orbit_plan_launch(orb_plan *plan, void *stream);
int orbit_plan_status(orb_plan *plan, void *stream);
int orbit_plan_destroy(orb_plan *plan);

/* Human-readable text of a status code (static storage). */
const char *orbit_strerror(int status);

/* GPU times (ms) of the kernels of the three 5-vertex orbit groups in the
 * calling thread's last call with ORB_TIMING ("pairs", "c5",
 * "clique2_k4terms"), each from events on the stream it ran on (they may
 * overlap): writes up to max_kernels values and names and returns how many. */
int orbit_last_kernel_times(float *ms, const char **names, int max_kernels);

/* Per-phase GPU times (ms) of the calling thread's last orbit_count_ex with
 * ORB_TIMING: writes up to max_phases values and their names (static
 * strings) and returns the number of phases. */
int orbit_last_phase_times(float *ms, const char **names, int max_phases);

/* ---- cost model (learned scheduler).  All pointers are device pointers;
 * the calls are asynchronous on `stream` and return after enqueueing. */

/* Initialise the ORB_MLP_PARAMS weights from `seed` (He-uniform weights,
 * zero biases). */
int orbit_mlp_init(float *weights, uint32_t seed, void *stream);

/* Predictions out[i] (log2 step count) for count feature rows (3 floats). */
int orbit_mlp_predict(const float *weights, const float *features, uint32_t count, float *out,
                      void *stream);

/* Full-batch gradient of the mean squared error between the predictions and
 * targets (floats), or log2(1 + steps) when targets is NULL: grad receives
 * ORB_MLP_PARAMS floats, loss one float.  Both are overwritten. */
int orbit_mlp_grad(const float *weights, const float *features, const float *targets,
                   const uint64_t *steps, uint32_t count, float *grad, float *loss,
                   void *stream);

/* Train the weights in place with Adam for `iters` mini-batch steps of
 * `batch` samples drawn (by a counter-based hash of seed and step) from the
 * count rows, target log2(1 + steps).  state: 3*ORB_MLP_PARAMS + 1 floats
 * of scratch (moments, gradient, last mini-batch loss in the final float). */
int orbit_mlp_train(const float *features, const uint64_t *steps, uint32_t count,
                    float *weights, float *state, uint32_t iters, uint32_t batch, float lr,
                    uint32_t seed, void *stream);

/* Work statistics of the calling thread's last orbit_count_ex with
 * ORB_TIMING, for throughput and roofline reporting: vals[0..5] = n, m,
 * triangles, degeneracy (largest peel level), wedges = sum over vertices of
 * C(d,2), diamonds = sum over edges of C(T(e),2) (the pattern counts W(G)
 * and D(G) in the running-time theorem of the paper's main-theorem
 * section); vals[6] = directed 3-paths i <- j <- k -> l walked by the
 * 5-cycle procedure (sum over k of d+(k) times the out-degrees of N+(k)).
 * Writes up to max_vals values and returns how many. */
int orbit_last_stats(uint64_t *vals, int max_vals);

#ifdef __cplusplus
}
#endif

#endif /* ORBIT_HIP_H */
