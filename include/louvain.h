/*
 * louvain.h -- C ABI of the MI355X (gfx950) synchronous parallel Louvain
 * library (liblouvain.so).
 *
 * Method: Lu, Halappanavar, Kalyanaraman, "Parallel heuristics for scalable
 * community detection".  The library runs the paper's parallel algorithm
 * (Sec. 5.4): optional vertex-following pre-merge (Sec. 5.3), optional
 * distance-1 coloring (Sec. 5.2), phases of synchronous local-moving
 * sweeps (Alg. 1) with the minimum-label heuristics (Sec. 5.1), and graph
 * rebuilding between phases; the coloring schedule and thresholds follow
 * Sec. 6.1.
 *
 * Graphs: undirected, integer edge weights >= 1 (Sec. 2), given as a
 * symmetric CSR: offsets int64[n+1] (offsets[0] = 0, offsets[n] = nnz),
 * cols int32[nnz] strictly ascending within each row (no multi-edges),
 * weights int32[nnz] or NULL for unit weights.  A self-loop (i,i) is stored
 * once and counts once in the degree k_i.  n < 2^31.
 *
 * Exactness: all arithmetic is integer.  Modularity (Eq. 3) is reported as
 * the exact rational N / D with D = (2m)^2 and N = 2m * (sum of CSR entries
 * inside communities) - sum_C a_C^2, plus its correctly rounded double.
 * Gains (Eq. 4) are compared as the integers G(c) = 2m*e_{i->c} - k_i*a_c.
 *
 * Conventions for every call:
 *  - Errors are status codes; nothing throws across the ABI.  A failed
 *    call leaves a message in louvain_last_error(g).  A HIP runtime error
 *    poisons the handle: afterwards only louvain_destroy is valid.
 *  - Work is ordered on the HIP stream given to louvain_init_csr (NULL = the
 *    null stream).  Calls that return host values synchronize that stream.
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - Device memory is owned by the handle and released by louvain_destroy.
 *  - Repeated launch sequences are captured once per phase as HIP graphs
 *    and replayed: by default the sweep stage of the batched form.  The
 *    environment variable LOUVAIN_HIP_GRAPHS, read when a handle is created,
 *    selects 0 (no capture), 1 (default) or 2 (also the colour classes of an
 *    iteration, which measured slightly slower than ordinary launches).
 *  - Lanes per vertex of the degree bins are autotuned: at the start of a
 *    phase, a bin of a kind and size not seen before in the process is swept
 *    once per candidate (without committing) and the fastest is kept for the
 *    process; LOUVAIN_AUTOTUNE=0 keeps the defaults and LOUVAIN_LANES=l1,l2,..
 *    fixes them for bins 1, 2, ...  Results do not depend on the choice.
 */
#ifndef LOUVAIN_H
#define LOUVAIN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct louvain_graph_s *louvain_graph_t;

typedef enum {
    LOUVAIN_OK = 0,
    LOUVAIN_E_INVALID_ARG = 1, /* null pointer, negative size, n >= 2^31, bad parameter */
    LOUVAIN_E_BAD_CSR = 2,     /* offsets, column range/order, weight < 1 or asymmetry */
    LOUVAIN_E_OOM = 3,         /* device allocation failed */
    LOUVAIN_E_HIP = 4,         /* HIP runtime error (handle poisoned) */
    LOUVAIN_E_OVERFLOW = 5,    /* 2m >= 2^62: gains could overflow the exact path */
    LOUVAIN_E_STATE = 6        /* call not valid in the handle's current state */
} louvain_status;

/* flags of louvain_init_csr */
#define LOUVAIN_DEVICE_PTRS 1u /* offsets/cols/weights are device pointers */
#define LOUVAIN_VALIDATE 2u    /* check the input contract (O(nnz log d) on device) */

typedef struct {
    int64_t num, den; /* threshold theta = num / den, num >= 0, den > 0 */
} louvain_ratio;

typedef struct {
    uint64_t lo; /* two's-complement 128-bit integer: value = hi * 2^64 + lo */
    int64_t hi;
} louvain_i128;

typedef struct {
    int32_t vf;                     /* vertex following before the first phase (Sec. 5.3): 0 none,
                                       1 single-degree vertices, 2 chain compression */
    int32_t color;                  /* coloring in early phases (Sec. 5.2, Sec. 6.1) */
    int32_t singlet_rule;           /* singlet minimum-label heuristic (Sec. 5.1) */
    int32_t threshold_mode;         /* 0: gain relative to |Q_prev|; 1: absolute gain */
    int32_t color_first_phase_only; /* color the first phase only (Table 4 variant) */
    int32_t max_iter;               /* iteration cap per phase */
    int32_t max_phases;             /* phase cap */
    int32_t color_balance;          /* balance the colour classes' sizes (1) or not (0) */
    louvain_ratio theta_color;      /* threshold while coloring (paper: 1e-2) */
    louvain_ratio theta_final;      /* threshold otherwise (paper: 1e-6) */
    int64_t color_cutoff;           /* color a phase only if it has >= this many vertices (100,000) */
    uint64_t color_seed;            /* coloring priority seed */
} louvain_params;

/* One synchronous iteration (Alg. 1 sweep + community totals + modularity). */
typedef struct {
    int64_t moves;      /* vertices whose community changed */
    louvain_i128 q_num; /* modularity numerator N of the partition after the iteration */
    int64_t pairs;      /* distinct (vertex, neighbouring community) pairs examined */
    int64_t entries;    /* CSR entries gathered */
    float ms;           /* device time of the iteration (0 unless profiling) */
    int32_t reserved;
} louvain_iter_stats;

typedef struct {
    int64_t n, nnz;          /* phase graph */
    int32_t colored;         /* phase ran colored sub-sweeps */
    int32_t num_colors;      /* colors used (0 if uncolored) */
    int32_t iterations;      /* iterations run in the phase (an undone one included) */
    int32_t hit_max_iter;    /* the iteration cap ended the phase */
    int32_t loss_undone;     /* the last iteration lowered Q and was undone (Sec. 5.1) */
    int32_t reserved;
    int64_t first_iter;      /* index of the phase's first record in louvain_result.iter */
    louvain_i128 q_num;      /* N at the end of the phase (after any undo) */
    double ms_color, ms_sweep, ms_coarsen;
} louvain_phase_stats;

typedef struct {
    int64_t n_orig;          /* input vertices */
    int64_t n_vf;            /* vertices after vertex following (= n_orig without it) */
    int64_t num_communities; /* K: labels are 0..K-1 */
    int64_t phases;
    int64_t iterations;      /* total over phases (records in iter) */
    louvain_i128 q_num, q_den, q0_num; /* final N, D = (2m)^2, singleton N of the first phase graph */
    double q;                /* correctly rounded N / D */
    int64_t sweep_entries;   /* CSR entries gathered by the sweeps of the iterations run */
    int64_t lookahead_entries; /* CSR entries gathered by look-ahead sweeps that only measured Q */
    int64_t vf_rounds;       /* rebuilds done by vertex following (chain mode: its rounds) */
    double ms_total, ms_vf, ms_color, ms_sweep, ms_coarsen; /* host wall-clock split */
    const louvain_phase_stats *phase; /* owned by the handle; valid until the next call */
    const louvain_iter_stats *iter;   /* owned by the handle; valid until the next call */
} louvain_result;

/* Fills the paper's defaults: baseline = minimum-label sweep with the
 * singlet rule, no VF, no coloring, theta_color = 1/100,
 * theta_final = 1/1000000, cutoff 100,000, max_iter 1000, max_phases 100. */
void louvain_params_default(louvain_params *p);

/*
 * Ingests a graph (Sec. 2, CSR as described above) and computes the weighted
 * degrees k_i and 2m.  The CSR is copied into handle-owned device memory;
 * the caller's buffers may be freed on return.  flags: LOUVAIN_DEVICE_PTRS,
 * LOUVAIN_VALIDATE.  On success *out is a handle at the first phase's
 * initial state (every vertex alone).  On failure *out is NULL and nothing
 * stays allocated; the message is available from louvain_last_error(NULL).
 */
louvain_status louvain_init_csr(int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols,
                                const int32_t *weights, uint32_t flags, void *hip_stream,
                                louvain_graph_t *out);

/*
 * Vertex following (Sec. 5.3): every vertex whose row is exactly one entry
 * (i, j), j != i, is merged into j (an isolated pair into its smaller id),
 * then the graph is rebuilt; the merged self-loop of j is w_jj + 2 w_ij so
 * that degrees, 2m and modularity are preserved.  Valid only on the input
 * graph before any sweep.  *n_new_out receives the new vertex count.
 */
louvain_status louvain_vf(louvain_graph_t g, int64_t *n_new_out);

/*
 * Chain-compressing vertex following (the extension closing Sec. 5.3):
 * rounds of the rule above for single-neighbour vertices (one neighbour
 * j != i besides an optional self-loop), each vertex merging only while the
 * bound in the proof of Lemma 3 stays positive, 2m * w_ij > k_i * k_j (the
 * exact gain of moving i into j's one-vertex community); each round rebuilds
 * the graph (the absorbed self-loops join the merged self-loop) and the
 * rounds repeat until no vertex qualifies.  Valid on the input graph before
 * any sweep.  *n_new_out: vertices after; *rounds_out (may be NULL): the
 * rounds that merged.
 */
louvain_status louvain_vf_chain(louvain_graph_t g, int64_t *n_new_out, int64_t *rounds_out);

/*
 * Distance-1 coloring of the current phase graph (Sec. 5.2) by
 * Jones-Plassmann rounds with priority pi(v) = SplitMix64 finalizer of
 * (seed << 32) ^ v; the result equals greedy coloring in descending
 * priority (self-loops ignored).  Subsequent louvain_sweep calls with
 * params->color != 0 process the color classes in ascending color until
 * the next louvain_coarsen.  *num_colors_out receives the class count.
 */
louvain_status louvain_color(louvain_graph_t g, uint64_t seed, int32_t *num_colors_out);

/*
 * Balanced colouring (Sec. 6.2 finds skewed colour classes costly and leaves
 * balanced sets to future work): after louvain_color, with chi colours on n
 * vertices and gamma = ceil(n / chi), the over-full classes (more than gamma
 * vertices) are taken in ascending colour c; in rounds, each waiting vertex of
 * K_c proposes the smallest colour c' != c that none of its neighbours has and
 * whose class holds fewer than gamma vertices (none: it stops waiting); each
 * c' takes its proposers in descending priority, at most gamma - |K_c'|, and of
 * all taken the first |K_c| - gamma in descending priority move; K_c is done at
 * gamma or after a round that moves nobody.  The colouring stays proper and
 * uses no new colour.  seed: the priority seed of the colouring.  At most 4096
 * colours (LOUVAIN_E_INVALID_ARG beyond).  *moved_out (may be NULL): vertices
 * that changed class.
 */
louvain_status louvain_color_balance(louvain_graph_t g, uint64_t seed, int64_t *moved_out);

/*
 * One synchronous iteration of Alg. 1 on the current phase graph: every
 * vertex (of each color class in turn, when colored) reads the communities
 * left by the previous iteration (class), gathers e_{i->c}, picks the
 * lexicographic max of (G(c), -c) over neighbouring communities c != C(i)
 * and moves iff G(c*) > G_stay = 2m*e_{i->C(i)\{i}} - k_i*(a_C(i) - k_i),
 * unless the singlet rule (params->singlet_rule) vetoes; then the community
 * degrees a_c are updated and the exact modularity numerator computed.
 * params is read for singlet_rule and color only.
 */
louvain_status louvain_sweep(louvain_graph_t g, const louvain_params *params, louvain_iter_stats *out);

/*
 * Graph rebuilding between phases (Sec. 3, Sec. 5.4 step 4): non-empty
 * communities are renumbered in ascending id, every CSR entry (u, v, w)
 * adds w to the coarse entry (C(u), C(v)), and the map from input vertices
 * to coarse vertices is composed.  The new graph starts with every vertex
 * alone.  *n_new_out receives the coarse vertex count.
 */
louvain_status louvain_coarsen(louvain_graph_t g, int64_t *n_new_out);

/*
 * The full method from the ingested input graph (any earlier step calls are
 * discarded): optional VF, then phases (colored while the schedule of
 * Sec. 6.1 allows), each iterated until an iteration loses modularity (that
 * iteration is undone: Sec. 5.1 continues a phase only on a net gain, and
 * Lemma 1 shows simultaneous moves can lose), a net gain below
 * theta * |Q_prev| (from the second iteration), no move, or max_iter, then
 * rebuilt; stops when a final-mode phase gains less than theta_final, does
 * not shrink the graph, or max_phases is reached.  labels_out receives
 * n_orig dense community labels 0..K-1 (host memory, or device memory if
 * labels_on_device != 0; may be NULL).  *out (may be NULL) receives the
 * summary; its arrays stay valid until the next call on g.
 */
louvain_status louvain_run(louvain_graph_t g, const louvain_params *params, int32_t *labels_out,
                           uint32_t labels_on_device, louvain_result *out);

/* Releases the handle and its device memory (NULL is a no-op). */
void louvain_destroy(louvain_graph_t g);

/* Size of the fixed device scratch of louvain_run_noalloc (64 MiB per GPU). */
#define LOUVAIN_NOALLOC_SCRATCH_BYTES (64ull << 20)

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * louvain_init_csr with device pointers followed by louvain_run, in one call
 * that makes no device allocation.  Every working buffer of the run is carved
 * from a fixed LOUVAIN_NOALLOC_SCRATCH_BYTES device array of the library; each
 * GPU the library runs on holds its own copy until the process ends.
 *   offsets, cols, weights: device CSR as in louvain_init_csr (weights NULL =
 *     unit); flags: 0 or LOUVAIN_VALIDATE.  labels_out: device int32[n] (may
 *     be NULL).  *out (may be NULL): as louvain_run; its phase and iter arrays
 *     stay valid until the next louvain_run_noalloc call of the same thread.
 * The result equals louvain_init_csr + louvain_run on the same input.  A graph
 * whose handle buffers (about 72 bytes per CSR entry plus 160 per vertex)
 * exceed the scratch is refused up front with LOUVAIN_E_INVALID_ARG; buffers
 * sized during the run (hub pair lists, colouring bitmaps) that no longer fit
 * end it with LOUVAIN_E_OOM.  Graphs of up to 65,536 vertices and 524,288 CSR
 * entries fit.  Errors are read with louvain_last_error(NULL).  All calls on
 * one GPU share its scratch, which keeps the last call's contents: calls that
 * overlap on one GPU (two threads, or two streams in flight) race and must
 * not be made.  The call synchronizes hip_stream before it returns.
 */
louvain_status louvain_run_noalloc(int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols,
                                   const int32_t *weights, uint32_t flags, const louvain_params *params,
                                   int32_t *labels_out, void *hip_stream, louvain_result *out);

/* Last error message of g (or of the last failed louvain_init_csr when g is
 * NULL); never NULL, "" when there was none. */
const char *louvain_last_error(louvain_graph_t g);

/* ---- state inspection (tests, tools) ---------------------------------- */

/* out[0..7] = n, nnz, 2m, n_orig, num_colors (0 if uncolored), weight kind
 * (0 unit, 1 int32, 2 int64), k_max, level (0 = input graph). */
louvain_status louvain_get_info(louvain_graph_t g, int64_t *out);

/* Current phase state: comm int32[n], a int64[n] (community degree by
 * community id), size int32[n] (members by id), k int64[n].  Any pointer may
 * be NULL.  Host buffers unless on_device != 0. */
louvain_status louvain_get_state(louvain_graph_t g, int32_t *comm, int64_t *a, int32_t *size, int64_t *k,
                                 uint32_t on_device);

/* Current phase graph: offsets int64[n+1], cols int32[nnz], weights as int64[nnz]
 * (expanded for unit and int32 inputs).  Any pointer may be NULL. */
louvain_status louvain_get_graph(louvain_graph_t g, int64_t *offsets, int32_t *cols, int64_t *weights,
                                 uint32_t on_device);

/* Color of each vertex of the current phase graph (after louvain_color). */
louvain_status louvain_get_colors(louvain_graph_t g, int32_t *color, uint32_t on_device);

/* Map from input vertices to current phase vertices: int32[n_orig]. */
louvain_status louvain_get_map(louvain_graph_t g, int32_t *orig_map, uint32_t on_device);

/* ---- measurement ------------------------------------------------------- */

/* Enables (1) or disables (0) per-launch HIP event timing of the hot kernels
 * on the handle's stream, and clears the accumulated records. */
louvain_status louvain_profile(louvain_graph_t g, int32_t enable);

/* Accumulated records, one per kernel family: idx in [0, count).  name is a
 * static string; launches, total device ms, and algorithmic bytes moved
 * (what the method must read and write, no over-fetch) over those launches.
 * Returns LOUVAIN_E_INVALID_ARG once idx >= count. */
louvain_status louvain_profile_get(louvain_graph_t g, int32_t idx, const char **name, int64_t *launches,
                                   double *total_ms, double *bytes, double *entries);

/* ---- batched form -------------------------------------------------------- */

/*
 * Many independent graphs in one handle, run together: the disjoint union is
 * given as one CSR whose vertex ids are global (graph g owns vertices
 * [graph_off[g], graph_off[g+1]) and no entry may leave its graph).  Every
 * sweep, update and rebuild kernel covers all graphs at once; each graph
 * keeps its own 2m and its own iteration and phase decisions, so each
 * graph's labels and statistics equal those of louvain_run on that graph
 * alone.  graph_off is a host array of num_graphs + 1 entries; the CSR
 * arrays follow louvain_init_csr (flags LOUVAIN_DEVICE_PTRS, LOUVAIN_VALIDATE).
 * The batched form runs uncolored phases (params->color must be 0).
 */
typedef struct louvain_batch_s *louvain_batch_t;

typedef struct {
    int64_t n, nnz;          /* the graph as given */
    int64_t num_communities; /* K: its labels are 0..K-1 */
    int64_t phases, iterations;
    louvain_i128 q_num, q_den, q0_num;
    double q;
    int64_t n_vf;
} louvain_graph_result;

louvain_status louvain_batch_init(int32_t num_graphs, const int64_t *graph_off, int64_t nnz, const int64_t *offsets,
                                  const int32_t *cols, const int32_t *weights, uint32_t flags, void *hip_stream,
                                  louvain_batch_t *out);

/* The same batch from separate host CSRs (graph i: n[i] vertices, nnz[i]
 * entries, offsets[i], cols[i], weights[i] or NULL, all in the layout of
 * louvain_init_csr with local vertex ids): the arrays are copied side by side
 * to device memory and renumbered there, so the caller needs no union CSR.
 * weights may be NULL (all unit) and any weights[i] may be NULL (unit).
 * flags: LOUVAIN_VALIDATE only. */
louvain_status louvain_batch_init_graphs(int32_t num_graphs, const int64_t *n, const int64_t *nnz,
                                         const int64_t *const *offsets, const int32_t *const *cols,
                                         const int32_t *const *weights, uint32_t flags, void *hip_stream,
                                         louvain_batch_t *out);

/* labels_out: graph_off[num_graphs] labels, local to each graph (may be NULL);
 * results: num_graphs records (may be NULL). */
louvain_status louvain_batch_run(louvain_batch_t b, const louvain_params *params, int32_t *labels_out,
                                 uint32_t labels_on_device, louvain_graph_result *results);

/* Per-phase and per-iteration records of one graph from the last batch run
 * (owned by the batch; valid until the next run or destroy). */
louvain_status louvain_batch_graph_stats(louvain_batch_t b, int32_t graph, const louvain_phase_stats **phases,
                                         int64_t *num_phases, const louvain_iter_stats **iters, int64_t *num_iters);

void louvain_batch_destroy(louvain_batch_t b);
const char *louvain_batch_last_error(louvain_batch_t b);

/* ---- served form --------------------------------------------------------- */

/*
 * A request loop with continuous batching: jobs (host CSRs, copied at submit,
 * or borrowed until they finish) queue in arrival order; a scheduler thread
 * admits a new batch whenever fewer than max_inflight_batches batches run and
 * the HBM budget covers its estimated device footprint (a large job at the
 * queue head alone, else the queued small jobs in order, passing large ones); each batch runs the batched form on its own
 * worker thread and HIP stream, so batches admitted at different times
 * overlap on the device, and memory returned by a finished batch admits the
 * next jobs.  A job of at least solo_min_vertices vertices is a batch of its
 * own and runs through louvain_init_csr + louvain_run.  Each job's result
 * equals the graph run alone.  A job larger than the whole budget fails with
 * LOUVAIN_E_OOM.  Uses the device current at louvain_server_create.
 */
typedef struct louvain_server_s *louvain_server_t;

typedef struct {
    uint64_t hbm_budget_bytes;     /* device memory the server may reserve (default 200 GiB) */
    int32_t max_inflight_batches;  /* concurrent batches / streams (default 4) */
    int32_t max_batch_graphs;      /* jobs per batch (default 4096) */
    int64_t max_batch_vertices;    /* vertices per batch, 0 = no limit */
    int64_t solo_min_vertices;     /* jobs this large run alone (default 100,000; 0 = never) */
} louvain_server_config;

typedef struct {
    louvain_graph_result result;
    int32_t status;                /* louvain_status of the job */
    int32_t reserved;
    double t_submit, t_admit, t_done; /* seconds since the server started */
    int64_t batch_id, batch_graphs;   /* the batch that ran the job and its size */
    double t_packed, t_ready;         /* its batch packed on the host / resident and checked on the device */
} louvain_job_result;

void louvain_server_config_default(louvain_server_config *cfg);
/* cfg may be NULL (defaults); params->color must be 0 */
louvain_status louvain_server_create(const louvain_server_config *cfg, const louvain_params *params,
                                     louvain_server_t *out);
/* host CSR in the layout of louvain_init_csr (weights NULL = unit), copied
 * before the call returns; offsets and column range are checked here
 * (LOUVAIN_E_BAD_CSR), order, weights and symmetry on the device when the job
 * runs (then the job's status is LOUVAIN_E_BAD_CSR) */
louvain_status louvain_server_submit(louvain_server_t s, int64_t n, int64_t nnz, const int64_t *offsets,
                                     const int32_t *cols, const int32_t *weights, uint64_t *ticket);
/* the same without the copy: the server reads the caller's arrays when the
 * job runs, so they must stay allocated and unchanged until poll reports the
 * job done (wait_all and destroy also wait for it); only offsets[0] and
 * offsets[n] are checked here, everything else on the device */
louvain_status louvain_server_submit_borrowed(louvain_server_t s, int64_t n, int64_t nnz, const int64_t *offsets,
                                              const int32_t *cols, const int32_t *weights, uint64_t *ticket);
/* *done = 1 once the job finished; then labels_out (n host entries, may be
 * NULL) and *out (may be NULL) are filled */
louvain_status louvain_server_poll(louvain_server_t s, uint64_t ticket, int32_t *labels_out, louvain_job_result *out,
                                   int32_t *done);
/* forgets a finished job */
louvain_status louvain_server_release(louvain_server_t s, uint64_t ticket);
/* blocks until every submitted job finished; LOUVAIN_E_HIP if a device error
 * occurred (an invalid job only fails itself: its batch is retried job by job) */
louvain_status louvain_server_wait_all(louvain_server_t s);
const char *louvain_server_last_error(louvain_server_t s);
/* waits for the submitted jobs, then stops the loop */
void louvain_server_destroy(louvain_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* LOUVAIN_H */
