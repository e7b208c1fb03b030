/*
 * libdsd -- k-clique-core densest-subgraph discovery on one AMD Instinct
 * MI355X (gfx950).  C ABI.
 *
 * Method: Fang, Yu, Cheng, Lakshmanan, Lin, "Efficient Algorithms for
 * Densest Subgraph Discovery", PVLDB 12(11), 2019.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every call returns a dsd_status; DSD_OK == 0.  No C++ exception crosses
 *    the ABI.  dsd_last_error() returns a thread-local message for the last
 *    failing call.
 *  - Psi is the h-clique, 2 <= h <= 6 (Definition 2 requires h >= 2; the paper
 *    evaluates h in [2, 6], Section 8).  Other h -> DSD_EINVAL.
 *  - Vertex ids are int32 in [0, n).  Outputs indexed by vertex use the
 *    caller's ids.
 *  - mem flags: DSD_MEM_HOST (0) means host memory; DSD_MEM_DEVICE (1) means
 *    device memory of the current HIP device (e.g. a torch tensor's
 *    data_ptr()).  Output buffers are caller-allocated, length n.
 *  - Every call is synchronous: on return the outputs are written, on the
 *    stream passed to dsd_build_csr (NULL = the null stream).
 *  - Counts are exact unsigned 64-bit integers; a count that would not fit
 *    returns DSD_EOVERFLOW.  Densities are exact reduced rationals num/den.
 *  - A graph without any h-clique has density 0/1 and an empty member set
 *    (also when n <= 1).
 *  - There is no CPU fallback: without a usable GPU every compute call
 *    returns DSD_EDEVICE.
 */
#ifndef DSD_H
#define DSD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DSD_OK = 0,
    DSD_EINVAL = -1,     /* bad argument: h outside [2,6], id outside [0,n), n < 0, NULL pointer */
    DSD_ENOMEM = -2,     /* device or host allocation failed */
    DSD_EDEVICE = -3,    /* HIP runtime error or no GPU */
    DSD_EOVERFLOW = -4,  /* a count or a scaled flow capacity would overflow 64 bits */
    DSD_EUNSUPPORTED = -5, /* graph shape beyond a documented limit: an out-neighbourhood above 2048
                              vertices for h >= 4, or an exact-step network above its limit (10^8
                              h-cliques for h >= 4; 2^31 residual arcs) */
    DSD_EBUSY = -6,       /* server: no free slot, or the request already runs */
    DSD_ETIMEDOUT = -7,   /* server: the request is not done within the wait */
    DSD_ECANCELED = -8    /* server: the request was cancelled */
} dsd_status;

enum { DSD_MEM_HOST = 0, DSD_MEM_DEVICE = 1 };

typedef struct dsd_graph_s *dsd_graph;

/* Exact density mu/|V| (Definition 4), reduced; 0/1 when there is no clique. */
typedef struct { uint64_t num, den; } dsd_rational;

/* Per-call timing and size statistics (all times in milliseconds, measured
 * with HIP events on the graph's stream).  Filled by every compute call when
 * the caller passes a non-NULL pointer to dsd_last_stats. */
typedef struct {
    double t_orient_ms, t_enum_ms, t_peel_ms, t_locate_ms, t_exact_ms, t_total_ms;
    uint64_t num_cliques;        /* mu(G, Psi) */
    uint64_t peel_rounds;        /* round-synchronous sub-rounds of the peel */
    uint64_t peel_levels;        /* distinct core values */
    uint64_t flow_calls;         /* min-cut computations of the exact step */
    uint64_t flow_nodes_max;     /* largest flow network built */
    uint64_t located_vertices;   /* vertices handed to the exact step */
    /* kernel families timed with HIP events on the graph's stream (whole-graph calls only):
     * k3 = clique-degree engine kernels, k4 = the peel (all of its kernels) */
    double k3_ms, k4_ms;
    uint64_t k3_launches, k4_launches;
    /* graph shape for the algorithmic byte model: n, m, the DAG's directed
     * 2-paths w2 = sum_v d-(v) d+(v) and s2 = sum_v deg(v) d+(v) */
    uint64_t n, m, w2, s2;
    /* host exact step: network construction and maximum-flow time */
    double t_flow_build_ms, t_flow_ms;
    /* the peel's main kernel: with dsd_set_kernel_timing on, every launch
     * timed on its own with HIP events (total time, launches; else 0); the
     * work it counted (pairs, nbrs) always.  Which kernel it was is
     * k4_main_kind:
     *   1  h = 2 edge pass: adjacency entries walked, frontier vertices;
     *   2  h = 3 triangle probe: out-list entries probed, neighbours expanded;
     *   3  h = 3 triangle lists: pairs walked, row items;
     *   4  x-star pattern frontier pass: adjacency entries walked, frontier vertices;
     *   5  4-loop pattern pass;
     *   6  h >= 4 arc discovery in the frontier vertices' neighbourhoods
     *      C_v: out-list entries probed, members of the sets C_v
     *      (k4_main_entries: row entries scanned to form them);
     *   0  none (h >= 4 with an out-list longer than 2048) */
    double k4_main_ms;
    uint64_t k4_main_launches, k4_main_pairs, k4_main_nbrs;
    /* minimum cuts of the exact step computed on the GPU (the others ran on
     * the host) */
    uint64_t flow_gpu_calls;
    uint64_t k4_main_kind;
    /* part of t_flow_ms: moving networks to the device (arcs up, residual CSR built there) */
    double t_flow_setup_ms;
    /* networks of the exact step built on the device (h = 3 components with
     * enough edges); the others were built on the host */
    uint64_t flow_gpu_networks;
    /* the peel's tail engine (h = 3 with triangle lists, and h = 2: one
     * workgroup takes every round once at most 16384 vertices are alive):
     * its time (HIP events around every launch, with dsd_set_kernel_timing
     * on; else 0), launches (one per peel that reaches it, one more after
     * every grid round), the row pairs it walked (each clique among the tail
     * vertices once per row) and the vertices it peeled */
    double k4_tail_ms;
    uint64_t k4_tail_launches, k4_tail_pairs, k4_tail_vertices;
    /* the tail's rounds whose frontier rows hold more than 2^18 pairs, which
     * the engine hands to a kernel on every CU: their time (HIP events, with
     * dsd_set_kernel_timing on; else 0), count and pairs */
    double k4_tail_grid_ms;
    uint64_t k4_tail_grid_rounds, k4_tail_grid_pairs;
    /* CoreExact's locate step (Section 6.1, Pruning1 and Pruning2), filled by
     * dsd_core_exact (else 0): rho' = the largest density mu(R_k)/|R_k| over
     * the level sets, k' = ceil(rho'); rho'' = the largest density of a
     * connected component of R_{k'}, of which there are locate_components;
     * k'' = max(k', ceil(rho'')); located_vertices above is |R_{k''}|, the
     * vertices handed to the exact search.  Densities as reduced num/den. */
    uint64_t locate_rho1_num, locate_rho1_den, locate_k1;
    uint64_t locate_rho2_num, locate_rho2_den, locate_k2;
    uint64_t locate_components;
    /* k4_main_kind 6: row entries the peel's main kernel scanned; the
     * second kernel of those rounds (the clique counting), timed like the
     * main kernel, and the 64-bit bitmap words it ANDed and counted at its
     * first level (all of its work for h = 4; counted with the kernel's work) */
    uint64_t k4_main_entries;
    double k4_main2_ms;
    uint64_t k4_main2_launches;
    uint64_t k4_main2_words;
} dsd_stats;

/*
 * Build a graph handle from raw vertex pairs (Section 3, data model: the graph
 * is undirected, unweighted and simple).  The pairs are copied, symmetrised,
 * and duplicates and self-loops dropped; the caller may free src/dst on
 * return.  The handle owns every device buffer until dsd_graph_free.
 * in_mem says where src/dst live.  stream: a hipStream_t or NULL.
 * Errors: DSD_EINVAL (n < 0, num_pairs < 0, NULL arrays with num_pairs > 0,
 * an id outside [0, n)), DSD_ENOMEM, DSD_EDEVICE.
 */
dsd_status dsd_build_csr(int32_t n, int64_t num_pairs, const int32_t *src, const int32_t *dst,
                         int in_mem, void *stream, dsd_graph *out);

/* n and the number of undirected edges after de-duplication. */
dsd_status dsd_graph_info(dsd_graph g, int32_t *n, int64_t *m);

/* Release the handle.  Its device memory goes to a process-wide cache of
 * chunks per device (at most 16 GiB), from which later handles draw before
 * they allocate; dsd_release_cache hands the cache back to the device.
 * NULL is accepted. */
dsd_status dsd_graph_free(dsd_graph g);

/* Free every cached chunk (memory of freed handles, kept for reuse) of every
 * device.  Handles still alive keep their own memory.  Always DSD_OK. */
dsd_status dsd_release_cache(void);

/*
 * Clique-degree (Definition 3): deg[v] = number of h-clique instances that
 * contain v; *num_cliques = mu(G, Psi) (Definition 4).  deg: length n,
 * residency out_mem.  num_cliques may be NULL.
 */
dsd_status dsd_clique_degrees(dsd_graph g, int h, int out_mem, uint64_t *deg,
                              uint64_t *num_cliques);

/*
 * dsd_clique_degrees for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same results, but the call allocates
 * nothing (no hipMalloc, hipFree or pinned host memory).  Its working memory
 * is one fixed device array of 112 MiB inside the library, which every GPU the
 * library runs on holds until the process ends.  The caller still passes the
 * output; the handle's CSR was allocated by dsd_build_csr.
 * Limit: n <= 2^22 vertices (DSD_EINVAL beyond).  Calls on one GPU share the
 * array: calls that overlap on one GPU (two threads, or two streams in
 * flight) race and must be serialised by the caller.  Every other error as
 * dsd_clique_degrees.
 */
dsd_status dsd_clique_degrees_noalloc(dsd_graph g, int h, int out_mem, uint64_t *deg,
                                      uint64_t *num_cliques);

/*
 * Launch tuning of the clique enumeration (the configuration of this
 * library's kernels, not a step of the method).  The enumeration bins DAG
 * roots into classes by out-degree, one launch each: h >= 4: class 0 up to
 * 64 (a wave per root), 1 up to 256, 2 up to 768, 3 up to 1,280 and 4 up to
 * 2,048 (workgroups with bitmaps in LDS for 1-2, in global memory for 3-4);
 * h = 3: class 0 up to 64, 1 up to 2,048, 2 larger.  Each launch's grid is
 * capped (workgroups loop over the class's roots).
 *
 * dsd_autotune times every class present in g's roots at h in [3, 6] under
 * a set of caps (the faster of two launches each), keeps the fastest cap per
 * (GPU architecture, h, class) in a process-wide table that every later
 * enumeration (single graphs, batches, peels' recounts) uses, and, with path
 * non-NULL, writes the table to that JSON file, merged over the entries the
 * file already holds: one flat object of "arch/hH/cC": cap pairs, e.g.
 * "gfx950/h4/c2": 1024.  out (capacity cap entries, may be NULL with cap 0)
 * receives one dsd_tune_result per measured class; *count (may be NULL) the
 * number of measured classes.  Results never depend on the caps.
 * dsd_tune_load replaces the table with a file's entries (path NULL: back
 * to the built-in caps); DSD_EINVAL for an unreadable or malformed file.
 * Without either call the environment variable DSD_TUNE_FILE, read once at
 * the first enumeration, names a file to load (a missing or malformed one
 * leaves the built-in caps).
 */
typedef struct {
    int32_t cls;          /* class (above) */
    int32_t roots;        /* roots in the class */
    int32_t cap_default;  /* built-in grid cap, workgroups */
    int32_t cap_best;     /* the fastest cap measured */
    double ms_default;    /* one launch of the class at the built-in cap, ms */
    double ms_best;       /* one launch at the chosen cap, ms */
} dsd_tune_result;

dsd_status dsd_autotune(dsd_graph g, int h, const char *path, int32_t cap, dsd_tune_result *out, int32_t *count);
dsd_status dsd_tune_load(const char *path);

/*
 * (k, Psi)-core decomposition (Definition 6, Algorithm 3): core[v] = the
 * clique-core number of v; *kmax = the largest one.  Computed by a
 * round-synchronous peel that removes every vertex of clique-degree <= k at
 * once.  core: length n, residency out_mem.  kmax may be NULL.
 */
dsd_status dsd_clique_core(dsd_graph g, int h, int out_mem, uint64_t *core, uint64_t *kmax);

/*
 * CoreApp (Algorithm 6): the (k_max, Psi)-core, which is a 1/h-approximation
 * of the densest subgraph (Lemma 8).  member[v] = 1 iff core(v) == k_max
 * (exactly the whole core, not a subset).  density = mu/|V| of that core.
 * member: length n bytes, residency out_mem.  kmax/density may be NULL.
 */
dsd_status dsd_core_app(dsd_graph g, int h, int out_mem, uint8_t *member, uint64_t *kmax,
                        dsd_rational *density);

/*
 * PeelApp (Algorithm 2): the densest residual graph of a peel by
 * clique-degree, a 1/h-approximation of the densest subgraph (Lemma 10).  A
 * round removes every vertex whose clique-degree in the residual graph S is
 * the smallest in S, with every h-clique through them (the 1/h argument
 * holds unchanged: the round that takes the first vertex of a densest
 * subgraph starts from an S whose minimum degree is at least rho_opt).  The
 * residual graph before every round, G itself included, is a candidate; of
 * equally dense ones the first (largest) is kept.
 *   member:     length n bytes, residency out_mem: 1 for the vertices of the
 *               answer (none when G holds no h-clique).
 *   density:    mu(S)/|S| of the answer, reduced; 0/1 when G has no h-clique.
 *   rounds:     rounds until S is empty.
 *   best_round: the round before which the answer was the residual graph
 *               (-1 when G has no h-clique).
 * density, rounds and best_round may be NULL.
 */
dsd_status dsd_peel_app(dsd_graph g, int h, int out_mem, uint8_t *member, dsd_rational *density,
                        int64_t *rounds, int64_t *best_round);

/*
 * CoreExact (Algorithm 4): the clique-densest subgraph (Problem 1).  The GPU
 * decomposes the graph, locates the densest subgraph with Pruning1 and
 * Pruning2 (Section 6.1), labels the components of the located core and
 * counts their h-cliques.  The search over alpha then visits those components
 * only, in descending density: each is tested at the best density found so
 * far and, while a denser set turns up, re-tested at that set's density (a
 * Dinkelbach iteration over the same minimum-cut tests as Algorithm 4's
 * binary search, on Algorithm 1's network, Goldberg's for h = 2).  A network
 * of at least 2^21 residual arcs gets its minimum cut on the GPU
 * (push-relabel), a smaller one on the host; the networks are built on the
 * host (h = 3 components of 8192 edges and more: on the GPU).
 * member[v] = 1 for the vertices of one densest subgraph; rho_opt its exact
 * density.  member: length n bytes, residency out_mem.  rho_opt may be NULL.
 * DSD_EUNSUPPORTED, after the locate step (whose figures dsd_last_stats then
 * holds), when a network would hold more than 10^8 h-cliques (about h arcs
 * each; DSD_EXACT_MAX_CLIQUES moves the limit) or more than 2^31 residual
 * arcs; the check counts before anything is built.
 */
dsd_status dsd_core_exact(dsd_graph g, int h, int out_mem, uint8_t *member,
                          dsd_rational *rho_opt);

/*
 * The densest subgraph that contains every vertex of a query set Q
 * (Section 6.3, the variant of the problem, here for h-cliques).  With x the
 * smallest clique-core number over Q, the (x, Psi)-core contains Q and has
 * density l >= x/h (Theorem 1); every densest set containing Q lies in the
 * (min(x, ceil(l)), Psi)-core, which the GPU locates; the host searches it
 * with minimum cuts of Algorithm 1's network (Goldberg's for h = 2) in which
 * Q is forced to the source side.
 *   q:      nq >= 1 caller ids in [0, n), host memory (repeats allowed).
 *   member: length n bytes, residency out_mem: 1 for the vertices of one
 *           densest set containing Q (Q itself, at density 0/1, when no set
 *           containing Q holds an h-clique).
 *   rho:    its density (may be NULL).
 * DSD_EINVAL for an empty query or an id outside [0, n); otherwise as
 * dsd_core_exact.
 */
dsd_status dsd_core_exact_query(dsd_graph g, int h, int32_t nq, const int32_t *q, int out_mem, uint8_t *member,
                                dsd_rational *rho);

/* ------------------------------------------------------------------ special patterns
 *
 * Pattern-degrees and (k, Psi)-cores for special patterns (the appendix on
 * core decomposition for special patterns; the (k, Psi)-core of a pattern is
 * the largest subgraph whose every vertex lies in >= k of its instances).
 * Instances are subgraphs, not necessarily induced. */
typedef enum {
    DSD_PATTERN_STAR = 1,  /* x-star: a centre joined to x tails, 2 <= x <= 8 */
    DSD_PATTERN_LOOP4 = 2  /* 4-loop: a cycle on four vertices (the appendix's
                              diamond: two 2-paths from a vertex to one other); x ignored */
} dsd_pattern;

/*
 * deg[v] = pattern instances containing v; *count = instances.  x-stars: a
 * pass over v's row, C(y, x) + sum over neighbours u of C(z_u - 1, x - 1)
 * (y, z_u degrees).  4-loops: sum over the vertices w two steps away of
 * C(c, 2), c the 2-paths from v to w, grouped in a table of v's 2-hop
 * neighbours.  deg: length n, residency out_mem; count may be NULL.
 * DSD_EINVAL for an unknown pattern or x outside [2, 8] (x-stars);
 * DSD_EOVERFLOW when a value could exceed 64 bits; DSD_EUNSUPPORTED when a
 * vertex's neighbours' degrees sum past 2^25 (4-loop tables).
 */
dsd_status dsd_pattern_degrees(dsd_graph g, int pattern, int x, int out_mem, uint64_t *deg, uint64_t *count);

/*
 * core[v] = the pattern-core number of v (round-synchronous peel over the
 * same closed form); *kmax = the largest.  core: length n, residency
 * out_mem; kmax may be NULL.  Errors as dsd_pattern_degrees.
 */
dsd_status dsd_pattern_core(dsd_graph g, int pattern, int x, int out_mem, uint64_t *core, uint64_t *kmax);

/* ------------------------------------------------------------------ batches
 *
 * dsd_batch_run runs one operation on many graphs at once and gives every
 * graph the result its single-graph entry point would give. */
typedef enum {
    DSD_OP_DEGREES = 0,   /* dsd_clique_degrees */
    DSD_OP_CORE = 1,      /* dsd_clique_core */
    DSD_OP_APP = 2,       /* dsd_core_app */
    DSD_OP_EXACT = 3,     /* dsd_core_exact */
    DSD_OP_PEEL = 4       /* dsd_peel_app */
} dsd_op;

/* Scalar outcome for one graph of a batch or one served request. */
typedef struct {
    dsd_status status;       /* this graph's outcome */
    int32_t h, op;
    uint64_t num_cliques;    /* mu(G, Psi) (Definition 4); 0 for DSD_OP_APP on a graph of
                                2^20 edges or more, where CoreApp runs alone (Algorithm 6
                                never counts the whole graph) */
    uint64_t kmax;           /* CORE, APP, EXACT: the largest clique-core number */
    dsd_rational density;    /* APP: density of the (k_max, Psi)-core; EXACT: rho_opt;
                                PEEL: density of the densest residual graph */
    uint64_t members;        /* APP, EXACT, PEEL: size of the member set */
    uint64_t peel_rounds;    /* rounds of the peel this graph took part in (PEEL: the
                                graph's own rounds, as dsd_peel_app reports them) */
    double t_ms;             /* wall time of the batch group that computed it */
} dsd_result;

/*
 * Graphs with the same h are enumerated and peeled together as one disjoint
 * union in which each graph keeps its own level: cliques never cross graphs,
 * so Definition 3 and the (k, Psi)-cores of Definition 6 hold graph by
 * graph, and the union needs as many peel rounds as its slowest graph
 * instead of their sum.  Every graph's decomposition is kept on its handle,
 * as a single-graph call would keep it.  DSD_OP_APP on a graph of 2^20
 * edges or more runs CoreApp's own top-down search (Algorithm 6) alone
 * instead, as dsd_core_app does.  DSD_OP_PEEL peels the union in
 * PeelApp's order (each graph removes its own minimum-degree vertices every
 * round) and keeps no decomposition.  DSD_OP_EXACT then runs the locate
 * steps and the host exact search of Algorithm 4 graph by graph, on up to 16
 * host threads.
 *   graphs: count distinct handles (a handle twice -> DSD_EINVAL).
 *   h:      count values in [2, 6].
 *   outs:   NULL, or count pointers, each NULL or an array of n_i entries:
 *           uint64_t for DEGREES (clique-degrees) and CORE (core numbers),
 *           uint8_t member flags for APP, EXACT and PEEL; residency out_mem.
 *   results: count entries, written for every graph.
 * Argument errors (DSD_EINVAL) are reported before any work.  Otherwise the
 * call returns DSD_OK when every graph succeeded, else the status of the
 * first graph that failed (its message in dsd_last_error); each graph's own
 * status is in its result.  Synchronous.
 */
dsd_status dsd_batch_run(int32_t count, const dsd_graph *graphs, const int *h, int op, int out_mem,
                         void *const *outs, dsd_result *results);

/* ------------------------------------------------------------------ serving
 *
 * Continuous batching.  A server owns worker threads (4, or
 * DSD_SERVER_WORKERS in [2, 16]), each with a non-blocking HIP stream of its
 * own.  A free worker takes the oldest queued request that fits the
 * device-memory budget left by running work and, when that request is on a
 * graph below 2^20 edges, every other queued small request with the same op
 * and h on a distinct graph that still fits; it runs that group through
 * dsd_batch_run on its stream (the group's handles are switched to it for
 * the run) and completes their tickets.  Requests that arrive while others
 * run therefore start as soon as a worker and budget are free, and the
 * groups of different workers overlap on the device.  A request on a larger
 * graph runs alone, and at most all workers but one hold such requests, so
 * small requests never wait behind large ones alone.  A request's footprint
 * is estimated as 160 bytes per vertex plus 192 bytes per edge (the peel's
 * buffers dominate); one that could never fit hbm_budget_bytes is refused at
 * submit with DSD_ENOMEM.  At most max_slots requests are queued or running
 * at once (DSD_EBUSY beyond).  A queued request may be overtaken by later
 * ones that fit while it does not. */
typedef struct dsd_server_s *dsd_server;

dsd_status dsd_server_create(size_t hbm_budget_bytes, int max_slots, dsd_server *out);

/* Queue op (a dsd_op) with h on g.  out: NULL, or n entries as in
 * dsd_batch_run, written before the ticket completes.  g must stay alive and
 * unused elsewhere until then.  *ticket identifies the request. */
dsd_status dsd_server_submit(dsd_server s, dsd_graph g, int h, int op, int out_mem, void *out, uint64_t *ticket);

/* Wait up to timeout_us microseconds (< 0: without limit) for a ticket.
 * DSD_OK: *out (may be NULL) holds the result and the ticket is released.
 * DSD_ETIMEDOUT: not done yet.  DSD_ECANCELED: it was cancelled (released).
 * DSD_EINVAL: unknown or already released ticket. */
dsd_status dsd_server_wait(dsd_server s, uint64_t ticket, int64_t timeout_us, dsd_result *out);

/* Cancel a request that has not started (DSD_OK); a started one runs to
 * its end (DSD_EBUSY). */
dsd_status dsd_server_cancel(dsd_server s, uint64_t ticket);

/* Cancel every queued request, finish the running group, stop the worker
 * and free the server.  NULL is accepted. */
dsd_status dsd_server_destroy(dsd_server s);

/* Statistics of the last compute call on g.  A handle keeps the core
 * decomposition of every h it has computed, so dsd_clique_core and
 * dsd_core_exact reuse it (their enumeration and peel figures then repeat
 * those of the call that computed it). */
dsd_status dsd_last_stats(dsd_graph g, dsd_stats *out);

/* With on != 0, later calls on g bracket every launch of the peel's main
 * kernel (the kernel named by k4_main_kind) with a pair of HIP events on the
 * graph's stream, and report their sum and count in k4_main_ms and
 * k4_main_launches; with on == 0 (the default) both stay 0.  A bracketed
 * launch costs the host some 20 microseconds, more than the round loop of
 * the peel spends on a round otherwise, so leave it off outside
 * measurements.  A decomposition already cached on g is not recomputed.
 * DSD_EINVAL: g is NULL. */
dsd_status dsd_set_kernel_timing(dsd_graph g, int on);

/* Human-readable name of a status; never NULL. */
const char *dsd_status_str(dsd_status s);

/* Message of the last failing call on this thread ("" if none). */
const char *dsd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
