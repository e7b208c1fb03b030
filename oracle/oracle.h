/*
 * CPU oracle for the k-clique-core densest-subgraph path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU baseline of the benchmark can check the GPU library's
 * results.  No product code may include, link or call it, and it shares no
 * code with the GPU library.  It is plain, single-threaded C99, written for
 * obviousness rather than speed; integers are exact (uint64 counts,
 * 128-bit intermediates, exact rational densities).
 *
 * Paper: Fang, Yu, Cheng, Lakshmanan, Lin, "Efficient Algorithms for Densest
 * Subgraph Discovery", PVLDB 12(11), 2019.
 *
 * Readings of points the paper leaves open (each one is also listed in the
 * design notes of the repository):
 *   - ties in "vertex with minimum clique-degree" (Alg. 3) are broken by id;
 *   - rho' of Pruning1 is the maximum density over the distinct core levels
 *     (the level sets R_k), which does not depend on removal order;
 *   - the components handed to the exact step are those of the
 *     (k'', Psi)-core (Alg. 4, line 3);
 *   - every "is there a subgraph denser than alpha" test is strict and reads
 *     the minimal minimum cut (vertices reachable from s in the residual
 *     network), which is what Lemma 14 characterises;
 *   - alpha lives on an integer grid p/Q so that capacities are integers;
 *   - CoreApp (Alg. 6): see orc_core_app;
 *   - PeelApp (Alg. 2) compares the residual graph before every step, G
 *     included, and keeps the first of equally dense ones: see orc_peel_app.
 */
#ifndef DSD_ORACLE_H
#define DSD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Simple undirected graph (Section 3, data model): rows sorted ascending,
 * no duplicates, no self-loops. */
typedef struct {
    int32_t n;
    int64_t m;        /* undirected edges */
    int64_t *off;     /* n + 1 */
    int32_t *adj;     /* 2m */
} orc_graph;

/* Returns NULL on an id outside [0, n) or n < 0. */
orc_graph *orc_graph_new(int32_t n, int64_t npairs, const int32_t *src, const int32_t *dst);
void orc_graph_free(orc_graph *g);
int32_t orc_graph_n(const orc_graph *g);
int64_t orc_graph_m(const orc_graph *g);
void orc_graph_adjacency(const orc_graph *g, int64_t *off, int32_t *adj);
/* Subgraph induced by mask[v] != 0, vertices relabelled in id order;
 * map[new] = old (map has room for n entries). */
orc_graph *orc_graph_induced(const orc_graph *g, const uint8_t *mask, int32_t *map);

/* Definition 3: deg[v] = number of h-clique instances containing v.
 * *mu = number of instances (Definition 4).  Returns 0, or -1 on h outside
 * [2, 8], -4 on uint64 overflow. */
int orc_clique_degrees(const orc_graph *g, int h, uint64_t *deg, uint64_t *mu);
/* Clique-degree of a single vertex: (h-1)-cliques inside its neighbourhood. */
int orc_clique_degree_of(const orc_graph *g, int h, int32_t v, uint64_t *deg);

/* Alg. 3, (k, Psi)-core decomposition: core[v] = clique-core number.
 * *kmax = max core.  Returns 0 or negative as above. */
int orc_core_decomposition(const orc_graph *g, int h, uint64_t *core, uint64_t *kmax);

/* Level table of the decomposition: for every distinct core value k (and
 * k = 0), rsize[i] = |R_k| and rmu[i] = mu(R_k), R_k = {v : core(v) >= k}.
 * levels/rsize/rmu have room for n + 1 entries; *nlevels is set. */
int orc_level_table(const orc_graph *g, int h, const uint64_t *core,
                    uint64_t *levels, uint64_t *rsize, uint64_t *rmu, int64_t *nlevels);

/* Alg. 5 (IncApp): member[v] = 1 iff core(v) == kmax; density as mu/|R|. */
int orc_inc_app(const orc_graph *g, int h, uint8_t *member, uint64_t *kmax,
                uint64_t *num, uint64_t *den);

/* Alg. 6 (CoreApp).  literal = 0: corrected reading (process W, then test the
 * stop rule, then double; peel a copy of W; start at max(k_l, kmax)).
 * literal = 1: the loop exactly as printed (stop test first, delete from W
 * itself, start at max(k_l, kmax + 1), double the post-peel |W|).
 * w0 <= 0 selects the default initial |W| = min(n, max(64, #{gamma = max})). */
int orc_core_app(const orc_graph *g, int h, int literal, int64_t w0,
                 uint8_t *member, uint64_t *kmax, uint64_t *num, uint64_t *den,
                 int64_t *iterations);

/* Alg. 2 (PeelApp).  A step removes vertices of minimum clique-degree from
 * the residual graph S (rounds = 0: the one of smallest id, as printed;
 * rounds = 1: all of them at once).  member marks the densest residual graph
 * seen before a step (G included; the first one on ties), num/den its
 * density; steps = number of steps, best_step = the step before which it was
 * seen (-1 and an empty member set when no residual graph holds a clique). */
int orc_peel_app(const orc_graph *g, int h, int rounds, uint8_t *member,
                 uint64_t *num, uint64_t *den, int64_t *steps, int64_t *best_step);

/* Special patterns (the appendix on core decomposition for special
 * patterns): pattern 1 = x-star (a centre with x >= 2 tails, x <= 8),
 * pattern 2 = 4-loop (a cycle on four vertices, the appendix's diamond;
 * x ignored).  Instances are subgraphs, not necessarily induced.
 * orc_pattern_degrees: deg[v] = instances containing v, *count = instances.
 * orc_pattern_core: Alg. 3 over pattern instances; core[v], *kmax.
 * Returns 0, -1 on bad arguments, -4 on overflow. */
int orc_pattern_degrees(const orc_graph *g, int pattern, int x, uint64_t *deg, uint64_t *count);
int orc_pattern_core(const orc_graph *g, int pattern, int x, uint64_t *core, uint64_t *kmax);

/* Pruning1/2 (Section 6.1): rho' = max level density, k' = ceil(rho');
 * components of R_{k'}; rho'' = max component density; k'' = max(k', ceil(rho'')).
 * label[v] = component id (>= 0) for v in R_{k'}, -1 otherwise. */
int orc_locate(const orc_graph *g, int h, const uint64_t *core,
               uint64_t *rho1_num, uint64_t *rho1_den, uint64_t *k1,
               uint64_t *rho2_num, uint64_t *rho2_den, uint64_t *k2,
               int32_t *label, int64_t *ncomp);

/* Exact CDS.  route 0: Alg. 1 (Exact) on the whole graph, binary search over
 * alpha with the (h-1)-clique network (h >= 3) or Goldberg's network (h = 2).
 * route 1: Alg. 4 (CoreExact) on the located components.
 * member marks the densest subgraph found; rho_opt = num/den reduced.
 * Returns 0, -1 on bad h, -4 on overflow. */
int orc_exact(const orc_graph *g, int h, int route, uint8_t *member,
              uint64_t *num, uint64_t *den, int64_t *flow_calls);

/* Densest subgraph that contains every vertex of q (nq >= 1 ids, repeats
 * allowed): member marks it, num/den its density (0/1 when no set containing
 * q holds a clique).  Minimum cuts of Alg. 1's network (Goldberg's for h = 2)
 * with q forced to the source side.  Returns 0, -1 on bad arguments. */
int orc_exact_query(const orc_graph *g, int h, int32_t nq, const int32_t *q, uint8_t *member,
                    uint64_t *num, uint64_t *den, int64_t *flow_calls);

/* Min-cut helper exposed for tests: strict test "is there a subgraph with
 * density > a/b", returns 1 and marks member if so, else 0. */
int orc_denser_than(const orc_graph *g, int h, uint64_t a, uint64_t b, uint8_t *member);

#ifdef __cplusplus
}
#endif
#endif
