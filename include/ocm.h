/*
 * ocm.h -- exact optimal cycle mean on one AMD Instinct MI355X (gfx950).
 *
 * The optimal cycle mean problem (Section 2.1, Definition "OCM problem"):
 * for a digraph G = (V, E) with integer edge weights w, the mean of a cycle is
 * its weight divided by its number of edges, and the minimum cycle mean is the
 * smallest mean over all cycles.  The maximum cycle mean (the worst sustainable
 * load of Sections 1 and 4) is minus the minimum over negated weights.
 *
 * The solver is Howard's policy iteration (Alg. 2, Section 2.5) decomposed
 * into data-parallel phases as in Section 3.1 (Alg. 3): policy improvement,
 * cycle detection in the one-successor policy graph, minimum-mean cycle
 * selection, rebuilding the policy graph around that cycle, and value
 * propagation from the cycle's smallest vertex.  All arithmetic is exact
 * (values scaled by the cycle length in int64, or in int128 once they leave
 * the int64 range; int128 comparisons of means), and
 * every choice the paper leaves open is fixed deterministically:
 *   - a vertex changes policy only on strict improvement, to the lowest CSR
 *     position attaining the best value;
 *   - cycles are ordered by mean, then by their smallest vertex index;
 *   - the source is the smallest vertex index on the chosen cycle;
 *   - vertices that cannot reach the chosen cycle through the policy are
 *     attached in breadth-first rounds, each taking its lowest-position edge
 *     into the set attached before the round.
 * Results therefore do not depend on scheduling: repeated calls return
 * identical bytes.
 *
 * Graph layout (Section 2.3, Fig. 2b): CSR.  row_ptr[n+1] holds the offset of
 * each vertex's first out-edge; col[m] holds edge targets ordered by source;
 * w[m] holds the weight of each edge in the same order (int32 or int64).
 * Edges are identified by their CSR position, so parallel edges and
 * self-loops are distinct.
 *
 * Memory: every array pointer is HIP device memory owned by the caller,
 * except ocm_result and ocm_profile, which are host memory.  Inputs are never
 * modified.  The library allocates no device memory in ocm_min / ocm_max: all
 * scratch space is the caller's workspace (see ocm_workspace_size).
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = null stream).
 * Every call enqueues its kernels on that stream and synchronises it before
 * returning (loop control reads small counters back to the host).  A cold
 * ocm_min / ocm_max on a graph of at least 131072 vertices also builds the
 * reverse CSR on a library-owned stream of the same device (created once,
 * default priority), ordered after the call's earlier work by an event; the
 * call waits for it before using it and before returning.
 *
 * Errors: functions return ocm_status; nothing aborts or throws across the
 * ABI.  ocm_last_error() returns a thread-local message for the last failure.
 * Calls are reentrant as long as concurrent calls use distinct workspaces.
 */
#ifndef OCM_H
#define OCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OCM_OK = 0,
    OCM_E_INVALID_ARG = -1,            /* null pointer, n < 1, m < 1, bad enum  */
    OCM_E_BAD_CSR = -2,                /* row_ptr not 0..m monotone, col outside [0,n) */
    OCM_E_NO_OUT_EDGE = -3,            /* a vertex without out-edges            */
    OCM_E_NOT_STRONGLY_CONNECTED = -4, /* some vertex cannot reach the chosen cycle */
    OCM_E_OVERFLOW = -5,               /* 2 n max|w| >= 2^62; or an int64 output
                                          (potential_out, ocm_phase_values,
                                          batched calls) cannot hold a value */
    OCM_E_CAPACITY = -6,               /* cycle_cap (or another cap) too small  */
    OCM_E_NOT_CONVERGED = -7,          /* max_iters reached with changes left   */
    OCM_E_WORKSPACE = -8,              /* workspace null or too small           */
    OCM_E_HIP = -9                     /* a HIP runtime call failed             */
} ocm_status;

enum { OCM_W_I32 = 0, OCM_W_I64 = 1 };

/* ocm_result.flags */
enum {
    OCM_F_TIE = 1u,            /* another critical cycle exists (exact test)   */
    OCM_F_TIE_UNCHECKED = 2u,  /* the uniqueness test was not run              */
    OCM_F_TIGHT_EDGES = 4u,    /* some non-policy edge is tight at the optimum */
    OCM_F_INT128 = 8u          /* values were carried in int128 (see below)    */
};

typedef struct {
    int64_t n, m;              /* 1 <= n, 1 <= m < 2^31                        */
    const int32_t *row_ptr;    /* device, n+1 entries                          */
    const int32_t *col;        /* device, m entries                            */
    const void *w;             /* device, m entries of int32 or int64          */
    int32_t wtype;             /* OCM_W_I32 or OCM_W_I64                       */
} ocm_graph;

typedef struct {
    int64_t p, q;              /* optimum = p/q, q >= 1, gcd(|p|, q) = 1       */
    int64_t cycle_len;         /* |C|, also set on OCM_E_CAPACITY              */
    int32_t source;            /* smallest vertex on C; C starts at its edge   */
    int32_t iterations;        /* policy-improvement sweeps, first and last included */
    uint32_t flags;            /* OCM_F_*                                      */
    int32_t connect_rounds;    /* breadth-first connect rounds, all iterations */
    int32_t jump_rounds;       /* pointer-jumping rounds, all iterations       */
    int32_t fast_iters;        /* iterations resolved by the fused fast path   */
    int64_t W, L;              /* unreduced optimum W/L: weight and length of C */
    int64_t tight_edges;       /* tight non-policy edges at the optimum        */
    int64_t push_frontier;     /* frontier vertices expanded by push rounds    */
    int64_t push_in_edges;     /* in-edges scanned by push rounds              */
    int32_t general_iters;     /* iterations that ran the cycle/select/rebuild phases */
    int32_t value_rounds;      /* pointer-jumping rounds of the value phases   */
} ocm_result;

/* Device time per kernel class, filled when ocm_options.profile is non-null
 * (hipEvents recorded around each launch on the call's stream). */
enum {
    OCM_K_VALIDATE = 0,   /* CSR validation and max |w|                      */
    OCM_K_SWEEP,          /* policy-improvement sweeps                       */
    OCM_K_TIESCAN,        /* tight-edge count at the optimum                 */
    OCM_K_CYCLES,         /* policy-graph cycles: init, jump rounds, final   */
    OCM_K_SELECT,         /* per-cycle sums and the minimum-mean select      */
    OCM_K_CONN_PULL,      /* rebuild: init and pull rounds                   */
    OCM_K_CONN_MARK,      /* rebuild: push-round marks                       */
    OCM_K_CONN_CLAIM,     /* rebuild: push-round claims                      */
    OCM_K_REVERSE,        /* reverse CSR build                               */
    OCM_K_VALUES,         /* value propagation after a rebuild               */
    OCM_K_FAST,           /* value propagation of the fast path              */
    OCM_K_RESULT,         /* cycle listing                                   */
    OCM_K_COUNT
};
typedef struct {
    double ms[OCM_K_COUNT];        /* summed kernel time per class             */
    int32_t launches[OCM_K_COUNT];
    double bytes[OCM_K_COUNT];     /* algorithmic bytes moved per class: each
                                      element the method reads or writes counted
                                      once at its size                        */
} ocm_profile;

typedef struct {
    int32_t max_iters;         /* 0 = unlimited                                */
    int32_t validate;          /* 1 = check the CSR on the device first        */
    int32_t schedule;          /* sweep schedule: 1..64 (power of two) lanes
                                  per vertex; 0 = vertex tiles with their
                                  edges staged in LDS (batched calls: lanes
                                  autotuned); same results either way          */
    int32_t tie_check;         /* 1 = run the exact uniqueness test of C       */
    int32_t fast_path;         /* 1 = fuse cycle/value phases while the critical
                                  cycle is unchanged (same results)            */
    int32_t connect_mode;      /* rebuild rounds: 0 = pick pull or push per
                                  round, 1 = pull only, 2 = push only (same
                                  results)                                     */
    int32_t tile;              /* batched calls: vertices per work chunk,
                                  512..4096, 0 = autotuned                     */
    const int32_t *init_policy;/* device int32[n] or NULL: warm start.  The
                                  given policy (one out-edge position per
                                  vertex) replaces the first sweep; the optimum
                                  is the same, the trajectory (and, with ties,
                                  the cycle) may differ.  An entry outside its
                                  vertex's edge range gives OCM_E_INVALID_ARG. */
    int32_t *policy_out;       /* device int32[n] or NULL: final policy (edge positions) */
    int64_t *potential_out;    /* device int64[n] or NULL: final values scaled by L.
                                  If they do not all fit int64 (OCM_F_INT128
                                  solves only) the call fills the result and
                                  returns OCM_E_OVERFLOW.                      */
    ocm_profile *profile;      /* host, or NULL                                */
    int32_t int128_values;     /* 0: values in int64 until one would leave
                                  [-2^62, 2^62], then int128 for the rest of
                                  the solve; 1: int128 from the start.  Same
                                  results either way (OCM_F_INT128 says which
                                  ran).                                         */
    int32_t multichain;        /* 0: Alg. 2 (one gain; the rebuild attaches
                                  every vertex to C).  1: multichain policy
                                  iteration, an alternative not in the paper:
                                  every policy cycle keeps its own gain W_r/L_r,
                                  a vertex's value is scaled by the length of
                                  the cycle it reaches, and the sweep compares
                                  (gain, bias) pairs; no rebuild.  Same optimum;
                                  its own trajectory and, among tied cycles, its
                                  own C (the policy cycle of smallest gain, then
                                  smallest vertex); potential_out holds those
                                  per-cycle scaled values.  ocm_min / ocm_max /
                                  ocm_min_noalloc only, without init_policy or
                                  int128_values; values stay int64 (one beyond
                                  2^62 gives OCM_E_OVERFLOW).                    */
} ocm_options;

/* Fills *o with the defaults: max_iters 0, validate 1, schedule 0,
 * tie_check 1, fast_path 1, connect_mode 0, no outputs, no profile. */
void ocm_default_options(ocm_options *o);

/* Bytes of workspace ocm_min / ocm_max / ocm_* phases need for this graph
 * (about 120 bytes per vertex plus 8 per edge).  Returns 0 on invalid input. */
size_t ocm_workspace_size(const ocm_graph *g, const ocm_options *o);

/* Minimum cycle mean (Definition "OCM problem", Section 2.1) by policy
 * iteration (Alg. 2, Alg. 3).  The graph must be strongly connected for a
 * guaranteed answer (Section 2.5); otherwise the call either returns the
 * optimum (still exact) or OCM_E_NOT_STRONGLY_CONNECTED.
 *   ws, ws_bytes   device workspace of at least ocm_workspace_size bytes;
 *   cycle_edges    device int32[cycle_cap]: receives C as CSR edge positions
 *                  in traversal order, starting with the edge leaving source;
 *   out            host result.
 * o may be NULL (defaults). */
ocm_status ocm_min(const ocm_graph *g, const ocm_options *o, void *ws,
                   size_t ws_bytes, int32_t *cycle_edges, int64_t cycle_cap,
                   ocm_result *out, void *stream);

/* Maximum cycle mean: minus the minimum over negated weights, with the same
 * rules (so the same cycle and iteration count as ocm_min on -w). */
ocm_status ocm_max(const ocm_graph *g, const ocm_options *o, void *ws,
                   size_t ws_bytes, int32_t *cycle_edges, int64_t cycle_cap,
                   ocm_result *out, void *stream);

/* Optimal cycle ratio (Section 2.2: every transition carries a cost and a
 * time, and the ratio of a cycle is its total cost over its total time; the
 * (v, w, t) edge record of Fig. 2).  The same policy iteration with
 * lambda = W / T (cost and time of the chosen cycle) and edge values
 * V[head] + T * w - W * t; the cycle mean is the case t = 1.
 *   t        device int32[m]: the time of each edge (CSR order), >= 1, so
 *            every cycle has positive time (OCM_E_INVALID_ARG otherwise);
 *   out      p/q = the optimal ratio in lowest terms; W and L are the
 *            critical cycle's cost and time; cycle_len its number of edges.
 * Values stay exact under 2 n max|w| max t < 2^62 (OCM_E_OVERFLOW beyond);
 * the workspace is ocm_workspace_size's.  Other arguments as ocm_min.
 * ocm_ratio_max is the maximum: minus the minimum over negated costs. */
ocm_status ocm_ratio_min(const ocm_graph *g, const int32_t *t, const ocm_options *o, void *ws,
                         size_t ws_bytes, int32_t *cycle_edges, int64_t cycle_cap,
                         ocm_result *out, void *stream);
ocm_status ocm_ratio_max(const ocm_graph *g, const int32_t *t, const ocm_options *o, void *ws,
                         size_t ws_bytes, int32_t *cycle_edges, int64_t cycle_cap,
                         ocm_result *out, void *stream);

/* Graphs that are not strongly connected (Prop. 2.2; Section 2.5 names the
 * decomposition into strongly connected components as the alternative to
 * augmenting the graph with a Hamiltonian cycle).  Every cycle lies inside
 * one component, so the optimum is the best optimum among the components
 * that hold a cycle.  The components are found on the device; those holding
 * a cycle (two or more vertices, or a self-loop) are solved together as a
 * batch (concurrent regions, Section 3.3).
 *   - vertices may have no out-edge; the graph must hold a cycle
 *     (OCM_E_NOT_STRONGLY_CONNECTED otherwise);
 *   - each component is solved with the rules of ocm_min on its own
 *     vertices, numbered in increasing original index, and its own edges in
 *     original CSR order; the result comes from the best component, ties to
 *     the one with the smallest vertex index;
 *   - out: p/q, W, L, the cycle (original CSR positions, from its smallest
 *     vertex), source (original vertex), iterations and flags of that
 *     component's solve; OCM_F_TIE also when another component reaches the
 *     same optimum; tight_edges = -1 (not counted);
 *   - *components (may be NULL): the number of components holding a cycle;
 *   - ws: ocm_general_workspace_size(g) bytes; o->init_policy, policy_out,
 *     potential_out and profile must be NULL. */
size_t ocm_general_workspace_size(const ocm_graph *g);
ocm_status ocm_min_general(const ocm_graph *g, const ocm_options *o, void *ws, size_t ws_bytes,
                           int32_t *cycle_edges, int64_t cycle_cap, ocm_result *out,
                           int64_t *components, void *stream);
ocm_status ocm_max_general(const ocm_graph *g, const ocm_options *o, void *ws, size_t ws_bytes,
                           int32_t *cycle_edges, int64_t cycle_cap, ocm_result *out,
                           int64_t *components, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ocm_min
 * without a caller workspace.  Its scratch is a library-owned device array of
 * OCM_NOALLOC_SCRATCH_BYTES (256 MiB) per GPU, part of the library's code
 * object: every GPU the library is loaded on holds it until the process ends.
 * Its address is looked up once per device (hipGetSymbolAddress), on the
 * first call with that device current.
 *   - Same arguments and results as ocm_min, minus the workspace; the caller
 *     still owns the graph, cycle_edges and out.
 *   - A graph whose workspace (ocm_workspace_size) exceeds the array gives
 *     OCM_E_WORKSPACE with the sizes in ocm_last_error(); o->profile must be
 *     NULL (OCM_E_INVALID_ARG).
 *   - The call allocates no device memory and no pinned host memory, creates
 *     no stream or event (control reads are synchronous copies into the
 *     calling thread's stack) and calls no hipMalloc / hipFree.  The
 *     uniqueness test's small host-side special-vertex graph, when that test
 *     needs it, lives on the host heap.
 *   - All calls on one GPU share that GPU's array, which keeps the last
 *     call's contents (the solver initialises everything it reads).  Calls
 *     on one device from threads of this process are serialised by a
 *     per-device lock, and each call synchronises `stream` before returning;
 *     work that another caller enqueues on the same array outside this entry
 *     point would race with it. */
#define OCM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
ocm_status ocm_min_noalloc(const ocm_graph *g, const ocm_options *o, int32_t *cycle_edges,
                           int64_t cycle_cap, ocm_result *out, void *stream);

/* ---------------------------------------------------------------------- */
/* Single phases of one policy-iteration step (Alg. 3), on caller arrays.  */
/* They share the workspace layout of ocm_min and exist so that each phase */
/* can be driven from a recorded state.  neg = 1 negates the weights.      */
/* ---------------------------------------------------------------------- */

/* Policy improvement sweep (Alg. 2 main loop; SPFPassIter of Alg. 3).  For
 * every vertex v: best = min over out-edges e = v->u of V[u] + L*w(e) - W,
 * taken at the lowest position; if first != 0 (pi = nil, V = 0, lambda = 0)
 * or best < V[v], pi[v] <- that position.  V may be NULL when first != 0.
 * *changed receives the number of vertices whose policy was written. */
ocm_status ocm_phase_sweep(const ocm_graph *g, int32_t neg, int32_t first,
                           const int64_t *V, int64_t W, int64_t L,
                           int32_t *pi, int32_t schedule, void *ws,
                           size_t ws_bytes, int64_t *changed, void *stream);

/* Policy-graph cycles (GpiPreprocess, elimination and cycleIdentification
 * of Alg. 3).  rep[v] = smallest vertex index on the cycle that v's policy
 * path enters; on_cycle[v] = 1 for cycle vertices.  *ncycles = cycles. */
ocm_status ocm_phase_cycles(const ocm_graph *g, const int32_t *pi,
                            int32_t *rep, uint8_t *on_cycle, void *ws,
                            size_t ws_bytes, int64_t *ncycles, void *stream);

/* Minimum-mean cycle (reduce_min, setMinCycle): among cycles of the policy
 * graph the smallest W/L, ties to the smallest rep.  s = that rep. */
ocm_status ocm_phase_select(const ocm_graph *g, int32_t neg, const int32_t *pi,
                            const int32_t *rep, const uint8_t *on_cycle,
                            void *ws, size_t ws_bytes, int32_t *s, int64_t *W,
                            int64_t *L, void *stream);

/* Rebuild (markMinComponent, connectGpi): vertices with rep == s keep pi
 * (layer 0); the others are attached in rounds k = 1, 2, ... (layer k).
 * *rounds = number of rounds; OCM_E_NOT_STRONGLY_CONNECTED if stuck. */
ocm_status ocm_phase_connect(const ocm_graph *g, const int32_t *rep, int32_t s,
                             int32_t *pi, int32_t *layer, void *ws,
                             size_t ws_bytes, int32_t *rounds, void *stream);

/* Value propagation (val[source] <- 0, valuePropagate of Alg. 4):
 * V[s] = 0 and V[v] = V[succ v] + L*w(pi v) - W over the policy tree cut at
 * s.  OCM_E_OVERFLOW if a value leaves [-2^62, 2^62]. */
ocm_status ocm_phase_values(const ocm_graph *g, int32_t neg, const int32_t *pi,
                            int32_t s, int64_t W, int64_t L, int64_t *V,
                            void *ws, size_t ws_bytes, int32_t *rounds,
                            void *stream);

/* ---------------------------------------------------------------------- */
/* Batched graphs: concurrent regions (Section 3.3, Alg. 5).               */
/* ---------------------------------------------------------------------- */

/* G independent graphs given as one disjoint-union CSR `u` (global vertex
 * ids): graph g owns vertices [vptr[g], vptr[g+1]) and edges [eptr[g],
 * eptr[g+1]) and no edge may leave its graph.  vptr and eptr are HOST
 * arrays of G+1 entries (vptr[0] = eptr[0] = 0, vptr[G] = n, eptr[G] = m,
 * every graph with >= 1 vertex and edge).  Every graph is solved with the
 * rules of ocm_min / ocm_max, concurrently: each keeps its own lambda, its
 * own minimum-mean vote and its own termination (finished graphs are retired
 * from all further kernels), so graph g's result equals ocm_min on graph g
 * alone (Prop. 2.2 makes min_g p_g/q_g the optimum of the union).
 *   p, q, iters, flags, status   HOST arrays of G entries (status: OCM_OK or
 *                                the graph's own error; may be NULL);
 *   cycle_ptr                    HOST array of G+1 entries: graph g's cycle
 *                                is cycle_edges[cycle_ptr[g] .. cycle_ptr[g+1]);
 *   cycle_edges                  DEVICE int32[cycle_cap] (<= n entries needed):
 *                                CSR positions in the union, from each
 *                                graph's source.
 * The uniqueness test runs the exact quick tests only; a graph they cannot
 * decide gets OCM_F_TIE_UNCHECKED.  o->init_policy must be NULL.  Returns
 * OCM_OK, the first failing graph's status, or a call-wide error. */
size_t ocm_batched_workspace_size(int64_t G, const int64_t *vptr, const int64_t *eptr,
                                  const ocm_graph *u, const ocm_options *o);
ocm_status ocm_min_batched(int64_t G, const int64_t *vptr, const int64_t *eptr,
                           const ocm_graph *u, const ocm_options *o, void *ws, size_t ws_bytes,
                           int64_t *p, int64_t *q, int64_t *cycle_ptr, int32_t *cycle_edges,
                           int64_t cycle_cap, int32_t *iters, uint32_t *flags, int32_t *status,
                           void *stream);
ocm_status ocm_max_batched(int64_t G, const int64_t *vptr, const int64_t *eptr,
                           const ocm_graph *u, const ocm_options *o, void *ws, size_t ws_bytes,
                           int64_t *p, int64_t *q, int64_t *cycle_ptr, int32_t *cycle_edges,
                           int64_t cycle_cap, int32_t *iters, uint32_t *flags, int32_t *status,
                           void *stream);

/* The schedule the last batched call on this thread used: sweep lanes per
 * vertex, chunk size, and whether it was timed now (1) or taken from the
 * autotuner's per-size-class cache (0).  The batched loop runs its first
 * iteration as two captured hipGraphs around host-driven rebuild rounds and
 * every later iteration as one captured hipGraph (device-driven rounds, one
 * host read per iteration); setting the environment variable
 * OCM_BATCH_GRAPH=0 enqueues the same kernels directly. */
void ocm_batched_last_schedule(int32_t *lanes, int32_t *tile, int32_t *tuned);

/* ---------------------------------------------------------------------- */
/* Differentiation (not in the paper).  Away from ties the optimum is a    */
/* smooth function of w with d(optimum)/d(w_e) = 1/|C| for the edges of   */
/* the critical cycle C and 0 for every other edge (the same holds for the */
/* maximum).                                                               */
/* ---------------------------------------------------------------------- */

/* Converts float64 weights to int64 on the device.  Every weight must be an
 * integer with |w| < 2^53, else OCM_E_INVALID_ARG.  ws: >= 256 bytes of
 * device scratch.  Synchronises `stream`. */
ocm_status ocm_weights_from_f64(int64_t m, const double *w_f64, int64_t *w_i64, void *ws,
                                size_t ws_bytes, void *stream);

/* Adjoint scatter: grad_w[e] = *grad_out / cycle_len for the cycle_len edge
 * positions in cycle_edges, 0 for every other e < m (zero-filled first).
 * grad_out points to one double in device memory (the incoming gradient), so
 * the call does not synchronise; the quotient is one correctly rounded IEEE
 * division. */
ocm_status ocm_adjoint_scatter(int64_t m, const int32_t *cycle_edges, int64_t cycle_len,
                               const double *grad_out, double *grad_w, void *stream);

const char *ocm_status_string(ocm_status s);
const char *ocm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* OCM_H */
