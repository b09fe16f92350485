/*
 * CPU oracle for the optimal (minimum / maximum) cycle mean.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the HIP path against a plain, slow,
 * obviously correct implementation.  It shares no code with the HIP path.
 *
 * Paper: Barnat, Bauch, Brim, Ceska, "Computing Optimal Cycle Mean in Parallel
 * on CUDA" (PDMC 2011).
 *
 * Contents
 *   orc_karp      Karp's characterisation of the minimum cycle mean (value
 *                 only).  Not in the paper; an independent exact pin.
 *   orc_solve     Sequential Howard policy iteration, Alg. 2 of Section 2.5,
 *                 with the tie-breaking readings listed below, in int128.
 *   orc_state_*   The same iteration exposed phase by phase, so that each GPU
 *                 phase can be fed the oracle's state and compared with the
 *                 oracle's next state.
 *   orc_certify   O(m) optimality certificate: a cycle of mean lambda plus a
 *                 potential feasible for w - lambda (Prop. 2.1 and the LP of
 *                 Eq. (1), Section 2.4) prove lambda is the optimum.
 *   *_ratio       The optimal cycle ratio (Section 2.2: every transition
 *                 carries a cost w and a time t, and the ratio of a cycle is
 *                 its cost over its time), by the same policy iteration with
 *                 lambda = W / T and edge values T * w - W * t; the cycle mean
 *                 is the case t = 1 on every edge.  Times are integers >= 1,
 *                 so every cycle has positive time.
 *
 * Readings where the paper leaves a choice open (Alg. 2 and Section 3.1):
 *   R1  the initial policy (pi = nil, val = 0, lambda = 0) picks, per vertex,
 *       the lowest CSR position among its minimum-weight out-edges;
 *   R2  a vertex changes its policy edge only when the current edge's value
 *       exceeds the best value strictly, and then takes the lowest CSR
 *       position attaining the best value;
 *   R3  among policy-graph cycles the one with the smallest mean is chosen,
 *       ties broken by the smallest minimum vertex index;
 *   R4  the source s is the smallest vertex index on the chosen cycle C;
 *   R5  vertices whose policy path reaches C keep their policy edge;
 *   R6  the other vertices are connected in breadth-first rounds: in round k
 *       every unconnected vertex with an out-edge into the set connected
 *       before round k takes the lowest-position such edge;
 *   R7  values are kept scaled by L = |C|: V(s) = 0 and
 *       V(v) = V(succ v) + L * w(pi v) - W with W = sum of w over C;
 *   R8  iteration stops at the first sweep after the first one that changes
 *       nothing; the iteration count is the number of sweeps;
 *   R9  the result is W/L in lowest terms with a positive denominator, and
 *       the cycle is listed as CSR edge positions starting with pi(s);
 *   R10 the maximum is minus the minimum over negated weights.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

enum {
    ORC_OK = 0,
    ORC_E_INVALID_ARG = -1,
    ORC_E_BAD_CSR = -2,
    ORC_E_NO_OUT_EDGE = -3,
    ORC_E_NOT_STRONGLY_CONNECTED = -4,
    ORC_E_OVERFLOW = -5,
    ORC_E_CAPACITY = -6,
    ORC_E_NOT_CONVERGED = -7,
    ORC_E_NOMEM = -10,
    ORC_E_CERT_CYCLE = -20,
    ORC_E_CERT_MEAN = -21,
    ORC_E_CERT_POTENTIAL = -22
};

static int64_t gcd64(int64_t a, int64_t b)
{
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b) { int64_t t = a % b; a = b; b = t; }
    return a;
}

/* Checks the CSR shape of Fig. 2b: offsets start at 0, never decrease, end
 * at m; every target is a vertex; every vertex has an out-edge. */
static int check_csr(int64_t n, int64_t m, const int32_t *row_ptr,
                     const int32_t *col)
{
    if (n < 1 || m < 1) return ORC_E_INVALID_ARG;
    if (row_ptr[0] != 0 || (int64_t)row_ptr[n] != m) return ORC_E_BAD_CSR;
    for (int64_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return ORC_E_BAD_CSR;
    for (int64_t e = 0; e < m; ++e)
        if (col[e] < 0 || (int64_t)col[e] >= n) return ORC_E_BAD_CSR;
    for (int64_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] == row_ptr[v]) return ORC_E_NO_OUT_EDGE;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Karp: with D_k(v) the least weight of a k-edge walk from vertex 0 to v,   */
/* the minimum cycle mean of a strongly connected graph is                   */
/*   min over v with D_n(v) finite of                                       */
/*   max over k < n with D_k(v) finite of (D_n(v) - D_k(v)) / (n - k).      */
/* Two passes keep memory at O(n): the first finds D_n, the second recomputes*/
/* D_0 .. D_{n-1} and keeps, per v, the largest ratio.                       */
/* ------------------------------------------------------------------------ */
#define INF64 INT64_MAX

static void karp_step(int64_t n, const int32_t *row_ptr, const int32_t *col,
                      const int64_t *w, const int64_t *prev, int64_t *next)
{
    for (int64_t v = 0; v < n; ++v) next[v] = INF64;
    for (int64_t u = 0; u < n; ++u) {
        if (prev[u] == INF64) continue;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int64_t c = prev[u] + w[e];
            if (c < next[col[e]]) next[col[e]] = c;
        }
    }
}

int orc_karp(int64_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
             const int64_t *w, int64_t *p_out, int64_t *q_out)
{
    int rc = check_csr(n, m, row_ptr, col);
    if (rc) return rc;
    int64_t *a = malloc(sizeof(int64_t) * n), *b = malloc(sizeof(int64_t) * n);
    int64_t *dn = malloc(sizeof(int64_t) * n);
    int64_t *bn = malloc(sizeof(int64_t) * n), *bd = malloc(sizeof(int64_t) * n);
    if (!a || !b || !dn || !bn || !bd) { rc = ORC_E_NOMEM; goto out; }

    for (int64_t v = 0; v < n; ++v) a[v] = INF64;
    a[0] = 0;
    for (int64_t k = 1; k <= n; ++k) {
        karp_step(n, row_ptr, col, w, a, b);
        int64_t *t = a; a = b; b = t;
    }
    memcpy(dn, a, sizeof(int64_t) * n);

    /* bn/bd: the best (largest) ratio seen so far for v; bd == 0 = none. */
    for (int64_t v = 0; v < n; ++v) { bn[v] = 0; bd[v] = 0; }
    for (int64_t v = 0; v < n; ++v) a[v] = INF64;
    a[0] = 0;
    for (int64_t k = 0; k < n; ++k) {
        for (int64_t v = 0; v < n; ++v) {
            if (dn[v] == INF64 || a[v] == INF64) continue;
            int64_t num = dn[v] - a[v], den = n - k;
            if (bd[v] == 0 || (i128)num * bd[v] > (i128)bn[v] * den) {
                bn[v] = num; bd[v] = den;
            }
        }
        karp_step(n, row_ptr, col, w, a, b);
        int64_t *t = a; a = b; b = t;
    }
    int64_t pn = 0, pd = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (dn[v] == INF64 || bd[v] == 0) continue;
        if (pd == 0 || (i128)bn[v] * pd < (i128)pn * bd[v]) { pn = bn[v]; pd = bd[v]; }
    }
    if (pd == 0) { rc = ORC_E_NOT_STRONGLY_CONNECTED; goto out; }
    int64_t g = gcd64(pn, pd);
    *p_out = pn / g;
    *q_out = pd / g;
    rc = ORC_OK;
out:
    free(a); free(b); free(dn); free(bn); free(bd);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Sequential policy iteration (Alg. 2).                                    */
/* ------------------------------------------------------------------------ */
typedef struct orc_state {
    int64_t n, m;
    const int32_t *row_ptr, *col;
    int64_t *w;          /* weights, negated for the maximum (R10) */
    int64_t *t;          /* times (ratio problem), NULL = 1 on every edge */
    int64_t clen;        /* number of edges of the chosen cycle */
    int32_t *src;        /* source vertex of every edge */
    /* backward adjacency: for every vertex x, the edges entering x */
    int64_t *in_ptr;
    int32_t *in_edge;
    /* Howard state */
    int32_t *pi;         /* policy: CSR position of the chosen out-edge, -1 = nil */
    i128 *val;           /* V, scaled by L */
    int64_t W, L;        /* lambda = W / L, unreduced (L = time of C for a ratio) */
    int32_t s;           /* source vertex */
    int32_t iter;        /* sweeps done */
    /* cycle phase outputs */
    int32_t *rep;        /* min vertex of the cycle each vertex reaches */
    uint8_t *on_cycle;
    int32_t *layer;      /* connect round: 0 = kept, k = connected in round k */
    int32_t rounds;      /* connect rounds in the last rebuild */
    /* scratch */
    int32_t *mark, *stack, *queue;
    int32_t *cyc_of;     /* index of the cycle a vertex reaches */
} orc_state;

void orc_state_free(orc_state *st)
{
    if (!st) return;
    free(st->w); free(st->t); free(st->src); free(st->in_ptr); free(st->in_edge);
    free(st->pi); free(st->val); free(st->rep); free(st->on_cycle);
    free(st->layer); free(st->mark); free(st->stack); free(st->queue);
    free(st->cyc_of);
    free(st);
}

/* Creates a solver state.  w64 holds the weights as int64 (the caller widens
 * int32 weights); t64 the times (NULL: the cycle mean, every time 1); negate
 * selects the maximum (R10).  The arrays must outlive the state.  *rc
 * receives the status. */
orc_state *orc_state_new_ratio(int64_t n, int64_t m, const int32_t *row_ptr,
                               const int32_t *col, const int64_t *w64,
                               const int64_t *t64, int negate, int *rc)
{
    *rc = check_csr(n, m, row_ptr, col);
    if (*rc) return NULL;
    if (t64)
        for (int64_t e = 0; e < m; ++e)
            if (t64[e] < 1) { *rc = ORC_E_INVALID_ARG; return NULL; }
    orc_state *st = calloc(1, sizeof(orc_state));
    if (!st) { *rc = ORC_E_NOMEM; return NULL; }
    st->n = n; st->m = m; st->row_ptr = row_ptr; st->col = col;
    st->w = malloc(sizeof(int64_t) * m);
    st->src = malloc(sizeof(int32_t) * m);
    st->in_ptr = calloc(n + 1, sizeof(int64_t));
    st->in_edge = malloc(sizeof(int32_t) * m);
    st->pi = malloc(sizeof(int32_t) * n);
    st->val = calloc(n, sizeof(i128));
    st->rep = malloc(sizeof(int32_t) * n);
    st->on_cycle = calloc(n, 1);
    st->layer = malloc(sizeof(int32_t) * n);
    st->mark = malloc(sizeof(int32_t) * n);
    st->stack = malloc(sizeof(int32_t) * n);
    st->queue = malloc(sizeof(int32_t) * n);
    st->cyc_of = malloc(sizeof(int32_t) * n);
    if (!st->w || !st->src || !st->in_ptr || !st->in_edge || !st->pi || !st->val ||
        !st->rep || !st->on_cycle || !st->layer || !st->mark || !st->stack ||
        !st->queue || !st->cyc_of) {
        orc_state_free(st); *rc = ORC_E_NOMEM; return NULL;
    }
    for (int64_t e = 0; e < m; ++e) st->w[e] = negate ? -w64[e] : w64[e];
    if (t64) {
        st->t = malloc(sizeof(int64_t) * m);
        if (!st->t) { orc_state_free(st); *rc = ORC_E_NOMEM; return NULL; }
        memcpy(st->t, t64, sizeof(int64_t) * m);
    }
    for (int64_t v = 0; v < n; ++v)
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) st->src[e] = (int32_t)v;
    /* backward edges, the G^-1 of Alg. 3, stored explicitly as in Sec. 2.3 */
    for (int64_t e = 0; e < m; ++e) st->in_ptr[col[e] + 1]++;
    for (int64_t v = 0; v < n; ++v) st->in_ptr[v + 1] += st->in_ptr[v];
    {
        int64_t *fill = malloc(sizeof(int64_t) * n);
        if (!fill) { orc_state_free(st); *rc = ORC_E_NOMEM; return NULL; }
        memcpy(fill, st->in_ptr, sizeof(int64_t) * n);
        for (int64_t e = 0; e < m; ++e) st->in_edge[fill[col[e]]++] = (int32_t)e;
        free(fill);
    }
    for (int64_t v = 0; v < n; ++v) st->pi[v] = -1;
    st->W = 0; st->L = 1; st->s = -1; st->iter = 0; st->rounds = 0; st->clen = 0;
    return st;
}

orc_state *orc_state_new(int64_t n, int64_t m, const int32_t *row_ptr,
                         const int32_t *col, const int64_t *w64, int negate,
                         int *rc)
{
    return orc_state_new_ratio(n, m, row_ptr, col, w64, NULL, negate, rc);
}

/* Time of edge e (1 for the cycle mean). */
static int64_t edge_time(const orc_state *st, int64_t e)
{
    return st->t ? st->t[e] : 1;
}

/* Value of edge e under the current lambda = W / L:
 * V(target) + L * w(e) - W * t(e). */
static i128 edge_value(const orc_state *st, int64_t e)
{
    return st->val[st->col[e]] + (i128)st->L * st->w[e] - (i128)st->W * edge_time(st, e);
}

/* Policy improvement: one pass of the main loop of Alg. 2.  For every vertex
 * the best value over its out-edges is computed; the policy edge is replaced
 * when it is nil or its value exceeds the best strictly (R1, R2). */
int64_t orc_state_sweep(orc_state *st)
{
    int64_t changed = 0;
    for (int64_t v = 0; v < st->n; ++v) {
        i128 best = 0;
        int32_t arg = -1;
        for (int64_t e = st->row_ptr[v]; e < st->row_ptr[v + 1]; ++e) {
            i128 k = edge_value(st, e);
            if (arg < 0 || k < best) { best = k; arg = (int32_t)e; }
        }
        if (st->pi[v] < 0 || edge_value(st, st->pi[v]) > best) {
            st->pi[v] = arg;
            ++changed;
        }
    }
    st->iter++;
    return changed;
}

/* Cycles of the policy graph.  Every vertex has one policy successor, so each
 * weakly connected component holds exactly one cycle (Section 2.5).  Walk from
 * every unvisited vertex, colouring the walk, until reaching a visited vertex;
 * if that vertex belongs to the current walk a new cycle has been found.
 * Fills on_cycle and rep (the smallest vertex index on the reached cycle).
 * Returns the number of cycles. */
int64_t orc_state_cycles(orc_state *st)
{
    const int64_t n = st->n;
    int64_t ncyc = 0;
    for (int64_t v = 0; v < n; ++v) { st->mark[v] = -1; st->on_cycle[v] = 0; }
    for (int64_t v0 = 0; v0 < n; ++v0) {
        if (st->mark[v0] != -1) continue;
        int64_t len = 0;
        int32_t x = (int32_t)v0;
        while (st->mark[x] == -1) {
            st->mark[x] = (int32_t)v0;  /* on the current walk */
            st->stack[len++] = x;
            x = st->col[st->pi[x]];
        }
        int32_t r;
        if (st->mark[x] == (int32_t)v0) {
            /* new cycle through x: find its smallest vertex */
            r = x;
            int32_t y = st->col[st->pi[x]];
            st->on_cycle[x] = 1;
            while (y != x) {
                if (y < r) r = y;
                st->on_cycle[y] = 1;
                y = st->col[st->pi[y]];
            }
            ++ncyc;
        } else {
            r = st->rep[x];  /* reached an earlier walk */
        }
        for (int64_t i = 0; i < len; ++i) {
            st->rep[st->stack[i]] = r;
            st->mark[st->stack[i]] = -2;  /* finished */
        }
    }
    return ncyc;
}

/* MinMeanWeightCycle and MinVertex of Alg. 2 (R3, R4): among the cycles of
 * the policy graph pick the smallest mean W/L (for a ratio: cost over time),
 * ties to the smallest rep. */
int orc_state_select(orc_state *st, int32_t *s, int64_t *W, int64_t *L)
{
    int32_t best_r = -1;
    i128 bw = 0, bl = 1;
    int64_t bc = 0;
    for (int64_t r = 0; r < st->n; ++r) {
        if (!st->on_cycle[r] || st->rep[r] != r) continue;
        i128 cw = 0, ct = 0;
        int64_t cl = 0;
        int32_t y = (int32_t)r;
        do {
            cw += st->w[st->pi[y]];
            ct += edge_time(st, st->pi[y]);
            ++cl;
            y = st->col[st->pi[y]];
        } while (y != r);
        /* cw / ct < bw / bl, both denominators positive */
        if (best_r < 0 || cw * bl < bw * ct) { best_r = (int32_t)r; bw = cw; bl = ct; bc = cl; }
    }
    if (bw > (i128)INT64_MAX || bw < (i128)INT64_MIN || bl > (i128)INT64_MAX)
        return ORC_E_OVERFLOW;
    st->s = best_r;
    st->W = (int64_t)bw;
    st->L = (int64_t)bl;
    st->clen = bc;
    *s = best_r; *W = st->W; *L = st->L;
    return ORC_OK;
}

/* Breaking every other cycle (Alg. 2; Section 2.5 describes it as two
 * backward reachabilities).  The component of C keeps its policy (R5); the
 * remaining vertices are attached breadth-first (R6).  Returns 0 or
 * ORC_E_NOT_STRONGLY_CONNECTED when some vertex cannot reach C. */
int orc_state_connect(orc_state *st)
{
    const int64_t n = st->n;
    int64_t left = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (st->rep[v] == st->s) st->layer[v] = 0;
        else { st->layer[v] = -1; ++left; }
    }
    int32_t k = 0;
    while (left > 0) {
        ++k;
        int64_t got = 0;
        for (int64_t u = 0; u < n; ++u) {
            if (st->layer[u] != -1) continue;
            for (int64_t e = st->row_ptr[u]; e < st->row_ptr[u + 1]; ++e) {
                int32_t t = st->layer[st->col[e]];
                if (t >= 0 && t < k) {      /* connected before round k */
                    st->pi[u] = (int32_t)e;
                    st->mark[got++] = (int32_t)u;
                    break;
                }
            }
        }
        if (got == 0) { st->rounds = k; return ORC_E_NOT_STRONGLY_CONNECTED; }
        for (int64_t i = 0; i < got; ++i) st->layer[st->mark[i]] = k;
        left -= got;
    }
    st->rounds = k;
    return ORC_OK;
}

/* Value update of Alg. 2: val(s) <- 0, then a backward breadth-first search
 * from s over policy edges sets val(u) = val(v) + L * w(u, v) - W for every
 * policy predecessor u != s of a reached vertex v (R7). */
void orc_state_values(orc_state *st)
{
    int64_t head = 0, tail = 0;
    st->val[st->s] = 0;
    st->queue[tail++] = st->s;
    while (head < tail) {
        int32_t v = st->queue[head++];
        for (int64_t i = st->in_ptr[v]; i < st->in_ptr[v + 1]; ++i) {
            int32_t e = st->in_edge[i];
            int32_t u = st->src[e];
            if (u != st->s && st->pi[u] == e) {
                st->val[u] = st->val[v] + (i128)st->L * st->w[e] - (i128)st->W * edge_time(st, e);
                st->queue[tail++] = u;
            }
        }
    }
}

/* Exact uniqueness test for the critical cycle at the optimum.  With V a
 * feasible potential, a cycle is critical exactly when all its edges are tight
 * (V(v) = V(u) + L*w - W for edge v->u).  Policy edges are tight and form one
 * cycle, C; so another critical cycle exists iff some tight non-policy edge
 * x->y has x and y in one strongly connected component of the tight subgraph.
 * Components by Tarjan's algorithm, written iteratively.  Returns 1 = another
 * critical cycle exists, 0 = C is the only one. */
int orc_state_tie(orc_state *st)
{
    const int64_t n = st->n;
    int32_t *index = malloc(sizeof(int32_t) * n), *low = malloc(sizeof(int32_t) * n);
    int32_t *comp = malloc(sizeof(int32_t) * n), *stk = malloc(sizeof(int32_t) * n);
    int32_t *cs_v = malloc(sizeof(int32_t) * n);
    int64_t *cs_e = malloc(sizeof(int64_t) * n);
    uint8_t *onstk = calloc(n, 1);
    int tie = -1;
    if (!index || !low || !comp || !stk || !cs_v || !cs_e || !onstk) goto out;
    for (int64_t v = 0; v < n; ++v) { index[v] = -1; comp[v] = -1; }
    int32_t counter = 0, ncomp = 0;
    int64_t sp = 0, csp = 0;
    for (int64_t r = 0; r < n; ++r) {
        if (index[r] != -1) continue;
        cs_v[csp] = (int32_t)r; cs_e[csp] = st->row_ptr[r]; ++csp;
        index[r] = low[r] = counter++;
        stk[sp++] = (int32_t)r; onstk[r] = 1;
        while (csp > 0) {
            int32_t v = cs_v[csp - 1];
            int64_t e = cs_e[csp - 1];
            if (e < st->row_ptr[v + 1]) {
                cs_e[csp - 1] = e + 1;
                int tight = (st->pi[v] == e) || (edge_value(st, e) == st->val[v]);
                if (!tight) continue;
                int32_t u = st->col[e];
                if (index[u] == -1) {
                    index[u] = low[u] = counter++;
                    stk[sp++] = u; onstk[u] = 1;
                    cs_v[csp] = u; cs_e[csp] = st->row_ptr[u]; ++csp;
                } else if (onstk[u] && index[u] < low[v]) {
                    low[v] = index[u];
                }
            } else {
                --csp;
                if (csp > 0) {
                    int32_t p = cs_v[csp - 1];
                    if (low[v] < low[p]) low[p] = low[v];
                }
                if (low[v] == index[v]) {
                    int32_t x;
                    do { x = stk[--sp]; onstk[x] = 0; comp[x] = ncomp; } while (x != v);
                    ++ncomp;
                }
            }
        }
    }
    tie = 0;
    for (int64_t v = 0; v < n && !tie; ++v)
        for (int64_t e = st->row_ptr[v]; e < st->row_ptr[v + 1]; ++e) {
            if (st->pi[v] == e) continue;
            if (edge_value(st, e) != st->val[v]) continue;
            if (comp[v] == comp[st->col[e]]) { tie = 1; break; }
        }
out:
    free(index); free(low); free(comp); free(stk); free(cs_v); free(cs_e); free(onstk);
    return tie;
}

/* Accessors for phase-by-phase comparison. */
void orc_state_get_pi(const orc_state *st, int32_t *out) { memcpy(out, st->pi, sizeof(int32_t) * st->n); }
void orc_state_get_rep(const orc_state *st, int32_t *out) { memcpy(out, st->rep, sizeof(int32_t) * st->n); }
void orc_state_get_on_cycle(const orc_state *st, uint8_t *out) { memcpy(out, st->on_cycle, st->n); }
void orc_state_get_layer(const orc_state *st, int32_t *out) { memcpy(out, st->layer, sizeof(int32_t) * st->n); }
int32_t orc_state_rounds(const orc_state *st) { return st->rounds; }
int32_t orc_state_iter(const orc_state *st) { return st->iter; }

/* V as int64; returns ORC_E_OVERFLOW if some value does not fit. */
int orc_state_get_val(const orc_state *st, int64_t *out)
{
    for (int64_t v = 0; v < st->n; ++v) {
        if (st->val[v] > (i128)INT64_MAX || st->val[v] < (i128)INT64_MIN) return ORC_E_OVERFLOW;
        out[v] = (int64_t)st->val[v];
    }
    return ORC_OK;
}

/* Overwrites the state with a given policy, lambda and values (int64), so a
 * test can start a phase from any recorded state. */
void orc_state_set(orc_state *st, const int32_t *pi, const int64_t *val,
                   int64_t W, int64_t L, int32_t s, int32_t iter)
{
    for (int64_t v = 0; v < st->n; ++v) {
        if (pi) st->pi[v] = pi[v];
        if (val) st->val[v] = val[v];
    }
    st->W = W; st->L = L; st->s = s; st->iter = iter;
}

/* Result of a full solve. */
typedef struct {
    int64_t p, q;
    int64_t cycle_len;
    int32_t source;
    int32_t iterations;
    int32_t tie;
    int32_t ncycles_first;   /* cycles in the first policy graph */
    int64_t W, L;            /* unreduced lambda */
    int64_t tight;           /* non-policy edges with V(v) = V(u) + L*w - W */
} orc_result;

/* Full sequential solve.  cycle_edges (capacity cap) receives the critical
 * cycle as CSR positions from pi(s); val_out (n, may be NULL) receives the
 * final potential scaled by L; pi_out (n, may be NULL) the final policy.
 * max_iters = 0 means no limit.  do_tie = 1 runs the exact uniqueness test.
 * t64 (may be NULL): edge times of the ratio problem; then p/q = W/L is the
 * optimal cost-to-time ratio, L the time of C and cycle_len its edge count. */
int orc_solve_ratio(int64_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
                    const int64_t *w64, const int64_t *t64, int negate, int32_t max_iters,
                    int do_tie, orc_result *res, int32_t *cycle_edges, int64_t cap,
                    int64_t *val_out, int32_t *pi_out)
{
    int rc;
    orc_state *st = orc_state_new_ratio(n, m, row_ptr, col, w64, t64, negate, &rc);
    if (!st) return rc;
    memset(res, 0, sizeof(*res));
    for (;;) {
        int64_t changed = orc_state_sweep(st);
        if (st->iter >= 2 && changed == 0) break;               /* R8 */
        if (max_iters > 0 && st->iter >= max_iters) { rc = ORC_E_NOT_CONVERGED; goto done; }
        int64_t nc = orc_state_cycles(st);
        if (st->iter == 1) res->ncycles_first = (int32_t)nc;
        int32_t s; int64_t W, L;
        rc = orc_state_select(st, &s, &W, &L);
        if (rc) goto done;
        rc = orc_state_connect(st);
        if (rc) goto done;
        orc_state_values(st);
    }
    {
        int64_t W = st->W, L = st->L;
        int64_t g = gcd64(W, L);
        res->p = (negate ? -W : W) / g;
        res->q = L / g;
        res->W = W; res->L = L;
        res->source = st->s;
        res->iterations = st->iter;
        res->cycle_len = st->clen;
        if (cycle_edges) {
            if (cap < st->clen) { rc = ORC_E_CAPACITY; goto done; }
            int32_t y = st->s;
            for (int64_t i = 0; i < st->clen; ++i) {
                cycle_edges[i] = st->pi[y];
                y = st->col[st->pi[y]];
            }
        }
        res->tie = do_tie ? orc_state_tie(st) : -1;
        res->tight = 0;
        for (int64_t v = 0; v < n; ++v)
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
                if (e != st->pi[v] && edge_value(st, e) == st->val[v]) res->tight++;
        if (pi_out) orc_state_get_pi(st, pi_out);
        if (val_out) {
            rc = orc_state_get_val(st, val_out);
            if (rc) goto done;
        }
        rc = ORC_OK;
    }
done:
    orc_state_free(st);
    return rc;
}

int orc_solve(int64_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
              const int64_t *w64, int negate, int32_t max_iters, int do_tie,
              orc_result *res, int32_t *cycle_edges, int64_t cap,
              int64_t *val_out, int32_t *pi_out)
{
    return orc_solve_ratio(n, m, row_ptr, col, w64, NULL, negate, max_iters, do_tie, res,
                           cycle_edges, cap, val_out, pi_out);
}

/* Optimality certificate.  Checks
 *   (a) cycle_edges is a closed walk over valid edges visiting no vertex twice,
 *   (b) its weight sum equals p/q times its length (for a ratio: its time),
 *   (c) V, scaled by K > 0 with K*p/q = Wk an integer, satisfies
 *       V(v) <= V(u) + K*w(e) - Wk*t(e) on every edge e = v->u (t = 1 for
 *       the mean)
 * for the minimum (negate = 0) or the maximum (negate = 1, on -w and -p).
 * (c) says p/q is feasible: summed around any cycle it gives
 * K*(cost) - Wk*(time) >= 0, so p/q <= optimum (Prop. 2.1 and Eq. (1));
 * (a)+(b) exhibit a cycle of value p/q.  Together: p/q is the optimum.  The
 * check is O(m) in int128 and independent of how V was computed. */
int orc_certify_ratio(int64_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
                      const int64_t *w64, const int64_t *t64, int negate, int64_t p,
                      int64_t q, const int32_t *cycle_edges, int64_t cycle_len,
                      const int64_t *V, int64_t K)
{
    int rc = check_csr(n, m, row_ptr, col);
    if (rc) return rc;
    if (q <= 0 || K <= 0 || cycle_len < 1 || cycle_len > n) return ORC_E_INVALID_ARG;
    int64_t pm = negate ? -p : p;   /* work on the minimum over -w */
    if (((i128)K * pm) % q != 0) return ORC_E_CERT_MEAN;
    i128 Wk = (i128)K * pm / q;
    /* (a) + (b) */
    uint8_t *seen = calloc(n, 1);
    if (!seen) return ORC_E_NOMEM;
    i128 sum = 0, tsum = 0;
    int32_t first_src = -1, at = -1;
    rc = ORC_OK;
    for (int64_t i = 0; i < cycle_len; ++i) {
        int64_t e = cycle_edges[i];
        if (e < 0 || e >= m) { rc = ORC_E_CERT_CYCLE; break; }
        /* source of e by binary search over the offsets */
        int64_t lo = 0, hi = n - 1;
        while (lo < hi) {
            int64_t mid = (lo + hi + 1) / 2;
            if (row_ptr[mid] <= e) lo = mid; else hi = mid - 1;
        }
        int32_t v = (int32_t)lo;
        if (i == 0) first_src = v;
        else if (v != at) { rc = ORC_E_CERT_CYCLE; break; }
        if (seen[v]) { rc = ORC_E_CERT_CYCLE; break; }
        seen[v] = 1;
        sum += negate ? -w64[e] : w64[e];
        tsum += t64 ? t64[e] : 1;
        at = col[e];
    }
    free(seen);
    if (rc) return rc;
    if (at != first_src) return ORC_E_CERT_CYCLE;
    if (sum * q != (i128)pm * tsum) return ORC_E_CERT_MEAN;
    /* (c) */
    for (int64_t v = 0; v < n; ++v)
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            i128 wv = negate ? -w64[e] : w64[e];
            i128 tv = t64 ? t64[e] : 1;
            if ((i128)V[v] > (i128)V[col[e]] + (i128)K * wv - Wk * tv) return ORC_E_CERT_POTENTIAL;
        }
    return ORC_OK;
}

int orc_certify(int64_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
                const int64_t *w64, int negate, int64_t p, int64_t q,
                const int32_t *cycle_edges, int64_t cycle_len,
                const int64_t *V, int64_t K)
{
    return orc_certify_ratio(n, m, row_ptr, col, w64, NULL, negate, p, q, cycle_edges,
                             cycle_len, V, K);
}

/* ------------------------------------------------------------------------ */
/* Strongly connected components (Tarjan's algorithm, iterative), for inputs */
/* that are not strongly connected: Prop. 2.2 makes the optimum of a graph   */
/* the best optimum over its components that hold a cycle (Section 2.5       */
/* names the SCC decomposition as the alternative to the Hamiltonian-cycle   */
/* augmentation).  Vertices may have no out-edge.  comp_out[v] receives the  */
/* smallest vertex index of v's component.  Returns ORC_OK or an error.      */
/* ------------------------------------------------------------------------ */
int orc_scc(int64_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
            int32_t *comp_out)
{
    if (n < 1 || m < 0) return ORC_E_INVALID_ARG;
    if (row_ptr[0] != 0 || (int64_t)row_ptr[n] != m) return ORC_E_BAD_CSR;
    for (int64_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return ORC_E_BAD_CSR;
    for (int64_t e = 0; e < m; ++e)
        if (col[e] < 0 || (int64_t)col[e] >= n) return ORC_E_BAD_CSR;
    int32_t *index = malloc(sizeof(int32_t) * n), *low = malloc(sizeof(int32_t) * n);
    int32_t *stk = malloc(sizeof(int32_t) * n), *cs_v = malloc(sizeof(int32_t) * n);
    int64_t *cs_e = malloc(sizeof(int64_t) * n);
    uint8_t *onstk = calloc(n, 1);
    int rc = ORC_E_NOMEM;
    if (!index || !low || !stk || !cs_v || !cs_e || !onstk) goto out;
    for (int64_t v = 0; v < n; ++v) index[v] = -1;
    int32_t counter = 0;
    int64_t sp = 0, csp = 0;
    for (int64_t r = 0; r < n; ++r) {
        if (index[r] != -1) continue;
        cs_v[csp] = (int32_t)r; cs_e[csp] = row_ptr[r]; ++csp;
        index[r] = low[r] = counter++;
        stk[sp++] = (int32_t)r; onstk[r] = 1;
        while (csp > 0) {
            int32_t v = cs_v[csp - 1];
            int64_t e = cs_e[csp - 1];
            if (e < row_ptr[v + 1]) {
                cs_e[csp - 1] = e + 1;
                int32_t u = col[e];
                if (index[u] == -1) {
                    index[u] = low[u] = counter++;
                    stk[sp++] = u; onstk[u] = 1;
                    cs_v[csp] = u; cs_e[csp] = row_ptr[u]; ++csp;
                } else if (onstk[u] && index[u] < low[v]) {
                    low[v] = index[u];
                }
            } else {
                --csp;
                if (csp > 0) {
                    int32_t p = cs_v[csp - 1];
                    if (low[v] < low[p]) low[p] = low[v];
                }
                if (low[v] == index[v]) {
                    /* pop the component; its id is its smallest vertex */
                    int64_t top = sp;
                    int32_t mn = v, x;
                    do { x = stk[--sp]; if (x < mn) mn = x; } while (x != v);
                    for (int64_t i = sp; i < top; ++i) {
                        onstk[stk[i]] = 0;
                        comp_out[stk[i]] = mn;
                    }
                }
            }
        }
    }
    rc = ORC_OK;
out:
    free(index); free(low); free(stk); free(cs_v); free(cs_e); free(onstk);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Multichain policy iteration (not in the paper: the variant that skips the */
/* rebuild of Alg. 2).  Every cycle of the policy graph keeps its own gain   */
/* lambda_r = W_r / L_r (weight and length of the cycle with smallest vertex */
/* r); a vertex's gain is that of the cycle its policy path reaches, and its */
/* value V is scaled by that cycle's L: V(r) = 0 at each cycle's smallest    */
/* vertex, V(v) = V(succ v) + L_r * w(pi v) - W_r.  An edge v->u offers the  */
/* pair (gain of u, bias (V(u) + L_u * w - W_u) / L_u); a vertex moves to the */
/* lowest-position edge with the lexicographically smallest pair when that   */
/* pair is strictly below its own (gain, V(v) / L_v).  The first sweep is   */
/* R1's, and the stop rule R8's.  At the end the optimum is the smallest     */
/* gain, C the policy cycle attaining it with the smallest vertex.           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t *cw, *cl;      /* per cycle rep: weight and length (0 elsewhere) */
} orc_mc;

/* gain of vertex v: (cw, cl) of its cycle */
#define MC_GW(st, mc, v) ((mc)->cw[(st)->rep[v]])
#define MC_GL(st, mc, v) ((mc)->cl[(st)->rep[v]])

static int64_t mc_sweep(orc_state *st, const orc_mc *mc)
{
    int64_t changed = 0;
    for (int64_t v = 0; v < st->n; ++v) {
        int64_t e0 = st->row_ptr[v], e1 = st->row_ptr[v + 1];
        if (st->pi[v] < 0) {   /* R1 */
            int32_t arg = -1;
            int64_t best = 0;
            for (int64_t e = e0; e < e1; ++e)
                if (arg < 0 || st->w[e] < best) { best = st->w[e]; arg = (int32_t)e; }
            st->pi[v] = arg;
            ++changed;
            continue;
        }
        /* best (gain bw/bl, bias bb/bl) over the out-edges, CSR order, strict < */
        int32_t arg = -1;
        i128 bw = 0, bl = 1, bb = 0;
        for (int64_t e = e0; e < e1; ++e) {
            int32_t u = st->col[e];
            i128 wu = MC_GW(st, mc, u), lu = MC_GL(st, mc, u);
            i128 nb = st->val[u] + lu * st->w[e] - wu;     /* bias numerator over lu */
            int less;
            if (arg < 0) less = 1;
            else if (wu * bl != bw * lu) less = wu * bl < bw * lu;
            else less = nb * bl < bb * lu;
            if (less) { arg = (int32_t)e; bw = wu; bl = lu; bb = nb; }
        }
        /* own pair: (gain of v, V(v) / L_v) */
        i128 ow = MC_GW(st, mc, v), ol = MC_GL(st, mc, v), ob = st->val[v];
        int better;
        if (bw * ol != ow * bl) better = bw * ol < ow * bl;
        else better = bb * ol < ob * bl;
        if (better) { st->pi[v] = arg; ++changed; }
    }
    st->iter++;
    return changed;
}

/* Per-cycle sums and the values toward every cycle's smallest vertex. */
static void mc_values(orc_state *st, orc_mc *mc)
{
    const int64_t n = st->n;
    for (int64_t v = 0; v < n; ++v) { mc->cw[v] = 0; mc->cl[v] = 0; }
    for (int64_t r = 0; r < n; ++r) {
        if (!st->on_cycle[r] || st->rep[r] != r) continue;
        int32_t y = (int32_t)r;
        do {
            mc->cw[r] += st->w[st->pi[y]];
            mc->cl[r] += 1;
            y = st->col[st->pi[y]];
        } while (y != r);
    }
    /* backward breadth-first search from every cycle's smallest vertex */
    int64_t head = 0, tail = 0;
    for (int64_t r = 0; r < n; ++r)
        if (st->on_cycle[r] && st->rep[r] == r) { st->val[r] = 0; st->queue[tail++] = (int32_t)r; }
    while (head < tail) {
        int32_t v = st->queue[head++];
        for (int64_t i = st->in_ptr[v]; i < st->in_ptr[v + 1]; ++i) {
            int32_t e = st->in_edge[i];
            int32_t u = st->src[e];
            if (st->pi[u] != e) continue;
            if (st->on_cycle[u] && st->rep[u] == u) continue;   /* a cycle's own source */
            int32_t r = st->rep[u];
            st->val[u] = st->val[v] + (i128)mc->cl[r] * st->w[e] - mc->cw[r];
            st->queue[tail++] = u;
        }
    }
}

/* Exact uniqueness of C for the multichain result: another policy cycle
 * with the optimal mean, or a tight non-policy edge inside a strongly
 * connected component of the tight subgraph among vertices of optimal gain
 * (an edge v->u is tight when u has the same gain and its bias equals
 * V(v) / L_v). */
static int mc_tight(const orc_state *st, const orc_mc *mc, int64_t e, int32_t v)
{
    int32_t u = st->col[e];
    i128 wu = MC_GW(st, mc, u), lu = MC_GL(st, mc, u);
    i128 wv = MC_GW(st, mc, v), lv = MC_GL(st, mc, v);
    if (wu * lv != wv * lu) return 0;
    i128 nb = st->val[u] + lu * st->w[e] - wu;
    return nb * lv == st->val[v] * lu;
}

static int mc_tie(orc_state *st, const orc_mc *mc, int64_t W, int64_t L, int64_t *tight)
{
    const int64_t n = st->n;
    int ncrit = 0;
    for (int64_t r = 0; r < n; ++r)
        if (st->on_cycle[r] && st->rep[r] == r && (i128)mc->cw[r] * L == (i128)W * mc->cl[r]) ++ncrit;
    *tight = 0;
    for (int64_t v = 0; v < n; ++v)
        for (int64_t e = st->row_ptr[v]; e < st->row_ptr[v + 1]; ++e)
            if (e != st->pi[v] && mc_tight(st, mc, e, (int32_t)v)) ++*tight;
    if (ncrit > 1) return 1;
    /* Tarjan over the tight subgraph of the optimal-gain vertices */
    int32_t *index = malloc(sizeof(int32_t) * n), *low = malloc(sizeof(int32_t) * n);
    int32_t *comp = malloc(sizeof(int32_t) * n), *stk = malloc(sizeof(int32_t) * n);
    int32_t *cs_v = malloc(sizeof(int32_t) * n);
    int64_t *cs_e = malloc(sizeof(int64_t) * n);
    uint8_t *onstk = calloc(n, 1), *opt = calloc(n, 1);
    int tie = -1;
    if (!index || !low || !comp || !stk || !cs_v || !cs_e || !onstk || !opt) goto out;
    for (int64_t v = 0; v < n; ++v) {
        index[v] = -1; comp[v] = -1;
        opt[v] = (i128)MC_GW(st, mc, v) * L == (i128)W * MC_GL(st, mc, v);
    }
    int32_t counter = 0, ncomp = 0;
    int64_t sp = 0, csp = 0;
    for (int64_t r = 0; r < n; ++r) {
        if (index[r] != -1 || !opt[r]) continue;
        cs_v[csp] = (int32_t)r; cs_e[csp] = st->row_ptr[r]; ++csp;
        index[r] = low[r] = counter++;
        stk[sp++] = (int32_t)r; onstk[r] = 1;
        while (csp > 0) {
            int32_t v = cs_v[csp - 1];
            int64_t e = cs_e[csp - 1];
            if (e < st->row_ptr[v + 1]) {
                cs_e[csp - 1] = e + 1;
                int32_t u = st->col[e];
                if (!opt[u]) continue;
                if (!(st->pi[v] == e || mc_tight(st, mc, e, v))) continue;
                if (index[u] == -1) {
                    index[u] = low[u] = counter++;
                    stk[sp++] = u; onstk[u] = 1;
                    cs_v[csp] = u; cs_e[csp] = st->row_ptr[u]; ++csp;
                } else if (onstk[u] && index[u] < low[v]) {
                    low[v] = index[u];
                }
            } else {
                --csp;
                if (csp > 0) {
                    int32_t p = cs_v[csp - 1];
                    if (low[v] < low[p]) low[p] = low[v];
                }
                if (low[v] == index[v]) {
                    int32_t x;
                    do { x = stk[--sp]; onstk[x] = 0; comp[x] = ncomp; } while (x != v);
                    ++ncomp;
                }
            }
        }
    }
    tie = 0;
    for (int64_t v = 0; v < n && !tie; ++v) {
        if (!opt[v]) continue;
        for (int64_t e = st->row_ptr[v]; e < st->row_ptr[v + 1]; ++e) {
            if (st->pi[v] == e || !opt[st->col[e]] || !mc_tight(st, mc, e, (int32_t)v)) continue;
            if (comp[v] == comp[st->col[e]]) { tie = 1; break; }
        }
    }
out:
    free(index); free(low); free(comp); free(stk); free(cs_v); free(cs_e); free(onstk); free(opt);
    return tie;
}

int orc_solve_mc(int64_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
                 const int64_t *w64, int negate, int32_t max_iters, int do_tie,
                 orc_result *res, int32_t *cycle_edges, int64_t cap, int64_t *val_out,
                 int32_t *pi_out)
{
    int rc;
    orc_state *st = orc_state_new(n, m, row_ptr, col, w64, negate, &rc);
    if (!st) return rc;
    orc_mc mc;
    mc.cw = calloc(n, sizeof(int64_t));
    mc.cl = calloc(n, sizeof(int64_t));
    memset(res, 0, sizeof(*res));
    if (!mc.cw || !mc.cl) { rc = ORC_E_NOMEM; goto done; }
    for (;;) {
        int64_t changed = mc_sweep(st, &mc);
        if (st->iter >= 2 && changed == 0) break;               /* R8 */
        if (max_iters > 0 && st->iter >= max_iters) { rc = ORC_E_NOT_CONVERGED; goto done; }
        int64_t nc = orc_state_cycles(st);
        if (st->iter == 1) res->ncycles_first = (int32_t)nc;
        mc_values(st, &mc);
    }
    {
        /* C: the smallest gain, then the smallest rep */
        int32_t s = -1;
        for (int64_t r = 0; r < n; ++r) {
            if (!st->on_cycle[r] || st->rep[r] != r) continue;
            if (s < 0 || (i128)mc.cw[r] * mc.cl[s] < (i128)mc.cw[s] * mc.cl[r]) s = (int32_t)r;
        }
        int64_t W = mc.cw[s], L = mc.cl[s];
        int64_t g = gcd64(W, L);
        res->p = (negate ? -W : W) / g;
        res->q = L / g;
        res->W = W; res->L = L;
        res->source = s;
        res->iterations = st->iter;
        res->cycle_len = L;
        if (cycle_edges) {
            if (cap < L) { rc = ORC_E_CAPACITY; goto done; }
            int32_t y = s;
            for (int64_t i = 0; i < L; ++i) {
                cycle_edges[i] = st->pi[y];
                y = st->col[st->pi[y]];
            }
        }
        int64_t tight = 0;
        res->tie = do_tie ? mc_tie(st, &mc, W, L, &tight) : -1;
        res->tight = tight;
        if (pi_out) orc_state_get_pi(st, pi_out);
        if (val_out) {
            rc = orc_state_get_val(st, val_out);
            if (rc) goto done;
        }
        rc = ORC_OK;
    }
done:
    free(mc.cw); free(mc.cl);
    orc_state_free(st);
    return rc;
}
