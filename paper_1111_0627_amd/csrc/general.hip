// Graphs that are not strongly connected (Prop. 2.2, Section 2.5): the
// optimum of a graph is the best optimum among its strongly connected
// components that hold a cycle.  The components are found on the device by
// repeated minimum-label colouring (forward) and backward closure; the ones
// holding a cycle are renumbered into one disjoint-union CSR and solved
// together by the batched solver (concurrent regions, Section 3.3).
#include "ocm.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "device_util.h"
#include "kernels.h"

namespace ocm {
namespace gen {

// Colouring state of the decomposition (device).
struct GCtl {
    unsigned changed;   // the last round changed a label or a member flag
    unsigned alive;     // vertices not yet assigned to a component
    unsigned kept;      // vertices of components that hold a cycle
    unsigned ncomp;     // components that hold a cycle
};

__global__ __launch_bounds__(kWG) void k_init(int n, unsigned char* __restrict__ alive,
                                              int* __restrict__ scc)
{
    for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < n; v += (int64_t)gridDim.x * kWG) {
        alive[v] = 1;
        scc[v] = -1;
    }
}

// label[v] = v for unassigned vertices; member[v]: v is its label's root
__global__ __launch_bounds__(kWG) void k_label_init(int n, const unsigned char* __restrict__ alive,
                                                    int* __restrict__ label,
                                                    unsigned char* __restrict__ member)
{
    for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < n; v += (int64_t)gridDim.x * kWG) {
        label[v] = alive[v] ? (int)v : INT32_MAX;
        member[v] = 0;
    }
}

// Forward colouring round: every unassigned vertex pushes its label along its
// out-edges into unassigned heads (atomic minimum).  The fixpoint is unique:
// label[v] = smallest unassigned vertex that reaches v.
__global__ __launch_bounds__(kWG) void k_label_round(int n, const int* __restrict__ row_ptr,
                                                     const int* __restrict__ col,
                                                     const unsigned char* __restrict__ alive,
                                                     int* __restrict__ label, GCtl* ctl)
{
    unsigned ch = 0;
    for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < n; v += (int64_t)gridDim.x * kWG) {
        if (!alive[v]) continue;
        const int lv = label[v];
        const int e1 = row_ptr[v + 1];
        for (int e = row_ptr[v]; e < e1; ++e) {
            const int u = col[e];
            if (alive[u] && lv < label[u] && atomicMin(&label[u], lv) > lv) ch = 1;
        }
    }
    if (__ballot(ch != 0) && (threadIdx.x & 63) == 0) atomicOr(&ctl->changed, 1u);
}

// Roots: vertices whose label is their own index.
__global__ __launch_bounds__(kWG) void k_roots(int n, const unsigned char* __restrict__ alive,
                                               const int* __restrict__ label,
                                               unsigned char* __restrict__ member)
{
    for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < n; v += (int64_t)gridDim.x * kWG)
        if (alive[v] && label[v] == (int)v) member[v] = 1;
}

// Backward closure round: an unassigned vertex with the root's label joins
// the root's component when one of its out-edges enters a member of that
// label (it reaches the root, and the root reaches it).
__global__ __launch_bounds__(kWG) void k_member_round(int n, const int* __restrict__ row_ptr,
                                                      const int* __restrict__ col,
                                                      const unsigned char* __restrict__ alive,
                                                      const int* __restrict__ label,
                                                      unsigned char* __restrict__ member, GCtl* ctl)
{
    unsigned ch = 0;
    for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < n; v += (int64_t)gridDim.x * kWG) {
        if (!alive[v] || member[v]) continue;
        const int lv = label[v];
        const int e1 = row_ptr[v + 1];
        for (int e = row_ptr[v]; e < e1; ++e) {
            const int u = col[e];
            if (alive[u] && label[u] == lv && member[u]) {
                member[v] = 1;
                ch = 1;
                break;
            }
        }
    }
    if (__ballot(ch != 0) && (threadIdx.x & 63) == 0) atomicOr(&ctl->changed, 1u);
}

// Members take their label (the component's smallest vertex) as component id.
__global__ __launch_bounds__(kWG) void k_assign(int n, unsigned char* __restrict__ alive,
                                                const int* __restrict__ label,
                                                const unsigned char* __restrict__ member,
                                                int* __restrict__ scc, GCtl* ctl)
{
    unsigned left = 0;
    for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < n; v += (int64_t)gridDim.x * kWG) {
        if (!alive[v]) continue;
        if (member[v]) {
            scc[v] = label[v];
            alive[v] = 0;
        } else {
            ++left;
        }
    }
    const unsigned long long t = block_sum_u64(left);
    if (threadIdx.x == 0 && t) atomicAdd(&ctl->alive, (unsigned)t);
}

// Component sizes and self-loops (a one-vertex component holds a cycle only
// through a self-loop).
__global__ __launch_bounds__(kWG) void k_comp_stats(int n, const int* __restrict__ row_ptr,
                                                    const int* __restrict__ col,
                                                    const int* __restrict__ scc,
                                                    unsigned* __restrict__ size,
                                                    unsigned char* __restrict__ self)
{
    for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < n; v += (int64_t)gridDim.x * kWG) {
        const int c = scc[v];
        atomicAdd(&size[c], 1u);
        const int e1 = row_ptr[v + 1];
        for (int e = row_ptr[v]; e < e1; ++e)
            if (col[e] == (int)v) self[c] = 1;
    }
}

// Sort keys: component id for vertices of components with a cycle, n for
// the others (sorted to the end).
__global__ __launch_bounds__(kWG) void k_keys(int n, const int* __restrict__ scc,
                                              const unsigned* __restrict__ size,
                                              const unsigned char* __restrict__ self,
                                              int* __restrict__ keys, int* __restrict__ vals,
                                              GCtl* ctl)
{
    unsigned kept = 0;
    for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < n; v += (int64_t)gridDim.x * kWG) {
        const int c = scc[v];
        const bool keep = size[c] >= 2 || self[c];
        keys[v] = keep ? c : n;
        vals[v] = (int)v;
        kept += keep;
    }
    const unsigned long long t = block_sum_u64(kept);
    if (threadIdx.x == 0 && t) atomicAdd(&ctl->kept, (unsigned)t);
}

// After the stable sort by component: position of every kept vertex in the
// union, and a flag at the first vertex of each component.
__global__ __launch_bounds__(kWG) void k_positions(int N, const int* __restrict__ keys_s,
                                                   const int* __restrict__ perm,
                                                   int* __restrict__ pos,
                                                   unsigned* __restrict__ first)
{
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < N; i += (int64_t)gridDim.x * kWG) {
        pos[perm[i]] = (int)i;
        first[i] = (i == 0 || keys_s[i] != keys_s[i - 1]) ? 1u : 0u;
    }
}

__global__ __launch_bounds__(kWG) void k_bounds(int N, const unsigned* __restrict__ first,
                                                const unsigned* __restrict__ idx,
                                                long long* __restrict__ vptr)
{
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < N; i += (int64_t)gridDim.x * kWG)
        if (first[i]) vptr[idx[i]] = i;
}

// Out-edges that stay inside the vertex's component, per union vertex.
__global__ __launch_bounds__(kWG) void k_degrees(int N, const int* __restrict__ perm,
                                                 const int* __restrict__ row_ptr,
                                                 const int* __restrict__ col,
                                                 const int* __restrict__ scc,
                                                 unsigned* __restrict__ deg)
{
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < N; i += (int64_t)gridDim.x * kWG) {
        const int v = perm[i];
        const int c = scc[v];
        unsigned d = 0;
        const int e1 = row_ptr[v + 1];
        for (int e = row_ptr[v]; e < e1; ++e) d += scc[col[e]] == c;
        deg[i] = d;
    }
}

// The union CSR: heads renumbered, weights copied, original edge positions
// kept in emap (edges in original CSR order within each row).
template <typename WT>
__global__ __launch_bounds__(kWG) void k_fill(int N, const int* __restrict__ perm,
                                              const int* __restrict__ row_ptr,
                                              const int* __restrict__ col,
                                              const WT* __restrict__ w,
                                              const int* __restrict__ scc,
                                              const int* __restrict__ pos,
                                              const unsigned* __restrict__ urp,
                                              int* __restrict__ ucol, WT* __restrict__ uw,
                                              int* __restrict__ emap)
{
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < N; i += (int64_t)gridDim.x * kWG) {
        const int v = perm[i];
        const int c = scc[v];
        unsigned k = urp[i];
        const int e1 = row_ptr[v + 1];
        for (int e = row_ptr[v]; e < e1; ++e) {
            const int u = col[e];
            if (scc[u] != c) continue;
            ucol[k] = pos[u];
            uw[k] = w[e];
            emap[k] = e;
            ++k;
        }
    }
}

__global__ __launch_bounds__(kWG) void k_edge_bounds(int G, const long long* __restrict__ vptr,
                                                     const unsigned* __restrict__ urp,
                                                     long long* __restrict__ eptr)
{
    for (int64_t g = (int64_t)blockIdx.x * kWG + threadIdx.x; g <= G; g += (int64_t)gridDim.x * kWG)
        eptr[g] = urp[vptr[g]];
}

// The chosen component's cycle in original edge positions, and its source
// (the tail of its first edge: components keep the original vertex order,
// so the smallest union vertex on the cycle is the smallest original one).
__global__ __launch_bounds__(kWG) void k_map_cycle(int len, const int* __restrict__ ucyc,
                                                   const int* __restrict__ emap,
                                                   int* __restrict__ out, int n,
                                                   const int* __restrict__ row_ptr,
                                                   int* __restrict__ source)
{
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < len; i += (int64_t)gridDim.x * kWG)
        out[i] = emap[ucyc[i]];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int e = emap[ucyc[0]];
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = lo + (hi - lo + 1) / 2;
            if (row_ptr[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        *source = lo;
    }
}

}  // namespace gen
}  // namespace ocm

namespace {

using ocm::gen::GCtl;

ocm_status gfail(ocm_status s, const char* what)
{
    ocm::set_last_error(what);
    return s;
}

#define GHIP(expr)                                                                     \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            char b_[256];                                                              \
            snprintf(b_, sizeof b_, "%s: %s", #expr, hipGetErrorString(e_));           \
            return gfail(OCM_E_HIP, b_);                                               \
        }                                                                              \
    } while (0)

size_t gal(size_t x) { return (x + 255) & ~size_t(255); }

struct GWs {
    GCtl* ctl;
    void* vctl;                 // control block of the validation kernel
    unsigned char *alive, *member, *self;
    int *label, *scc, *keys, *vals, *keys_s, *perm, *pos;
    unsigned *size, *first, *idx, *stot, *deg, *urp;
    long long *vptr, *eptr;
    int* ucol;
    void* uw;
    int* emap;
    int* ucyc;                  // union positions of the components' cycles
    int* src;                   // the chosen cycle's source
    void* sort_tmp;
    size_t sort_bytes;
    void* bws;                  // the batched solver's workspace
    size_t bws_bytes;
    size_t total;
};

size_t sort_temp_bytes(int n)
{
    size_t b = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, b, (const int*)nullptr, (int*)nullptr,
                                             (const int*)nullptr, (int*)nullptr, n, 0, 32);
    return b;
}

GWs gcarve(void* base, int64_t n, int64_t m)
{
    char* b = (char*)base;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        size_t o = off;
        off += gal(bytes);
        return b ? (void*)(b + o) : nullptr;
    };
    const size_t N = (size_t)n, M = (size_t)m;
    GWs w;
    w.ctl = (GCtl*)take(sizeof(GCtl));
    w.vctl = take(sizeof(ocm::Ctl));
    w.alive = (unsigned char*)take(N);
    w.member = (unsigned char*)take(N);
    w.self = (unsigned char*)take(N);
    w.label = (int*)take(4 * N);
    w.scc = (int*)take(4 * N);
    w.keys = (int*)take(4 * N);
    w.vals = (int*)take(4 * N);
    w.keys_s = (int*)take(4 * N);
    w.perm = (int*)take(4 * N);
    w.pos = (int*)take(4 * N);
    w.size = (unsigned*)take(4 * N);
    w.first = (unsigned*)take(4 * (N + 1));
    w.idx = (unsigned*)take(4 * (N + 1));
    w.stot = (unsigned*)take(4 * ((N + 1) / 2048 + 2));
    w.deg = (unsigned*)take(4 * (N + 1));
    w.urp = (unsigned*)take(4 * (N + 1));
    w.vptr = (long long*)take(8 * (N + 1));
    w.eptr = (long long*)take(8 * (N + 1));
    w.ucol = (int*)take(4 * M);
    w.uw = take(8 * M);
    w.emap = (int*)take(4 * M);
    w.ucyc = (int*)take(4 * N);
    w.src = (int*)take(256);
    w.sort_bytes = sort_temp_bytes((int)n);
    w.sort_tmp = take(w.sort_bytes);
    // the union has at most n vertices, m edges and n graphs, the largest
    // graph at most n vertices and m edges
    w.bws_bytes = ocm::batched_ws_bound(n, n, m, n, m);
    w.bws = take(w.bws_bytes);
    w.total = off;
    return w;
}

// Reads the decomposition's control block.
ocm_status read_gctl(const GWs& w, GCtl* h, hipStream_t st)
{
    GHIP(ocm::host_read(w.ctl, h, sizeof(GCtl), st));
    return OCM_OK;
}

ocm_status solve_general(const ocm_graph* g, const ocm_options* o_in, void* wsp, size_t ws_bytes,
                         int32_t* cycle_edges, int64_t cap, ocm_result* out, int64_t* ncomp_out,
                         void* stream, int neg)
{
    if (!out) return gfail(OCM_E_INVALID_ARG, "result pointer is null");
    memset(out, 0, sizeof *out);
    if (!g) return gfail(OCM_E_INVALID_ARG, "graph is null");
    if (g->n < 1 || g->m < 1 || g->n >= (int64_t(1) << 31) - 1 || g->m >= (int64_t(1) << 31))
        return gfail(OCM_E_INVALID_ARG, "n and m must be in [1, 2^31)");
    if (!g->row_ptr || !g->col || !g->w) return gfail(OCM_E_INVALID_ARG, "null graph array");
    if (g->wtype != OCM_W_I32 && g->wtype != OCM_W_I64) return gfail(OCM_E_INVALID_ARG, "bad wtype");
    ocm_options o;
    if (o_in) o = *o_in;
    else ocm_default_options(&o);
    if (o.init_policy || o.policy_out || o.potential_out || o.profile)
        return gfail(OCM_E_INVALID_ARG, "general graphs take no policy, potential or profile");
    const int n = (int)g->n, m = (int)g->m;
    hipStream_t st = (hipStream_t)stream;
    GWs w = gcarve(nullptr, n, m);
    if (!wsp || ws_bytes < w.total) return gfail(OCM_E_WORKSPACE, "workspace missing or too small");
    w = gcarve(wsp, n, m);
    const unsigned grid = ocm::stride_grid(n);

    // the CSR's shape (a vertex may have no out-edge here)
    {
        ocm::Ctl* vc = (ocm::Ctl*)w.vctl;
        ocm::launch_ctl_clear(vc, ocm::kClrAll, st);
        ocm::launch_validate(n, m, g->row_ptr, g->col, g->w, g->wtype, o.validate != 0, vc, st);
        ocm::CtlView h;
        GHIP(ocm::host_read_ctl(vc, &h, st));
        if (h.err & ocm::kErrBadCsr) return gfail(OCM_E_BAD_CSR, "malformed CSR");
    }

    // components: colour from the smallest unassigned vertex forward, close
    // each root's component backward, repeat on what is left
    GCtl h;
    ocm::gen::k_init<<<grid, ocm::kWG, 0, st>>>(n, w.alive, w.scc);
    for (int pass = 0;; ++pass) {
        if (pass > n) return gfail(OCM_E_HIP, "component passes did not finish");
        ocm::gen::k_label_init<<<grid, ocm::kWG, 0, st>>>(n, w.alive, w.label, w.member);
        for (int r = 0;; ++r) {
            if (r > n + 1) return gfail(OCM_E_HIP, "colouring did not converge");
            ocm::launch_fill_u32(&w.ctl->changed, 1, 0u, st);
            ocm::gen::k_label_round<<<grid, ocm::kWG, 0, st>>>(n, g->row_ptr, g->col, w.alive,
                                                               w.label, w.ctl);
            GHIP(hipGetLastError());
            if (read_gctl(w, &h, st) != OCM_OK) return OCM_E_HIP;
            if (!h.changed) break;
        }
        ocm::gen::k_roots<<<grid, ocm::kWG, 0, st>>>(n, w.alive, w.label, w.member);
        for (int r = 0;; ++r) {
            if (r > n + 1) return gfail(OCM_E_HIP, "backward closure did not converge");
            ocm::launch_fill_u32(&w.ctl->changed, 1, 0u, st);
            ocm::gen::k_member_round<<<grid, ocm::kWG, 0, st>>>(n, g->row_ptr, g->col, w.alive,
                                                                w.label, w.member, w.ctl);
            GHIP(hipGetLastError());
            if (read_gctl(w, &h, st) != OCM_OK) return OCM_E_HIP;
            if (!h.changed) break;
        }
        ocm::launch_fill_u32(&w.ctl->alive, 1, 0u, st);
        ocm::gen::k_assign<<<grid, ocm::kWG, 0, st>>>(n, w.alive, w.label, w.member, w.scc, w.ctl);
        GHIP(hipGetLastError());
        if (read_gctl(w, &h, st) != OCM_OK) return OCM_E_HIP;
        if (h.alive == 0) break;
    }

    // the components that hold a cycle, renumbered into one union CSR
    ocm::launch_fill_u32(w.size, n, 0u, st);
    ocm::launch_fill_u8(w.self, n, 0, st);
    ocm::launch_fill_u32(&w.ctl->kept, 1, 0u, st);
    ocm::gen::k_comp_stats<<<grid, ocm::kWG, 0, st>>>(n, g->row_ptr, g->col, w.scc, w.size, w.self);
    ocm::gen::k_keys<<<grid, ocm::kWG, 0, st>>>(n, w.scc, w.size, w.self, w.keys, w.vals, w.ctl);
    size_t sb = w.sort_bytes;
    GHIP(hipcub::DeviceRadixSort::SortPairs(w.sort_tmp, sb, w.keys, w.keys_s, w.vals, w.perm, n, 0,
                                            32, st));
    if (read_gctl(w, &h, st) != OCM_OK) return OCM_E_HIP;
    const int N = (int)h.kept;
    if (N == 0) return gfail(OCM_E_NOT_STRONGLY_CONNECTED, "the graph has no cycle");
    const unsigned gN = ocm::stride_grid(N);
    ocm::gen::k_positions<<<gN, ocm::kWG, 0, st>>>(N, w.keys_s, w.perm, w.pos, w.first);
    ocm::launch_exclusive_scan(N, w.first, w.idx, w.stot, st);
    unsigned G = 0, lastf = 0;
    GHIP(hipMemcpyAsync(&G, w.idx + N - 1, 4, hipMemcpyDeviceToHost, st));
    GHIP(hipMemcpyAsync(&lastf, w.first + N - 1, 4, hipMemcpyDeviceToHost, st));
    GHIP(hipStreamSynchronize(st));
    G += lastf;
    ocm::gen::k_bounds<<<gN, ocm::kWG, 0, st>>>(N, w.first, w.idx, w.vptr);
    ocm::gen::k_degrees<<<gN, ocm::kWG, 0, st>>>(N, w.perm, g->row_ptr, g->col, w.scc, w.deg);
    ocm::launch_fill_u32(w.deg + N, 1, 0u, st);
    ocm::launch_exclusive_scan(N + 1, w.deg, w.urp, w.stot, st);
    GHIP(hipGetLastError());
    if (g->wtype == OCM_W_I64)
        ocm::gen::k_fill<long long><<<gN, ocm::kWG, 0, st>>>(
            N, w.perm, g->row_ptr, g->col, (const long long*)g->w, w.scc, w.pos, w.urp, w.ucol,
            (long long*)w.uw, w.emap);
    else
        ocm::gen::k_fill<int><<<gN, ocm::kWG, 0, st>>>(N, w.perm, g->row_ptr, g->col,
                                                        (const int*)g->w, w.scc, w.pos, w.urp,
                                                        w.ucol, (int*)w.uw, w.emap);
    long long NN = N;
    GHIP(hipMemcpyAsync(w.vptr + G, &NN, 8, hipMemcpyHostToDevice, st));
    ocm::gen::k_edge_bounds<<<ocm::stride_grid(G + 1), ocm::kWG, 0, st>>>((int)G, w.vptr, w.urp,
                                                                         w.eptr);
    GHIP(hipGetLastError());
    std::vector<int64_t> vptr(G + 1), eptr(G + 1);
    GHIP(hipMemcpyAsync(vptr.data(), w.vptr, 8 * (size_t)(G + 1), hipMemcpyDeviceToHost, st));
    GHIP(hipMemcpyAsync(eptr.data(), w.eptr, 8 * (size_t)(G + 1), hipMemcpyDeviceToHost, st));
    GHIP(hipStreamSynchronize(st));
    const int64_t M = eptr[G];

    // every component at once (batched solver)
    ocm_graph u{N, M, (const int32_t*)w.urp, w.ucol, w.uw, g->wtype};
    std::vector<int64_t> p(G), q(G), cptr(G + 1);
    std::vector<int32_t> it(G), status(G);
    std::vector<uint32_t> fl(G);
    ocm_options bo;
    ocm_default_options(&bo);
    bo.max_iters = o.max_iters;
    bo.tie_check = o.tie_check;
    bo.fast_path = o.fast_path;
    bo.validate = 0;
    const ocm_status rc = (neg ? ocm_max_batched : ocm_min_batched)(
        G, vptr.data(), eptr.data(), &u, &bo, w.bws, w.bws_bytes, p.data(), q.data(), cptr.data(),
        w.ucyc, N, it.data(), fl.data(), status.data(), stream);
    if (rc != OCM_OK) return rc;

    // the best component; ties to the smallest component id (the union keeps
    // the components in increasing id order)
    int64_t best = 0;
    int same = 1;
    for (int64_t k = 1; k < (int64_t)G; ++k) {
        const __int128 a = (__int128)p[k] * q[best], b = (__int128)p[best] * q[k];
        const bool better = neg ? a > b : a < b;
        if (better) {
            best = k;
            same = 1;
        } else if (a == b) {
            ++same;
        }
    }
    const int64_t len = cptr[best + 1] - cptr[best];
    out->p = p[best];
    out->q = q[best];
    out->cycle_len = len;
    out->iterations = it[best];
    out->flags = fl[best];
    if (same > 1) out->flags = (out->flags & ~(uint32_t)OCM_F_TIE_UNCHECKED) | OCM_F_TIE;
    // unreduced W / L of C: its weight sum over its length
    out->L = len;
    out->W = p[best] * (len / q[best]);
    out->tight_edges = -1;
    if (ncomp_out) *ncomp_out = G;
    if (cap < len) return gfail(OCM_E_CAPACITY, "cycle_cap smaller than the critical cycle");
    if (len > 0 && !cycle_edges) return gfail(OCM_E_INVALID_ARG, "cycle_edges is null");
    ocm::gen::k_map_cycle<<<ocm::stride_grid(len), ocm::kWG, 0, st>>>(
        (int)len, w.ucyc + cptr[best], w.emap, cycle_edges, n, g->row_ptr, w.src);
    GHIP(hipGetLastError());
    int s = -1;
    GHIP(hipMemcpyAsync(&s, w.src, 4, hipMemcpyDeviceToHost, st));
    GHIP(hipStreamSynchronize(st));
    out->source = s;
    return OCM_OK;
}

}  // namespace

extern "C" {

size_t ocm_general_workspace_size(const ocm_graph* g)
{
    if (!g || g->n < 1 || g->m < 1 || g->n >= (int64_t(1) << 31) - 1 || g->m >= (int64_t(1) << 31))
        return 0;
    return gcarve(nullptr, g->n, g->m).total;
}

ocm_status ocm_min_general(const ocm_graph* g, const ocm_options* o, void* ws, size_t ws_bytes,
                           int32_t* cycle_edges, int64_t cycle_cap, ocm_result* out,
                           int64_t* components, void* stream)
{
    return solve_general(g, o, ws, ws_bytes, cycle_edges, cycle_cap, out, components, stream, 0);
}

ocm_status ocm_max_general(const ocm_graph* g, const ocm_options* o, void* ws, size_t ws_bytes,
                           int32_t* cycle_edges, int64_t cycle_cap, ocm_result* out,
                           int64_t* components, void* stream)
{
    return solve_general(g, o, ws, ws_bytes, cycle_edges, cycle_cap, out, components, stream, 1);
}

}  // extern "C"
