// Host driver of the exact optimal-cycle-mean solver: the loop of Alg. 3
// (Howard's policy iteration, Alg. 2) over the device phases, behind the
// C ABI declared in include/ocm.h.
#include "ocm.h"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

using ocm::Ctl;
using ocm::Jmp;

namespace {

thread_local std::string g_last_error;

ocm_status fail(ocm_status s, const char* what)
{
    g_last_error = what;
    return s;
}

}  // namespace

void ocm::set_last_error(const char* what) { g_last_error = what; }

namespace {

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            char b_[256];                                                              \
            snprintf(b_, sizeof b_, "%s: %s", #expr, hipGetErrorString(e_));           \
            return fail(OCM_E_HIP, b_);                                                \
        }                                                                              \
    } while (0)

#define OCM_TRY(expr)                                                                  \
    do {                                                                               \
        ocm_status s_ = (expr);                                                        \
        if (s_ != OCM_OK) return s_;                                                   \
    } while (0)

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Hard bound on policy iterations when the caller sets none.
constexpr int kIterCap = 1 << 20;

// The exact uniqueness test lists at most this many tight non-policy edges;
// beyond it the result is flagged OCM_F_TIE_UNCHECKED.
constexpr int64_t kTieListCap = 1 << 20;

// Workspace carved into the solver's device arrays.
struct Ws {
    Ctl* ctl;
    long long* V;        // values scaled by L (int128 values: their low words)
    long long* Vhi;      // int128 values: high words
    int* V32;            // int32 copy of V (valid while every value fits int32)
    long long* Dhi[2];   // int128 value rounds: high words of the jump entries' sums
    int* pi;             // policy: CSR position of each vertex's edge
    int* succ;           // policy successor
    int* hop;            // policy hops to the source (value phase)
    Jmp* Q[2];           // pointer-jumping buffers (values; cycles alias them)
    int* rep;            // smallest vertex of the reached cycle
    unsigned char* onc;  // on a policy-graph cycle
    unsigned char* onC;  // on the chosen cycle C
    int* layer;          // connect round of each vertex
    int* list[2];        // tie check: special-vertex list and jump pointers
    unsigned* rdeg;      // reverse CSR: in-degree, then fill cursor (n+1)
    unsigned* stot;      // prefix-sum block totals
    int* rin_ptr;        // reverse CSR offsets (n+1)
    int* rin;            // reverse CSR entries: the tail of each in-edge (m)
    void* rscratch;      // reverse CSR build: partition scratch (pairs and histograms)
    unsigned* abits[2];  // connect: attached-vertex bitmaps (alternating by round)
    unsigned char* marks[2];  // push rounds: marked vertices (bytes), by round parity
    unsigned char* touched;  // tie check: special-vertex flags
    void* sel;           // select: per-block best candidates
    int* xs;             // tie check: tight non-policy edges (tail), xcap entries
    int* ys;             //            and head
    unsigned xcap;
    long long* wsum;     // per-cycle weight sums, keyed by rep
    unsigned* lcnt;      // per-cycle lengths, keyed by rep
    long long* tsum;     // cycle ratio: per-cycle times, keyed by rep
    int* cyc;            // cycle heads
    // giant rows (more than kGiantRow edges): the listed triples, the chunk
    // table, the rows' chunk ranges and the chunks' partial results
    unsigned gcap, ccap;
    int* gtri;
    int* cv;
    int* cs;
    int* ce;
    int* gv;
    int* gc0;
    int* gc1;
    void* gparts;
    size_t total;
};

Ws carve(void* base, int64_t n, int64_t m)
{
    char* b = (char*)base;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        size_t o = off;
        off += align_up(bytes);
        return b ? (void*)(b + o) : nullptr;
    };
    Ws w;
    const size_t N = (size_t)n;
    w.ctl = (Ctl*)take(sizeof(Ctl));
    w.V = (long long*)take(8 * N);
    w.Vhi = (long long*)take(8 * N);
    w.V32 = (int*)take(4 * N);
    w.Dhi[0] = (long long*)take(8 * N);
    w.Dhi[1] = (long long*)take(8 * N);
    w.pi = (int*)take(4 * N);
    w.succ = (int*)take(4 * N);
    w.hop = (int*)take(4 * N);
    w.Q[0] = (Jmp*)take(sizeof(Jmp) * N);
    w.Q[1] = (Jmp*)take(sizeof(Jmp) * N);
    w.rep = (int*)take(4 * N);
    w.onc = (unsigned char*)take(N);
    w.onC = (unsigned char*)take(N);
    w.layer = (int*)take(4 * N);
    w.list[0] = (int*)take(4 * N);
    w.list[1] = (int*)take(4 * N);
    const size_t M = (size_t)m;
    w.rdeg = (unsigned*)take(4 * (N + 1));
    w.stot = (unsigned*)take(4 * ((N + 1) / 2048 + 2));
    w.rin_ptr = (int*)take(4 * (N + 1));
    w.rin = (int*)take(4 * M);
    w.rscratch = take(ocm::rev_scratch_bytes(n, m));
    w.abits[0] = (unsigned*)take(4 * ((N + 31) / 32 + 1));
    w.abits[1] = (unsigned*)take(4 * ((N + 31) / 32 + 1));
    w.marks[0] = (unsigned char*)take(N + 16);
    w.marks[1] = (unsigned char*)take(N + 16);
    w.touched = (unsigned char*)take(N + 16);
    w.sel = take(32 * ocm::kSelectParts);
    w.xcap = (unsigned)(m < kTieListCap ? m : kTieListCap);
    w.xs = (int*)take(4 * (size_t)w.xcap);
    w.ys = (int*)take(4 * (size_t)w.xcap);
    w.wsum = (long long*)take(8 * N);
    w.lcnt = (unsigned*)take(4 * N);
    w.tsum = (long long*)take(8 * N);
    w.cyc = (int*)take(4 * N);
    w.gcap = (unsigned)(M / ocm::kGiantRow + 1);
    w.ccap = (unsigned)(M / ocm::kGiantChunk + w.gcap + 1);
    w.gtri = (int*)take(12 * (size_t)w.gcap);
    w.cv = (int*)take(4 * (size_t)w.ccap);
    w.cs = (int*)take(4 * (size_t)w.ccap);
    w.ce = (int*)take(4 * (size_t)w.ccap);
    w.gv = (int*)take(4 * (size_t)w.gcap);
    w.gc0 = (int*)take(4 * (size_t)w.gcap);
    w.gc1 = (int*)take(4 * (size_t)w.gcap);
    w.gparts = take(32 * (size_t)w.ccap);
    w.total = off;
    return w;
}

// Per-phase timing with hipEvents, when requested.
struct Prof {
    ocm_profile* out = nullptr;
    hipStream_t st = nullptr;
    struct Rec {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    int open = -1;
    void begin(int ph)
    {
        if (!out) return;
        Rec r{ph, nullptr, nullptr};
        if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
        (void)hipEventRecord(r.a, st);
        recs.push_back(r);
        open = (int)recs.size() - 1;
    }
    void end()
    {
        if (!out || open < 0) return;
        (void)hipEventRecord(recs[open].b, st);
        open = -1;
    }
    void bytes(int cls, double b)
    {
        if (out) out->bytes[cls] += b;
    }
    void finish()
    {
        if (!out) return;
        for (auto& r : recs) {
            float ms = 0.f;
            if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                out->ms[r.phase] += ms;
                out->launches[r.phase] += 1;
            }
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        recs.clear();
    }
};

struct Ctx {
    int n, m;
    const int* row_ptr;
    const int* col;
    const void* w;
    const int* t = nullptr;   // cycle ratio: edge times (>= 1); null for the mean
    int wtype;
    int neg;
    hipStream_t st;
    Ws ws;
    ocm::CtlView h;      // host snapshot of the control block
    Prof prof;
    int G;               // lanes per vertex in the sweep
    int sw;              // bytes per weight
    unsigned sweep_grid;
    bool tile_sweep = true;   // schedule 0: sweeps over vertex tiles, else G lanes per vertex
    bool count_tight = false;   // sweeps also count tight edges (tie check requested)
    bool swept_tie = false;     // the last sweep's counts are the tie scan's first pass
    // ws.succ holds col[pi] for every vertex of the workspace's policy: the
    // cycle and value inits then read it instead of gathering col[pi]; the
    // sweeps that count tight edges keep it so (the rebuild does not: its
    // scattered stores cost more than the gather they save)
    bool succ_ok = false;
    bool sweep_fused = false;   // the last sweep launched counts tight edges
    double sweep_vbytes = 8.0;  // bytes per value the last sweep gathered
    unsigned long long swept_tight = 0, swept_certain = 0;
    int jump_rounds = 0;
    int connect_rounds = 0;
    int connect_mode = 0;   // 0 auto, 1 pull only, 2 push only
    bool rev_built = false;
    // reverse CSR built early on a side stream: rev_done is recorded there
    // when it is complete; the solve's stream waits for it before use
    bool rev_pending = false;
    hipEvent_t rev_in = nullptr, rev_done = nullptr;
    int64_t push_frontier = 0;
    int general_iters = 0;
    int value_rounds = 0;
    // the call may not allocate: control reads go through a stack copy
    // instead of the pinned mailbox, and no side stream or event is created
    bool noalloc = false;
    // values are int128 (split lo / hi): set once a value leaves the int64
    // range (or on request), for the rest of the solve
    bool wide = false;
    bool allow_wide = false;
    // ws.V32 holds V as int32 (every value of the last value phase fit):
    // sweeps then gather 4-byte values
    bool v32 = false;
    // rows of more than kGiantRow edges, swept by several workgroups each
    // (tile sweeps only; empty when there are none)
    ocm::GiantTab giant;

    Ctx() = default;
    Ctx(const Ctx&) = delete;
    Ctx& operator=(const Ctx&) = delete;
    ~Ctx()
    {
        // every exit path: the side stream's writes into the workspace end
        // before the solve returns
        if (rev_pending) {
            (void)hipStreamWaitEvent(st, rev_done, 0);
            (void)hipEventSynchronize(rev_done);
        }
        if (rev_in) (void)hipEventDestroy(rev_in);
        if (rev_done) (void)hipEventDestroy(rev_done);
    }
};

// Push rounds pay off once many vertices are unattached and the frontier is
// small next to them; below this size pull rounds are cheap anyway.
constexpr unsigned kPushMinUnattached = 1u << 16;

ocm_status read_ctl(Ctx& c)
{
    if (c.noalloc) {
        HIP_TRY(ocm::host_read_ctl_copy(c.ws.ctl, &c.h, c.st));
        return OCM_OK;
    }
    HIP_TRY(ocm::host_read_ctl(c.ws.ctl, &c.h, c.st));
    return OCM_OK;
}

int choose_lanes(int64_t n, int64_t m, int schedule)
{
    if (schedule > 0) return schedule;
    const double d = (double)m / (double)n;
    int G = 1;
    while (G < 64 && G < d) G <<= 1;
    return G;
}

unsigned sweep_grid(int64_t n, int G)
{
    const int64_t vpb = ocm::kWG / G;
    int64_t g = (n + vpb - 1) / vpb;
    if (g > 8192) g = 8192;
    if (g >= 8) g &= ~int64_t(7);
    return (unsigned)(g < 1 ? 1 : g);
}

bool valid_lanes(int G) { return G == 1 || G == 2 || G == 4 || G == 8 || G == 16 || G == 32 || G == 64; }

ocm_status check_graph(const ocm_graph* g)
{
    if (!g) return fail(OCM_E_INVALID_ARG, "graph is null");
    if (g->n < 1 || g->m < 1) return fail(OCM_E_INVALID_ARG, "n and m must be >= 1");
    if (g->n >= (int64_t(1) << 31) - 1 || g->m >= (int64_t(1) << 31))
        return fail(OCM_E_INVALID_ARG, "n and m must stay below 2^31");
    if (!g->row_ptr || !g->col || !g->w) return fail(OCM_E_INVALID_ARG, "null graph array");
    if (g->wtype != OCM_W_I32 && g->wtype != OCM_W_I64) return fail(OCM_E_INVALID_ARG, "bad wtype");
    return OCM_OK;
}

ocm_status setup(Ctx& c, const ocm_graph* g, int neg, void* ws, size_t ws_bytes, void* stream,
                 ocm_profile* prof)
{
    OCM_TRY(check_graph(g));
    c.n = (int)g->n;
    c.m = (int)g->m;
    c.row_ptr = g->row_ptr;
    c.col = g->col;
    c.w = g->w;
    c.wtype = g->wtype;
    c.sw = g->wtype == OCM_W_I64 ? 8 : 4;
    c.neg = neg;
    c.st = (hipStream_t)stream;
    c.ws = carve(nullptr, g->n, g->m);
    if (!ws || ws_bytes < c.ws.total) return fail(OCM_E_WORKSPACE, "workspace missing or too small");
    c.ws = carve(ws, g->n, g->m);
    c.prof.out = prof;
    c.prof.st = c.st;
    memset(&c.h, 0, sizeof c.h);
    // the workspace may hold anything: every entry point starts from a clean
    // control block
    ocm::launch_ctl_clear(c.ws.ctl, ocm::kClrAll | ocm::kClrCount | ocm::kClrChanged, c.st);
    HIP_TRY(hipGetLastError());
    return OCM_OK;
}

// Validation kernel, then the bound that keeps every value inside int64:
// |L*w - W| <= 2 n max|w| must stay below 2^62.
ocm_status validate(Ctx& c, int check_csr)
{
    ocm::launch_ctl_clear(c.ws.ctl, ocm::kClrAll | ocm::kClrCount | ocm::kClrChanged, c.st);
    c.prof.begin(OCM_K_VALIDATE);
    ocm::launch_validate(c.n, c.m, c.row_ptr, c.col, c.w, c.wtype, check_csr, c.ws.ctl, c.st);
    c.prof.end();
    c.prof.bytes(OCM_K_VALIDATE, 4.0 * (c.n + 1) + (check_csr ? 4.0 * c.m : 0.0) + c.sw * (double)c.m);
    HIP_TRY(hipGetLastError());
    OCM_TRY(read_ctl(c));
    if (c.h.err & ocm::kErrBadCsr) return fail(OCM_E_BAD_CSR, "malformed CSR");
    if (c.h.err & ocm::kErrNoOut) return fail(OCM_E_NO_OUT_EDGE, "a vertex has no out-edge");
    const unsigned long long maxw = c.h.maxabsw;
    unsigned long long maxt = 1;
    if (c.t) {
        // |T w - W t| <= 2 n max|w| max t for a cycle's (W, T)
        ocm::launch_ctl_clear(c.ws.ctl, ocm::kClrAll, c.st);
        ocm::launch_validate_t(c.m, c.t, c.ws.ctl, c.st);
        HIP_TRY(hipGetLastError());
        OCM_TRY(read_ctl(c));
        if (c.h.bad) return fail(OCM_E_INVALID_ARG, "edge times must be integers >= 1");
        maxt = c.h.maxabsw;
    }
    const unsigned __int128 bound = (unsigned __int128)2 * (unsigned)c.n * maxw * maxt;
    if (bound >= ((unsigned __int128)1 << 62)) return fail(OCM_E_OVERFLOW, "weights too large for int64 values");
    return OCM_OK;
}

// Policy improvement sweep; afterwards c.h.changed / cbroken are current.
// The sweep's bookkeeping once c.h holds the control block after it.
void sweep_done(Ctx& c, bool first, bool tie, bool fused)
{
    c.swept_tie = fused;
    c.swept_tight = c.h.tight;
    c.swept_certain = c.h.certain;
    // col + w per edge, row_ptr per vertex; after the first sweep also the
    // gathered V per edge and the own V per vertex; the tie scan (and a
    // sweep that counts tight edges) reads pi; policy writes of changed
    // vertices
    const double n = c.n, m = c.m;
    double b = m * (4.0 + c.sw) + 4.0 * (n + 1);
    // values gathered as int64, int128 (two words) or from the int32 copy
    const double sv = c.sweep_vbytes;
    if (!first) b += sv * m + sv * n;
    if (tie || fused) b += 4.0 * n;
    if (!tie) b += 4.0 * (double)c.h.changed;
    c.prof.bytes(tie ? OCM_K_TIESCAN : OCM_K_SWEEP, b);
}

// read = false: the caller reads the control block later (after more work
// queued behind the sweep) and then calls sweep_done.
ocm_status phase_sweep(Ctx& c, bool first, bool tie, const long long* V, long long W, long long L,
                       int* pi, const unsigned char* onC, bool collect = false,
                       bool with_hop = false, bool read = true)
{
    ocm::launch_ctl_clear(c.ws.ctl, ocm::kClrChanged, c.st);
    ocm::SweepArgs a;
    a.n = c.n;
    a.neg = c.neg;
    a.row_ptr = c.row_ptr;
    a.col = c.col;
    a.V = V;
    a.Vhi = c.wide && V == c.ws.V ? c.ws.Vhi : nullptr;
    a.V32 = !c.wide && c.v32 && V == c.ws.V && !first ? c.ws.V32 : nullptr;
    a.t = first ? nullptr : c.t;
    a.W = W;
    a.L = L;
    a.pi = pi;
    a.succ = nullptr;
    a.onC = onC;
    a.ctl = c.ws.ctl;
    a.giant = c.tile_sweep ? c.giant : ocm::GiantTab{};
    a.hop = tie && with_hop ? c.ws.hop : nullptr;
    a.xs = a.ys = nullptr;
    a.xcnt = nullptr;
    a.xcap = 0;
    if (tie && collect) {
        a.xs = c.ws.xs;
        a.ys = c.ws.ys;
        a.xcnt = &c.ws.ctl->xcnt;
        a.xcap = c.ws.xcap;
    }
    const int cls = tie ? OCM_K_TIESCAN : OCM_K_SWEEP;
    const bool fused = !tie && !first && c.tile_sweep && c.count_tight;
    // a sweep that changes pi without updating succ leaves it stale; the
    // first tile sweep writes every vertex's, so succ is whole after it
    const bool keep = pi == c.ws.pi && (first ? c.tile_sweep : fused && c.succ_ok);
    a.succ = keep ? c.ws.succ : nullptr;
    if (!tie && !keep) c.succ_ok = false;
    if (keep && first) c.succ_ok = true;
    c.prof.begin(cls);
    ocm::launch_sweep(a, c.w, c.wtype, c.tile_sweep ? 0 : c.G, first, tie, fused, c.sweep_grid,
                      c.st);
    c.prof.end();
    HIP_TRY(hipGetLastError());
    c.sweep_fused = fused;
    c.sweep_vbytes = a.Vhi ? 16.0 : a.V32 ? 4.0 : 8.0;
    if (!read) return OCM_OK;
    OCM_TRY(read_ctl(c));
    sweep_done(c, first, tie, fused);
    return OCM_OK;
}

// Giant rows: listed on the device; their chunk table is built on the host
// (rows by vertex, each row's chunks in position order, so that the merge
// keeps the lowest position among equal keys) and copied to the workspace.
// Only the tile sweeps use it.
ocm_status build_giant(Ctx& c)
{
    Ws& w = c.ws;
    c.giant = ocm::GiantTab{};
    if (!c.tile_sweep || c.m <= ocm::kGiantRow) return OCM_OK;
    ocm::launch_ctl_clear(w.ctl, ocm::kClrGiant, c.st);
    ocm::launch_giant_list(c.n, c.row_ptr, w.gtri, w.gcap, w.ctl, c.st);
    HIP_TRY(hipGetLastError());
    OCM_TRY(read_ctl(c));
    const unsigned ng = c.h.ngiant;
    if (ng == 0) return OCM_OK;
    if (ng > w.gcap) return fail(OCM_E_HIP, "more giant rows than the edges allow");
    std::vector<int> tri(3 * (size_t)ng);
    HIP_TRY(hipMemcpyAsync(tri.data(), w.gtri, 12 * (size_t)ng, hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    std::vector<int> order(ng);
    for (unsigned i = 0; i < ng; ++i) order[i] = (int)i;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return tri[3 * x] < tri[3 * y]; });
    std::vector<int> cv, cs, ce, gv(ng), gc0(ng), gc1(ng);
    for (unsigned k = 0; k < ng; ++k) {
        const int i = order[k], v = tri[3 * i], b = tri[3 * i + 1], e = tri[3 * i + 2];
        gv[k] = v;
        gc0[k] = (int)cv.size();
        for (int x = b; x < e; x += ocm::kGiantChunk) {
            cv.push_back(v);
            cs.push_back(x);
            ce.push_back(e - x > ocm::kGiantChunk ? x + ocm::kGiantChunk : e);
        }
        gc1[k] = (int)cv.size();
    }
    const size_t nc = cv.size();
    if (nc > w.ccap) return fail(OCM_E_HIP, "more giant-row chunks than the workspace holds");
    HIP_TRY(hipMemcpyAsync(w.cv, cv.data(), 4 * nc, hipMemcpyHostToDevice, c.st));
    HIP_TRY(hipMemcpyAsync(w.cs, cs.data(), 4 * nc, hipMemcpyHostToDevice, c.st));
    HIP_TRY(hipMemcpyAsync(w.ce, ce.data(), 4 * nc, hipMemcpyHostToDevice, c.st));
    HIP_TRY(hipMemcpyAsync(w.gv, gv.data(), 4 * (size_t)ng, hipMemcpyHostToDevice, c.st));
    HIP_TRY(hipMemcpyAsync(w.gc0, gc0.data(), 4 * (size_t)ng, hipMemcpyHostToDevice, c.st));
    HIP_TRY(hipMemcpyAsync(w.gc1, gc1.data(), 4 * (size_t)ng, hipMemcpyHostToDevice, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));   // the host vectors end here
    c.giant.cv = w.cv;
    c.giant.cs = w.cs;
    c.giant.ce = w.ce;
    c.giant.nchunks = (int)nc;
    c.giant.gv = w.gv;
    c.giant.gc0 = w.gc0;
    c.giant.gc1 = w.gc1;
    c.giant.ngiant = (int)ng;
    c.giant.parts = w.gparts;
    return OCM_OK;
}

// Cycles of the policy graph: rep and on_cycle for every vertex.  At most
// K = ceil(log2 n) jump rounds; the stop test of k_pj_round ends the phase as
// soon as every jump pointer is on its cycle and the window minima are fixed.
// Rounds queued between two host reads of the control block when the device
// decides when rounds end (rebuild, cycles, values).
constexpr int kRoundsPerRead = 8;

// Cycle rounds with the stop test decided on the device: K rounds at most,
// queued kRoundsPerRead at a time with the final after each batch.
ocm_status cycle_rounds_on_device(Ctx& c, int K, unsigned long long* P0, unsigned long long* P1,
                                  unsigned char* const tag[2], int* rep, unsigned char* onc)
{
    unsigned long long* P[2] = {P0, P1};
    ocm::launch_jump_setup(c.ws.ctl, false, false, c.st);
    int r = 0;
    for (;;) {
        for (int j = 0; j < kRoundsPerRead && r < K; ++j) {
            ++r;
            ocm::launch_pj_round_dev(c.n, r, P[(r - 1) & 1], P[r & 1], tag[(r - 1) & 1], tag[r & 1],
                                     c.ws.ctl, c.st);
        }
        ocm::launch_pj_final_dev(c.n, P0, P1, K, rep, onc, c.ws.ctl, c.st);
        HIP_TRY(hipGetLastError());
        OCM_TRY(read_ctl(c));
        if (c.h.jmode == 0 || c.h.jk == (unsigned)K) break;
        if (r >= K) return fail(OCM_E_HIP, "cycle rounds did not finish");
    }
    c.jump_rounds += (int)c.h.jk;
    return OCM_OK;
}

ocm_status phase_cycles(Ctx& c, const int* pi, int* rep, unsigned char* onc)
{
    auto* P0 = (unsigned long long*)c.ws.Q[0];
    auto* P1 = (unsigned long long*)c.ws.Q[1];
    int K = 0;
    while ((int64_t(1) << K) < c.n) ++K;
    const double n = c.n;
    // the two tag arrays live in the layer array, which the rebuild rewrites
    unsigned char* tag[2] = {(unsigned char*)c.ws.layer, (unsigned char*)c.ws.layer + c.n};
    const bool stop_test = K > 2;
    c.prof.begin(OCM_K_CYCLES);
    if (stop_test) ocm::launch_fill_u32((unsigned*)c.ws.layer, ((int64_t)c.n * 2 + 3) / 4, 0u, c.st);
    const bool have_succ = c.succ_ok && pi == c.ws.pi;
    ocm::launch_pj_init(c.n, c.col, pi, c.ws.succ, have_succ, P0, onc, stop_test ? tag[0] : nullptr,
                        stop_test && c.prof.out ? c.ws.ctl->lane[0].pjc : nullptr, c.st);
    c.prof.end();
    c.succ_ok = pi == c.ws.pi;
    // pi, col[pi], succ, packed entry, on-cycle (+ tag clear and mark)
    c.prof.bytes(OCM_K_CYCLES, 21.0 * n + (stop_test ? 3.0 * n : 0.0));
    HIP_TRY(hipGetLastError());
    if (stop_test && !c.prof.out) return cycle_rounds_on_device(c, K, P0, P1, tag, rep, onc);
    long long img_prev = -1;
    int r = 0;
    while (r < K) {
        ++r;
        c.prof.begin(OCM_K_CYCLES);
        if (stop_test)
            ocm::launch_pj_round_tagged(c.n, r, P0, P1, tag[(r - 1) & 1], tag[r & 1],
                                        c.ws.ctl->lane[0].pjc, c.st);
        else
            ocm::launch_pj_round(c.n, P0, P1, c.st);
        c.prof.end();
        // own entry, gathered entry, new entry (+ tag read and mark)
        c.prof.bytes(OCM_K_CYCLES, (stop_test ? 26.0 : 24.0) * n);
        std::swap(P0, P1);
        if (stop_test && r < K) {
            HIP_TRY(hipGetLastError());
            OCM_TRY(read_ctl(c));
            const long long img = c.h.pjc[2 * (r & 1)];
            const unsigned chg = c.h.pjc[2 * (r & 1) + 1];
            if (r >= 2 && img == img_prev && chg == 0) break;
            img_prev = img;
        }
    }
    c.prof.begin(OCM_K_CYCLES);
    ocm::launch_pj_final(c.n, P0, rep, onc, c.st);
    c.prof.end();
    c.prof.bytes(OCM_K_CYCLES, 21.0 * n);
    c.jump_rounds += r;
    HIP_TRY(hipGetLastError());
    return OCM_OK;
}

// Minimum-mean cycle in the order (W/L, rep); c.h gets s, W, L, ncyc.
ocm_status phase_select(Ctx& c, const int* pi, const int* rep, const unsigned char* onc)
{
    ocm::launch_ctl_clear(c.ws.ctl, ocm::kClrCount, c.st);
    c.prof.begin(OCM_K_SELECT);
    long long* tsum = c.t ? c.ws.tsum : nullptr;
    ocm::launch_cyc_zero(c.n, rep, onc, c.ws.wsum, c.ws.lcnt, c.ws.cyc, c.ws.ctl, c.st, tsum);
    ocm::launch_cyc_sum(c.n, rep, onc, pi, c.w, c.wtype, c.neg, c.ws.wsum, c.ws.lcnt, c.st, c.t,
                        tsum);
    ocm::launch_select(c.ws.cyc, c.ws.wsum, c.ws.lcnt, c.ws.ctl, c.ws.sel, c.st, tsum);
    c.prof.end();
    c.prof.bytes(OCM_K_SELECT, 6.0 * c.n);   // rep and on-cycle flags, twice
    HIP_TRY(hipGetLastError());
    OCM_TRY(read_ctl(c));
    if (c.h.ncyc == 0 || c.h.s < 0) return fail(OCM_E_HIP, "no policy cycle found");
    return OCM_OK;
}

// The rebuild rounds without a host round trip per round: each round's
// direction is picked on the device by the round before it (same rule as the
// host loop below), two kernels are queued per round (marks or a pull round,
// then the claims and the next round's marks), and the host reads the state
// back every kRoundsPerRead rounds.  Rounds queued after the last one do
// nothing.

// Reverse CSR for push rounds, once per solve, on stream st; both mark
// arrays start clear.
void launch_reverse(Ctx& c, hipStream_t st)
{
    Ws& w = c.ws;
    ocm::launch_rev_build(c.n, c.m, c.row_ptr, c.col, w.rdeg, w.stot, w.rin_ptr, w.rin,
                          w.marks[0], w.rscratch, st);
    ocm::launch_fill_u32((unsigned*)w.marks[1], ((int64_t)c.n + 3) / 4, 0u, st);
}

// The reverse CSR, ready on the solve's stream: the early build's (waited
// for) or one built now.
void build_reverse(Ctx& c)
{
    if (c.rev_pending) {
        (void)hipStreamWaitEvent(c.st, c.rev_done, 0);
        c.rev_pending = false;
    } else {
        launch_reverse(c, c.st);
    }
    c.rev_built = true;
}

// One side stream per device (default priority, non-blocking), kept for
// the life of the process.
hipStream_t side_stream()
{
    static std::mutex mu;
    static std::map<int, hipStream_t> streams;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = streams.find(dev);
    if (it != streams.end()) return it->second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    streams[dev] = s;
    return s;
}

// A cold solve's first iteration always rebuilds; on a large graph that
// rebuild pushes and needs the reverse CSR, which depends on the graph only.
// Build it on a side stream right after validation, so that it overlaps the
// first sweep and the cycle phase.  Not with the per-phase profile (its
// timings stay per kernel), not for pull-only rebuilds.
void start_reverse_early(Ctx& c)
{
    if (c.noalloc || c.prof.out || c.rev_built || c.connect_mode == 1 ||
        c.n < 2 * (int64_t)kPushMinUnattached)
        return;
    hipStream_t side = side_stream();
    if (!side) return;
    if (hipEventCreateWithFlags(&c.rev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c.rev_done, hipEventDisableTiming) != hipSuccess)
        return;
    if (hipEventRecord(c.rev_in, c.st) != hipSuccess || hipStreamWaitEvent(side, c.rev_in, 0) != hipSuccess)
        return;
    launch_reverse(c, side);
    if (hipEventRecord(c.rev_done, side) != hipSuccess) {
        // the build is queued; make the solve's stream wait for it anyway
        (void)hipStreamSynchronize(side);
        return;
    }
    c.rev_pending = true;
}

ocm_status connect_rounds_on_device(Ctx& c, int* pi, int* layer, unsigned left, unsigned front,
                                    int* rounds)
{
    Ws& w = c.ws;
    const int policy = c.connect_mode;   // 0 automatic, 1 pull, 2 push
    const bool may_push = policy == 2 || (policy == 0 && left >= kPushMinUnattached);
    if (may_push && !c.rev_built) {
        build_reverse(c);
        HIP_TRY(hipGetLastError());
    }
    ocm::launch_round_setup(w.ctl, left, front, policy, kPushMinUnattached, c.st);
    unsigned long long* pedges = &w.ctl->lane[0].pedges;
    // the host's guess of the next rounds' direction (the device's rule on
    // the counts it last read): while it says push, rounds after the first
    // take one kernel each; a wrong guess costs time, not results
    bool guess_push = left > 0 && (policy == 2 || (policy == 0 && left >= kPushMinUnattached &&
                                                   2ull * front < left));
    int k = 0;
    for (;;) {
        for (int j = 0; j < kRoundsPerRead; ++j) {
            ++k;
            ocm::launch_round(k, c.n, c.row_ptr, c.col, w.rin_ptr, w.rin, w.abits[k & 1],
                              w.abits[(k + 1) & 1], w.marks[k & 1], w.marks[(k + 1) & 1], pi,
                              layer, w.ctl, pedges, policy, kPushMinUnattached, may_push,
                              k > 1 && guess_push, c.st);
        }
        HIP_TRY(hipGetLastError());
        OCM_TRY(read_ctl(c));
        if (c.h.rerr || c.h.rleft == 0) break;
        if (k > c.n + kRoundsPerRead) return fail(OCM_E_HIP, "rebuild rounds did not finish");
        guess_push = c.h.rmode == 1u;
    }
    if (rounds) *rounds = (int)c.h.rk;
    c.connect_rounds += (int)c.h.rk;
    if (c.h.rerr) return fail(OCM_E_NOT_STRONGLY_CONNECTED, "some vertex cannot reach the chosen cycle");
    return OCM_OK;
}

// Rebuild around C: component of C keeps pi, the rest attaches breadth-first.
// Each round is a pull or a push round (same result, see k_conn_claim).
ocm_status phase_connect(Ctx& c, const int* rep, const unsigned char* onc, int s, int* pi,
                         int* layer, unsigned char* onC, int* rounds)
{
    Ws& w = c.ws;
    c.succ_ok = false;   // the rebuild rewires pi and leaves succ behind
    ocm::launch_ctl_clear(w.ctl, ocm::kClrCount, c.st);
    c.prof.begin(OCM_K_CONN_PULL);
    // round 1 reads abits[1] (C's component) and completes abits[0]
    ocm::launch_conn_init(c.n, rep, onc, s, layer, onC, w.abits[1], w.abits[0], w.ctl, c.st);
    c.prof.end();
    HIP_TRY(hipGetLastError());
    OCM_TRY(read_ctl(c));
    // rep, layer and on-C flags per vertex; the two bitmaps
    c.prof.bytes(OCM_K_CONN_PULL, 6.25 * c.n);
    unsigned long long pe0 = c.h.pedges, le0 = c.h.ledges;
    unsigned left = c.h.left, front = c.h.got;
    if (!c.prof.out && left > 0) return connect_rounds_on_device(c, pi, layer, left, front, rounds);
    const double bitmaps = 0.125 * c.n;   // one attached-vertex bitmap
    unsigned long long* pedges = &w.ctl->lane[0].pedges;
    // the scanned-edge counts only feed the profile's byte figures
    unsigned long long* ledges = c.prof.out ? &w.ctl->lane[0].ledges : nullptr;
    int k = 0;
    int marked = 0;   // the round whose marks the last push round left
    ocm_status rc = OCM_OK;
    while (left > 0) {
        ++k;
        bool push = false;
        if (c.connect_mode == 2) push = front > 0;
        else if (c.connect_mode == 0)
            push = left >= kPushMinUnattached && (uint64_t)front * 2 < left;
        if (push && !c.rev_built) {
            c.prof.begin(OCM_K_REVERSE);
            build_reverse(c);
            c.prof.end();
            // count: col + counter per edge; fill, scan and copy of the
            // counters; fill: row_ptr, col, cursor and the 4-byte tail per
            // edge; mark reset
            c.prof.bytes(OCM_K_REVERSE, 20.0 * c.m + 29.0 * c.n);
            HIP_TRY(hipGetLastError());
        }
        // round k reads abits[k&1] and completes abits[(k+1)&1]
        const unsigned* acur = w.abits[k & 1];
        unsigned* anext = w.abits[(k + 1) & 1];
        ocm::launch_ctl_clear(w.ctl, ocm::kClrCount, c.st);
        const bool standalone = push && marked != k;
        if (push) {
            if (standalone) {
                c.prof.begin(OCM_K_CONN_MARK);
                ocm::launch_conn_mark(c.n, w.rin_ptr, w.rin, acur, anext, w.marks[k & 1], pedges,
                                      nullptr, nullptr, c.st);
                c.prof.end();
                HIP_TRY(hipGetLastError());
                OCM_TRY(read_ctl(c));
                // both bitmaps; per frontier vertex its offsets, per in-edge
                // the 4-byte tail (its mark bytes are booked below)
                c.prof.bytes(OCM_K_CONN_MARK,
                             2.0 * bitmaps + 8.0 * front + 4.0 * (double)(c.h.pedges - pe0));
                pe0 = c.h.pedges;
            }
            c.prof.begin(OCM_K_CONN_CLAIM);
            ocm::launch_conn_claim(k, c.n, c.row_ptr, c.col, acur, anext, w.marks[k & 1], pi, layer,
                                   w.ctl, ledges, nullptr, nullptr, w.rin_ptr, w.rin,
                                   w.marks[(k + 1) & 1], pedges, c.st);
            c.prof.end();
            marked = k + 1;
            c.push_frontier += front;
        } else {
            c.prof.begin(OCM_K_CONN_PULL);
            ocm::launch_conn_pull(k, c.n, c.row_ptr, c.col, acur, anext, layer, pi, w.ctl, ledges,
                                  nullptr, nullptr, marked == k ? w.marks[k & 1] : nullptr, c.st);
            c.prof.end();
        }
        HIP_TRY(hipGetLastError());
        OCM_TRY(read_ctl(c));
        const unsigned got = c.h.got;
        const double S = (double)(c.h.ledges - le0);
        if (push) {
            // claims: the mark bytes and both bitmaps (acur read, anext
            // written); per attached vertex its offsets, pi and (when
            // requested) layer; per scanned out-edge col and a bit.  The
            // next round's marks: per attached vertex its in-edge offsets,
            // per in-edge the 4-byte tail.  This round's attachments are the
            // vertices marked for it, a byte each, booked to the step that
            // marked them
            const double E = (double)(c.h.pedges - pe0);
            c.prof.bytes(OCM_K_CONN_CLAIM, (double)c.n + 2.0 * bitmaps + (layer ? 16.0 : 12.0) * got +
                                               4.125 * S + 8.0 * got + 4.0 * E);
            c.prof.bytes(standalone ? OCM_K_CONN_MARK : OCM_K_CONN_CLAIM, (double)got);
        } else {
            // both bitmaps; per unattached vertex its offsets, per scanned
            // out-edge col and a bit; pi (and layer) of the attached
            c.prof.bytes(OCM_K_CONN_PULL, 3.0 * bitmaps + 8.0 * left + 4.125 * S + (layer ? 8.0 : 4.0) * got);
        }
        pe0 = c.h.pedges;
        le0 = c.h.ledges;
        if (got == 0) {
            rc = fail(OCM_E_NOT_STRONGLY_CONNECTED, "some vertex cannot reach the chosen cycle");
            break;
        }
        left -= got;
        front = got;
    }
    if (rounds) *rounds = k;
    c.connect_rounds += k;
    return rc;
}

// Values by pointer jumping toward s.  With `probe` set the policy graph may
// hold vertices that never reach s; the phase then stops as soon as a round
// finishes no vertex and reports *stalled = true (no values written).
// Otherwise every vertex must reach s.  *qfinal is the buffer holding the
// final entries (their hop counts list C).
// Value rounds decided on the device after the init: kRoundsPerRead rounds
// and the final per host read, until every vertex finished or a round
// finished none (a stall: the policy graph does not reach s).
ocm_status value_rounds_on_device(Ctx& c, int s, long long* V, int* hop, bool probe, bool* stalled,
                                  int* rounds, bool gated)
{
    ocm::launch_jump_setup(c.ws.ctl, true, gated, c.st);
    Ws& w = c.ws;
    int r = 0;
    for (;;) {
        for (int j = 0; j < kRoundsPerRead; ++j) {
            ++r;
            if (c.wide)
                ocm::launch_val_round_dev(c.n, s, r, w.Q[(r - 1) & 1], w.Q[r & 1], w.ctl, c.st,
                                          w.Dhi[(r - 1) & 1], w.Dhi[r & 1]);
            else
                ocm::launch_val_round_dev(c.n, s, r, w.Q[(r - 1) & 1], w.Q[r & 1], w.ctl, c.st);
        }
        if (c.wide)
            ocm::launch_val_final_dev(c.n, w.Q[0], w.Q[1], V, hop, w.ctl, c.st, w.Dhi[0], w.Dhi[1],
                                      w.Vhi);
        else
            ocm::launch_val_final_dev(c.n, w.Q[0], w.Q[1], V, hop, w.ctl, c.st, nullptr, nullptr,
                                      nullptr, V == w.V ? w.V32 : nullptr);
        HIP_TRY(hipGetLastError());
        OCM_TRY(read_ctl(c));
        if (c.h.jmode == 0) break;
        if (r > 64) return fail(OCM_E_HIP, "value propagation did not converge");
    }
    const int k = (int)c.h.jk;
    c.jump_rounds += k;
    c.value_rounds += k;
    if (rounds) *rounds = k;
    // the int32 copy is current when the phase ran to its end (a gated phase
    // runs iff the sweep queued before it changed a policy edge and no
    // vertex of C)
    if (V == c.ws.V && !c.h.jstall && (!gated || (!c.h.cbroken && c.h.changed > 0)))
        c.v32 = !c.wide && !c.h.wide32;
    if (c.h.jstall) {
        if (probe) {
            if (stalled) *stalled = true;
            return OCM_OK;
        }
        return fail(OCM_E_NOT_STRONGLY_CONNECTED, "policy graph does not reach the source");
    }
    if (c.h.overflow) return fail(OCM_E_OVERFLOW, "a value left [-2^62, 2^62]");
    return OCM_OK;
}

// gated (rounds decided on the device only): the phase runs only if
// ctl->jgate is open (k_fast_gate); a closed gate leaves V as it was.
ocm_status phase_values_once(Ctx& c, const int* pi, int s, long long W, long long L, long long* V,
                             int* hop, bool probe, bool* stalled, int* rounds, bool gated)
{
    if (stalled) *stalled = false;
    ocm::launch_ctl_clear(c.ws.ctl, ocm::kClrCount, c.st);
    const int ph = probe ? OCM_K_FAST : OCM_K_VALUES;
    c.prof.begin(ph);
    const bool have_succ = c.succ_ok && pi == c.ws.pi;
    ocm::launch_val_init(c.n, c.col, pi, c.w, c.wtype, c.neg, s, W, L, c.ws.succ, have_succ,
                         c.ws.Q[0], c.ws.ctl, gated ? &c.ws.ctl->jgate : nullptr, c.st,
                         c.wide ? c.ws.Dhi[0] : nullptr, c.t);
    // a gated init that does not run leaves succ as it was
    if (!gated) c.succ_ok = pi == c.ws.pi;
    c.prof.end();
    c.prof.bytes(ph, (28.0 + c.sw) * c.n);   // pi, col[pi], w[pi], succ, 16-byte entry
    HIP_TRY(hipGetLastError());
    if (!c.prof.out) return value_rounds_on_device(c, s, V, hop, probe, stalled, rounds, gated);
    OCM_TRY(read_ctl(c));
    unsigned act = c.h.active;
    int a = 0, k = 0;
    while (act > 0) {
        if (k > 64) return fail(OCM_E_HIP, "value propagation did not converge");
        ++k;
        ++c.value_rounds;
        const int b = a ^ 1;
        ocm::launch_ctl_clear(c.ws.ctl, ocm::kClrActive2, c.st);
        c.prof.begin(ph);
        if (c.wide)
            ocm::launch_val_round(c.n, s, c.ws.Q[a], c.ws.Q[b], &c.ws.ctl->lane[0].active2, c.st,
                                  c.ws.Dhi[a], c.ws.Dhi[b]);
        else
            ocm::launch_val_round(c.n, s, c.ws.Q[a], c.ws.Q[b], &c.ws.ctl->lane[0].active2, c.st);
        c.prof.end();
        c.prof.bytes(ph, 32.0 * c.n + 16.0 * act);   // own + new entry; gather if unfinished
        HIP_TRY(hipGetLastError());
        OCM_TRY(read_ctl(c));
        const unsigned now = c.h.active2;
        a = b;
        if (now == act) {
            c.jump_rounds += k;
            if (rounds) *rounds = k;
            if (probe) {
                if (stalled) *stalled = true;
                return OCM_OK;
            }
            return fail(OCM_E_NOT_STRONGLY_CONNECTED, "policy graph does not reach the source");
        }
        act = now;
    }
    c.jump_rounds += k;
    if (rounds) *rounds = k;
    c.prof.begin(ph);
    if (c.wide) ocm::launch_val_final(c.n, c.ws.Q[a], V, hop, c.ws.ctl, c.st, c.ws.Dhi[a], c.ws.Vhi);
    else
        ocm::launch_val_final(c.n, c.ws.Q[a], V, hop, c.ws.ctl, c.st, nullptr, nullptr,
                              V == c.ws.V ? c.ws.V32 : nullptr);
    c.prof.end();
    c.prof.bytes(ph, 24.0 * c.n);
    HIP_TRY(hipGetLastError());
    OCM_TRY(read_ctl(c));
    if (V == c.ws.V) c.v32 = !c.wide && !c.h.wide32;
    if (c.h.overflow) return fail(OCM_E_OVERFLOW, "a value left [-2^62, 2^62]");
    return OCM_OK;
}

// Value phase; when a value leaves the int64 range (only int64 values are
// checked), the phase is run again with int128 values, which the rest of the
// solve keeps (sweeps and the tie check read them).  The overflowing phase's
// V is discarded: its inputs (pi, s, W, L) are unchanged.
ocm_status phase_values(Ctx& c, const int* pi, int s, long long W, long long L, long long* V,
                        int* hop, bool probe, bool* stalled, int* rounds, bool gated = false)
{
    const ocm_status rc = phase_values_once(c, pi, s, W, L, V, hop, probe, stalled, rounds, gated);
    if (rc != OCM_E_OVERFLOW || c.wide || !c.allow_wide || V != c.ws.V) return rc;
    c.wide = true;
    return phase_values_once(c, pi, s, W, L, V, hop, probe, stalled, rounds, false);
}

// Does the small graph (nodes 0..N-1, edges from adjacency lists) hold a
// cycle?  Iterative three-colour depth-first search.
bool has_cycle(int N, const std::vector<int>& head, const std::vector<int>& next,
               const std::vector<int>& to)
{
    std::vector<unsigned char> col(N, 0);
    std::vector<std::pair<int, int>> st;
    for (int r = 0; r < N; ++r) {
        if (col[r]) continue;
        col[r] = 1;
        st.push_back({r, head[r]});
        while (!st.empty()) {
            auto& top = st.back();
            if (top.second < 0) {
                col[top.first] = 2;
                st.pop_back();
                continue;
            }
            const int e = top.second;
            top.second = next[e];
            const int u = to[e];
            if (col[u] == 1) return true;
            if (col[u] == 0) {
                col[u] = 1;
                st.push_back({u, head[u]});
            }
        }
    }
    return false;
}

// Exact uniqueness of C at the optimum.  A cycle is critical iff all its
// edges are tight (the potential is feasible and reduced costs sum to zero
// around critical cycles); policy edges are tight and hold only C.  So C is
// the unique critical cycle iff no tight non-policy edge closes a cycle of
// the tight subgraph.  Quick exact answers first (no such edge; a tight
// self-loop; a tight edge leaving C), then the compressed special-vertex
// graph described at k_tie_mark.
ocm_status tie_from_list(Ctx& c, unsigned kx, ocm_result* out);

ocm_status tie_check(Ctx& c, long long W, long long L, ocm_result* out)
{
    Ws& w = c.ws;
    // the solve's last sweep changed nothing; if it counted tight edges, its
    // counts are this first scan's
    if (!c.swept_tie) OCM_TRY(phase_sweep(c, false, true, w.V, W, L, w.pi, w.onC));
    const unsigned long long k = c.swept_tie ? c.swept_tight : c.h.tight;
    const unsigned long long certain = c.swept_tie ? c.swept_certain : c.h.certain;
    c.swept_tie = false;
    out->tight_edges = (int64_t)k;
    if (k == 0) return OCM_OK;
    out->flags |= OCM_F_TIGHT_EDGES;
    if (certain > 0) {
        out->flags |= OCM_F_TIE;
        return OCM_OK;
    }
    // second scan, now with the hop test (a random read per tight edge)
    OCM_TRY(phase_sweep(c, false, true, w.V, W, L, w.pi, w.onC, false, true));
    // With hop = policy hops to s, every policy edge lowers hop by one except
    // s's own; a cycle of tight edges other than C, with no tight edge
    // leaving C (certain == 0), needs a tight non-policy edge whose head is
    // not nearer to s than its tail.
    if (c.h.nondec == 0) return OCM_OK;
    {
        ocm::SweepArgs a;
        a.n = c.n;
        a.neg = c.neg;
        a.row_ptr = c.row_ptr;
        a.col = c.col;
        a.V = w.V;
        a.Vhi = c.wide ? w.Vhi : nullptr;
        a.V32 = !c.wide && c.v32 ? w.V32 : nullptr;
        a.t = c.t;
        a.W = W;
        a.L = L;
        a.pi = w.pi;
        a.onC = w.onC;
        a.ctl = w.ctl;
        a.hop = w.hop;
        a.xs = a.ys = nullptr;
        a.xcnt = nullptr;
        a.xcap = 0;
        a.giant = c.tile_sweep ? c.giant : ocm::GiantTab{};
        c.prof.begin(OCM_K_TIESCAN);
        ocm::launch_tie_short_walk(a, c.w, c.wtype, c.G, w.succ, c.sweep_grid, c.st);
        c.prof.end();
        HIP_TRY(hipGetLastError());
        OCM_TRY(read_ctl(c));
        if (c.h.certain > 0) {
            out->flags |= OCM_F_TIE;
            return OCM_OK;
        }
    }
    if (k > w.xcap) {
        out->flags |= OCM_F_TIE_UNCHECKED;
        return OCM_OK;
    }
    OCM_TRY(phase_sweep(c, false, true, w.V, W, L, w.pi, w.onC, true, true));
    const unsigned kx = c.h.xcnt;
    if (kx != k) return fail(OCM_E_HIP, "tie scan listed a different edge count");
    return tie_from_list(c, kx, out);
}

// The tie decision from the listed tight non-policy edges (w.xs, w.ys; kx of
// them) whose tails have the optimal gain: the special-vertex graph below.
// Every policy path from such a vertex reaches C.
ocm_status tie_from_list(Ctx& c, unsigned kx, ocm_result* out)
{
    Ws& w = c.ws;
    int* spid = w.layer;
    int* slist = w.list[1];
    int* P = w.list[0];
    c.prof.begin(OCM_K_TIESCAN);
    ocm::launch_tie_special(c.n, kx, w.xs, w.ys, w.succ, w.onC, w.touched, spid, slist,
                            &w.ctl->scnt, c.st);
    c.prof.end();
    HIP_TRY(hipGetLastError());
    OCM_TRY(read_ctl(c));
    const unsigned ns = c.h.scnt;
    c.prof.begin(OCM_K_TIESCAN);
    ocm::launch_tie_walk(c.n, ns, slist, w.succ, w.touched, w.onC, spid, P, kx, w.xs, w.ys, c.st);
    c.prof.end();
    HIP_TRY(hipGetLastError());
    std::vector<int> hp(ns), hx(kx), hy(kx);
    if (ns) HIP_TRY(hipMemcpyAsync(hp.data(), P, 4 * (size_t)ns, hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipMemcpyAsync(hx.data(), w.xs, 4 * (size_t)kx, hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipMemcpyAsync(hy.data(), w.ys, 4 * (size_t)kx, hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    // nodes: special vertices 0..ns-1, c* = ns; a special vertex on C is c*
    const int N = (int)ns + 1;
    auto node = [&](int id) { return (id < 0 || hp[id] == -2) ? (int)ns : id; };
    std::vector<int> head(N, -1), next, to;
    auto add = [&](int a, int b) {
        to.push_back(b);
        next.push_back(head[a]);
        head[a] = (int)to.size() - 1;
    };
    for (unsigned i = 0; i < ns; ++i) {
        if (hp[i] == -2) continue;
        if (hp[i] == -3) return fail(OCM_E_HIP, "policy path does not reach the critical cycle");
        add((int)i, hp[i] == -1 ? (int)ns : node(hp[i]));
    }
    for (unsigned i = 0; i < kx; ++i) add(node(hx[i]), node(hy[i]));
    if (has_cycle(N, head, next, to)) out->flags |= OCM_F_TIE;
    return OCM_OK;
}

long long gcd_ll(long long a, long long b)
{
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b) {
        long long t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Multichain policy iteration (ocm_options.multichain): every policy cycle
// keeps its own gain and no rebuild runs.  The first sweep is R1's, the stop
// rule R8's; each later iteration finds the policy graph's cycles, sums them,
// propagates every vertex's value toward the smallest vertex of the cycle it
// reaches, and sweeps with (gain, bias) pairs.  At the end C is the policy
// cycle with the smallest gain (ties: the smallest vertex), the same order as
// the select of Alg. 2.
struct McRun {
    const Jmp* R = nullptr;   // records of the last value phase
};

ocm_status mc_values(Ctx& c, McRun& run)
{
    Ws& w = c.ws;
    ocm::launch_ctl_clear(w.ctl, ocm::kClrCount, c.st);
    c.prof.begin(OCM_K_SELECT);
    ocm::launch_cyc_zero(c.n, w.rep, w.onc, w.wsum, w.lcnt, w.cyc, w.ctl, c.st);
    ocm::launch_cyc_sum(c.n, w.rep, w.onc, w.pi, c.w, c.wtype, c.neg, w.wsum, w.lcnt, c.st);
    c.prof.end();
    c.prof.bytes(OCM_K_SELECT, 6.0 * c.n);
    c.prof.begin(OCM_K_VALUES);
    const bool have_succ = c.succ_ok;
    ocm::launch_mc_val_init(c.n, c.col, w.pi, c.w, c.wtype, c.neg, w.rep, w.onc, w.wsum, w.lcnt,
                            w.succ, have_succ, w.Q[0], w.ctl, c.st);
    c.succ_ok = true;
    c.prof.end();
    // pi, succ, rep, on-cycle flag, w[pi], the entry
    c.prof.bytes(OCM_K_VALUES, (29.0 + c.sw) * c.n);
    HIP_TRY(hipGetLastError());
    ocm::launch_jump_setup(w.ctl, true, false, c.st);
    int r = 0;
    for (;;) {
        c.prof.begin(OCM_K_VALUES);
        for (int j = 0; j < kRoundsPerRead; ++j) {
            ++r;
            ocm::launch_mc_round_dev(c.n, r, w.Q[(r - 1) & 1], w.Q[r & 1], w.ctl, c.st);
        }
        ocm::launch_mc_final_dev(c.n, w.Q[0], w.Q[1], w.V, w.hop, w.ctl, c.st);
        c.prof.end();
        HIP_TRY(hipGetLastError());
        OCM_TRY(read_ctl(c));
        if (c.h.jmode == 0) break;
        if (r > 64) return fail(OCM_E_HIP, "value propagation did not converge");
    }
    const int k = (int)c.h.jk;
    c.jump_rounds += k;
    c.value_rounds += k;
    // own entry, gathered entry, new entry per round; the final's record
    c.prof.bytes(OCM_K_VALUES, 48.0 * c.n * k + 44.0 * c.n);
    if (c.h.jstall) return fail(OCM_E_HIP, "a policy path reaches no cycle");
    if (c.h.overflow)
        return fail(OCM_E_OVERFLOW, "a multichain value left [-2^62, 2^62] (int64 only)");
    run.R = w.Q[k & 1];
    return OCM_OK;
}

ocm_status mc_sweep(Ctx& c, const McRun& run, bool tie, long long W, long long L, bool list)
{
    Ws& w = c.ws;
    ocm::launch_ctl_clear(w.ctl, ocm::kClrChanged, c.st);
    ocm::McArgs a;
    a.n = c.n;
    a.neg = c.neg;
    a.row_ptr = c.row_ptr;
    a.col = c.col;
    a.R = run.R;
    a.wsum = w.wsum;
    a.lcnt = w.lcnt;
    a.pi = w.pi;
    a.succ = w.succ;
    a.ctl = w.ctl;
    a.W = W;
    a.L = L;
    a.onC = w.onC;
    a.xs = list ? w.xs : nullptr;
    a.ys = list ? w.ys : nullptr;
    a.xcnt = &w.ctl->xcnt;
    a.xcap = w.xcap;
    a.giant = c.giant;
    const int cls = tie ? OCM_K_TIESCAN : OCM_K_SWEEP;
    c.prof.begin(cls);
    ocm::launch_mc_sweep(a, c.w, c.wtype, c.G, tie, c.st);
    c.prof.end();
    // row_ptr, own record + gain; per edge col, w, the head's record and gain
    c.prof.bytes(cls, 28.0 * c.n + (4.0 + c.sw + 28.0) * c.m);
    HIP_TRY(hipGetLastError());
    return read_ctl(c);
}

ocm_status solve_mc(Ctx& c, const ocm_options& o, int32_t* cycle_edges, int64_t cap,
                    ocm_result* out)
{
    Ws& w = c.ws;
    McRun run;
    ocm_status rc = phase_sweep(c, true, false, w.V, 0, 1, w.pi, nullptr, false, false, false);
    int iter = 1;
    unsigned long long tight = 0;
    while (rc == OCM_OK) {
        if ((o.max_iters > 0 && iter >= o.max_iters) || iter >= kIterCap) {
            rc = fail(OCM_E_NOT_CONVERGED, "max_iters reached");
            break;
        }
        ++c.general_iters;
        rc = phase_cycles(c, w.pi, w.rep, w.onc);
        if (rc != OCM_OK) break;
        rc = mc_values(c, run);
        if (rc != OCM_OK) break;
        rc = mc_sweep(c, run, false, 0, 1, false);
        if (rc != OCM_OK) break;
        ++iter;
        tight = c.h.tight;
        if (c.h.changed == 0) break;   // no strict improvement left
    }
    out->iterations = iter;
    out->jump_rounds = c.jump_rounds;
    out->general_iters = c.general_iters;
    out->value_rounds = c.value_rounds;
    if (rc != OCM_OK) {
        c.prof.finish();
        return rc;
    }
    // C: the last policy's cycle of smallest gain (the sums are recomputed)
    rc = phase_select(c, w.pi, w.rep, w.onc);
    if (rc != OCM_OK) {
        c.prof.finish();
        return rc;
    }
    const int s = c.h.s;
    const long long W = c.h.W, L = c.h.L, clen = c.h.clen;
    const long long gg = gcd_ll(W, L);
    out->p = (c.neg ? -W : W) / gg;
    out->q = L / gg;
    out->W = c.neg ? -W : W;
    out->L = L;
    out->source = s;
    out->cycle_len = clen;
    if (cap < clen) {
        c.prof.finish();
        return fail(OCM_E_CAPACITY, "cycle_cap smaller than the critical cycle");
    }
    c.prof.begin(OCM_K_RESULT);
    ocm::launch_mc_mark_c(c.n, w.rep, w.onc, s, w.onC, c.st);
    ocm::launch_cycle_list(c.n, s, clen, w.onC, w.pi, w.hop, cycle_edges, c.st);
    c.prof.end();
    c.prof.bytes(OCM_K_RESULT, 7.0 * c.n + 28.0 * clen);
    HIP_TRY(hipGetLastError());
    if (o.tie_check) {
        // tight edges: those of the last sweep (it changed nothing)
        out->tight_edges = (int64_t)tight;
        if (tight > 0) out->flags |= OCM_F_TIGHT_EDGES;
        // a second policy cycle of optimal gain is a second critical cycle;
        // otherwise every vertex of optimal gain reaches C, and the
        // single-gain test applies to the tight edges among them
        ocm::launch_ctl_clear(w.ctl, ocm::kClrChanged, c.st);
        ocm::launch_mc_ncrit(w.cyc, w.wsum, w.lcnt, W, L, w.ctl, c.st);
        HIP_TRY(hipGetLastError());
        OCM_TRY(read_ctl(c));
        if (c.h.ncrit > 1) {
            out->flags |= OCM_F_TIE;
        } else if (tight > 0) {
            OCM_TRY(mc_sweep(c, run, true, W, L, false));
            const unsigned long long k = c.h.tight;
            if (c.h.certain > 0) {
                out->flags |= OCM_F_TIE;
            } else if (k > 0 && c.h.nondec > 0) {
                if (k > w.xcap) {
                    out->flags |= OCM_F_TIE_UNCHECKED;
                } else {
                    OCM_TRY(mc_sweep(c, run, true, W, L, true));
                    if (c.h.xcnt != k) return fail(OCM_E_HIP, "tie scan listed a different edge count");
                    OCM_TRY(tie_from_list(c, (unsigned)k, out));
                }
            }
        }
    } else {
        out->flags |= OCM_F_TIE_UNCHECKED;
        out->tight_edges = -1;
    }
    if (o.policy_out)
        HIP_TRY(hipMemcpyAsync(o.policy_out, w.pi, 4 * (size_t)c.n, hipMemcpyDeviceToDevice, c.st));
    if (o.potential_out)
        HIP_TRY(hipMemcpyAsync(o.potential_out, w.V, 8 * (size_t)c.n, hipMemcpyDeviceToDevice, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    c.prof.finish();
    return OCM_OK;
}

// t (nullable): edge times, the optimal cycle ratio instead of the mean.
ocm_status solve(const ocm_graph* g, const ocm_options* o_in, void* wsp, size_t ws_bytes,
                 int32_t* cycle_edges, int64_t cap, ocm_result* out, void* stream, int neg,
                 bool noalloc = false, const int32_t* t = nullptr)
{
    if (!out) return fail(OCM_E_INVALID_ARG, "result pointer is null");
    memset(out, 0, sizeof *out);
    ocm_options o;
    if (o_in) o = *o_in;
    else ocm_default_options(&o);
    if (o.profile) memset(o.profile, 0, sizeof *o.profile);
    Ctx c;
    c.noalloc = noalloc;
    c.t = t;
    OCM_TRY(setup(c, g, neg, wsp, ws_bytes, stream, o.profile));
    if (cap > 0 && !cycle_edges) return fail(OCM_E_INVALID_ARG, "cycle_edges is null");
    c.G = choose_lanes(c.n, c.m, o.schedule);
    if (!valid_lanes(c.G)) return fail(OCM_E_INVALID_ARG, "schedule must be a power of two <= 64");
    c.sweep_grid = sweep_grid(c.n, c.G);
    c.tile_sweep = o.schedule <= 0;
    c.count_tight = o.tie_check != 0;
    c.connect_mode = o.connect_mode;
    c.allow_wide = true;
    c.wide = o.int128_values != 0;
    if (c.connect_mode < 0 || c.connect_mode > 2) return fail(OCM_E_INVALID_ARG, "bad connect_mode");

    if (o.multichain && (o.init_policy || t || o.int128_values))
        return fail(OCM_E_INVALID_ARG,
                    "multichain runs without init_policy, edge times or int128 values");
    ocm_status rc = validate(c, o.validate != 0);
    if (rc == OCM_OK) rc = build_giant(c);
    if (rc != OCM_OK) { c.prof.finish(); return rc; }
    if (o.multichain) return solve_mc(c, o, cycle_edges, cap, out);
    start_reverse_early(c);
    HIP_TRY(hipGetLastError());

    Ws& w = c.ws;
    const bool warm = o.init_policy != nullptr;
    if (warm) {
        // warm start: the given policy replaces the first sweep
        ocm::launch_ctl_clear(w.ctl, ocm::kClrChanged, c.st);
        ocm::launch_check_policy(c.n, c.row_ptr, o.init_policy, &w.ctl->lane[0].bad, c.st);
        HIP_TRY(hipGetLastError());
        OCM_TRY(read_ctl(c));
        if (c.h.bad) return fail(OCM_E_INVALID_ARG, "init_policy picks an edge of another vertex");
        HIP_TRY(hipMemcpyAsync(w.pi, o.init_policy, 4 * (size_t)c.n, hipMemcpyDeviceToDevice, c.st));
    }
    int iter = 0, fast = 0;
    bool have_c = false, need_sweep = !warm;
    int s = -1;
    long long W = 0, L = 1;
    long long clen = 1;   // edges of C (L itself for the mean; L is C's time for a ratio)
    for (;;) {
        // with the rounds decided on the device, the fast path's value phase
        // is queued behind the sweep, gated on the sweep's outcome, and both
        // are read back at once
        const bool ahead = need_sweep && o.fast_path && have_c && !c.prof.out;
        bool stalled = false;
        if (need_sweep) {
            const bool first = iter == 0 && !warm;
            // a cold start's first sweep decides nothing (the stop test needs a
            // second sweep; the iteration cap is at least 2 then): no read
            const bool blind = first && !c.prof.out && (o.max_iters <= 0 || o.max_iters > 1);
            rc = phase_sweep(c, first, false, w.V, W, L, w.pi, have_c ? w.onC : nullptr, false,
                             false, !ahead && !blind);
            if (rc != OCM_OK) break;
            if (blind) c.h.changed = 1;   // FIRST always picks an edge per vertex
            if (ahead) {
                // the sweep count test below only spares a warm start's first
                // sweep, which never runs here (no C yet)
                ocm::launch_fast_gate(w.ctl, false, c.st);
                rc = phase_values(c, w.pi, s, W, L, w.V, w.hop, true, &stalled, nullptr, true);
                if (rc != OCM_OK) break;
                sweep_done(c, first, false, c.sweep_fused);
            }
            ++iter;
            // no strict improvement left (a cold start's first sweep always changes)
            if (iter >= (warm ? 1 : 2) && c.h.changed == 0) break;
            if ((o.max_iters > 0 && iter >= o.max_iters) || iter >= kIterCap) {
                rc = fail(OCM_E_NOT_CONVERGED, "max_iters reached");
                break;
            }
        }
        need_sweep = true;
        if (o.fast_path && have_c && !c.h.cbroken) {
            // C is still a cycle of the new policy.  If every vertex still
            // reaches s, C is the policy graph's only cycle: the cycle, select
            // and connect phases would change nothing, so only values remain.
            if (!ahead) {
                rc = phase_values(c, w.pi, s, W, L, w.V, w.hop, true, &stalled, nullptr);
                if (rc != OCM_OK) break;
            }
            if (!stalled) {
                ++fast;
                continue;
            }
        }
        ++c.general_iters;
        rc = phase_cycles(c, w.pi, w.rep, w.onc);
        if (rc != OCM_OK) break;
        rc = phase_select(c, w.pi, w.rep, w.onc);
        if (rc != OCM_OK) break;
        s = c.h.s;
        W = c.h.W;
        L = c.h.L;
        clen = c.h.clen;
        // the solve itself needs no layers, only the rewired policy
        rc = phase_connect(c, w.rep, w.onc, s, w.pi, nullptr, w.onC, nullptr);
        if (rc != OCM_OK) break;
        rc = phase_values(c, w.pi, s, W, L, w.V, w.hop, false, nullptr, nullptr);
        if (rc != OCM_OK) break;
        have_c = true;
    }
    out->iterations = iter;
    if (c.wide) out->flags |= OCM_F_INT128;
    out->connect_rounds = c.connect_rounds;
    out->jump_rounds = c.jump_rounds;
    out->fast_iters = fast;
    out->general_iters = c.general_iters;
    out->value_rounds = c.value_rounds;
    out->push_frontier = c.push_frontier;
    // the last read came after the last rebuild: its in-edge count is final
    out->push_in_edges = (int64_t)c.h.pedges;
    if (rc != OCM_OK) {
        c.prof.finish();
        return rc;
    }
    const long long gg = gcd_ll(W, L);
    out->p = (neg ? -W : W) / gg;
    out->q = L / gg;
    out->W = neg ? -W : W;
    out->L = L;
    out->source = s;
    out->cycle_len = clen;
    if (cap < clen) {
        c.prof.finish();
        return fail(OCM_E_CAPACITY, "cycle_cap smaller than the critical cycle");
    }
    c.prof.begin(OCM_K_RESULT);
    ocm::launch_cycle_list(c.n, s, clen, w.onC, w.pi, w.hop, cycle_edges, c.st);
    c.prof.end();
    c.prof.bytes(OCM_K_RESULT, (double)c.n + 28.0 * clen);
    HIP_TRY(hipGetLastError());
    if (o.tie_check) {
        rc = tie_check(c, W, L, out);
        if (rc != OCM_OK) {
            c.prof.finish();
            return rc;
        }
    } else {
        out->flags |= OCM_F_TIE_UNCHECKED;
        out->tight_edges = -1;
    }
    if (o.policy_out)
        HIP_TRY(hipMemcpyAsync(o.policy_out, w.pi, 4 * (size_t)c.n, hipMemcpyDeviceToDevice, c.st));
    if (o.potential_out && c.wide) {
        // int128 values: exported only if every one fits int64
        ocm::launch_ctl_clear(w.ctl, ocm::kClrChanged, c.st);
        ocm::launch_fits64(c.n, w.V, w.Vhi, &w.ctl->lane[0].bad, c.st);
        HIP_TRY(hipGetLastError());
        OCM_TRY(read_ctl(c));
        if (c.h.bad) {
            c.prof.finish();
            return fail(OCM_E_OVERFLOW, "the optimum's values need int128; potential_out holds int64");
        }
    }
    if (o.potential_out)
        HIP_TRY(hipMemcpyAsync(o.potential_out, w.V, 8 * (size_t)c.n, hipMemcpyDeviceToDevice, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    c.prof.finish();
    return OCM_OK;
}

// Workspace of ocm_min_noalloc: one array per GPU (each device that loads
// the library holds its own copy until the process ends).  Host code must
// never pass `scratch` itself to a kernel (in host code it names a host-side
// stand-in); it uses the device address from hipGetSymbolAddress instead.
static __device__ __align__(256) unsigned char scratch[OCM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

struct ScratchSlot {
    std::mutex call;           // serialises calls on this device within the process
    void* ptr = nullptr;       // device address of this device's `scratch`
    bool init = false;
};
ScratchSlot g_scratch[kMaxDevices];
std::mutex g_scratch_init;

// The calling thread's current device and the address of its `scratch`,
// looked up once per device with that device current.
ocm_status scratch_slot(ScratchSlot** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(OCM_E_INVALID_ARG, "device index out of range");
    ScratchSlot& sl = g_scratch[dev];
    std::lock_guard<std::mutex> lock(g_scratch_init);
    if (!sl.init) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(OCM_E_HIP, "no device address for the static scratch array");
        sl.ptr = p;
        sl.init = true;
    }
    *out = &sl;
    return OCM_OK;
}

}  // namespace

extern "C" {

ocm_status ocm_min_noalloc(const ocm_graph* g, const ocm_options* o, int32_t* cycle_edges,
                           int64_t cycle_cap, ocm_result* out, void* stream)
{
    if (o && o->profile) return fail(OCM_E_INVALID_ARG, "ocm_min_noalloc takes no profile");
    OCM_TRY(check_graph(g));
    const size_t need = carve(nullptr, g->n, g->m).total;
    if (need > (size_t)OCM_NOALLOC_SCRATCH_BYTES) {
        char b[192];
        snprintf(b, sizeof b,
                 "graph needs %zu bytes of scratch; ocm_min_noalloc holds %zu (use ocm_min with a "
                 "caller workspace)",
                 need, (size_t)OCM_NOALLOC_SCRATCH_BYTES);
        return fail(OCM_E_WORKSPACE, b);
    }
    ScratchSlot* sl = nullptr;
    OCM_TRY(scratch_slot(&sl));
    std::lock_guard<std::mutex> lock(sl->call);
    const ocm_status rc = solve(g, o, sl->ptr, OCM_NOALLOC_SCRATCH_BYTES, cycle_edges, cycle_cap,
                                out, stream, 0, true);
    // the array is free for the next call only once this call's kernels end
    const hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (rc == OCM_OK && e != hipSuccess) return fail(OCM_E_HIP, hipGetErrorString(e));
    return rc;
}

ocm_status ocm_weights_from_f64(int64_t m, const double* w_f64, int64_t* w_i64, void* ws,
                                size_t ws_bytes, void* stream)
{
    if (m < 1 || !w_f64 || !w_i64) return fail(OCM_E_INVALID_ARG, "null argument or m < 1");
    if (!ws || ws_bytes < 256) return fail(OCM_E_WORKSPACE, "workspace must hold 256 bytes");
    hipStream_t st = (hipStream_t)stream;
    unsigned* bad = (unsigned*)ws;
    ocm::launch_zero2(bad, bad, st);
    ocm::launch_w_from_f64(m, w_f64, (long long*)w_i64, bad, st);
    HIP_TRY(hipGetLastError());
    unsigned h = 0;
    HIP_TRY(hipMemcpyAsync(&h, bad, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h) return fail(OCM_E_INVALID_ARG, "weights must be integers with |w| < 2^53");
    return OCM_OK;
}

ocm_status ocm_adjoint_scatter(int64_t m, const int32_t* cycle_edges, int64_t cycle_len,
                               const double* grad_out, double* grad_w, void* stream)
{
    if (m < 1 || !grad_w || !grad_out || (cycle_len > 0 && !cycle_edges) || cycle_len < 0 ||
        cycle_len > m)
        return fail(OCM_E_INVALID_ARG, "bad adjoint arguments");
    ocm::launch_adjoint_scatter(m, cycle_edges, cycle_len, grad_out, grad_w, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return OCM_OK;
}

void ocm_default_options(ocm_options* o)
{
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->validate = 1;
    o->tie_check = 1;
    o->fast_path = 1;
}

size_t ocm_workspace_size(const ocm_graph* g, const ocm_options* o)
{
    (void)o;
    if (check_graph(g) != OCM_OK) return 0;
    return carve(nullptr, g->n, g->m).total;
}

ocm_status ocm_min(const ocm_graph* g, const ocm_options* o, void* ws, size_t ws_bytes,
                   int32_t* cycle_edges, int64_t cycle_cap, ocm_result* out, void* stream)
{
    return solve(g, o, ws, ws_bytes, cycle_edges, cycle_cap, out, stream, 0);
}

ocm_status ocm_max(const ocm_graph* g, const ocm_options* o, void* ws, size_t ws_bytes,
                   int32_t* cycle_edges, int64_t cycle_cap, ocm_result* out, void* stream)
{
    return solve(g, o, ws, ws_bytes, cycle_edges, cycle_cap, out, stream, 1);
}

ocm_status ocm_ratio_min(const ocm_graph* g, const int32_t* t, const ocm_options* o, void* ws,
                         size_t ws_bytes, int32_t* cycle_edges, int64_t cycle_cap,
                         ocm_result* out, void* stream)
{
    if (!t) return fail(OCM_E_INVALID_ARG, "edge times are null");
    return solve(g, o, ws, ws_bytes, cycle_edges, cycle_cap, out, stream, 0, false, t);
}

ocm_status ocm_ratio_max(const ocm_graph* g, const int32_t* t, const ocm_options* o, void* ws,
                         size_t ws_bytes, int32_t* cycle_edges, int64_t cycle_cap,
                         ocm_result* out, void* stream)
{
    if (!t) return fail(OCM_E_INVALID_ARG, "edge times are null");
    return solve(g, o, ws, ws_bytes, cycle_edges, cycle_cap, out, stream, 1, false, t);
}

ocm_status ocm_phase_sweep(const ocm_graph* g, int32_t neg, int32_t first, const int64_t* V,
                           int64_t W, int64_t L, int32_t* pi, int32_t schedule, void* ws,
                           size_t ws_bytes, int64_t* changed, void* stream)
{
    Ctx c;
    OCM_TRY(setup(c, g, neg != 0, ws, ws_bytes, stream, nullptr));
    if (!pi || !changed || (!first && !V)) return fail(OCM_E_INVALID_ARG, "null argument");
    if (!first && L < 1) return fail(OCM_E_INVALID_ARG, "L must be >= 1");
    c.G = choose_lanes(c.n, c.m, schedule);
    if (!valid_lanes(c.G)) return fail(OCM_E_INVALID_ARG, "schedule must be a power of two <= 64");
    c.sweep_grid = sweep_grid(c.n, c.G);
    c.tile_sweep = schedule <= 0;
    OCM_TRY(phase_sweep(c, first != 0, false, (const long long*)V, W, L, pi, nullptr));
    *changed = (int64_t)c.h.changed;
    return OCM_OK;
}

ocm_status ocm_phase_cycles(const ocm_graph* g, const int32_t* pi, int32_t* rep,
                            uint8_t* on_cycle, void* ws, size_t ws_bytes, int64_t* ncycles,
                            void* stream)
{
    Ctx c;
    OCM_TRY(setup(c, g, 0, ws, ws_bytes, stream, nullptr));
    if (!pi || !rep || !on_cycle) return fail(OCM_E_INVALID_ARG, "null argument");
    OCM_TRY(phase_cycles(c, pi, rep, on_cycle));
    if (ncycles) {
        // count cycle heads with the select phase's first kernel
        ocm::launch_ctl_clear(c.ws.ctl, ocm::kClrCount, c.st);
        ocm::launch_cyc_zero(c.n, rep, on_cycle, c.ws.wsum, c.ws.lcnt, c.ws.cyc, c.ws.ctl, c.st);
        HIP_TRY(hipGetLastError());
        OCM_TRY(read_ctl(c));
        *ncycles = c.h.ncyc;
    }
    HIP_TRY(hipStreamSynchronize(c.st));
    return OCM_OK;
}

ocm_status ocm_phase_select(const ocm_graph* g, int32_t neg, const int32_t* pi,
                            const int32_t* rep, const uint8_t* on_cycle, void* ws,
                            size_t ws_bytes, int32_t* s, int64_t* W, int64_t* L, void* stream)
{
    Ctx c;
    OCM_TRY(setup(c, g, neg != 0, ws, ws_bytes, stream, nullptr));
    if (!pi || !rep || !on_cycle || !s || !W || !L) return fail(OCM_E_INVALID_ARG, "null argument");
    OCM_TRY(phase_select(c, pi, rep, on_cycle));
    *s = c.h.s;
    *W = c.h.W;
    *L = c.h.L;
    return OCM_OK;
}

ocm_status ocm_phase_connect(const ocm_graph* g, const int32_t* rep, int32_t s, int32_t* pi,
                             int32_t* layer, void* ws, size_t ws_bytes, int32_t* rounds,
                             void* stream)
{
    Ctx c;
    OCM_TRY(setup(c, g, 0, ws, ws_bytes, stream, nullptr));
    if (!rep || !pi || !layer) return fail(OCM_E_INVALID_ARG, "null argument");
    if (s < 0 || s >= c.n) return fail(OCM_E_INVALID_ARG, "source out of range");
    int r = 0;
    ocm_status rc = phase_connect(c, rep, nullptr, s, pi, layer, nullptr, &r);
    if (rounds) *rounds = r;
    HIP_TRY(hipStreamSynchronize(c.st));
    return rc;
}

ocm_status ocm_phase_values(const ocm_graph* g, int32_t neg, const int32_t* pi, int32_t s,
                            int64_t W, int64_t L, int64_t* V, void* ws, size_t ws_bytes,
                            int32_t* rounds, void* stream)
{
    Ctx c;
    OCM_TRY(setup(c, g, neg != 0, ws, ws_bytes, stream, nullptr));
    if (!pi || !V) return fail(OCM_E_INVALID_ARG, "null argument");
    if (s < 0 || s >= c.n || L < 1) return fail(OCM_E_INVALID_ARG, "bad source or L");
    int r = 0;
    ocm_status rc = phase_values(c, pi, s, W, L, (long long*)V, nullptr, false, nullptr, &r);
    if (rounds) *rounds = r;
    HIP_TRY(hipStreamSynchronize(c.st));
    return rc;
}

const char* ocm_status_string(ocm_status s)
{
    switch (s) {
        case OCM_OK: return "ok";
        case OCM_E_INVALID_ARG: return "invalid argument";
        case OCM_E_BAD_CSR: return "malformed CSR";
        case OCM_E_NO_OUT_EDGE: return "vertex without out-edge";
        case OCM_E_NOT_STRONGLY_CONNECTED: return "graph not strongly connected";
        case OCM_E_OVERFLOW: return "int64 overflow";
        case OCM_E_CAPACITY: return "capacity too small";
        case OCM_E_NOT_CONVERGED: return "not converged within max_iters";
        case OCM_E_WORKSPACE: return "workspace missing or too small";
        case OCM_E_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char* ocm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
