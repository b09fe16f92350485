// Shared declarations of the device kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ocm {

constexpr int kWG = 256;        // threads per workgroup (4 waves of 64)
constexpr int kWI32 = 0, kWI64 = 1;
constexpr int kListItems = 4096;  // LDS list buffer of the connect kernels (16 KiB)
constexpr int kShortWalk = 64;    // tie test: policy steps walked from a tight edge's head

constexpr unsigned kErrBadCsr = 1u;
constexpr unsigned kErrNoOut = 2u;

constexpr unsigned kClrChanged = 1u;
constexpr unsigned kClrCount = 2u;
constexpr unsigned kClrAll = 4u;
constexpr unsigned kClrActive2 = 8u;
constexpr unsigned kClrGiant = 16u;

// |V| must stay within 2^62 so that V[u] + (L*w - W) cannot leave int64 when
// |L*w - W| < 2^62 as well.
constexpr long long kValLimit = (1ll << 62);
constexpr unsigned kHopOverflow = 0x80000000u;

// Counters that many workgroups update.  Same-address atomics from
// thousands of workgroups serialise (about 11 ns apiece measured on MI355X,
// i.e. ~90 us for one atomic from each of 8192 workgroups), so every
// workgroup updates copy blockIdx % kLanes and readers fold the copies.
constexpr int kLanes = 16;
constexpr int kLaneWords = 32;   // one copy per 128-byte line

struct alignas(128) CtlLane {
    unsigned long long changed;    // sweep: vertices whose policy changed
    unsigned long long tight;      // tie scan: tight non-policy edges
    unsigned long long certain;    // tie scan: edges that certainly close a second critical cycle
    unsigned long long nondec;     // tie scan: tight non-policy edges not nearer the source
    unsigned long long pedges;     // connect: in-edges scanned by push marks
    unsigned long long ledges;     // connect: out-edges scanned by pull rounds and push claims
    unsigned long long maxabsw;    // validation: max |w| (max-folded)
    unsigned active, active2;      // values: unfinished vertices
    unsigned got;                  // connect: vertices attached in the round (init: C's component)
    unsigned left;                 // connect init: unattached vertices
    unsigned err;                  // validation error bits (or-folded, like the next three)
    unsigned cbroken;              // sweep: a vertex of C changed policy
    unsigned overflow;             // values: a value left [-2^62, 2^62]
    unsigned bad;                  // conversion / policy check failure
    unsigned pjc[4];               // cycles: per round parity, image size and M changes
    unsigned long long rpack;      // device-driven rounds: this copy's workgroups done with
                                   //   the running round kernel, and their counts
    unsigned wide32;               // values: some value does not fit int32 (no int32 copy)
    unsigned ncrit;                // multichain tie check: policy cycles of optimal gain
    unsigned pad_[2];
};
static_assert(sizeof(CtlLane) == 4 * kLaneWords, "one lane per 128-byte line");

// Device control block: the current lambda = W / L, list counters, and the
// striped counters.
struct alignas(128) Ctl {
    long long W, L;                // current lambda, unreduced
    int s;                         // current source (min vertex of C)
    unsigned ncyc;                 // cycles found by the cycle phase
    unsigned rmode;                // connect, device-driven rounds: 0 done, 1 push, 2 pull
    unsigned rleft;                //   unattached vertices
    unsigned rfront;               //   vertices attached by the last round
    unsigned rerr;                 //   a round attached nobody while vertices were left
    unsigned rk;                   //   rounds run
    unsigned rmarks;               //   the round whose marks a push round left
    unsigned long long rpack;      //   lanes done with a round kernel, and their counts
    unsigned jk;                   // jump rounds on the device (values, cycles): rounds run
    unsigned jmode;                //   1 while rounds are left, 0 once they are over
    unsigned jlast;                //   the last round's count (unfinished vertices, image size)
    unsigned jstall;               //   values: a round finished no vertex
    unsigned jgate;                //   values: 0 = the queued value phase is skipped
    unsigned xcnt;                 // tie scan: tight non-policy edges listed
    unsigned scnt;                 // tie check: special vertices
    unsigned clen;                 // select: edges of the chosen cycle (its L for a mean)
    unsigned ngiant;               // rows longer than kGiantRow
    CtlLane lane[kLanes];
};

// Host snapshot of a Ctl with the lanes folded (sums, or / max for flags).
struct CtlView {
    long long W, L;
    int s;
    unsigned ncyc;
    unsigned rmode, rleft, rfront, rerr, rk;
    unsigned jk, jmode, jlast, jstall;
    unsigned xcnt, scnt, clen, ngiant;
    unsigned long long changed, tight, certain, nondec, pedges, ledges, maxabsw;
    unsigned active, active2, got, left, err, cbroken, overflow, bad;
    unsigned pjc[4];
    unsigned wide32, ncrit;
};

__host__ __device__ inline void fold_lanes(const Ctl& c, CtlView& v)
{
    v.W = c.W;
    v.L = c.L;
    v.s = c.s;
    v.ncyc = c.ncyc;
    v.rmode = c.rmode;
    v.rleft = c.rleft;
    v.rfront = c.rfront;
    v.rerr = c.rerr;
    v.rk = c.rk;
    v.jk = c.jk;
    v.jmode = c.jmode;
    v.jlast = c.jlast;
    v.jstall = c.jstall;
    v.xcnt = c.xcnt;
    v.scnt = c.scnt;
    v.clen = c.clen;
    v.ngiant = c.ngiant;
    v.changed = v.tight = v.certain = v.nondec = v.pedges = v.ledges = v.maxabsw = 0;
    v.active = v.active2 = v.got = v.left = v.err = v.cbroken = v.overflow = v.bad = 0;
    v.wide32 = v.ncrit = 0;
    for (int j = 0; j < 4; ++j) v.pjc[j] = 0;
    for (int l = 0; l < kLanes; ++l) {
        const CtlLane& ln = c.lane[l];
        v.changed += ln.changed;
        v.tight += ln.tight;
        v.certain += ln.certain;
        v.nondec += ln.nondec;
        v.pedges += ln.pedges;
        v.ledges += ln.ledges;
        v.maxabsw = ln.maxabsw > v.maxabsw ? ln.maxabsw : v.maxabsw;
        v.active += ln.active;
        v.active2 += ln.active2;
        v.got += ln.got;
        v.left += ln.left;
        v.err |= ln.err;
        v.cbroken |= ln.cbroken;
        v.overflow |= ln.overflow;
        v.bad |= ln.bad;
        v.wide32 |= ln.wide32;
        v.ncrit += ln.ncrit;
        for (int j = 0; j < 4; ++j) v.pjc[j] += ln.pjc[j];
    }
}

// copy of a striped counter used by the calling workgroup
__device__ __forceinline__ CtlLane& my_lane(Ctl* c) { return c->lane[blockIdx.x & (kLanes - 1)]; }
template <typename T>
__device__ __forceinline__ T* my_copy(T* lane0_field)
{
    return (T*)((char*)lane0_field + (blockIdx.x & (kLanes - 1)) * (4 * kLaneWords));
}

// Pointer-jumping entry of the value phase: the first H edges of v's policy
// path lead to J and carry the sum D of (L*w - W).  Bit 31 of H flags an
// int64 overflow of D.
struct alignas(16) Jmp {
    long long D;
    int J;
    unsigned H;
};

// Rows of more than kGiantRow edges are swept by several workgroups: one per
// chunk of at most kGiantChunk consecutive edges (k_giant_part), then one
// merge per row in chunk order (k_giant_merge); the tile kernels skip them.
// Built once per solve; ngiant = 0 leaves every row to the tile kernels.
constexpr int kGiantRow = 8192;
constexpr int kGiantChunk = 8192;

struct GiantTab {
    const int* cv = nullptr;       // chunk: its row's vertex,
    const int* cs = nullptr;       //        first edge position
    const int* ce = nullptr;       //        and end
    int nchunks = 0;
    const int* gv = nullptr;       // giant rows: vertex,
    const int* gc0 = nullptr;      //             first chunk
    const int* gc1 = nullptr;      //             and end chunk
    int ngiant = 0;
    void* parts = nullptr;         // per chunk: its best key, position and head (32 bytes)
};

struct SweepArgs {
    int n;
    int neg;
    const int* row_ptr;
    const int* col;
    const long long* V;
    const long long* Vhi;          // int128 values: high words of V (else null)
    const int* V32;                // int32 copy of V when every value fits (else null)
    const int* t;                  // cycle ratio: edge times (else null: the mean)
    long long W, L;
    int* pi;
    int* succ;                     // optional: col[pi] kept up to date where pi changes
    const unsigned char* onC;      // optional: flags vertices of the current C
    Ctl* ctl;
    const int* hop;                // tie scan: policy hops to the source, or null
    int* xs;                       // tie scan: optional list of tight edges (tail)
    int* ys;                       //           and head
    unsigned* xcnt;
    unsigned xcap;
    GiantTab giant;                // rows swept by several workgroups (tile sweeps only)
};

// Giant rows: (vertex, first, end) triples of every row longer than
// kGiantRow edges, appended in any order (at most cap; ctl->ngiant counts
// them all).
void launch_giant_list(int n, const int* row_ptr, int* triples, unsigned cap, Ctl* ctl,
                       hipStream_t st);

void launch_validate(int n, int m, const int* row_ptr, const int* col, const void* w, int wtype,
                     int check_csr, Ctl* ctl, hipStream_t st);
// G = 0: vertex tiles (k_sweep_tile, k_tiescan_tile), else G lanes per
// vertex.  tie: the tie scan instead of a sweep.  count_tight (tiles, not
// first): the sweep also counts tight and certain edges as the tie scan's
// first pass does (valid as such when it changes nothing).
void launch_sweep(const SweepArgs& a, const void* w, int wtype, int G, bool first, bool tie,
                  bool count_tight, unsigned grid, hipStream_t st);
// tag0 (optional): byte array marked with 1 at every successor; cnt: the
// four stop-test counters, cleared
// have_succ: succ already holds col[pi]; otherwise it is written.
void launch_pj_init(int n, const int* col, const int* pi, int* succ, bool have_succ,
                    unsigned long long* P, unsigned char* onc, unsigned char* tag0, unsigned* cnt,
                    hipStream_t st);
void launch_pj_round(int n, const unsigned long long* Pin, unsigned long long* Pout,
                     hipStream_t st);
// round r >= 1 with the stop-test counters: cnt[2*(r&1)] = size of
// image(J_{r-1}), cnt[2*(r&1)+1] = M values changed; tprev / tcur alternate
void launch_pj_round_tagged(int n, int r, const unsigned long long* Pin, unsigned long long* Pout,
                            const unsigned char* tprev, unsigned char* tcur, unsigned* cnt,
                            hipStream_t st);
// Device-driven jump rounds (cycles and values): setup arms round 1 (for
// values only if the init left unfinished vertices); round r runs only if it
// is the next one and the rounds are not over; the final runs once they are,
// on the buffer of the last round run (round r reads buffer (r-1)&1 and
// writes r&1).  Progress: jk, jmode, jstall.
void launch_jump_setup(Ctl* ctl, bool values, bool gated, hipStream_t st);
// Opens ctl->jgate iff the sweep just run changed a policy edge (or force)
// and no vertex of C changed: the fast-path value phase queued behind the
// sweep (init and jump setup gated) then runs only if the host would have
// started it.
void launch_fast_gate(Ctl* ctl, bool force, hipStream_t st);
void launch_pj_round_dev(int n, int r, const unsigned long long* Pin, unsigned long long* Pout,
                         const unsigned char* tprev, unsigned char* tcur, Ctl* ctl, hipStream_t st);
void launch_pj_final_dev(int n, const unsigned long long* P0, const unsigned long long* P1, int K,
                         int* rep, unsigned char* onc, const Ctl* ctl, hipStream_t st);
// int128 values (hin/hout, h0/h1 non-null): the entries' high words live in
// parallel arrays and Vhi receives the values' high words.
void launch_val_round_dev(int n, int s, int r, const Jmp* Qin, Jmp* Qout, Ctl* ctl,
                          hipStream_t st, const long long* hin = nullptr,
                          long long* hout = nullptr);
// V32 (nullable, int64 values only): also the int32 copy of V; the lanes'
// wide32 flag says some value did not fit.
void launch_val_final_dev(int n, const Jmp* Q0, const Jmp* Q1, long long* V, int* hop, Ctl* ctl,
                          hipStream_t st, const long long* h0 = nullptr,
                          const long long* h1 = nullptr, long long* Vhi = nullptr,
                          int* V32 = nullptr);
void launch_pj_final(int n, const unsigned long long* P, int* rep, unsigned char* onc,
                     hipStream_t st);
// Cycle ratio (t non-null): tsum receives each cycle's time, and the order
// is cost over time; ctl->clen gets the chosen cycle's edge count.
void launch_cyc_zero(int n, const int* rep, const unsigned char* onc, long long* wsum,
                     unsigned* lcnt, int* cyc_list, Ctl* ctl, hipStream_t st,
                     long long* tsum = nullptr);
void launch_cyc_sum(int n, const int* rep, const unsigned char* onc, const int* pi, const void* w,
                    int wtype, int neg, long long* wsum, unsigned* lcnt, hipStream_t st,
                    const int* t = nullptr, long long* tsum = nullptr);
// scratch: kSelectParts * 32 bytes of device memory
constexpr int kSelectParts = 512;
void launch_select(const int* cyc_list, const long long* wsum, const unsigned* lcnt, Ctl* ctl,
                   void* scratch, hipStream_t st, const long long* tsum = nullptr);
// Edge times of a cycle ratio: lane bad |= some t < 1, lane maxabsw = max t
// (the caller clears both first).
void launch_validate_t(int m, const int* t, Ctl* ctl, hipStream_t st);
// Rebuild (breadth-first attachment to C's component); layer (the round that
// attached each vertex) may be null.  a[0], a[1]: the two
// attached-vertex bitmaps (ceil(n/32) words each); marks: push-round mark
// bytes (n + 16).  Counts go to the control block's lanes: init -> got (C's
// component) and left (unattached); every round -> got (attached in it).
void launch_conn_init(int n, const int* rep, const unsigned char* onc, int s, int* layer,
                      unsigned char* onC, unsigned* a1, unsigned* a0, Ctl* ctl, hipStream_t st);
// Round kernels work on spans of kWG * round_wpt(n) bitmap words; `spans`
// (device list of span indices, *nspans of them) restricts a round to those
// spans, nullptr means every span.
int round_wpt(int n);
int64_t round_spans(int n);
// Host-driven round steps (the host picks each round's direction).  Push
// round k: the marks (frontier in-edges -> mark bytes), unless round k-1
// left them, then the claims, which with marks_next also mark round k+1's
// frontier there (the next round's mark array).  A pull round given `stale`
// clears those mark bytes (marks a push round left for it).  Any superset
// of the marked vertices gives the same attachments.
void launch_conn_pull(int k, int n, const int* row_ptr, const int* col, const unsigned* acur,
                      unsigned* anext, int* layer, int* pi, Ctl* ctl, unsigned long long* ledges,
                      const int* spans, const unsigned* nspans, unsigned char* stale,
                      hipStream_t st);
void launch_conn_mark(int n, const int* rin_ptr, const int* rin, const unsigned* acur,
                      const unsigned* anext, unsigned char* marks, unsigned long long* pedges,
                      const int* spans, const unsigned* nspans, hipStream_t st);
void launch_conn_claim(int k, int n, const int* row_ptr, const int* col, const unsigned* acur,
                       unsigned* anext, unsigned char* marks, int* pi, int* layer, Ctl* ctl,
                       unsigned long long* cedges, const int* spans, const unsigned* nspans,
                       const int* rin_ptr, const int* rin, unsigned char* marks_next,
                       unsigned long long* pedges, hipStream_t st);
// Device-driven rounds: setup stores the counts after the init and picks
// round 1's direction (policy 0: push while left >= push_min and 2 * front <
// left, 1: pull, 2: push); launch_round queues round k (a push or pull round
// as the device decides, nothing once the rebuild is over).  Rounds are
// queued in order k = 1, 2, ...; with may_push false (no reverse CSR) every
// round must be a pull round.  single (k > 1, may_push): one kernel for the
// round instead of two, for rounds the host expects to push with the marks
// the round before left; any other round then runs as a pull round (same
// attachments).  Progress: rk, rleft, rerr, rmode.
void launch_round_setup(Ctl* ctl, unsigned left, unsigned front, int policy, unsigned push_min,
                        hipStream_t st);
// launch_round_setup with left / front taken on the device from the lanes'
// counts of the rebuild init (ctl cleared with kClrCount before the init).
void launch_round_setup_dev(Ctl* ctl, int policy, unsigned push_min, hipStream_t st);
void launch_round(int k, int n, const int* row_ptr, const int* col, const int* rin_ptr,
                  const int* rin, const unsigned* acur, unsigned* anext, unsigned char* marks,
                  unsigned char* marks_next, int* pi, int* layer, Ctl* ctl,
                  unsigned long long* pedges, int policy, unsigned push_min, bool may_push,
                  bool single, hipStream_t st);
// Reverse CSR (rin_ptr, rin) of the graph.  With `scratch` of
// rev_scratch_bytes(n, m) bytes (0 when the plan does not apply) the build
// is partitioned by head bucket; otherwise it counts and fills with global
// atomics (deg and tot are its counters).  Also clears the mark bytes.
struct RevPlan {
    int64_t buckets, chunk, nblk, hist_len;
    int bits;   // heads per bucket = 2^bits
    bool partition;
};
RevPlan rev_plan(int64_t n, int64_t m);
size_t rev_scratch_bytes(int64_t n, int64_t m);
void launch_rev_build(int n, int m, const int* row_ptr, const int* col, unsigned* deg,
                      unsigned* tot, int* rin_ptr, int* rin, unsigned char* marks, void* scratch,
                      hipStream_t st);
// gate (nullable): the init does nothing while *gate is 0.  have_succ: succ
// already holds col[pi]; otherwise it is written.
// Dhi (nullable): int128 entries, whose high words start sign-extended.
// t (nullable): cycle ratio, the entries start at L * w - W * t.
void launch_val_init(int n, const int* col, const int* pi, const void* w, int wtype, int neg,
                     int s, long long W, long long L, int* succ, bool have_succ, Jmp* Q, Ctl* ctl,
                     const unsigned* gate, hipStream_t st, long long* Dhi = nullptr,
                     const int* t = nullptr);
void launch_val_round(int n, int s, const Jmp* Qin, Jmp* Qout, unsigned* active, hipStream_t st,
                      const long long* hin = nullptr, long long* hout = nullptr);
void launch_val_final(int n, const Jmp* Q, long long* V, int* hop, Ctl* ctl, hipStream_t st,
                      const long long* hin = nullptr, long long* Vhi = nullptr,
                      int* V32 = nullptr);
// *bad |= some int128 value (lo, hi) does not fit int64.
void launch_fits64(int n, const long long* lo, const long long* hi, unsigned* bad,
                   hipStream_t st);
void launch_cycle_list(int n, int s, long long L, const unsigned char* onC, const int* pi,
                       const int* hop, int* out, hipStream_t st);
void launch_tie_short_walk(const SweepArgs& a, const void* w, int wtype, int G, const int* succ,
                           unsigned grid, hipStream_t st);
void launch_ctl_clear(Ctl* ctl, unsigned what, hipStream_t st);
void launch_ctl_set(Ctl* ctl, int s, long long W, long long L, hipStream_t st);
void launch_zero2(unsigned* a, unsigned* b, hipStream_t st);
// exclusive prefix sum of len values; tot needs len/2048 + 1 entries
void launch_exclusive_scan(int64_t len, const unsigned* in, unsigned* out, unsigned* tot,
                           hipStream_t st);

// Reads `bytes` (a multiple of 4, at most 256) of device memory into host
// memory once the stream's earlier work is done.
hipError_t host_read(const void* dsrc, void* hdst, size_t bytes, hipStream_t st);
// Folds a control block's lanes and reads the snapshot.
hipError_t host_read_ctl(const Ctl* ctl, CtlView* out, hipStream_t st);
// The same through a copy into the caller's stack and a stream
// synchronisation: no pinned mailbox is created (used by the entry point
// that allocates nothing).
hipError_t host_read_ctl_copy(const Ctl* ctl, CtlView* out, hipStream_t st);

// Multichain policy iteration (every policy cycle keeps its own gain).
// Value entries are Jmp: D sums L_r * w - W_r over the first H policy edges
// of v's path, where r is the smallest vertex of the cycle that path reaches
// and W_r, L_r are that cycle's weight and length; J is the vertex reached,
// or ~r once the path has reached r.  After the final the entries are the
// records the sweep gathers: D = V(v), J = r, H = hops from v to r.
struct McArgs {
    int n;
    int neg;
    const int* row_ptr;
    const int* col;
    const Jmp* R;                  // per-vertex records (value, cycle, hops)
    const long long* wsum;         // per cycle (keyed by r): weight
    const unsigned* lcnt;          //                         length
    int* pi;
    int* succ;                     // col[pi], kept up to date where pi changes
    Ctl* ctl;
    // tie scan only: the optimal gain W / L, C's flags, hops, list of the
    // tight non-policy edges between vertices of optimal gain
    long long W, L;
    const unsigned char* onC;
    int* xs;
    int* ys;
    unsigned* xcnt;
    unsigned xcap;
    GiantTab giant;                // rows swept by several workgroups (as in the tile sweeps)
};
// Entries of every vertex: roots (the smallest vertex of each policy cycle)
// finished with D = 0; succ gets col[pi] unless have_succ; lanes' active =
// unfinished vertices.
void launch_mc_val_init(int n, const int* col, const int* pi, const void* w, int wtype, int neg,
                        const int* rep, const unsigned char* onc, const long long* wsum,
                        const unsigned* lcnt, int* succ, bool have_succ, Jmp* Q, Ctl* ctl,
                        hipStream_t st);
// Device-driven rounds as launch_val_round_dev (jump setup with values).
void launch_mc_round_dev(int n, int r, const Jmp* Qin, Jmp* Qout, Ctl* ctl, hipStream_t st);
// After the rounds: V, hop, the lanes' overflow flag, and the records in
// place (buffer jk & 1).
void launch_mc_final_dev(int n, Jmp* Q0, Jmp* Q1, long long* V, int* hop, Ctl* ctl,
                         hipStream_t st);
// G lanes per vertex (power of two <= 64).  Not tie: the improvement sweep
// (lanes' changed) that also counts every tight non-policy edge (lanes'
// tight).  tie: counts (tight), and lists when a.xs is set, the tight
// non-policy edges whose tail has the optimal gain a.W / a.L, with certain
// (a tight self-loop or a tail on C) and nondec (head not nearer its root).
void launch_mc_sweep(const McArgs& a, const void* w, int wtype, int G, bool tie, hipStream_t st);
// Lanes' ncrit = policy cycles whose gain equals W / L.
void launch_mc_ncrit(const int* cyc_list, const long long* wsum, const unsigned* lcnt, long long W,
                     long long L, Ctl* ctl, hipStream_t st);
// onC = vertices of the policy cycle whose smallest vertex is s.
void launch_mc_mark_c(int n, const int* rep, const unsigned char* onc, int s, unsigned char* onC,
                      hipStream_t st);

// Upper bound of the batched workspace for G graphs over n vertices and m
// edges, the largest graph at most max_n vertices and max_m edges.
size_t batched_ws_bound(int64_t G, int64_t n, int64_t m, int64_t max_n, int64_t max_m);

// thread-local message returned by ocm_last_error()
void set_last_error(const char* what);

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kWG - 1) / kWG); }
inline unsigned stride_grid(int64_t n)
{
    const unsigned b = blocks_for(n);
    return b < 2048 ? b : 2048;
}
void launch_tie_special(int n, unsigned k, int* xs, int* ys, const int* succ,
                        const unsigned char* onC, unsigned char* sp, int* spid, int* slist,
                        unsigned* scnt, hipStream_t st);
void launch_tie_walk(int n, unsigned ns, const int* slist, const int* succ,
                     const unsigned char* sp, const unsigned char* onC, const int* spid, int* P,
                     unsigned k, int* xs, int* ys, hipStream_t st);
void launch_adjoint_scatter(int64_t m, const int* cyc, int64_t len, const double* g, double* grad,
                            hipStream_t st);
void launch_w_from_f64(int64_t m, const double* w, long long* out, unsigned* bad, hipStream_t st);
void launch_check_policy(int n, const int* row_ptr, const int* pi, unsigned* bad, hipStream_t st);
void launch_fill_u8(unsigned char* p, int64_t n, unsigned char v, hipStream_t st);
void launch_fill_u32(unsigned* p, int64_t len, unsigned v, hipStream_t st);

}  // namespace ocm
