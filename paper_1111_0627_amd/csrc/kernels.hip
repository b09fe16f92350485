// Device kernels of the exact optimal-cycle-mean solver (gfx950, wave64).
//
// Howard's policy iteration (Alg. 2) decomposed into data-parallel phases as
// in Alg. 3.  Phase names follow the paper's kernels:
//   sweep    SPFPassIter: policy improvement over the CSR out-edges
//   cycles   GpiPreprocess + elimination + cycleIdentification, done here by
//            pointer jumping over the one-successor policy graph
//   select   reduce_min + setMinCycle: minimum-mean cycle, exact order
//   connect  markMinComponent + connectGpi: breadth-first rebuild rounds
//   values   val[source] <- 0 + valuePropagate (Alg. 4), by pointer jumping
// All values are exact integers: V is scaled by L = |C| so that lambda = W/L
// never has to be divided.
#include <cstdlib>
#include <cstring>

#include "kernels.h"
#include "device_util.h"

namespace ocm {

// ---------------------------------------------------------------------------
// validation: CSR shape of Fig. 2b, out-degree >= 1, max |w|
// ---------------------------------------------------------------------------
template <typename WT>
__global__ __launch_bounds__(kWG) void k_validate(int n, int m, const int* __restrict__ row_ptr,
                                                  const int* __restrict__ col,
                                                  const WT* __restrict__ w, int check_csr,
                                                  Ctl* ctl)
{
    unsigned err = 0;
    unsigned long long mx = 0;
    const int64_t total = (int64_t)(n > m ? n : m);
    const int64_t stride = (int64_t)gridDim.x * kWG;
    constexpr int U = 8;   // independent elements in flight per thread
    for (int64_t ib = (int64_t)blockIdx.x * kWG + threadIdx.x; ib < total; ib += U * stride) {
        int ra[U], rb[U], c[U];
        WT wv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = ib + u * stride;
            ra[u] = rb[u] = c[u] = 0;
            wv[u] = 0;
            if (check_csr && i < n) {
                ra[u] = row_ptr[i];
                rb[u] = row_ptr[i + 1];
            }
            if (i < m) {
                if (check_csr) c[u] = col[i];
                wv[u] = w[i];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = ib + u * stride;
            if (check_csr && i < n) {
                if (rb[u] < ra[u]) err |= kErrBadCsr;
                if (rb[u] == ra[u]) err |= kErrNoOut;
                if (i == 0 && (ra[u] != 0 || row_ptr[n] != m)) err |= kErrBadCsr;
            }
            if (i < m) {
                if (check_csr && (c[u] < 0 || c[u] >= n)) err |= kErrBadCsr;
                const unsigned long long a = uabs64((int64_t)wv[u]);
                mx = a > mx ? a : mx;
            }
        }
    }
    mx = block_max_u64(mx);
    __shared__ unsigned eor;
    if (threadIdx.x == 0) eor = 0;
    __syncthreads();
    if (err) atomicOr(&eor, err);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (mx) atomicMax(&my_lane(ctl).maxabsw, mx);
        if (eor) atomicOr(&my_lane(ctl).err, eor);
    }
}

// ---------------------------------------------------------------------------
// sweep (SPFPassIter): G lanes per vertex, segmented argmin over out-edges
// ---------------------------------------------------------------------------
#ifndef OCM_SWEEP_UNROLL
#define OCM_SWEEP_UNROLL 2
#endif

// Improvement sweep with U vertices per lane group and step: the offsets,
// each lane's first out-edge and its gathered value are loaded for all U
// vertices before any of them is reduced, so every wave keeps U independent
// load chains in flight.  Same result as k_sweep: within a lane edges are
// visited in CSR order with a strict "<", and the cross-lane reduction
// breaks ties by the lower position.
template <int G, typename WT, bool FIRST, int U>
__global__ __launch_bounds__(kWG) void k_sweep_u(SweepArgs a, const WT* __restrict__ w)
{
    constexpr int VPB = kWG / G;             // vertices per block per step and unroll slot
    const int64_t L = FIRST ? 1 : a.L;
    const int64_t W = FIRST ? 0 : a.W;
    const int lane = threadIdx.x & (G - 1);
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int64_t per = ((int64_t)a.n + gridDim.x - 1) / gridDim.x;
    const int64_t v0 = (int64_t)b * per;
    const int64_t v1 = v0 + per < a.n ? v0 + per : a.n;
    unsigned long long cnt = 0;
    unsigned cbroken = 0;
    for (int64_t vb = v0; vb < v1; vb += U * VPB) {
        int64_t v[U], own[U], best[U];
        int beg[U], end[U], bpos[U], c0[U];
        int64_t w0[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            v[u] = vb + u * VPB + threadIdx.x / G;
            beg[u] = end[u] = 0;
            own[u] = 0;
            if (v[u] < v1) {
                beg[u] = a.row_ptr[v[u]];
                end[u] = a.row_ptr[v[u] + 1];
                if (!FIRST) own[u] = a.V[v[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = beg[u] + lane;
            c0[u] = 0;
            w0[u] = 0;
            if (e < end[u]) {
                w0[u] = wval(w, e, a.neg);
                if (!FIRST) c0[u] = a.col[e];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = beg[u] + lane;
            best[u] = INT64_MAX;
            bpos[u] = INT32_MAX;
            if (e < end[u]) {
                best[u] = FIRST ? w0[u] : a.V[c0[u]] + L * w0[u] - W;
                bpos[u] = e;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            for (int e = beg[u] + lane + G; e < end[u]; e += G) {
                const int64_t we = wval(w, e, a.neg);
                const int64_t key = FIRST ? we : a.V[a.col[e]] + L * we - W;
                if (key < best[u]) {
                    best[u] = key;
                    bpos[u] = e;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) {
                const int64_t ob = __shfl_xor(best[u], off, G);
                const int op = __shfl_xor(bpos[u], off, G);
                if (ob < best[u] || (ob == best[u] && op < bpos[u])) {
                    best[u] = ob;
                    bpos[u] = op;
                }
            }
            if (v[u] < v1 && lane == 0 && (FIRST || best[u] < own[u])) {
                a.pi[v[u]] = bpos[u];
                cnt++;
                if (!FIRST && a.onC && a.onC[v[u]]) cbroken = 1;
            }
        }
    }
    cnt = block_sum_u64(cnt);
    const unsigned long long brk = block_sum_u64(cbroken);
    if (threadIdx.x == 0) {
        CtlLane& ln = my_lane(a.ctl);
        if (cnt) atomicAdd(&ln.changed, cnt);
        if (brk) atomicOr(&ln.cbroken, 1u);
    }
}

// Sweep over a tile: a workgroup takes kWG consecutive vertices, whose
// out-edges form one contiguous CSR range.  The range is processed in
// batches of kTileEdges: every thread loads kTileEdges / kWG edges (col, w,
// then the gathered V, all independent loads) and stores their keys in LDS;
// then each thread walks its own vertex's part of the batch in CSR order,
// keeping the minimum key at the lowest position.  Three dependent global
// loads per batch instead of per vertex step; same result as k_sweep_u.
constexpr int kTileEdges = 2048;

// First position at or after eb (below e1) outside the tile's giant rows
// (beg: the tile's nv + 1 row offsets).  The same in every thread.
__device__ __forceinline__ int skip_giant(const int* beg, int nv, int eb, int e1)
{
    while (eb < e1) {
        int lo = 0, hi = nv - 1;   // the row holding eb: the last x with beg[x] <= eb
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (beg[mid] <= eb) lo = mid;
            else hi = mid - 1;
        }
        if (beg[lo + 1] - beg[lo] <= kGiantRow) break;
        eb = beg[lo + 1];
    }
    return eb;
}

// VM: how V is read (0 int64, 1 int128 in a.V / a.Vhi with int128 keys, 2
// the int32 copy a.V32).  RATIO: cycle ratio, the key is
// V[head] + L * w - W * t (a.t: edge times).
template <typename WT, bool FIRST, int VM = 0, bool RATIO = false>
__global__ __launch_bounds__(kWG) void k_sweep_tile(SweepArgs a, const WT* __restrict__ w)
{
    using KT = typename ValT<VM>::type;
    __shared__ int beg[kWG + 1];
    __shared__ KT key[kTileEdges];
    const int64_t L = FIRST ? 1 : a.L;
    const int64_t W = FIRST ? 0 : a.W;
    const int64_t v0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kWG;
    const int nv = a.n - v0 < kWG ? (int)(a.n - v0) : kWG;
    const int t = threadIdx.x;
    KT own = 0, best = val_max<KT>();
    int pos = INT32_MAX;
    if (t < nv) {
        beg[t] = a.row_ptr[v0 + t];
        if (!FIRST) own = load_val<VM>(a.V, a.Vhi, a.V32, v0 + t);
    }
    if (t == 0) beg[nv] = a.row_ptr[v0 + nv];
    __syncthreads();
    const int e0 = beg[0], e1 = beg[nv];
    // giant rows are left to k_giant_part / k_giant_merge
    const bool giant = a.giant.ngiant > 0 && t < nv && beg[t + 1] - beg[t] > kGiantRow;
    const bool skip = a.giant.ngiant > 0 && __syncthreads_or(giant);
    const int mb = t < nv && !giant ? beg[t] : 0, me = t < nv && !giant ? beg[t + 1] : 0;
    constexpr int U = kTileEdges / kWG;
    for (int eb = skip ? skip_giant(beg, nv, e0, e1) : e0; eb < e1;) {
        const int cnt = e1 - eb < kTileEdges ? e1 - eb : kTileEdges;
        if (FIRST) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = t + u * kWG;
                if (j < cnt) key[j] = wval(w, eb + j, a.neg);
            }
        } else {
            int c[U];
            long long wl[U], tl[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = t + u * kWG;
                c[u] = 0;
                wl[u] = 0;
                tl[u] = 1;
                if (j < cnt) {
                    c[u] = a.col[eb + j];
                    wl[u] = wval(w, eb + j, a.neg);
                    if (RATIO) tl[u] = a.t[eb + j];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = t + u * kWG;
                if (j < cnt)
                    key[j] = load_val<VM>(a.V, a.Vhi, a.V32, c[u]) +
                             (KT)(L * wl[u] - (RATIO ? W * tl[u] : W));
            }
        }
        __syncthreads();
        // this vertex's edges inside the batch, in CSR order
        const int lo = mb > eb ? mb : eb, hi = me < eb + cnt ? me : eb + cnt;
        const bool long_row = hi - lo > kLongRow;
        if (!long_row)
            for (int e = lo; e < hi; ++e) {
                const KT k = key[e - eb];
                if (k < best) {
                    best = k;
                    pos = e;
                }
            }
        // the wave's long rows, one after the other, by all its lanes
        for (unsigned long long lm = __ballot(long_row); lm; lm &= lm - 1) {
            const int l = __ffsll((long long)lm) - 1;
            const int rlo = __shfl(lo, l, 64), rhi = __shfl(hi, l, 64);
            KT rb = val_max<KT>();
            int rp = INT32_MAX, rh = 0;
            for (int e = rlo + (t & 63); e < rhi; e += 64) {
                const KT k = key[e - eb];
                if (k < rb) {
                    rb = k;
                    rp = e;
                }
            }
            wave_argmin<KT, false>(rb, rp, rh);
            if ((t & 63) == l && rb < best) {   // earlier batches hold lower positions
                best = rb;
                pos = rp;
            }
        }
        __syncthreads();
        eb += cnt;
        if (skip) eb = skip_giant(beg, nv, eb, e1);
    }
    unsigned long long changed = 0;
    unsigned cbroken = 0;
    if (t < nv && pos != INT32_MAX && (FIRST || best < own)) {
        a.pi[v0 + t] = pos;
        if (a.succ) a.succ[v0 + t] = a.col[pos];   // the batch just read it
        changed = 1;
        if (!FIRST && a.onC && a.onC[v0 + t]) cbroken = 1;
    }
    unsigned long long sums[2] = {changed, cbroken};
    block_sums_u64(sums);
    if (t == 0) {
        CtlLane& ln = my_lane(a.ctl);
        if (sums[0]) atomicAdd(&ln.changed, sums[0]);
        if (sums[1]) atomicOr(&ln.cbroken, 1u);
    }
}

// Tie scan over a tile (batches as k_sweep_tile; the heads are kept in LDS
// too).  Counts the tight edges other than the policy edge, those that
// certainly close a second critical cycle (a tight self-loop, or a tight
// edge leaving C: every policy path leads back to C), and those whose head
// is not nearer the source; optionally lists them.  SWEEP: also the
// improvement sweep of k_sweep_tile (not FIRST) in the same pass; when it
// changes no policy edge its counts are the tie scan's (no hop test, no
// list), so the solve's last sweep doubles as the tie check's first scan.
// Edges per batch of the tie scan: keys and heads (12 bytes each) in LDS;
// 1536 keeps 8 workgroups per CU (measured 13 % faster than 2048 here).
constexpr int kTieTileEdges = 1536;

// The mean with int64 or int32 values is held to 64 VGPRs (8 waves per
// SIMD, as many as its LDS allows); left alone, the long-row walk would take
// it to 72 VGPRs and 7 waves.
template <typename WT, bool SWEEP, int VM = 0, bool RATIO = false>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(RATIO || VM == 1 ? 4 : 8, 8)))
void k_tiescan_tile(SweepArgs a, const WT* __restrict__ w)
{
    using KT = typename ValT<VM>::type;
    __shared__ int beg[kWG + 1];
    __shared__ KT key[kTieTileEdges];
    __shared__ int head[kTieTileEdges];
    const int64_t L = a.L, W = a.W;
    const int64_t v0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kWG;
    const int nv = a.n - v0 < kWG ? (int)(a.n - v0) : kWG;
    const int t = threadIdx.x;
    KT own = 0;
    int cur = -1, hv = 0;
    bool onc = false;
    if (t < nv) {
        beg[t] = a.row_ptr[v0 + t];
        own = load_val<VM>(a.V, a.Vhi, a.V32, v0 + t);
        cur = a.pi[v0 + t];
        if (a.hop) hv = a.hop[v0 + t];
        onc = a.onC && a.onC[v0 + t];
    }
    if (t == 0) beg[nv] = a.row_ptr[v0 + nv];
    __syncthreads();
    const int e0 = beg[0], e1 = beg[nv];
    // giant rows are left to k_giant_part / k_giant_merge
    const bool giant = a.giant.ngiant > 0 && t < nv && beg[t + 1] - beg[t] > kGiantRow;
    const bool skip = a.giant.ngiant > 0 && __syncthreads_or(giant);
    const int mb = t < nv && !giant ? beg[t] : 0, me = t < nv && !giant ? beg[t + 1] : 0;
    unsigned long long cnt = 0, certain = 0, nondec = 0;
    KT best = val_max<KT>();
    int pos = INT32_MAX, bhead = 0;
    constexpr int U = kTieTileEdges / kWG;
    for (int eb = skip ? skip_giant(beg, nv, e0, e1) : e0; eb < e1;) {
        const int n_e = e1 - eb < kTieTileEdges ? e1 - eb : kTieTileEdges;
        int c[U];
        long long wl[U], tl[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = t + u * kWG;
            c[u] = 0;
            wl[u] = 0;
            tl[u] = 1;
            if (j < n_e) {
                c[u] = a.col[eb + j];
                wl[u] = wval(w, eb + j, a.neg);
                if (RATIO) tl[u] = a.t[eb + j];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = t + u * kWG;
            if (j < n_e) {
                key[j] = load_val<VM>(a.V, a.Vhi, a.V32, c[u]) +
                         (KT)(L * wl[u] - (RATIO ? W * tl[u] : W));
                head[j] = c[u];
            }
        }
        __syncthreads();
        const int lo = mb > eb ? mb : eb, hi = me < eb + n_e ? me : eb + n_e;
        const bool long_row = hi - lo > kLongRow;
        for (int e = lo; e < (long_row ? lo : hi); ++e) {
            const KT k = key[e - eb];
            const int h = head[e - eb];
            if (SWEEP && k < best) {
                best = k;
                pos = e;
                bhead = h;
            }
            const bool tight = k == own && e != cur;
            if (tight) {
                cnt++;
                if (h == v0 + t || onc) certain++;
                if (a.hop && a.hop[h] >= hv) nondec++;
            }
            if (a.xs) {   // one counter atomic per wave and step
                const unsigned slot = wave_append(tight, a.xcnt);
                if (tight && slot < a.xcap) {
                    a.xs[slot] = (int)(v0 + t);
                    a.ys[slot] = h;
                }
            }
        }
        // the wave's long rows, one after the other, by all its lanes
        for (unsigned long long lm = __ballot(long_row); lm; lm &= lm - 1) {
            const int l = __ffsll((long long)lm) - 1;
            const int rlo = __shfl(lo, l, 64), rhi = __shfl(hi, l, 64);
            const KT rown = shfl_kt(own, l);
            const int rcur = __shfl(cur, l, 64), rhv = __shfl(hv, l, 64);
            const bool ronc = __shfl((int)onc, l, 64) != 0;
            const int rv = (int)(v0 + (t & ~63) + l);
            KT rb = val_max<KT>();
            int rp = INT32_MAX, rh = 0;
            for (int e = rlo + (t & 63); e < rhi; e += 64) {
                const KT k = key[e - eb];
                const int h = head[e - eb];
                if (SWEEP && k < rb) {
                    rb = k;
                    rp = e;
                    rh = h;
                }
                const bool tight = k == rown && e != rcur;
                if (tight) {
                    cnt++;
                    if (h == rv || ronc) certain++;
                    if (a.hop && a.hop[h] >= rhv) nondec++;
                }
                if (a.xs) {
                    const unsigned slot = wave_append(tight, a.xcnt);
                    if (tight && slot < a.xcap) {
                        a.xs[slot] = rv;
                        a.ys[slot] = h;
                    }
                }
            }
            if (SWEEP) {
                wave_argmin<KT, true>(rb, rp, rh);
                if ((t & 63) == l && rb < best) {   // earlier batches hold lower positions
                    best = rb;
                    pos = rp;
                    bhead = rh;
                }
            }
        }
        __syncthreads();
        eb += n_e;
        if (skip) eb = skip_giant(beg, nv, eb, e1);
    }
    unsigned long long changed = 0;
    unsigned cbroken = 0;
    if (SWEEP && t < nv && pos != INT32_MAX && best < own) {
        a.pi[v0 + t] = pos;
        if (a.succ) a.succ[v0 + t] = bhead;
        changed = 1;
        if (onc) cbroken = 1;
    }
    unsigned long long sums[5] = {cnt, certain, nondec, changed, cbroken};
    block_sums_u64(sums);
    if (t == 0) {
        CtlLane& ln = my_lane(a.ctl);
        if (sums[0]) atomicAdd(&ln.tight, sums[0]);
        if (sums[1]) atomicAdd(&ln.certain, sums[1]);
        if (sums[2]) atomicAdd(&ln.nondec, sums[2]);
        if (SWEEP && sums[3]) atomicAdd(&ln.changed, sums[3]);
        if (SWEEP && sums[4]) atomicOr(&ln.cbroken, 1u);
    }
}

// ---------------------------------------------------------------------------
// giant rows: several workgroups per row
// ---------------------------------------------------------------------------
struct alignas(16) GiantPart {
    __int128 key;   // the chunk's smallest key (any value mode, widened)
    int pos;        // its lowest position (INT32_MAX: none)
    int head;
    int pad[2];
};

__global__ __launch_bounds__(kWG) void k_giant_list(int n, const int* __restrict__ row_ptr,
                                                    int* __restrict__ triples, unsigned cap,
                                                    Ctl* ctl)
{
    for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kWG) {
        const int b = row_ptr[v], e = row_ptr[v + 1];
        if (e - b <= kGiantRow) continue;
        const unsigned i = atomicAdd(&ctl->ngiant, 1u);
        if (i < cap) {
            triples[3 * i] = (int)v;
            triples[3 * i + 1] = b;
            triples[3 * i + 2] = e;
        }
    }
}

// One workgroup per chunk (grid-stride over the chunks).  MODE 0: the first
// sweep (keys are the weights); 1: an improvement sweep (COUNT: it also
// counts tight edges, as k_tiescan_tile<SWEEP> does); 2: the tie scan
// (counts, and lists when a.xs is set; no best).  The chunk's best key at its
// lowest position goes to parts[c] (modes 0 and 1).
template <typename WT, int MODE, bool COUNT, int VM, bool RATIO>
__global__ __launch_bounds__(kWG) void k_giant_part(SweepArgs a, const WT* __restrict__ w)
{
    using KT = typename ValT<VM>::type;
    __shared__ KT sk[kWG / 64];
    __shared__ int sp[kWG / 64], sh[kWG / 64];
    const GiantTab& g = a.giant;
    GiantPart* parts = (GiantPart*)g.parts;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    unsigned long long cnt = 0, certain = 0, nondec = 0;
    for (int c = blockIdx.x; c < g.nchunks; c += gridDim.x) {
        const int v = g.cv[c], c0 = g.cs[c], c1 = g.ce[c];
        const KT own = MODE == 0 ? (KT)0 : load_val<VM>(a.V, a.Vhi, a.V32, v);
        int cur = -1, hv = 0;
        bool onc = false;
        if (COUNT) {
            cur = a.pi[v];
            if (a.hop) hv = a.hop[v];
            onc = a.onC && a.onC[v];
        }
        KT best = val_max<KT>();
        int pos = INT32_MAX, bh = 0;
        // lanes stride over the chunk: each keeps its lowest position among
        // equal keys
        for (int e = c0 + t; e < c1; e += kWG) {
            const int h = a.col[e];
            const long long wl = wval(w, e, a.neg);
            KT k;
            if (MODE == 0) k = (KT)wl;
            else
                k = load_val<VM>(a.V, a.Vhi, a.V32, h) +
                    (KT)(a.L * wl - (RATIO ? a.W * (long long)a.t[e] : a.W));
            if (MODE != 2 && k < best) {
                best = k;
                pos = e;
                bh = h;
            }
            if (COUNT) {
                const bool tight = k == own && e != cur;
                if (tight) {
                    ++cnt;
                    if (h == v || onc) ++certain;
                    if (a.hop && a.hop[h] >= hv) ++nondec;
                }
                if (MODE == 2 && a.xs) {   // one counter atomic per wave and step
                    const unsigned slot = wave_append(tight, a.xcnt);
                    if (tight && slot < a.xcap) {
                        a.xs[slot] = v;
                        a.ys[slot] = h;
                    }
                }
            }
        }
        if (MODE != 2) {
            wave_argmin<KT, true>(best, pos, bh);
            if (lane == 0) {
                sk[wave] = best;
                sp[wave] = pos;
                sh[wave] = bh;
            }
            __syncthreads();
            if (t == 0) {
                // the best wave by index (not a running record: see
                // k_mc_giant_part)
                int bi = 0;
                for (int i = 1; i < kWG / 64; ++i)
                    if (sk[i] < sk[bi] || (sk[i] == sk[bi] && sp[i] < sp[bi])) bi = i;
                GiantPart p;
                p.key = (__int128)sk[bi];
                p.pos = sp[bi];
                p.head = sh[bi];
                p.pad[0] = p.pad[1] = 0;
                parts[c] = p;
            }
            __syncthreads();   // sk is reused by the next chunk
        }
    }
    if (COUNT) {
        unsigned long long sums[3] = {cnt, certain, nondec};
        block_sums_u64(sums);
        if (t == 0) {
            CtlLane& ln = my_lane(a.ctl);
            if (sums[0]) atomicAdd(&ln.tight, sums[0]);
            if (sums[1]) atomicAdd(&ln.certain, sums[1]);
            if (sums[2]) atomicAdd(&ln.nondec, sums[2]);
        }
    }
}

// Each giant row's best over its chunks (in position order: a strict
// compare keeps the lowest position), then the sweep's write rule.
template <int VM, bool FIRST>
__global__ __launch_bounds__(kWG) void k_giant_merge(SweepArgs a)
{
    using KT = typename ValT<VM>::type;
    const GiantTab& g = a.giant;
    const GiantPart* parts = (const GiantPart*)g.parts;
    unsigned long long changed = 0, cbroken = 0;
    for (int i = blockIdx.x * kWG + threadIdx.x; i < g.ngiant; i += gridDim.x * kWG) {
        const int v = g.gv[i];
        // the best chunk by index, position order (strict keeps the lowest)
        int bi = -1;
        for (int c = g.gc0[i]; c < g.gc1[i]; ++c)
            if (parts[c].pos != INT32_MAX && (bi < 0 || (KT)parts[c].key < (KT)parts[bi].key))
                bi = c;
        if (bi < 0) continue;
        const KT best = (KT)parts[bi].key;
        if (!FIRST && !(best < load_val<VM>(a.V, a.Vhi, a.V32, v))) continue;
        a.pi[v] = parts[bi].pos;
        if (a.succ) a.succ[v] = parts[bi].head;
        ++changed;
        if (!FIRST && a.onC && a.onC[v]) cbroken = 1;
    }
    unsigned long long sums[2] = {changed, cbroken};
    block_sums_u64(sums);
    if (threadIdx.x == 0) {
        CtlLane& ln = my_lane(a.ctl);
        if (sums[0]) atomicAdd(&ln.changed, sums[0]);
        if (sums[1]) atomicOr(&ln.cbroken, 1u);
    }
}

// Start of device-driven jump rounds.  values: round 1 runs if init left
// unfinished vertices (their count, in the lanes' active, becomes jlast);
// cycles: round 1 runs.  gated (values): nothing runs unless jgate is open
// (set by k_fast_gate); otherwise the gate is opened here.
__global__ void k_jump_setup(Ctl* c, int values, int gated)
{
    if (threadIdx.x < kLanes) c->lane[threadIdx.x].rpack = 0;
    if (threadIdx.x == 0) {
        unsigned act = 0;
        for (int l = 0; l < kLanes; ++l) act += c->lane[l].active;
        if (!gated) c->jgate = 1;
        const bool open = c->jgate != 0;
        c->rpack = 0;
        c->jk = 0;
        c->jstall = 0;
        c->jlast = values ? act : 0u;
        c->jmode = values ? (act > 0 && open ? 1u : 0u) : 1u;
    }
}

// After a sweep whose value phase is queued behind it: open jgate only if
// the sweep changed a policy edge (or force) and no vertex of C changed.
__global__ void k_fast_gate(Ctl* c, int force)
{
    if (threadIdx.x == 0) {
        unsigned long long changed = 0;
        unsigned broken = 0;
        for (int l = 0; l < kLanes; ++l) {
            changed += c->lane[l].changed;
            broken |= c->lane[l].cbroken;
        }
        c->jgate = !broken && (changed > 0 || force) ? 1u : 0u;
    }
}

// ---------------------------------------------------------------------------
// cycles: pointer jumping over the policy graph.  Entry P[v] packs
// (J = succ^(2^k)(v), M = min vertex among the first 2^k vertices of v's
// policy path).  After K rounds with 2^K >= n, J is on v's cycle and M at a
// cycle vertex is the whole cycle's minimum.
//
// The host may stop earlier, after round r, when both of these hold:
//  * image(J_{r-1}) and image(J_{r-2}) have the same size.  J_{r-1} is
//    J_{r-2} applied twice, so J_{r-2} then maps its image S onto S, i.e.
//    permutes S; a permuted vertex returns to itself under succ, so S holds
//    cycle vertices only and every J_{r-2}(v), hence J_r(v), is on a cycle;
//  * no M changed in round r.  The update M' = min(M, M o J) at such a fixed
//    point stays fixed in every later round (J only advances to vertices
//    whose M is no smaller), so M_r is the minimum over v's whole path, which
//    at a cycle vertex is the cycle's minimum.
// Round r marks image(J_r) with tag r+1 in one of two byte arrays
// (alternating) and counts the vertices tagged r by the round before.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long pj_pack(int j, int mn)
{
    return ((unsigned long long)(unsigned)j << 32) | (unsigned)mn;
}

// have_succ: succ already holds col[pi] (kept up to date where pi changed);
// otherwise it is written here.
__global__ __launch_bounds__(kWG) void k_pj_init(int n, const int* __restrict__ col,
                                                 const int* __restrict__ pi, int* __restrict__ succ,
                                                 int have_succ,
                                                 unsigned long long* __restrict__ P,
                                                 unsigned char* __restrict__ onc,
                                                 unsigned char* __restrict__ tag0, unsigned* cnt)
{
    const int v = blockIdx.x * kWG + threadIdx.x;
    if (v == 0 && cnt)
        for (int l = 0; l < kLanes; ++l)
            for (int j = 0; j < 4; ++j) cnt[l * kLaneWords + j] = 0;
    if (v >= n) return;
    int s;
    if (have_succ) {
        s = succ[v];
    } else {
        s = col[pi[v]];
        succ[v] = s;
    }
    P[v] = pj_pack(s, v);
    onc[v] = 0;
    if (tag0) tag0[s] = 1;
}

constexpr int kJumpUnroll = 4;   // entries in flight per thread in grid-stride jump rounds

__global__ __launch_bounds__(kWG) void k_pj_round(int n, const unsigned long long* __restrict__ Pin,
                                                  unsigned long long* __restrict__ Pout)
{
    const int v = blockIdx.x * kWG + threadIdx.x;
    if (v >= n) return;
    const unsigned long long p = Pin[v];
    const int j = (int)(p >> 32);
    const unsigned long long q = Pin[j];
    const unsigned m0 = (unsigned)p, m1 = (unsigned)q;
    Pout[v] = (q & 0xffffffff00000000ull) | (m0 < m1 ? m0 : m1);
}

// A jump round with the stop test's tags: image(J) of this round is tagged
// tag_cur in tcur; returns (in thread 0) the vertices tagged tag_prev in
// tprev (the previous image) and the M changes.
__device__ __forceinline__ void pj_tagged_body(int n, const unsigned long long* __restrict__ Pin,
                                               unsigned long long* __restrict__ Pout,
                                               const unsigned char* __restrict__ tprev,
                                               unsigned char* __restrict__ tcur,
                                               unsigned char tag_prev, unsigned char tag_cur,
                                               unsigned long long* img_out,
                                               unsigned long long* chg_out)
{
    unsigned long long img = 0, chg = 0;
    // grid-stride with kJumpUnroll independent entries in flight per thread
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t v0 = (int64_t)blockIdx.x * kWG + threadIdx.x; v0 < n;
         v0 += kJumpUnroll * stride) {
        unsigned long long p[kJumpUnroll], q[kJumpUnroll];
#pragma unroll
        for (int u = 0; u < kJumpUnroll; ++u) {
            const int64_t v = v0 + u * stride;
            p[u] = v < n ? Pin[v] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < kJumpUnroll; ++u) {
            const int64_t v = v0 + u * stride;
            q[u] = v < n ? Pin[(int)(p[u] >> 32)] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < kJumpUnroll; ++u) {
            const int64_t v = v0 + u * stride;
            if (v < n) {
                const unsigned m0 = (unsigned)p[u], m1 = (unsigned)q[u];
                Pout[v] = (q[u] & 0xffffffff00000000ull) | (m0 < m1 ? m0 : m1);
                chg += m1 < m0;
                // the image shrinks fast: most targets are already tagged
                const int t = (int)(q[u] >> 32);
                if (tcur[t] != tag_cur) tcur[t] = tag_cur;
                img += tprev[v] == tag_prev;
            }
        }
    }
    *img_out = block_sum_u64(img);
    *chg_out = block_sum_u64(chg);
}

// Host-driven: cnt = {image count, M changes} of this round; nxt = the next
// round's pair (cleared here).
__global__ __launch_bounds__(kWG) void k_pj_round_tagged(
    int n, const unsigned long long* __restrict__ Pin, unsigned long long* __restrict__ Pout,
    const unsigned char* __restrict__ tprev, unsigned char* __restrict__ tcur,
    unsigned char tag_prev, unsigned char tag_cur, unsigned* cnt, unsigned* nxt)
{
    if (blockIdx.x == 0 && threadIdx.x < kLanes) {
        nxt[threadIdx.x * kLaneWords] = 0;
        nxt[threadIdx.x * kLaneWords + 1] = 0;
    }
    unsigned long long img, chg;
    pj_tagged_body(n, Pin, Pout, tprev, tcur, tag_prev, tag_cur, &img, &chg);
    if (threadIdx.x == 0) {
        unsigned* mine = my_copy(cnt);
        if (img) atomicAdd(&mine[0], (unsigned)img);
        if (chg) atomicAdd(&mine[1], (unsigned)chg);
    }
}

// Device-driven round r: the last workgroup applies the stop test (the
// image size repeated and no M changed) and ends the rounds when it holds.
__global__ __launch_bounds__(kWG) void k_pj_round_dev(
    int n, int r, const unsigned long long* __restrict__ Pin, unsigned long long* __restrict__ Pout,
    const unsigned char* __restrict__ tprev, unsigned char* __restrict__ tcur, Ctl* ctl)
{
    if (!jump_round_is(ctl, r)) return;
    unsigned long long img, chg;
    pj_tagged_body(n, Pin, Pout, tprev, tcur, (unsigned char)r, (unsigned char)(r + 1), &img, &chg);
    if (threadIdx.x != 0) return;
    unsigned long long tot;
    if (!last_arrival(ctl, arrival_word(img, chg != 0), &tot)) return;
    const unsigned image = (unsigned)tot;
    const bool changed = ((tot >> 32) & 0xffffu) != 0;
    const bool stop = r >= 2 && image == ctl->jlast && !changed;
    ctl->jlast = image;
    ctl->jk = (unsigned)r;
    if (stop) ctl->jmode = 0;
}

__global__ __launch_bounds__(kWG) void k_pj_final(int n, const unsigned long long* __restrict__ P,
                                                  int* __restrict__ rep,
                                                  unsigned char* __restrict__ onc)
{
    const int v = blockIdx.x * kWG + threadIdx.x;
    if (v >= n) return;
    const int c = (int)(P[v] >> 32);
    rep[v] = (int)(unsigned)P[c];
    onc[c] = 1;
}

// Device-driven: runs once the rounds are over (stopped, or all K run), on
// the entries of the last round run.
__global__ __launch_bounds__(kWG) void k_pj_final_dev(int n, const unsigned long long* __restrict__ P0,
                                                      const unsigned long long* __restrict__ P1,
                                                      int K, int* __restrict__ rep,
                                                      unsigned char* __restrict__ onc, const Ctl* ctl)
{
    if (ctl->jmode != 0 && ctl->jk != (unsigned)K) return;
    const unsigned long long* __restrict__ P = (ctl->jk & 1) ? P1 : P0;
    const int v = blockIdx.x * kWG + threadIdx.x;
    if (v >= n) return;
    const int c = (int)(P[v] >> 32);
    rep[v] = (int)(unsigned)P[c];
    onc[c] = 1;
}

// ---------------------------------------------------------------------------
// select: per-cycle (W, L) keyed by rep, then the minimum in exact order
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_cyc_zero(int n, const int* __restrict__ rep,
                                                  const unsigned char* __restrict__ onc,
                                                  unsigned per, long long* __restrict__ wsum,
                                                  unsigned* __restrict__ lcnt,
                                                  int* __restrict__ cyc_list, Ctl* ctl,
                                                  long long* __restrict__ tsum)
{
    __shared__ int hbuf[kListItems];
    __shared__ unsigned nh;
    if (threadIdx.x == 0) nh = 0;
    __syncthreads();
    BlockList bl{hbuf, &nh};
    const int64_t v0 = (int64_t)blockIdx.x * per;
    const int64_t v1 = v0 + per < n ? v0 + per : n;
    for (int64_t vb = v0; vb < v1; vb += kWG) {
        const int64_t v = vb + threadIdx.x;
        const bool head = v < v1 && onc[v] && rep[v] == v;
        if (head) {
            wsum[v] = 0;
            lcnt[v] = 0;
            if (tsum) tsum[v] = 0;
        }
        blist_push(bl, head, (int)v);
    }
    blist_flush(bl, cyc_list, &ctl->ncyc);
}

template <typename WT>
__global__ __launch_bounds__(kWG) void k_cyc_sum(int n, const int* __restrict__ rep,
                                                 const unsigned char* __restrict__ onc,
                                                 const int* __restrict__ pi,
                                                 const WT* __restrict__ w, int neg,
                                                 long long* __restrict__ wsum,
                                                 unsigned* __restrict__ lcnt,
                                                 const int* __restrict__ tm,
                                                 long long* __restrict__ tsum)
{
    const int v = blockIdx.x * kWG + threadIdx.x;
    if (v >= n || !onc[v]) return;
    const int r = rep[v];
    const int e = pi[v];
    atomicAdd((unsigned long long*)&wsum[r], (unsigned long long)wval(w, e, neg));
    atomicAdd(&lcnt[r], 1u);
    if (tsum) atomicAdd((unsigned long long*)&tsum[r], (unsigned long long)tm[e]);
}

struct Cand {
    long long W;
    long long L;
    int r;
};

// a < b in the order (W/L, r); L > 0.
__device__ __forceinline__ bool cand_less(const Cand& a, const Cand& b)
{
    if (b.r < 0) return a.r >= 0;
    if (a.r < 0) return false;
    const __int128 x = (__int128)a.W * b.L, y = (__int128)b.W * a.L;
    if (x != y) return x < y;
    return a.r < b.r;
}

__device__ __forceinline__ Cand cand_shfl_xor(const Cand& c, int off)
{
    Cand o;
    o.W = __shfl_xor(c.W, off, 64);
    o.L = __shfl_xor(c.L, off, 64);
    o.r = __shfl_xor(c.r, off, 64);
    return o;
}

// Best candidate of the workgroup (valid in thread 0).
__device__ __forceinline__ Cand block_best(Cand best)
{
    __shared__ Cand sh[kWG / 64];
    for (int off = 32; off > 0; off >>= 1) {
        const Cand o = cand_shfl_xor(best, off);
        if (cand_less(o, best)) best = o;
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 1; i < kWG / 64; ++i)
            if (cand_less(sh[i], best)) best = sh[i];
    return best;
}

// tsum (cycle ratio): a cycle's denominator is its time, not its length.
__global__ __launch_bounds__(kWG) void k_select_part(const int* __restrict__ cyc_list,
                                                     const long long* __restrict__ wsum,
                                                     const unsigned* __restrict__ lcnt,
                                                     const long long* __restrict__ tsum,
                                                     const Ctl* ctl, Cand* __restrict__ part)
{
    const unsigned nc = ctl->ncyc;
    Cand best{0, 1, -1};
    for (unsigned i = blockIdx.x * kWG + threadIdx.x; i < nc; i += gridDim.x * kWG) {
        const int r = cyc_list[i];
        const Cand c{wsum[r], tsum ? tsum[r] : (long long)lcnt[r], r};
        if (cand_less(c, best)) best = c;
    }
    best = block_best(best);
    if (threadIdx.x == 0) part[blockIdx.x] = best;
}

__global__ __launch_bounds__(kWG) void k_select_final(const Cand* __restrict__ part, int nparts,
                                                      const unsigned* __restrict__ lcnt, Ctl* ctl)
{
    Cand best{0, 1, -1};
    for (int i = threadIdx.x; i < nparts; i += kWG)
        if (cand_less(part[i], best)) best = part[i];
    best = block_best(best);
    if (threadIdx.x == 0) {
        ctl->s = best.r;
        ctl->W = best.W;
        ctl->L = best.L;
        ctl->clen = best.r >= 0 ? lcnt[best.r] : 0u;
    }
}

// Edge times of a cycle ratio must be >= 1; their maximum bounds the values.
__global__ __launch_bounds__(kWG) void k_validate_t(int m, const int* __restrict__ t, Ctl* ctl)
{
    unsigned bad = 0;
    unsigned long long mx = 0;
    for (int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * kWG) {
        const int x = t[e];
        bad |= x < 1 ? 1u : 0u;
        mx = (unsigned long long)x > mx ? (unsigned long long)x : mx;
    }
    mx = block_max_u64(mx);
    const unsigned anybad = (unsigned)block_sum_u64(bad);
    if (threadIdx.x == 0) {
        CtlLane& ln = my_lane(ctl);
        if (mx) atomicMax(&ln.maxabsw, mx);
        if (anybad) atomicOr(&ln.bad, 1u);
    }
}

// ---------------------------------------------------------------------------
// connect: keep the chosen cycle's component, attach the rest breadth-first
// ---------------------------------------------------------------------------
// Each block owns a contiguous range of at most kListItems inputs; outputs
// are buffered in LDS and written with one global atomic per block.
//
// The rebuild attaches vertices in rounds.  In round k an unattached vertex u
// can only have out-edges into layer k-1 (an edge into an earlier layer would
// have attached it earlier), so "the lowest-position out-edge into the set
// attached before round k" is u's lowest out-edge whose head is attached.
//
// Two bitmaps (one bit per vertex) alternate: at the start of round k,
// A[k&1] holds the layers <= k-1 and A[(k+1)&1] the layers <= k-2, so the
// frontier (layer k-1) is A[k&1] & ~A[(k+1)&1].  Round k only reads A[k&1];
// it adds the frontier and its own attachments (layer k) to A[(k+1)&1],
// which restores the invariant for round k+1.  No vertex lists are kept:
// every round kernel owns 64 bitmap words (2048 vertices) per workgroup, so
// each word has one writer and needs no atomics.
//   pull: the workgroup lists its unattached vertices and scans their
//         out-edges (k_conn_pull);
//   push: the frontier's in-edges mark their unattached tails in a byte
//         array (k_conn_mark) and only the marked vertices scan
//         (k_conn_claim).
// Both find, for every vertex that attaches, the same (lowest) edge; the host
// picks the cheaper direction per round.
// A round workgroup owns kWG consecutive bitmap words, one per thread (32
// vertices).  Claims and pull rounds: each wave handles its 64 words on its
// own: it ranks its candidates (marked or unattached vertices) in word order
// and gives rank r to lane r % 64, so the lanes share the work evenly without
// workgroup barriers; a lane scans its vertex's out-row itself, four entries
// per step, and stops at the first attached head (the lowest one); rows
// longer than kLaneRow are scanned by the whole wave, 64 entries per step.
// Marks: the workgroup lists its frontier vertices in LDS batches and spreads
// all their in-edges over its threads (every in-edge is visited, and spread
// rows give coalesced loads; measured faster than the per-wave scheme here).
constexpr int kLaneRow = 32;
constexpr int kWaves = kWG / 64;

__device__ __forceinline__ bool attached(const unsigned* __restrict__ abits, int v)
{
    return (abits[v >> 5] >> (v & 31)) & 1u;
}

__device__ __forceinline__ unsigned valid_bits(int64_t word, int n)
{
    const int64_t lo = word * 32;
    return lo + 32 <= n ? 0xffffffffu : (lo >= n ? 0u : (1u << (unsigned)(n - lo)) - 1u);
}

// Rebuild init: C's component (rep == s) keeps pi (layer 0), every other
// vertex is unattached (layer -1).  Writes the round-1 bitmaps (a1 = layer
// 0, a0 = empty) and counts both sets into the lanes (got, left).
__global__ __launch_bounds__(kWG) void k_conn_init(int n, const int* __restrict__ rep,
                                                   const unsigned char* __restrict__ onc, int s,
                                                   int* __restrict__ layer,
                                                   unsigned char* __restrict__ onC,
                                                   unsigned* __restrict__ a1,
                                                   unsigned* __restrict__ a0, Ctl* ctl)
{
    const int64_t words = ((int64_t)n + 31) / 32;
    const int64_t span = (int64_t)gridDim.x * kWG;
    const int lane = threadIdx.x & 63;
    unsigned long long ncomp = 0, nleft = 0;
    // 64 consecutive vertices per wave, two words per ballot
    for (int64_t vb = ((int64_t)blockIdx.x * kWG + threadIdx.x) & ~(int64_t)63; vb < (int64_t)n;
         vb += span) {
        const int64_t v = vb + lane;
        bool comp = false;
        if (v < n) {
            comp = rep[v] == s;
            if (layer) layer[v] = comp ? 0 : -1;
            if (onC) onC[v] = (unsigned char)(comp && onc && onc[v]);
        }
        const unsigned long long b = __ballot(comp);
        const unsigned long long live = __ballot(v < n);
        const int64_t wd = (vb >> 5) + (lane >> 5);
        if ((lane & 31) == 0 && wd < words) {
            a1[wd] = (unsigned)(b >> (lane & 32));
            a0[wd] = 0u;
        }
        if (lane == 0) {
            ncomp += (unsigned long long)__popcll(b);
            nleft += (unsigned long long)__popcll(live & ~b);
        }
    }
    ncomp = block_sum_u64(ncomp);
    nleft = block_sum_u64(nleft);
    if (threadIdx.x == 0) {
        if (ncomp) atomicAdd(&my_lane(ctl).got, (unsigned)ncomp);
        if (nleft) atomicAdd(&my_lane(ctl).left, (unsigned)nleft);
    }
}

// LDS of the mark step: the frontier of a workgroup's words is processed
// in batches of kBatch vertices whose in-edges are spread over all its
// threads (the rows are short, so spreading keeps the loads coalesced).
constexpr int kBatch = 1024;
constexpr int kExpand = 4;   // in-edges per thread in flight: 2 * kExpand

struct MarkLds {
    int todo[kBatch];
    int beg[kBatch];
    unsigned off[kBatch];
    unsigned wsum[kWG / 64];
};

// Exclusive rank of each thread's count c over the workgroup; *total = sum.
// All threads call it.
__device__ __forceinline__ unsigned block_rank(unsigned c, unsigned* wsum, unsigned* total)
{
    const unsigned incl = wave_incl_scan(c);
    if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = incl;
    __syncthreads();
    unsigned wbase = 0, t = 0;
    for (int w = 0; w < kWG / 64; ++w) {
        if (w < (int)(threadIdx.x >> 6)) wbase += wsum[w];
        t += wsum[w];
    }
    __syncthreads();   // wsum may be reused
    *total = t;
    return wbase + incl - c;
}

// Exclusive prefix sum of a[0, cnt) in LDS (cnt <= kBatch); returns the
// total.  All threads call it.
__device__ __forceinline__ unsigned block_excl_scan(unsigned* a, unsigned cnt, unsigned* wsum)
{
    constexpr int kRun = kBatch / kWG;
    const unsigned r0 = threadIdx.x * kRun;
    unsigned run = 0;
    for (int j = 0; j < kRun; ++j)
        if (r0 + j < cnt) run += a[r0 + j];
    unsigned total = 0;
    const unsigned ex = block_rank(run, wsum, &total);
    unsigned acc = ex;
    for (int j = 0; j < kRun; ++j) {
        if (r0 + j < cnt) {
            const unsigned d = a[r0 + j];
            a[r0 + j] = acc;
            acc += d;
        }
    }
    __syncthreads();
    return total;
}

// Last i in [0, cnt) with off[i] <= t (off non-decreasing, off[0] = 0).
__device__ __forceinline__ unsigned owner_of(const unsigned* off, unsigned cnt, unsigned t)
{
    unsigned lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const unsigned mid = (lo + hi + 1) >> 1;
        if (off[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Writes this thread's items (set bits of mask, item = base_id + bit) whose
// workgroup rank lies in [b0, b0 + kBatch) to todo[rank - b0].
__device__ __forceinline__ void emit_batch(unsigned long long mask, int64_t base_id, unsigned rank,
                                           unsigned b0, int* todo)
{
    const unsigned c = (unsigned)__popcll(mask);
    if (c == 0 || rank + c <= b0 || rank >= b0 + kBatch) return;
    unsigned r = rank;
    while (mask && r < b0 + kBatch) {
        const int b = __ffsll((long long)mask) - 1;
        mask &= mask - 1;
        if (r >= b0) todo[r - b0] = (int)(base_id + b);
        ++r;
    }
}

// beg[i], off[i] = first position and length of the row of todo[i] (i < cnt),
// four rows per thread in flight.
__device__ __forceinline__ void gather_rows(const int* __restrict__ ptr, const int* todo,
                                            unsigned cnt, int* beg, unsigned* off)
{
    constexpr int R = 4;
    for (unsigned i0 = threadIdx.x; i0 < cnt; i0 += R * kWG) {
        int a[R], b[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const unsigned i = i0 + j * kWG;
            const int u = i < cnt ? todo[i] : -1;
            a[j] = u >= 0 ? ptr[u] : 0;
            b[j] = u >= 0 ? ptr[u + 1] : 0;
        }
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const unsigned i = i0 + j * kWG;
            if (i < cnt) {
                beg[i] = a[j];
                off[i] = (unsigned)(b[j] - a[j]);
            }
        }
    }
}

// Per-wave LDS of the round kernels.
struct WaveLds {
    unsigned pre[kWaves][64];   // exclusive rank of each word's first candidate
    unsigned msk[kWaves][64];   // candidates of each word
    unsigned nb[kWaves][64];    // vertices attached in the round, per word
};

// LDS of a round kernel that claims and then marks (used one after the other).
union RoundLds {
    WaveLds wave;
    MarkLds mark;
};

// LDS written by some lanes of a wave and read by others.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Position of the k-th (from 0) set bit of m; k < popcount(m).
__device__ __forceinline__ int select_bit(unsigned m, unsigned k)
{
    int pos = 0;
    unsigned c = __popc(m & 0xffffu);
    if (k >= c) { k -= c; m >>= 16; pos += 16; }
    c = __popc(m & 0xffu);
    if (k >= c) { k -= c; m >>= 8; pos += 8; }
    c = __popc(m & 0xfu);
    if (k >= c) { k -= c; m >>= 4; pos += 4; }
    c = __popc(m & 0x3u);
    if (k >= c) { k -= c; m >>= 2; pos += 2; }
    if (k >= (m & 1u)) pos += 1;
    return pos;
}

// Publishes this lane's candidate mask; returns the wave's candidate count.
__device__ __forceinline__ unsigned wave_rank(unsigned mask, unsigned* pre, unsigned* msk)
{
    const int lane = threadIdx.x & 63;
    const unsigned c = __popc(mask);
    const unsigned incl = wave_incl_scan(c);
    pre[lane] = incl - c;
    msk[lane] = mask;
    wave_lds_sync();
    return __shfl(incl, 63);
}

// Word (0..63, within the wave's words) and bit of the candidate of rank r.
__device__ __forceinline__ void wave_candidate(const unsigned* pre, const unsigned* msk, unsigned r,
                                               int* word, int* bit)
{
    int lo = 0, hi = 63;   // the last word whose first rank is <= r holds r
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    *word = lo;
    *bit = select_bit(msk[lo], r - pre[lo]);
}

// Every candidate of the wave (v0: first vertex of the wave's words)
// attaches with its lowest out-edge whose head is in acur, if it has one
// (pi, layer = k, bit in nb).  Returns the lane's attachments; out-edges
// examined are added to *scanned.
__device__ __forceinline__ unsigned wave_attach(int k, int64_t v0, unsigned mask,
                                                const int* __restrict__ row_ptr,
                                                const int* __restrict__ col,
                                                const unsigned* __restrict__ acur,
                                                int* __restrict__ pi, int* __restrict__ layer,
                                                unsigned* pre, unsigned* msk, unsigned* nb,
                                                unsigned long long* scanned)
{
    const int lane = threadIdx.x & 63;
    nb[lane] = 0;
    const unsigned total = wave_rank(mask, pre, msk);
    unsigned got = 0;
    for (unsigned r0 = 0; r0 < total; r0 += 64) {
        const unsigned r = r0 + lane;
        int word = 0, bit = 0, u = -1, b = 0, end = 0;
        if (r < total) {
            wave_candidate(pre, msk, r, &word, &bit);
            u = (int)(v0 + 32 * word + bit);
            b = row_ptr[u];
            end = row_ptr[u + 1];
        }
        const bool heavy = end - b > kLaneRow;
        int best = INT32_MAX;
        if (u >= 0 && !heavy) {
            for (int e = b; e < end; e += 4) {
                int h[4];
                unsigned a[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) h[j] = e + j < end ? col[e + j] : -1;
#pragma unroll
                for (int j = 0; j < 4; ++j) a[j] = h[j] >= 0 ? acur[h[j] >> 5] : 0u;
                int hit = -1;
#pragma unroll
                for (int j = 3; j >= 0; --j)
                    if ((a[j] >> (h[j] & 31)) & 1u) hit = j;
                *scanned += (unsigned)(end - e < 4 ? end - e : 4);
                if (hit >= 0) {
                    best = e + hit;
                    break;
                }
            }
        }
        // long rows, one at a time, by the whole wave
        for (unsigned long long hv = __ballot(heavy); hv; hv &= hv - 1) {
            const int src = __ffsll((long long)hv) - 1;
            const int hb = __shfl(b, src), he = __shfl(end, src);
            int found = INT32_MAX;
            for (int e0 = hb; e0 < he; e0 += 64) {
                const int e = e0 + lane;
                const unsigned long long bal = __ballot(e < he && attached(acur, col[e]));
                if (lane == src) *scanned += (unsigned)(he - e0 < 64 ? he - e0 : 64);
                if (bal) {
                    found = e0 + __ffsll((long long)bal) - 1;
                    break;
                }
            }
            if (lane == src) best = found;
        }
        if (best != INT32_MAX) {
            pi[u] = best;
            if (layer) layer[u] = k;
            atomicOr(&nb[word], 1u << bit);
            ++got;
        }
    }
    wave_lds_sync();
    return got;
}

// Spans of the round kernels: span i covers bitmap words [i * kWG,
// (i + 1) * kWG).  A workgroup strides over the spans (all of them, or only
// those listed in `spans`, *nspans of them).
template <typename F>
__device__ __forceinline__ void for_each_span(const int* __restrict__ spans, const unsigned* nspans,
                                              int64_t nall, F&& f)
{
    const int64_t cnt = spans ? (int64_t)*nspans : nall;
    for (int64_t i = blockIdx.x; i < cnt; i += gridDim.x) f(spans ? (int64_t)spans[i] : i);
}

// The 32 mark bytes of word w as a bit mask, cleared on the way (marks are
// 0 or 1).
__device__ __forceinline__ unsigned take_marks(unsigned char* __restrict__ marks, int64_t w, int n)
{
    const int64_t v0 = w * 32;
    unsigned mask = 0;
    if (v0 + 32 <= n) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const uint4 t = *(const uint4*)(marks + v0 + 16 * q);
            if (t.x | t.y | t.z | t.w) *(uint4*)(marks + v0 + 16 * q) = make_uint4(0, 0, 0, 0);
            const unsigned wd[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
            for (int i = 0; i < 4; ++i)   // four 0/1 bytes -> four bits
                mask |= (((wd[i] & 0x01010101u) * 0x01020408u) >> 24) << (16 * q + 4 * i);
        }
    } else {
        for (int q = 0; q < 32 && v0 + q < n; ++q) {
            if (marks[v0 + q]) {
                mask |= 1u << q;
                marks[v0 + q] = 0;
            }
        }
    }
    return mask;
}

// Pull round k: the unattached vertices (~acur) scan their out-edges; anext
// becomes acur plus this round's attachments.  With stale (marks left by a
// push round before it for this round), their bytes are cleared.  Returns (in
// thread 0) the workgroup's attachment count.
__device__ __forceinline__ unsigned long long pull_body(
    int k, int n, const int* __restrict__ row_ptr, const int* __restrict__ col,
    const unsigned* __restrict__ acur, unsigned* __restrict__ anext, int* __restrict__ layer,
    int* __restrict__ pi, unsigned long long* ledges, const int* __restrict__ spans,
    const unsigned* nspans, unsigned char* __restrict__ stale, WaveLds& L)
{
    const int64_t words = ((int64_t)n + 31) / 32;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    unsigned got = 0;
    unsigned long long scanned = 0;
    for_each_span(spans, nspans, (words + kWG - 1) / kWG, [&](int64_t span) {
        const int64_t w = span * kWG + threadIdx.x;
        const unsigned a = w < words ? acur[w] : 0u;
        const unsigned mask = w < words ? ~a & valid_bits(w, n) : 0u;
        if (stale && w < words) (void)take_marks(stale, w, n);
        got += wave_attach(k, (w - lane) * 32, mask, row_ptr, col, acur, pi, layer, L.pre[wave],
                           L.msk[wave], L.nb[wave], &scanned);
        if (w < words) anext[w] = a | L.nb[wave][lane];
    });
    const unsigned long long g = block_sum_u64(got);
    scanned = block_sum_u64(scanned);
    if (threadIdx.x == 0 && ledges && scanned) atomicAdd(my_copy(ledges), scanned);
    return g;
}

// Marks the tails of the in-edges of the workgroup's listed vertices (mask:
// this thread's word w0) in marks: marks[u] = 1, a plain byte store
// (idempotent).  The vertices go through LDS in batches of kBatch and their
// in-edges are spread over the workgroup.  Returns the in-edges visited
// (the same in every thread).  All threads call it; it ends with a barrier.
__device__ __forceinline__ unsigned mark_in_edges(unsigned mask, int64_t w0,
                                                  const int* __restrict__ rin_ptr,
                                                  const int* __restrict__ rin,
                                                  unsigned char* __restrict__ marks, MarkLds& L)
{
    unsigned total = 0, visited = 0;
    const unsigned rank = block_rank((unsigned)__popc(mask), L.wsum, &total);
    for (unsigned b0 = 0; b0 < total; b0 += kBatch) {
        emit_batch(mask, w0 * 32, rank, b0, L.todo);
        __syncthreads();
        const unsigned cnt = total - b0 < kBatch ? total - b0 : kBatch;
        gather_rows(rin_ptr, L.todo, cnt, L.beg, L.off);
        __syncthreads();
        const unsigned tot = block_excl_scan(L.off, cnt, L.wsum);
        constexpr int U = 2 * kExpand;
        for (unsigned t0 = threadIdx.x; t0 < tot; t0 += U * kWG) {
            int x[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const unsigned t = t0 + j * kWG;
                const unsigned i = t < tot ? owner_of(L.off, cnt, t) : 0;
                x[j] = t < tot ? L.beg[i] + (int)(t - L.off[i]) : -1;
            }
#pragma unroll
            for (int j = 0; j < U; ++j) x[j] = x[j] >= 0 ? rin[x[j]] : -1;
#pragma unroll
            for (int j = 0; j < U; ++j)
                if (x[j] >= 0) marks[x[j]] = 1;
        }
        visited += tot;
        __syncthreads();
    }
    return visited;
}

// Push round k, mark: the frontier (acur & ~anext) marks the tails of its
// in-edges.  Attached tails are dropped by the claim, which reads its words
// of acur anyway.  Used for a push round whose marks the previous round did
// not leave (the first one, or one after a pull round).
__device__ __forceinline__ void mark_body(int n, const int* __restrict__ rin_ptr,
                                          const int* __restrict__ rin,
                                          const unsigned* __restrict__ acur,
                                          const unsigned* __restrict__ anext,
                                          unsigned char* __restrict__ marks,
                                          unsigned long long* pedges, const int* __restrict__ spans,
                                          const unsigned* nspans, MarkLds& L)
{
    const int64_t words = ((int64_t)n + 31) / 32;
    unsigned long long scanned = 0;
    for_each_span(spans, nspans, (words + kWG - 1) / kWG, [&](int64_t span) {
        const int64_t w0 = span * kWG + threadIdx.x;
        const unsigned f = w0 < words ? acur[w0] & ~anext[w0] : 0u;
        scanned += mark_in_edges(f, w0, rin_ptr, rin, marks, L);
    });
    if (pedges && threadIdx.x == 0 && scanned) atomicAdd(my_copy(pedges), scanned);
}

// Push round k, claim: each word takes its mark bytes (clearing them); the
// marked vertices not attached yet find their lowest out-edge into the
// attached set.  One exists: the edge that marked the vertex.  The vertex
// attaches with it (pi, layer = k); anext gets acur plus the attachments
// (whole words).  With marks_next, the workgroup then marks the in-edge
// tails of its attachments, the next round's frontier, in marks_next (the
// next round's mark array; this round's is marks).  Returns (in thread 0)
// the workgroup's attachment count.
__device__ __forceinline__ unsigned long long claim_body(
    int k, int n, const int* __restrict__ row_ptr, const int* __restrict__ col,
    const unsigned* __restrict__ acur, unsigned* __restrict__ anext,
    unsigned char* __restrict__ marks, int* __restrict__ pi, int* __restrict__ layer,
    unsigned long long* cedges, const int* __restrict__ spans, const unsigned* nspans,
    const int* __restrict__ rin_ptr, const int* __restrict__ rin,
    unsigned char* __restrict__ marks_next, unsigned long long* pedges, RoundLds& L)
{
    const int64_t words = ((int64_t)n + 31) / 32;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    unsigned got = 0;
    unsigned long long scanned = 0, marked = 0;
    for_each_span(spans, nspans, (words + kWG - 1) / kWG, [&](int64_t span) {
        const int64_t w = span * kWG + threadIdx.x;
        const unsigned a = w < words ? acur[w] : 0u;
        // marked tails that are already attached drop out
        const unsigned mask = w < words ? take_marks(marks, w, n) & ~a : 0u;
        got += wave_attach(k, (w - lane) * 32, mask, row_ptr, col, acur, pi, layer,
                           L.wave.pre[wave], L.wave.msk[wave], L.wave.nb[wave], &scanned);
        const unsigned x = L.wave.nb[wave][lane];
        if (w < words) anext[w] = a | x;
        if (marks_next) {
            __syncthreads();   // the LDS turns into the mark step's
            marked += mark_in_edges(x, w, rin_ptr, rin, marks_next, L.mark);
        }
    });
    const unsigned long long g = block_sum_u64(got);
    scanned = block_sum_u64(scanned);
    if (threadIdx.x == 0) {
        if (cedges && scanned) atomicAdd(my_copy(cedges), scanned);
        if (pedges && marked) atomicAdd(my_copy(pedges), marked);
    }
    return g;
}

// Host-driven rounds: one kernel per step.
__global__ __launch_bounds__(kWG) void k_conn_pull(int k, int n, const int* __restrict__ row_ptr,
                                                   const int* __restrict__ col,
                                                   const unsigned* __restrict__ acur,
                                                   unsigned* __restrict__ anext,
                                                   int* __restrict__ layer, int* __restrict__ pi,
                                                   Ctl* ctl, unsigned long long* ledges,
                                                   const int* __restrict__ spans,
                                                   const unsigned* nspans,
                                                   unsigned char* __restrict__ stale)
{
    __shared__ WaveLds L;
    const unsigned long long g =
        pull_body(k, n, row_ptr, col, acur, anext, layer, pi, ledges, spans, nspans, stale, L);
    if (threadIdx.x == 0 && g) atomicAdd(&my_lane(ctl).got, (unsigned)g);
}

__global__ __launch_bounds__(kWG) void k_conn_mark(int n, const int* __restrict__ rin_ptr,
                                                   const int* __restrict__ rin,
                                                   const unsigned* __restrict__ acur,
                                                   const unsigned* __restrict__ anext,
                                                   unsigned char* __restrict__ marks,
                                                   unsigned long long* pedges,
                                                   const int* __restrict__ spans,
                                                   const unsigned* nspans)
{
    __shared__ MarkLds L;
    mark_body(n, rin_ptr, rin, acur, anext, marks, pedges, spans, nspans, L);
}

__global__ __launch_bounds__(kWG) void k_conn_claim(int k, int n, const int* __restrict__ row_ptr,
                                                    const int* __restrict__ col,
                                                    const unsigned* __restrict__ acur,
                                                    unsigned* __restrict__ anext,
                                                    unsigned char* __restrict__ marks,
                                                    int* __restrict__ pi, int* __restrict__ layer,
                                                    Ctl* ctl, unsigned long long* cedges,
                                                    const int* __restrict__ spans,
                                                    const unsigned* nspans,
                                                    const int* __restrict__ rin_ptr,
                                                    const int* __restrict__ rin,
                                                    unsigned char* __restrict__ marks_next,
                                                    unsigned long long* pedges)
{
    __shared__ RoundLds L;
    const unsigned long long g = claim_body(k, n, row_ptr, col, acur, anext, marks, pi, layer,
                                            cedges, spans, nspans, rin_ptr, rin, marks_next,
                                            pedges, L);
    if (threadIdx.x == 0 && g) atomicAdd(&my_lane(ctl).got, (unsigned)g);
}

// Device-driven rebuild rounds.  The control block holds the rounds run
// (rk), the direction of the next one (rmode: 1 push, 2 pull, 0 the rebuild
// is over) and its counts; round k's kernels run only while rk + 1 == k and
// rmode names them.  The last workgroup of a round's final kernel books the
// round (round_close).

// Direction of the next round: policy 0 pushes while many vertices are left
// and the frontier is small against them, 1 always pulls, 2 always pushes.
__device__ __forceinline__ unsigned round_mode(unsigned left, unsigned front, int policy,
                                               unsigned push_min)
{
    if (left == 0) return 0;
    if (policy == 1) return 2;
    if (policy == 2) return front > 0 ? 1 : 2;
    return left >= push_min && 2ull * front < left ? 1 : 2;
}

// Called by thread 0 of every workgroup of round k's final kernel with the
// workgroup's attachment count g.  The last workgroup to arrive books the
// round's attachments and picks round k + 1's direction (a round that
// attached nobody while vertices were left ends the rebuild with rerr set);
// marked_next: the round left round k + 1's marks.
__device__ __forceinline__ void round_close(Ctl* c, int k, unsigned long long g, int policy,
                                            unsigned push_min, bool marked_next)
{
    unsigned long long tot;
    if (!last_arrival(c, arrival_word(g, 0), &tot)) return;
    const unsigned got = (unsigned)tot;
    c->rk = (unsigned)k;
    if (marked_next) c->rmarks = (unsigned)k + 1;
    if (got == 0) {
        c->rerr = 1;
        c->rmode = 0;
        return;
    }
    const unsigned left = c->rleft - got;
    c->rleft = left;
    c->rfront = got;
    c->rmode = round_mode(left, got, policy, push_min);
}

__device__ __forceinline__ bool round_is(const Ctl* c, int k, unsigned mode)
{
    return c->rk + 1 == (unsigned)k && c->rmode == mode;
}

// Round k's first kernel: the marks of a push round (unless round k-1 left
// them), or a whole pull round (clearing marks round k-1 left).  marks is
// round k's mark array (marks[k & 1] of the pair).  Not launched when the
// host expects pushes with their marks left (single, below).
__global__ __launch_bounds__(kWG) void k_round_mark_pull(
    int k, int n, const int* __restrict__ row_ptr, const int* __restrict__ col,
    const int* __restrict__ rin_ptr, const int* __restrict__ rin, const unsigned* __restrict__ acur,
    unsigned* __restrict__ anext, unsigned char* __restrict__ marks, int* __restrict__ pi,
    int* __restrict__ layer, Ctl* ctl, unsigned long long* pedges, int policy, unsigned push_min)
{
    __shared__ RoundLds L;
    const bool left_marks = ctl->rmarks == (unsigned)k;
    if (round_is(ctl, k, 1u)) {
        if (!left_marks)
            mark_body(n, rin_ptr, rin, acur, anext, marks, pedges, nullptr, nullptr, L.mark);
    } else if (round_is(ctl, k, 2u)) {
        const unsigned long long g =
            pull_body(k, n, row_ptr, col, acur, anext, layer, pi, nullptr, nullptr, nullptr,
                      left_marks ? marks : nullptr, L.wave);
        if (threadIdx.x == 0) round_close(ctl, k, g, policy, push_min, false);
    }
}

// Round k's second kernel: the claims of a push round, and the marks of
// round k + 1 in marks_next.  single: k_round_mark_pull was not launched
// for round k (the host expected a push with its marks left by round k - 1);
// this kernel then runs a pull round itself, and a push round that finds no
// marks left (a pull came first) as a pull round too, which attaches the
// same vertices by the same edges.
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_round_claim(
    int k, int n, const int* __restrict__ row_ptr, const int* __restrict__ col,
    const int* __restrict__ rin_ptr, const int* __restrict__ rin, const unsigned* __restrict__ acur,
    unsigned* __restrict__ anext, unsigned char* __restrict__ marks,
    unsigned char* __restrict__ marks_next, int* __restrict__ pi, int* __restrict__ layer, Ctl* ctl,
    unsigned long long* pedges, int policy, unsigned push_min, int single)
{
    const bool push = round_is(ctl, k, 1u);
    if (!push && !(single && round_is(ctl, k, 2u))) return;
    __shared__ RoundLds L;
    const bool left_marks = ctl->rmarks == (unsigned)k;
    if (push && (!single || left_marks)) {
        const unsigned long long g = claim_body(k, n, row_ptr, col, acur, anext, marks, pi, layer,
                                                nullptr, nullptr, nullptr, rin_ptr, rin,
                                                marks_next, pedges, L);
        if (threadIdx.x == 0) round_close(ctl, k, g, policy, push_min, true);
    } else {
        const unsigned long long g =
            pull_body(k, n, row_ptr, col, acur, anext, layer, pi, nullptr, nullptr, nullptr,
                      left_marks ? marks : nullptr, L.wave);
        if (threadIdx.x == 0) round_close(ctl, k, g, policy, push_min, false);
    }
}

// ---------------------------------------------------------------------------
// reverse CSR (the tail of every in-edge), built once per solve when the
// rebuild needs push rounds
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_rev_count(int n, const int* __restrict__ row_ptr,
                                                   const int* __restrict__ col,
                                                   unsigned* __restrict__ deg)
{
    for (int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x; e < row_ptr[n];
         e += (int64_t)gridDim.x * kWG)
        atomicAdd(&deg[col[e]], 1u);
}

__global__ __launch_bounds__(kWG) void k_rev_fill(int n, const int* __restrict__ row_ptr,
                                                  const int* __restrict__ col,
                                                  unsigned* __restrict__ cursor,
                                                  int* __restrict__ rin)
{
    constexpr int G = 8;
    const int lane = threadIdx.x & (G - 1);
    const int64_t ngroups = (int64_t)gridDim.x * (kWG / G);
    for (int64_t u = ((int64_t)blockIdx.x * kWG + threadIdx.x) / G; u < n; u += ngroups) {
        for (int e = row_ptr[u] + lane, end = row_ptr[u + 1]; e < end; e += G) {
            const unsigned pos = atomicAdd(&cursor[col[e]], 1u);
            rin[pos] = (int)u;
        }
    }
}

// Partitioned build (no global atomics): edges are binned by head bucket
// (2^bits heads, bits = 12..14) in LDS, scattered bucket by bucket as
// (head offset in the bucket: 16 bits, tail: 32 bits) in two arrays, and one
// workgroup per bucket then counts its edges per head and places them.  When the bucket's in-edges fit in LDS they are
// placed there and written out in order (scattered 4-byte stores over a
// bucket's region in HBM cost several times their size in write traffic).
// The order of a vertex's in-edges is arbitrary; the rounds only test
// membership.
constexpr int kRevMinBits = 12;
constexpr int kRevMaxBits = 14;
constexpr int kRevMaxBuckets = 8192;
constexpr int kPlaceWG = 1024;
constexpr int kPlaceUnroll = 16;

// Adds one to cnt[key] for every lane with key >= 0 and returns the lane's
// old count.  Locality in a graph sends many of a wave's edges into one head
// bucket, and such adds serialise in the LDS: for up to kClaimRounds keys,
// the lanes that share the first remaining lane's key take one atomic
// together; the rest add one each.
constexpr int kClaimRounds = 1;

__device__ __forceinline__ unsigned lds_claim(unsigned* cnt, int key)
{
    const unsigned lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    bool open = key >= 0;
    unsigned pos = 0;
#pragma unroll
    for (int r = 0; r < kClaimRounds; ++r) {
        const unsigned long long live = __ballot(open);
        if (!live) break;
        const int leader = __ffsll((long long)live) - 1;
        const int k = __builtin_amdgcn_readlane(key, leader);
        const bool grp = open && key == k;
        const unsigned long long mask = __ballot(grp);
        unsigned base = 0;
        if ((int)lane == leader) base = atomicAdd(&cnt[k], (unsigned)__popcll(mask));
        base = (unsigned)__builtin_amdgcn_readlane((int)base, leader);
        if (grp) {
            pos = base + (unsigned)__popcll(mask & below);
            open = false;
        }
    }
    if (open) pos = atomicAdd(&cnt[key], 1u);
    return pos;
}

__global__ __launch_bounds__(kWG) void k_rev_hist(int64_t m, const int* __restrict__ col,
                                                  int64_t chunk, int nblk, int B, int bits,
                                                  unsigned* __restrict__ hist)
{
    extern __shared__ unsigned h[];   // B counters
    for (int i = threadIdx.x; i < B; i += kWG) h[i] = 0;
    __syncthreads();
    const int64_t e0 = (int64_t)blockIdx.x * chunk;
    const int64_t e1 = e0 + chunk < m ? e0 + chunk : m;
    constexpr int U = 8;   // independent loads in flight per thread
    for (int64_t e = e0 + threadIdx.x; e < e1; e += U * kWG) {
        int v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) v[j] = e + j * kWG < e1 ? col[e + j * kWG] : -1;
#pragma unroll
        for (int j = 0; j < U; ++j) (void)lds_claim(h, v[j] >= 0 ? v[j] >> bits : -1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < B; i += kWG) hist[(int64_t)i * nblk + blockIdx.x] = h[i];
}

// last u in [0, n) with row_ptr[u] <= e
__device__ __forceinline__ int source_of(const int* __restrict__ row_ptr, int n, int64_t e)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_ptr[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kWG) void k_rev_scatter(int n, const int* __restrict__ row_ptr,
                                                     const int* __restrict__ col, int64_t m,
                                                     int64_t chunk, int nblk, int B, int bits,
                                                     const unsigned* __restrict__ hoff,
                                                     unsigned short* __restrict__ hlo,
                                                     int* __restrict__ tails)
{
    extern __shared__ unsigned cur[];   // B cursors
    __shared__ int su[2];
    const int64_t e0 = (int64_t)blockIdx.x * chunk;
    const int64_t e1 = e0 + chunk < m ? e0 + chunk : m;
    for (int i = threadIdx.x; i < B; i += kWG) cur[i] = hoff[(int64_t)i * nblk + blockIdx.x];
    if (threadIdx.x == 0) su[0] = source_of(row_ptr, n, e0);
    if (threadIdx.x == 64) su[1] = source_of(row_ptr, n, e1 - 1);
    __syncthreads();
    const int hmask = (1 << bits) - 1;
    // G lanes per source, U sources per group in flight
    constexpr int G = 8, U = 4;
    const int lane = threadIdx.x & (G - 1);
    constexpr int kGroups = kWG / G;
    for (int ub = su[0] + threadIdx.x / G; ub <= su[1]; ub += U * kGroups) {
        int lo[U], hi[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int u = ub + j * kGroups;
            lo[j] = hi[j] = 0;
            if (u <= su[1]) {
                const int a = row_ptr[u], b = row_ptr[u + 1];
                lo[j] = a > e0 ? a : (int)e0;
                hi[j] = b < e1 ? b : (int)e1;
            }
        }
        int v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) v[j] = lo[j] + lane < hi[j] ? col[lo[j] + lane] : -1;
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int u = ub + j * kGroups;
            const unsigned pos = lds_claim(cur, v[j] >= 0 ? v[j] >> bits : -1);
            if (v[j] >= 0) {
                hlo[pos] = (unsigned short)(v[j] & hmask);
                tails[pos] = u;
            }
            for (int e = lo[j] + lane + G; e < hi[j]; e += G) {   // out-degree above G
                const int x = col[e];
                const unsigned pos = atomicAdd(&cur[x >> bits], 1u);
                hlo[pos] = (unsigned short)(x & hmask);
                tails[pos] = u;
            }
        }
    }
}

// One workgroup per bucket.  Dynamic LDS: 2^bits head counters, then `cap`
// staged entries (cap = 0: the bucket is placed straight into rin).
__global__ __launch_bounds__(kPlaceWG) void k_rev_place(int n, int64_t m, int B, int nblk,
                                                        int bits, int64_t cap,
                                                        const unsigned* __restrict__ hoff,
                                                        const unsigned short* __restrict__ hlo,
                                                        const int* __restrict__ tails,
                                                        int* __restrict__ rin_ptr,
                                                        int* __restrict__ rin)
{
    extern __shared__ unsigned lds[];
    __shared__ unsigned wsum[kPlaceWG / 64];
    const int H = 1 << bits;
    unsigned* cnt = lds;
    int* stage = (int*)(lds + H);
    const int bkt = blockIdx.x;
    const int64_t lo = (int64_t)bkt << bits;
    const int64_t hi = lo + H < n ? lo + H : n;
    const int64_t start = hoff[(int64_t)bkt * nblk];
    const int64_t end = bkt + 1 < B ? (int64_t)hoff[(int64_t)(bkt + 1) * nblk] : m;
    for (int i = threadIdx.x; i < H; i += kPlaceWG) cnt[i] = 0;
    __syncthreads();
    // one workgroup per CU (the LDS): many loads in flight per thread
    constexpr int U = kPlaceUnroll;
    for (int64_t p = start + threadIdx.x; p < end; p += U * kPlaceWG) {
        int h[U];
#pragma unroll
        for (int j = 0; j < U; ++j) h[j] = p + j * kPlaceWG < end ? (int)hlo[p + j * kPlaceWG] : -1;
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (h[j] >= 0) atomicAdd(&cnt[h[j]], 1u);
    }
    __syncthreads();
    // exclusive scan of cnt: each thread owns a run of H / kPlaceWG heads
    const int run = H / kPlaceWG;
    const int r0 = threadIdx.x * run;
    unsigned sum = 0;
    for (int j = 0; j < run; ++j) sum += cnt[r0 + j];
    const unsigned incl = wave_incl_scan(sum);
    if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = incl;
    __syncthreads();
    unsigned acc = incl - sum;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) acc += wsum[w];
    for (int j = 0; j < run; ++j) {
        const unsigned d = cnt[r0 + j];
        cnt[r0 + j] = acc;
        acc += d;
    }
    __syncthreads();
    for (int64_t v = lo + threadIdx.x; v < hi; v += kPlaceWG) rin_ptr[v] = (int)(start + cnt[v - lo]);
    if (bkt == B - 1 && threadIdx.x == 0) rin_ptr[n] = (int)m;
    const bool staged = end - start <= cap;   // uniform
    int* out = staged ? stage : rin + start;
    for (int64_t p = start + threadIdx.x; p < end; p += U * kPlaceWG) {
        int h[U], t[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const bool in = p + j * kPlaceWG < end;
            h[j] = in ? (int)hlo[p + j * kPlaceWG] : -1;
            t[j] = in ? tails[p + j * kPlaceWG] : 0;
        }
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (h[j] >= 0) out[atomicAdd(&cnt[h[j]], 1u)] = t[j];
    }
    if (staged) {
        __syncthreads();
        const int len = (int)(end - start);
        for (int i = threadIdx.x; i < len; i += kPlaceWG) rin[start + i] = stage[i];
    }
}

RevPlan rev_plan(int64_t n, int64_t m)
{
    RevPlan p;
    int bits = kRevMinBits;
    while (bits < kRevMaxBits && ((n + (1 << bits) - 1) >> bits) > kRevMaxBuckets) ++bits;
    // OCM_REV_BUCKET_BITS raises the bucket size (up to 2^kRevMaxBits heads),
    // so that small graphs reach the placements of large ones
    if (const char* env = getenv("OCM_REV_BUCKET_BITS")) {
        const int b = atoi(env);
        if (b > bits && b <= kRevMaxBits) bits = b;
    }
    p.bits = bits;
    p.buckets = (n + (1 << bits) - 1) >> bits;
    // edges per histogram / scatter block: at least 4096, and at most 1024
    // blocks (four per CU).  Longer chunks give longer per-bucket runs in the
    // scatter's writes, and a build on a side stream leaves CUs to the solve
    // it overlaps; 512 or fewer blocks no longer hide the loads.
    int64_t chunk = 4096;
    while ((m + chunk - 1) / chunk > 1024) chunk <<= 1;
    p.chunk = chunk;
    p.nblk = (m + chunk - 1) / chunk;
    p.hist_len = p.buckets * p.nblk;
    p.partition = p.buckets <= kRevMaxBuckets && m < (int64_t(1) << 31);
    return p;
}

size_t rev_scratch_bytes(int64_t n, int64_t m)
{
    const RevPlan p = rev_plan(n, m);
    if (!p.partition) return 0;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    return al(4 * (size_t)m) + al(2 * (size_t)m) + 2 * al(4 * (size_t)p.hist_len) +
           al(4 * ((size_t)p.hist_len / 2048 + 2));
}

// Exclusive prefix sum of len unsigned values (three launches: per-block
// scans, a single-block scan of the block totals, and the offsets added).
constexpr int kScanItems = 8;
constexpr int kScanBlock = kWG * kScanItems;

__global__ __launch_bounds__(kWG) void k_scan_a(int64_t len, const unsigned* __restrict__ in,
                                                unsigned* __restrict__ out,
                                                unsigned* __restrict__ tot)
{
    __shared__ unsigned wt[kWG / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    unsigned v[kScanItems];
    unsigned sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const unsigned t = base + i < len ? in[base + i] : 0u;
        v[i] = sum;
        sum += t;
    }
    const unsigned incl = wave_incl_scan(sum);
    if ((threadIdx.x & 63) == 63) wt[threadIdx.x >> 6] = incl;
    __syncthreads();
    unsigned wbase = 0;
    for (int wv = 0; wv < (int)(threadIdx.x >> 6); ++wv) wbase += wt[wv];
    const unsigned excl = wbase + incl - sum;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < len) out[base + i] = v[i] + excl;
    if (threadIdx.x == kWG - 1) tot[blockIdx.x] = wbase + incl;
}

// One workgroup; kScanTotals consecutive totals per thread, so that up to
// 1024 * kScanTotals block totals take a single pass.
constexpr int kScanTotals = 4;

__global__ __launch_bounds__(1024) void k_scan_b(unsigned nb, unsigned* __restrict__ tot)
{
    __shared__ unsigned wt[16];
    __shared__ unsigned carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (unsigned b0 = 0; b0 < nb; b0 += 1024 * kScanTotals) {
        const unsigned i0 = b0 + threadIdx.x * kScanTotals;
        unsigned v[kScanTotals], sum = 0;
#pragma unroll
        for (int j = 0; j < kScanTotals; ++j) {
            const unsigned x = i0 + j < nb ? tot[i0 + j] : 0u;
            v[j] = sum;
            sum += x;
        }
        const unsigned incl = wave_incl_scan(sum);
        if ((threadIdx.x & 63) == 63) wt[threadIdx.x >> 6] = incl;
        __syncthreads();
        unsigned wbase = 0;
        for (int wv = 0; wv < (int)(threadIdx.x >> 6); ++wv) wbase += wt[wv];
        const unsigned excl = carry + wbase + incl - sum;
#pragma unroll
        for (int j = 0; j < kScanTotals; ++j)
            if (i0 + j < nb) tot[i0 + j] = excl + v[j];
        __syncthreads();
        if (threadIdx.x == 1023) carry = excl + sum;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kWG) void k_scan_c(int64_t len, unsigned* __restrict__ out,
                                                const unsigned* __restrict__ tot)
{
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kWG)
        out[i] += tot[i / kScanBlock];
}

__global__ __launch_bounds__(kWG) void k_copy_u32(int64_t len, const unsigned* __restrict__ in,
                                                  unsigned* __restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kWG)
        out[i] = in[i];
}

__global__ __launch_bounds__(kWG) void k_fill_u32(int64_t len, unsigned* __restrict__ p,
                                                  unsigned v)
{
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kWG)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// values: pointer jumping toward the source over the policy tree cut at s.
// Entry: D = sum of (L*w - W) over the first H edges of v's path, J = the
// vertex reached.  A vertex is finished once J == s.
// ---------------------------------------------------------------------------
template <typename WT>
__global__ __launch_bounds__(kWG) void k_val_init(int n, const int* __restrict__ col,
                                                  const int* __restrict__ pi,
                                                  const WT* __restrict__ w, int neg, int s,
                                                  long long W, long long L,
                                                  int* __restrict__ succ, int have_succ,
                                                  Jmp* __restrict__ Q, Ctl* ctl,
                                                  const unsigned* gate, long long* __restrict__ Dhi,
                                                  const int* __restrict__ tm)
{
    if (gate && *gate == 0u) return;   // the value phase is skipped (uniform)
    unsigned long long act = 0;
    constexpr int U = 4;   // independent vertices in flight per thread
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t vb = (int64_t)blockIdx.x * kWG + threadIdx.x; vb < n; vb += U * stride) {
        int e[U], t[U];
        long long wv[U], tv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t v = vb + u * stride;
            e[u] = v < n ? pi[v] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t v = vb + u * stride;
            t[u] = 0;
            wv[u] = 0;
            tv[u] = 1;
            if (v < n) {
                t[u] = have_succ ? succ[v] : col[e[u]];
                wv[u] = wval(w, e[u], neg);
                if (tm) tv[u] = tm[e[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t v = vb + u * stride;
            if (v >= n) continue;
            if (!have_succ) succ[v] = t[u];
            Jmp q;
            if (v == s) {
                q.D = 0;
                q.J = s;
                q.H = 0;
            } else {
                q.D = L * wv[u] - W * tv[u];
                q.J = t[u];
                q.H = 1;
                act += t[u] != s;
            }
            Q[v] = q;
            if (Dhi) Dhi[v] = q.D < 0 ? -1ll : 0ll;   // int128 entries: sign-extended
        }
    }
    act = block_sum_u64(act);
    if (threadIdx.x == 0 && act) atomicAdd(&my_lane(ctl).active, (unsigned)act);
}

// int128 entries: the sum's low word stays in the Jmp entry, its high word in
// a parallel array (hin / hout); no overflow is possible (|sum| < n * 2^62).
__device__ __forceinline__ void jmp_combine_wide(Jmp& q, long long& qh, const Jmp& r, long long rh)
{
    const unsigned __int128 a = ((unsigned __int128)(unsigned long long)qh << 64) |
                                (unsigned long long)q.D;
    const unsigned __int128 b = ((unsigned __int128)(unsigned long long)rh << 64) |
                                (unsigned long long)r.D;
    const unsigned __int128 d = a + b;
    q.D = (long long)(unsigned long long)d;
    qh = (long long)(unsigned long long)(d >> 64);
    q.J = r.J;
    q.H = q.H + r.H;
}

// One jump round over all entries; returns (in thread 0) the vertices still
// unfinished after it.
template <bool WIDE = false>
__device__ __forceinline__ unsigned long long val_round_body(int n, int s,
                                                             const Jmp* __restrict__ Qin,
                                                             Jmp* __restrict__ Qout,
                                                             const long long* __restrict__ hin = nullptr,
                                                             long long* __restrict__ hout = nullptr)
{
    unsigned long long act = 0;
    // grid-stride with kJumpUnroll independent entries in flight per thread
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t v0 = (int64_t)blockIdx.x * kWG + threadIdx.x; v0 < n;
         v0 += kJumpUnroll * stride) {
        Jmp q[kJumpUnroll], r[kJumpUnroll];
        long long qh[kJumpUnroll], rh[kJumpUnroll];
#pragma unroll
        for (int u = 0; u < kJumpUnroll; ++u) {
            const int64_t v = v0 + u * stride;
            qh[u] = rh[u] = 0;
            if (v < n) {
                q[u] = Qin[v];
                if (WIDE) qh[u] = hin[v];
            } else {
                q[u].J = s;
            }
        }
#pragma unroll
        for (int u = 0; u < kJumpUnroll; ++u)
            if (q[u].J != s) {
                r[u] = Qin[q[u].J];
                if (WIDE) rh[u] = hin[q[u].J];
            }
#pragma unroll
        for (int u = 0; u < kJumpUnroll; ++u) {
            const int64_t v = v0 + u * stride;
            if (v >= n) continue;
            if (q[u].J != s) {
                if (WIDE) jmp_combine_wide(q[u], qh[u], r[u], rh[u]);
                else q[u] = jmp_combine(q[u], r[u]);
                act += q[u].J != s;
            }
            Qout[v] = q[u];
            if (WIDE) hout[v] = qh[u];
        }
    }
    return block_sum_u64(act);
}

template <bool WIDE>
__global__ __launch_bounds__(kWG) void k_val_round(int n, int s, const Jmp* __restrict__ Qin,
                                                   Jmp* __restrict__ Qout, unsigned* active,
                                                   const long long* __restrict__ hin,
                                                   long long* __restrict__ hout)
{
    const unsigned long long act = val_round_body<WIDE>(n, s, Qin, Qout, hin, hout);
    if (threadIdx.x == 0 && act) atomicAdd(my_copy(active), (unsigned)act);
}

// Device-driven round r: the last workgroup ends the rounds once no vertex
// is unfinished, or with jstall once a round finished none.
template <bool WIDE>
__global__ __launch_bounds__(kWG) void k_val_round_dev(int n, int s, int r,
                                                       const Jmp* __restrict__ Qin,
                                                       Jmp* __restrict__ Qout, Ctl* ctl,
                                                       const long long* __restrict__ hin,
                                                       long long* __restrict__ hout)
{
    if (!jump_round_is(ctl, r)) return;
    const unsigned long long act = val_round_body<WIDE>(n, s, Qin, Qout, hin, hout);
    if (threadIdx.x != 0) return;
    unsigned long long tot;
    if (!last_arrival(ctl, arrival_word(act, 0), &tot)) return;
    const unsigned now = (unsigned)tot;
    ctl->jk = (unsigned)r;
    if (now == 0) {
        ctl->jmode = 0;
    } else if (now == ctl->jlast) {
        ctl->jstall = 1;
        ctl->jmode = 0;
    } else {
        ctl->jlast = now;
    }
}

// WIDE: V gets the low words, Vhi the high words (hin: the entries' high
// words); int128 values cannot overflow.
// V32 (int64 values only, nullable): the int32 copy, with wide32 flagged
// when some value does not fit it.
template <bool WIDE>
__device__ __forceinline__ void val_final_body(int n, const Jmp* __restrict__ Q,
                                               long long* __restrict__ V, int* __restrict__ hop,
                                               Ctl* ctl, const long long* __restrict__ hin,
                                               long long* __restrict__ Vhi,
                                               int* __restrict__ V32)
{
    const int v = blockIdx.x * kWG + threadIdx.x;
    unsigned bad = 0, big = 0;
    if (v < n) {
        const Jmp q = Q[v];
        V[v] = q.D;
        if (hop) hop[v] = (int)(q.H & ~kHopOverflow);
        if (WIDE) Vhi[v] = hin[v];
        else if ((q.H & kHopOverflow) || q.D > kValLimit || q.D < -kValLimit) bad = 1;
        if (!WIDE && V32) {
            V32[v] = (int)q.D;
            big = q.D > INT32_MAX || q.D < INT32_MIN;
        }
    }
    if (!WIDE && __ballot(bad != 0) && (threadIdx.x & 63) == 0)
        atomicOr(&my_lane(ctl).overflow, 1u);
    if (!WIDE && __ballot(big != 0) && (threadIdx.x & 63) == 0)
        atomicOr(&my_lane(ctl).wide32, 1u);
}

template <bool WIDE>
__global__ __launch_bounds__(kWG) void k_val_final(int n, const Jmp* __restrict__ Q,
                                                   long long* __restrict__ V,
                                                   int* __restrict__ hop, Ctl* ctl,
                                                   const long long* __restrict__ hin,
                                                   long long* __restrict__ Vhi,
                                                   int* __restrict__ V32)
{
    val_final_body<WIDE>(n, Q, V, hop, ctl, hin, Vhi, V32);
}

// Device-driven: runs once every vertex finished (not after a stall), on the
// entries of the last round run.
template <bool WIDE>
__global__ __launch_bounds__(kWG) void k_val_final_dev(int n, const Jmp* __restrict__ Q0,
                                                       const Jmp* __restrict__ Q1,
                                                       long long* __restrict__ V,
                                                       int* __restrict__ hop, Ctl* ctl,
                                                       const long long* __restrict__ h0,
                                                       const long long* __restrict__ h1,
                                                       long long* __restrict__ Vhi,
                                                       int* __restrict__ V32)
{
    if (ctl->jmode != 0 || ctl->jstall || !ctl->jgate) return;
    const bool odd = (ctl->jk & 1) != 0;
    val_final_body<WIDE>(n, odd ? Q1 : Q0, V, hop, ctl, odd ? h1 : h0, Vhi, V32);
}

// Cycle C listed from the source: vertex c_j (j steps after s) is H = L - j
// hops before s on the tree cut at s.
__global__ __launch_bounds__(kWG) void k_cycle_list(int n, int s, long long L,
                                                    const unsigned char* __restrict__ onC,
                                                    const int* __restrict__ pi,
                                                    const int* __restrict__ hop,
                                                    int* __restrict__ out)
{
    const int v = blockIdx.x * kWG + threadIdx.x;
    if (v >= n || !onC[v]) return;
    const long long j = v == s ? 0 : L - (long long)hop[v];
    if (j >= 0 && j < L) out[j] = pi[v];
}

// Short-walk test: for every tight non-policy edge x->y whose head is not
// nearer the source (hop[y] >= hop[x]), follow y's policy path for at most
// kShortWalk steps; meeting x closes a cycle of tight edges other than C.

template <int G, typename WT, int VM = 0>
__global__ __launch_bounds__(kWG) void k_tie_short_walk(SweepArgs a, const WT* __restrict__ w,
                                                        const int* __restrict__ succ)
{
    using KT = typename ValT<VM>::type;
    constexpr int VPB = kWG / G;
    const int lane = threadIdx.x & (G - 1);
    const int64_t per = ((int64_t)a.n + gridDim.x - 1) / gridDim.x;
    const int64_t v0 = (int64_t)blockIdx.x * per;
    const int64_t v1 = v0 + per < a.n ? v0 + per : a.n;
    unsigned long long found = 0;
    for (int64_t vb = v0; vb < v1; vb += VPB) {
        const int64_t v = vb + threadIdx.x / G;
        if (v >= v1) continue;
        const int beg = a.row_ptr[v], end = a.row_ptr[v + 1];
        if (a.giant.ngiant > 0 && end - beg > kGiantRow) continue;   // k_giant_short_walk
        const KT own = load_val<VM>(a.V, a.Vhi, a.V32, v);
        const int cur = a.pi[v];
        for (int e = beg + lane; e < end; e += G) {
            if (e == cur) continue;
            const int y = a.col[e];
            if (a.hop[y] < a.hop[v]) continue;
            const long long te = a.t ? a.t[e] : 1;
            if (load_val<VM>(a.V, a.Vhi, a.V32, y) + (KT)(a.L * wval(w, e, a.neg) - a.W * te) != own)
                continue;
            int x = y;
            for (int st = 0; st < kShortWalk && x != (int)v; ++st) x = succ[x];
            found += x == (int)v;
        }
    }
    found = block_sum_u64(found);
    if (threadIdx.x == 0 && found) atomicAdd(&my_lane(a.ctl).certain, found);
}

// The same test on the giant rows, one workgroup per chunk.
template <typename WT, int VM>
__global__ __launch_bounds__(kWG) void k_giant_short_walk(SweepArgs a, const WT* __restrict__ w,
                                                          const int* __restrict__ succ)
{
    using KT = typename ValT<VM>::type;
    const GiantTab& g = a.giant;
    unsigned long long found = 0;
    for (int c = blockIdx.x; c < g.nchunks; c += gridDim.x) {
        const int v = g.cv[c];
        const KT own = load_val<VM>(a.V, a.Vhi, a.V32, v);
        const int cur = a.pi[v], hv = a.hop[v];
        for (int e = g.cs[c] + (int)threadIdx.x; e < g.ce[c]; e += kWG) {
            if (e == cur) continue;
            const int y = a.col[e];
            if (a.hop[y] < hv) continue;
            const long long te = a.t ? a.t[e] : 1;
            if (load_val<VM>(a.V, a.Vhi, a.V32, y) + (KT)(a.L * wval(w, e, a.neg) - a.W * te) != own)
                continue;
            int x = y;
            for (int st = 0; st < kShortWalk && x != v; ++st) x = succ[x];
            found += x == v;
        }
    }
    found = block_sum_u64(found);
    if (threadIdx.x == 0 && found) atomicAdd(&my_lane(a.ctl).certain, found);
}

// ---------------------------------------------------------------------------
// exact uniqueness of the critical cycle (used when no quick test decided).
// The tight subgraph T is the policy graph plus the tight non-policy edges
// X = {x_i -> y_i}.  Contract C to one node c*; the policy is then an in-tree
// rooted at c*.  Every vertex that is an endpoint of an X edge is "special";
// each special vertex z gets P(z) = the first special vertex (or c*) strictly
// after z on its policy path.  T has a second critical cycle iff the graph on
// special vertices + c* with edges z -> P(z) and x_i -> y_i has a cycle,
// which the host checks on that small graph.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_tie_mark(unsigned k, const int* __restrict__ xs,
                                                  const int* __restrict__ ys,
                                                  unsigned char* __restrict__ sp)
{
    for (unsigned i = blockIdx.x * kWG + threadIdx.x; i < k; i += gridDim.x * kWG) {
        sp[xs[i]] = 1;
        sp[ys[i]] = 1;
    }
}

// Lists the special vertices and gives each its index in the list.
__global__ __launch_bounds__(kWG) void k_tie_compact(int n, unsigned char* __restrict__ sp,
                                                     int* __restrict__ spid,
                                                     int* __restrict__ slist, unsigned* scnt)
{
    __shared__ int buf[kWG * 16];
    __shared__ unsigned nb, base;
    if (threadIdx.x == 0) nb = 0;
    __syncthreads();
    BlockList bl{buf, &nb};
    const int64_t v0 = (int64_t)blockIdx.x * (kWG * 16) + (int64_t)threadIdx.x * 16;
    for (int q = 0; q < 16; ++q) {
        const int64_t v = v0 + q;
        const bool hit = v < n && sp[v] != 0;
        blist_push(bl, hit, (int)v);
    }
    __syncthreads();
    const unsigned cnt = nb;
    if (threadIdx.x == 0) base = cnt ? atomicAdd(scnt, cnt) : 0u;
    __syncthreads();
    for (unsigned j = threadIdx.x; j < cnt; j += kWG) {
        slist[base + j] = buf[j];
        spid[buf[j]] = (int)(base + j);
    }
}

// P(z) for every special z: -2 if z is on C (z is c* itself), -1 if the walk
// reaches C first, else the index of the special vertex reached.  Every
// policy path reaches C; the walk is still capped at n steps (-3).
__global__ __launch_bounds__(kWG) void k_tie_walk(int n, unsigned ns, const int* __restrict__ slist,
                                                  const int* __restrict__ succ,
                                                  const unsigned char* __restrict__ sp,
                                                  const unsigned char* __restrict__ onC,
                                                  const int* __restrict__ spid,
                                                  int* __restrict__ P)
{
    for (unsigned i = blockIdx.x * kWG + threadIdx.x; i < ns; i += gridDim.x * kWG) {
        const int z = slist[i];
        if (onC[z]) {
            P[i] = -2;
            continue;
        }
        int x = succ[z];
        int64_t steps = 0;
        while (!sp[x] && !onC[x] && steps < n) {
            x = succ[x];
            ++steps;
        }
        P[i] = onC[x] ? -1 : (sp[x] ? spid[x] : -3);
    }
}

// Endpoints of the X edges as special-vertex indices (-1 = on C).
__global__ __launch_bounds__(kWG) void k_tie_ends(unsigned k, int* __restrict__ xs,
                                                  int* __restrict__ ys,
                                                  const unsigned char* __restrict__ onC,
                                                  const int* __restrict__ spid,
                                                  unsigned char* __restrict__ sp)
{
    for (unsigned i = blockIdx.x * kWG + threadIdx.x; i < k; i += gridDim.x * kWG) {
        const int x = xs[i], y = ys[i];
        xs[i] = onC[x] ? -1 : spid[x];
        ys[i] = onC[y] ? -1 : spid[y];
    }
    (void)sp;
}

__global__ __launch_bounds__(kWG) void k_clear_u8(int64_t len, unsigned char* __restrict__ p)
{
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kWG)
        p[i] = 0;
}

// ---------------------------------------------------------------------------
// adjoint: d(optimum)/d(w_e) = 1/|C| on the edges of C, 0 elsewhere
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_fill_f64(int64_t len, double* __restrict__ p, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kWG)
        p[i] = v;
}

__global__ __launch_bounds__(kWG) void k_adjoint_scatter(int64_t len, const int* __restrict__ cyc,
                                                         const double* __restrict__ g,
                                                         double* __restrict__ grad)
{
    const double v = *g / (double)len;   // one IEEE division: correctly rounded
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kWG)
        grad[cyc[i]] = v;
}

// float64 weights -> int64; flags non-integral values and |w| >= 2^53.
__global__ __launch_bounds__(kWG) void k_w_from_f64(int64_t m, const double* __restrict__ w,
                                                    long long* __restrict__ out, unsigned* bad)
{
    unsigned b = 0;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kWG) {
        const double x = w[i];
        const bool ok = x == __builtin_trunc(x) && __builtin_fabs(x) < 9007199254740992.0;
        out[i] = ok ? (long long)x : 0;
        b |= ok ? 0u : 1u;
    }
    if (__ballot(b != 0) && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
}

// A given policy must pick one of each vertex's own out-edges.
__global__ __launch_bounds__(kWG) void k_check_policy(int n, const int* __restrict__ row_ptr,
                                                      const int* __restrict__ pi, unsigned* bad)
{
    unsigned b = 0;
    for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kWG) {
        const int e = pi[v];
        b |= (e < row_ptr[v] || e >= row_ptr[v + 1]) ? 1u : 0u;
    }
    if (__ballot(b != 0) && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
}

// Does every int128 value (lo, hi) fit int64, i.e. is hi the sign of lo?
__global__ __launch_bounds__(kWG) void k_fits64(int n, const long long* __restrict__ lo,
                                                const long long* __restrict__ hi, unsigned* bad)
{
    unsigned b = 0;
    for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kWG)
        b |= hi[v] != (lo[v] < 0 ? -1ll : 0ll) ? 1u : 0u;
    if (__ballot(b != 0) && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
}

// Thread l < kLanes clears lane l; thread 0 also the header fields.
__global__ void k_ctl_clear(Ctl* ctl, unsigned what)
{
    const int t = threadIdx.x;
    if (what & kClrAll) {
        unsigned* p = (unsigned*)ctl;
        for (unsigned i = t; i < sizeof(Ctl) / sizeof(unsigned); i += blockDim.x) p[i] = 0;
        return;
    }
    if (t < kLanes) {
        CtlLane& ln = ctl->lane[t];
        if (what & kClrChanged) {
            ln.changed = 0;
            ln.cbroken = 0;
            ln.tight = 0;
            ln.certain = 0;
            ln.nondec = 0;
            ln.bad = 0;
            ln.ncrit = 0;
        }
        if (what & kClrCount) {
            ln.active = 0;
            ln.active2 = 0;
            ln.got = 0;
            ln.left = 0;
            ln.overflow = 0;
            ln.wide32 = 0;
        }
        if (what & kClrActive2) ln.active2 = 0;
    }
    if (t == 0) {
        if (what & kClrGiant) ctl->ngiant = 0;
        if (what & kClrChanged) {
            ctl->xcnt = 0;
            ctl->scnt = 0;
        }
        if (what & kClrCount) {
            ctl->ncyc = 0;
            ctl->rmode = ctl->rleft = ctl->rfront = ctl->rerr = ctl->rk = 0;
        }
    }
}

__global__ void k_zero2(unsigned* a, unsigned* b)
{
    if (threadIdx.x == 0) {
        *a = 0;
        *b = 0;
    }
}

__global__ void k_ctl_set(Ctl* ctl, int s, long long W, long long L)
{
    if (threadIdx.x != 0) return;
    ctl->s = s;
    ctl->W = W;
    ctl->L = L;
}

__global__ __launch_bounds__(kWG) void k_fill_u8(unsigned char* p, int64_t n, unsigned char v)
{
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Items per block for list-producing kernels: spread over about 2048 blocks,
// at most kListItems so the LDS buffer cannot overflow.
static unsigned list_per_block(int64_t items)
{
    int64_t per = (items + 2047) / 2048;
    per = (per + kWG - 1) / kWG * kWG;
    if (per < kWG) per = kWG;
    if (per > kListItems) per = kListItems;
    return (unsigned)per;
}

template <typename WT>
static void launch_sweep_t(const SweepArgs& a, const void* w, int G, bool first, bool tie,
                           unsigned grid, hipStream_t st)
{
    const WT* ww = (const WT*)w;
#define OCM_SWEEP_CASE(GG)                                                                        \
    case GG:                                                                                      \
        if (first)                                                                                \
            k_sweep_u<GG, WT, true, OCM_SWEEP_UNROLL><<<grid, kWG, 0, st>>>(a, ww);               \
        else k_sweep_u<GG, WT, false, OCM_SWEEP_UNROLL><<<grid, kWG, 0, st>>>(a, ww);             \
        break;
    switch (G) {
        OCM_SWEEP_CASE(1)
        OCM_SWEEP_CASE(2)
        OCM_SWEEP_CASE(4)
        OCM_SWEEP_CASE(8)
        OCM_SWEEP_CASE(16)
        OCM_SWEEP_CASE(32)
        OCM_SWEEP_CASE(64)
        default: break;
    }
#undef OCM_SWEEP_CASE
}

void launch_validate(int n, int m, const int* row_ptr, const int* col, const void* w, int wtype,
                     int check_csr, Ctl* ctl, hipStream_t st)
{
    const int64_t total = n > m ? n : m;
    const unsigned grid = stride_grid(total);
    if (wtype == kWI64)
        k_validate<long long><<<grid, kWG, 0, st>>>(n, m, row_ptr, col, (const long long*)w,
                                                    check_csr, ctl);
    else
        k_validate<int><<<grid, kWG, 0, st>>>(n, m, row_ptr, col, (const int*)w, check_csr, ctl);
}

// Sweeps after the first with int128 values, an int32 copy of V or edge
// times: always over vertex tiles.
// The giant rows' part of a tile sweep (after the tile kernel, on the same
// stream): chunk bests, then one merge per row (not for the tie scan).
template <typename WT, int VM, bool RATIO>
static void launch_giant(const SweepArgs& a, const WT* ww, bool first, bool tie, bool fused,
                         hipStream_t st)
{
    if (a.giant.ngiant <= 0) return;
    const unsigned grid = a.giant.nchunks < 2048 ? (unsigned)a.giant.nchunks : 2048u;
    const unsigned mgrid = blocks_for(a.giant.ngiant);
    if (first) {
        k_giant_part<WT, 0, false, 0, false><<<grid, kWG, 0, st>>>(a, ww);
        k_giant_merge<0, true><<<mgrid, kWG, 0, st>>>(a);
    } else if (tie) {
        k_giant_part<WT, 2, true, VM, RATIO><<<grid, kWG, 0, st>>>(a, ww);
    } else {
        if (fused) k_giant_part<WT, 1, true, VM, RATIO><<<grid, kWG, 0, st>>>(a, ww);
        else k_giant_part<WT, 1, false, VM, RATIO><<<grid, kWG, 0, st>>>(a, ww);
        k_giant_merge<VM, false><<<mgrid, kWG, 0, st>>>(a);
    }
}

template <typename WT, int VM, bool RATIO>
static void launch_sweep_tiles(const SweepArgs& a, const WT* ww, bool tie, bool fused,
                               hipStream_t st)
{
    const unsigned tiles = blocks_for(a.n);
    if (tie) k_tiescan_tile<WT, false, VM, RATIO><<<tiles, kWG, 0, st>>>(a, ww);
    else if (fused) k_tiescan_tile<WT, true, VM, RATIO><<<tiles, kWG, 0, st>>>(a, ww);
    else k_sweep_tile<WT, false, VM, RATIO><<<tiles, kWG, 0, st>>>(a, ww);
    launch_giant<WT, VM, RATIO>(a, ww, false, tie, fused, st);
}

template <typename WT, int VM>
static void launch_sweep_vm(const SweepArgs& a, const WT* ww, bool tie, bool fused, hipStream_t st)
{
    if (a.t) launch_sweep_tiles<WT, VM, true>(a, ww, tie, fused, st);
    else launch_sweep_tiles<WT, VM, false>(a, ww, tie, fused, st);
}

template <typename WT>
static void launch_sweep_general(const SweepArgs& a, const WT* ww, bool tie, bool fused,
                                 hipStream_t st)
{
    if (a.Vhi) launch_sweep_vm<WT, 1>(a, ww, tie, fused, st);
    else if (a.V32) launch_sweep_vm<WT, 2>(a, ww, tie, fused, st);
    else launch_sweep_vm<WT, 0>(a, ww, tie, fused, st);
}

void launch_sweep(const SweepArgs& a, const void* w, int wtype, int G, bool first, bool tie,
                  bool count_tight, unsigned grid, hipStream_t st)
{
    if ((a.Vhi || a.t || (a.V32 && (G == 0 || tie))) && !first) {
        const bool fused = !tie && count_tight;
        if (wtype == kWI64) launch_sweep_general(a, (const long long*)w, tie, fused, st);
        else launch_sweep_general(a, (const int*)w, tie, fused, st);
        return;
    }
    if (G == 0) {   // sweep over vertex tiles
        const unsigned tiles = blocks_for(a.n);
        const bool fused = !tie && !first && count_tight;
        if (wtype == kWI64) {
            const long long* ww = (const long long*)w;
            if (tie) k_tiescan_tile<long long, false><<<tiles, kWG, 0, st>>>(a, ww);
            else if (fused) k_tiescan_tile<long long, true><<<tiles, kWG, 0, st>>>(a, ww);
            else if (first) k_sweep_tile<long long, true><<<tiles, kWG, 0, st>>>(a, ww);
            else k_sweep_tile<long long, false><<<tiles, kWG, 0, st>>>(a, ww);
            launch_giant<long long, 0, false>(a, ww, first, tie, fused, st);
        } else {
            const int* ww = (const int*)w;
            if (tie) k_tiescan_tile<int, false><<<tiles, kWG, 0, st>>>(a, ww);
            else if (fused) k_tiescan_tile<int, true><<<tiles, kWG, 0, st>>>(a, ww);
            else if (first) k_sweep_tile<int, true><<<tiles, kWG, 0, st>>>(a, ww);
            else k_sweep_tile<int, false><<<tiles, kWG, 0, st>>>(a, ww);
            launch_giant<int, 0, false>(a, ww, first, tie, fused, st);
        }
        return;
    }
    if (tie) {   // the tie scan always runs over vertex tiles
        const unsigned tiles = blocks_for(a.n);
        if (wtype == kWI64) {
            k_tiescan_tile<long long, false><<<tiles, kWG, 0, st>>>(a, (const long long*)w);
            launch_giant<long long, 0, false>(a, (const long long*)w, false, true, false, st);
        } else {
            k_tiescan_tile<int, false><<<tiles, kWG, 0, st>>>(a, (const int*)w);
            launch_giant<int, 0, false>(a, (const int*)w, false, true, false, st);
        }
        return;
    }
    if (wtype == kWI64) launch_sweep_t<long long>(a, w, G, first, tie, grid, st);
    else launch_sweep_t<int>(a, w, G, first, tie, grid, st);
}

void launch_giant_list(int n, const int* row_ptr, int* triples, unsigned cap, Ctl* ctl,
                       hipStream_t st)
{
    k_giant_list<<<stride_grid(n), kWG, 0, st>>>(n, row_ptr, triples, cap, ctl);
}

void launch_pj_init(int n, const int* col, const int* pi, int* succ, bool have_succ,
                    unsigned long long* P, unsigned char* onc, unsigned char* tag0, unsigned* cnt,
                    hipStream_t st)
{
    k_pj_init<<<blocks_for(n), kWG, 0, st>>>(n, col, pi, succ, have_succ ? 1 : 0, P, onc, tag0,
                                             cnt);
}

void launch_jump_setup(Ctl* ctl, bool values, bool gated, hipStream_t st)
{
    k_jump_setup<<<1, 64, 0, st>>>(ctl, values ? 1 : 0, gated ? 1 : 0);
}

void launch_fast_gate(Ctl* ctl, bool force, hipStream_t st)
{
    k_fast_gate<<<1, 64, 0, st>>>(ctl, force ? 1 : 0);
}

void launch_pj_round_dev(int n, int r, const unsigned long long* Pin, unsigned long long* Pout,
                         const unsigned char* tprev, unsigned char* tcur, Ctl* ctl, hipStream_t st)
{
    k_pj_round_dev<<<stride_grid(n), kWG, 0, st>>>(n, r, Pin, Pout, tprev, tcur, ctl);
}

void launch_pj_final_dev(int n, const unsigned long long* P0, const unsigned long long* P1, int K,
                         int* rep, unsigned char* onc, const Ctl* ctl, hipStream_t st)
{
    k_pj_final_dev<<<blocks_for(n), kWG, 0, st>>>(n, P0, P1, K, rep, onc, ctl);
}

void launch_val_round_dev(int n, int s, int r, const Jmp* Qin, Jmp* Qout, Ctl* ctl,
                          hipStream_t st, const long long* hin, long long* hout)
{
    if (hin)
        k_val_round_dev<true><<<stride_grid(n), kWG, 0, st>>>(n, s, r, Qin, Qout, ctl, hin, hout);
    else
        k_val_round_dev<false><<<stride_grid(n), kWG, 0, st>>>(n, s, r, Qin, Qout, ctl, nullptr,
                                                               nullptr);
}

void launch_val_final_dev(int n, const Jmp* Q0, const Jmp* Q1, long long* V, int* hop, Ctl* ctl,
                          hipStream_t st, const long long* h0, const long long* h1,
                          long long* Vhi, int* V32)
{
    if (Vhi)
        k_val_final_dev<true><<<blocks_for(n), kWG, 0, st>>>(n, Q0, Q1, V, hop, ctl, h0, h1, Vhi,
                                                             nullptr);
    else
        k_val_final_dev<false><<<blocks_for(n), kWG, 0, st>>>(n, Q0, Q1, V, hop, ctl, nullptr,
                                                              nullptr, nullptr, V32);
}

void launch_pj_round(int n, const unsigned long long* Pin, unsigned long long* Pout,
                     hipStream_t st)
{
    k_pj_round<<<blocks_for(n), kWG, 0, st>>>(n, Pin, Pout);
}

void launch_pj_round_tagged(int n, int r, const unsigned long long* Pin, unsigned long long* Pout,
                            const unsigned char* tprev, unsigned char* tcur, unsigned* cnt,
                            hipStream_t st)
{
    k_pj_round_tagged<<<stride_grid(n), kWG, 0, st>>>(n, Pin, Pout, tprev, tcur, (unsigned char)r,
                                                      (unsigned char)(r + 1), cnt + 2 * (r & 1),
                                                      cnt + 2 * ((r + 1) & 1));
}

void launch_pj_final(int n, const unsigned long long* P, int* rep, unsigned char* onc,
                     hipStream_t st)
{
    k_pj_final<<<blocks_for(n), kWG, 0, st>>>(n, P, rep, onc);
}

void launch_cyc_zero(int n, const int* rep, const unsigned char* onc, long long* wsum,
                     unsigned* lcnt, int* cyc_list, Ctl* ctl, hipStream_t st, long long* tsum)
{
    const unsigned per = list_per_block(n);
    const unsigned grid = (unsigned)(((int64_t)n + per - 1) / per);
    k_cyc_zero<<<grid, kWG, 0, st>>>(n, rep, onc, per, wsum, lcnt, cyc_list, ctl, tsum);
}

void launch_cyc_sum(int n, const int* rep, const unsigned char* onc, const int* pi, const void* w,
                    int wtype, int neg, long long* wsum, unsigned* lcnt, hipStream_t st,
                    const int* t, long long* tsum)
{
    if (wtype == kWI64)
        k_cyc_sum<long long><<<blocks_for(n), kWG, 0, st>>>(n, rep, onc, pi, (const long long*)w,
                                                            neg, wsum, lcnt, t, tsum);
    else
        k_cyc_sum<int><<<blocks_for(n), kWG, 0, st>>>(n, rep, onc, pi, (const int*)w, neg, wsum,
                                                      lcnt, t, tsum);
}

void launch_select(const int* cyc_list, const long long* wsum, const unsigned* lcnt, Ctl* ctl,
                   void* scratch, hipStream_t st, const long long* tsum)
{
    Cand* part = (Cand*)scratch;
    k_select_part<<<kSelectParts, kWG, 0, st>>>(cyc_list, wsum, lcnt, tsum, ctl, part);
    k_select_final<<<1, kWG, 0, st>>>(part, kSelectParts, lcnt, ctl);
}

void launch_validate_t(int m, const int* t, Ctl* ctl, hipStream_t st)
{
    k_validate_t<<<stride_grid(m), kWG, 0, st>>>(m, t, ctl);
}

void launch_conn_init(int n, const int* rep, const unsigned char* onc, int s, int* layer,
                      unsigned char* onC, unsigned* a1, unsigned* a0, Ctl* ctl, hipStream_t st)
{
    k_conn_init<<<stride_grid(n), kWG, 0, st>>>(n, rep, onc, s, layer, onC, a1, a0, ctl);
}

// Words per thread of the round kernels: 2 when one word per thread would
// need more than 1024 workgroups.
// One bitmap word (32 vertices) per thread: on the 16.7M-vertex product
// graph two words per thread (half the workgroups) made the push rounds
// 20 % slower, the gathers there being latency-bound.
int round_wpt(int n)
{
    (void)n;
    return 1;
}

int64_t round_spans(int n)
{
    const int64_t words = ((int64_t)n + 31) / 32;
    const int64_t per = (int64_t)kWG * round_wpt(n);
    return (words + per - 1) / per;
}

// one workgroup per span (with a span list the ones past its length leave
// at once)
static unsigned round_grid(int n, const int* spans)
{
    (void)spans;
    return (unsigned)round_spans(n);
}

void launch_conn_pull(int k, int n, const int* row_ptr, const int* col, const unsigned* acur,
                      unsigned* anext, int* layer, int* pi, Ctl* ctl, unsigned long long* ledges,
                      const int* spans, const unsigned* nspans, unsigned char* stale,
                      hipStream_t st)
{
    k_conn_pull<<<round_grid(n, spans), kWG, 0, st>>>(k, n, row_ptr, col, acur, anext, layer, pi,
                                                      ctl, ledges, spans, nspans, stale);
}

void launch_conn_mark(int n, const int* rin_ptr, const int* rin, const unsigned* acur,
                      const unsigned* anext, unsigned char* marks, unsigned long long* pedges,
                      const int* spans, const unsigned* nspans, hipStream_t st)
{
    k_conn_mark<<<round_grid(n, spans), kWG, 0, st>>>(n, rin_ptr, rin, acur, anext, marks,
                                                         pedges, spans, nspans);
}

void launch_conn_claim(int k, int n, const int* row_ptr, const int* col, const unsigned* acur,
                       unsigned* anext, unsigned char* marks, int* pi, int* layer, Ctl* ctl,
                       unsigned long long* cedges, const int* spans, const unsigned* nspans,
                       const int* rin_ptr, const int* rin, unsigned char* marks_next,
                       unsigned long long* pedges, hipStream_t st)
{
    k_conn_claim<<<round_grid(n, spans), kWG, 0, st>>>(k, n, row_ptr, col, acur, anext, marks, pi,
                                                       layer, ctl, cedges, spans, nspans, rin_ptr,
                                                       rin, marks_next, pedges);
}

// Device-driven rebuild rounds (one wave each).
__global__ void k_round_setup(Ctl* c, unsigned left, unsigned front, int policy,
                              unsigned push_min)
{
    if (threadIdx.x < kLanes) c->lane[threadIdx.x].rpack = 0;
    if (threadIdx.x == 0) {
        c->rleft = left;
        c->rfront = front;
        c->rerr = 0;
        c->rk = 0;
        c->rmarks = 0;
        c->rpack = 0;
        c->rmode = round_mode(left, front, policy, push_min);
    }
}

// The same start, from the counts the rebuild init left in the lanes (got:
// C's component, left: unattached), with no host read in between (one wave).
__global__ void k_round_setup_dev(Ctl* c, int policy, unsigned push_min)
{
    const int l = threadIdx.x;
    unsigned long long got = 0, left = 0;
    if (l < kLanes) {
        got = c->lane[l].got;
        left = c->lane[l].left;
        c->lane[l].rpack = 0;
    }
    got = wave_sum_u64(got);
    left = wave_sum_u64(left);
    if (l == 0) {
        c->rleft = (unsigned)left;
        c->rfront = (unsigned)got;
        c->rerr = 0;
        c->rk = 0;
        c->rmarks = 0;
        c->rpack = 0;
        c->rmode = round_mode((unsigned)left, (unsigned)got, policy, push_min);
    }
}

void launch_round_setup_dev(Ctl* ctl, int policy, unsigned push_min, hipStream_t st)
{
    k_round_setup_dev<<<1, 64, 0, st>>>(ctl, policy, push_min);
}

void launch_round_setup(Ctl* ctl, unsigned left, unsigned front, int policy, unsigned push_min,
                        hipStream_t st)
{
    k_round_setup<<<1, 64, 0, st>>>(ctl, left, front, policy, push_min);
}

void launch_round(int k, int n, const int* row_ptr, const int* col, const int* rin_ptr,
                  const int* rin, const unsigned* acur, unsigned* anext, unsigned char* marks,
                  unsigned char* marks_next, int* pi, int* layer, Ctl* ctl,
                  unsigned long long* pedges, int policy, unsigned push_min, bool may_push,
                  bool single, hipStream_t st)
{
    const unsigned grid = (unsigned)round_spans(n);
    const bool one = single && may_push;
    if (!one)
        k_round_mark_pull<<<grid, kWG, 0, st>>>(k, n, row_ptr, col, rin_ptr, rin, acur, anext,
                                                marks, pi, layer, ctl, pedges, policy, push_min);
    if (may_push)
        k_round_claim<<<grid, kWG, 0, st>>>(k, n, row_ptr, col, rin_ptr, rin, acur, anext, marks,
                                            marks_next, pi, layer, ctl, pedges, policy, push_min,
                                            one ? 1 : 0);
}

void launch_exclusive_scan(int64_t len, const unsigned* in, unsigned* out, unsigned* tot,
                           hipStream_t st)
{
    const unsigned nb = (unsigned)((len + kScanBlock - 1) / kScanBlock);
    k_scan_a<<<nb, kWG, 0, st>>>(len, in, out, tot);
    k_scan_b<<<1, 1024, 0, st>>>(nb, tot);
    k_scan_c<<<stride_grid(len), kWG, 0, st>>>(len, out, tot);
}

void launch_rev_build(int n, int m, const int* row_ptr, const int* col, unsigned* deg,
                      unsigned* tot, int* rin_ptr, int* rin, unsigned char* marks, void* scratch,
                      hipStream_t st)
{
    const RevPlan p = rev_plan(n, m);
    // OCM_REV_BUILD=atomic selects the two-pass atomic build (it also serves
    // graphs with too many head buckets); both give the same in-edge sets
    const char* env = getenv("OCM_REV_BUILD");
    const bool atomic_build = env && env[0] == 'a';
    if (p.partition && scratch && !atomic_build) {
        auto al = [](size_t b) { return (b + 255) / 256 * 256; };
        char* sp = (char*)scratch;
        int* tails = (int*)sp;
        auto* hlo = (unsigned short*)(sp + al(4 * (size_t)m));
        unsigned* hist = (unsigned*)((char*)hlo + al(2 * (size_t)m));
        unsigned* hoff = (unsigned*)((char*)hist + al(4 * (size_t)p.hist_len));
        unsigned* htot = (unsigned*)((char*)hoff + al(4 * (size_t)p.hist_len));
        const size_t lds = 4 * (size_t)p.buckets;
        k_rev_hist<<<(unsigned)p.nblk, kWG, lds, st>>>(m, col, p.chunk, (int)p.nblk,
                                                       (int)p.buckets, p.bits, hist);
        launch_exclusive_scan(p.hist_len, hist, hoff, htot, st);
        k_rev_scatter<<<(unsigned)p.nblk, kWG, lds, st>>>(n, row_ptr, col, m, p.chunk,
                                                          (int)p.nblk, (int)p.buckets, p.bits,
                                                          hoff, hlo, tails);
        // the placement's LDS: head counters, then as many staged entries as
        // the device's per-workgroup limit leaves room for
        const size_t counters = (size_t)4 << p.bits;
        int limit = 65536, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            limit = 65536;
        const size_t room = (size_t)limit - 1024;   // static LDS of the kernel
        const int64_t cap = room > counters ? (int64_t)((room - counters) / 4) : 0;
        const size_t place_lds = counters + 4 * (size_t)cap;
        if (place_lds > 65536)
            (void)hipFuncSetAttribute((const void*)k_rev_place,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)place_lds);
        k_rev_place<<<(unsigned)p.buckets, kPlaceWG, place_lds, st>>>(
            n, m, (int)p.buckets, (int)p.nblk, p.bits, cap, hoff, hlo, tails, rin_ptr, rin);
    } else {
        const int64_t len = (int64_t)n + 1;
        k_fill_u32<<<stride_grid(len), kWG, 0, st>>>(len, deg, 0u);
        k_rev_count<<<stride_grid(m), kWG, 0, st>>>(n, row_ptr, col, deg);
        const unsigned nb = (unsigned)((len + kScanBlock - 1) / kScanBlock);
        k_scan_a<<<nb, kWG, 0, st>>>(len, deg, (unsigned*)rin_ptr, tot);
        k_scan_b<<<1, 1024, 0, st>>>(nb, tot);
        k_scan_c<<<stride_grid(len), kWG, 0, st>>>(len, (unsigned*)rin_ptr, tot);
        k_copy_u32<<<stride_grid(n), kWG, 0, st>>>(n, (const unsigned*)rin_ptr, deg);
        k_rev_fill<<<stride_grid(n), kWG, 0, st>>>(n, row_ptr, col, deg, rin);
    }
    const int64_t words = ((int64_t)n + 3) / 4;
    k_fill_u32<<<stride_grid(words), kWG, 0, st>>>(words, (unsigned*)marks, 0u);
}

void launch_val_init(int n, const int* col, const int* pi, const void* w, int wtype, int neg,
                     int s, long long W, long long L, int* succ, bool have_succ, Jmp* Q, Ctl* ctl,
                     const unsigned* gate, hipStream_t st, long long* Dhi, const int* t)
{
    if (wtype == kWI64)
        k_val_init<long long><<<stride_grid(n), kWG, 0, st>>>(n, col, pi, (const long long*)w, neg,
                                                             s, W, L, succ, have_succ ? 1 : 0, Q, ctl,
                                                             gate, Dhi, t);
    else
        k_val_init<int><<<stride_grid(n), kWG, 0, st>>>(n, col, pi, (const int*)w, neg, s, W, L,
                                                       succ, have_succ ? 1 : 0, Q, ctl, gate, Dhi,
                                                       t);
}

void launch_val_round(int n, int s, const Jmp* Qin, Jmp* Qout, unsigned* active, hipStream_t st,
                      const long long* hin, long long* hout)
{
    if (hin)
        k_val_round<true><<<stride_grid(n), kWG, 0, st>>>(n, s, Qin, Qout, active, hin, hout);
    else
        k_val_round<false><<<stride_grid(n), kWG, 0, st>>>(n, s, Qin, Qout, active, nullptr,
                                                           nullptr);
}

void launch_val_final(int n, const Jmp* Q, long long* V, int* hop, Ctl* ctl, hipStream_t st,
                      const long long* hin, long long* Vhi, int* V32)
{
    if (Vhi) k_val_final<true><<<blocks_for(n), kWG, 0, st>>>(n, Q, V, hop, ctl, hin, Vhi, nullptr);
    else
        k_val_final<false><<<blocks_for(n), kWG, 0, st>>>(n, Q, V, hop, ctl, nullptr, nullptr,
                                                          V32);
}

void launch_cycle_list(int n, int s, long long L, const unsigned char* onC, const int* pi,
                       const int* hop, int* out, hipStream_t st)
{
    k_cycle_list<<<blocks_for(n), kWG, 0, st>>>(n, s, L, onC, pi, hop, out);
}

template <typename WT>
static void launch_short_walk_t(const SweepArgs& a, const void* w, int G, const int* succ,
                                unsigned grid, hipStream_t st)
{
    const WT* ww = (const WT*)w;
    if (a.giant.ngiant > 0) {
        const unsigned gg = a.giant.nchunks < 2048 ? (unsigned)a.giant.nchunks : 2048u;
        if (a.Vhi) k_giant_short_walk<WT, 1><<<gg, kWG, 0, st>>>(a, ww, succ);
        else k_giant_short_walk<WT, 0><<<gg, kWG, 0, st>>>(a, ww, succ);
    }
    if (a.Vhi) {   // int128 values: one lane group size (a rare fallback)
        k_tie_short_walk<8, WT, 1><<<grid, kWG, 0, st>>>(a, ww, succ);
        return;
    }
    switch (G) {
        case 1: k_tie_short_walk<1, WT><<<grid, kWG, 0, st>>>(a, ww, succ); break;
        case 2: k_tie_short_walk<2, WT><<<grid, kWG, 0, st>>>(a, ww, succ); break;
        case 4: k_tie_short_walk<4, WT><<<grid, kWG, 0, st>>>(a, ww, succ); break;
        case 8: k_tie_short_walk<8, WT><<<grid, kWG, 0, st>>>(a, ww, succ); break;
        case 16: k_tie_short_walk<16, WT><<<grid, kWG, 0, st>>>(a, ww, succ); break;
        case 32: k_tie_short_walk<32, WT><<<grid, kWG, 0, st>>>(a, ww, succ); break;
        default: k_tie_short_walk<64, WT><<<grid, kWG, 0, st>>>(a, ww, succ); break;
    }
}

void launch_tie_short_walk(const SweepArgs& a, const void* w, int wtype, int G, const int* succ,
                           unsigned grid, hipStream_t st)
{
    if (wtype == kWI64) launch_short_walk_t<long long>(a, w, G, succ, grid, st);
    else launch_short_walk_t<int>(a, w, G, succ, grid, st);
}

void launch_tie_special(int n, unsigned k, int* xs, int* ys, const int* succ,
                        const unsigned char* onC, unsigned char* sp, int* spid, int* slist,
                        unsigned* scnt, hipStream_t st)
{
    const int64_t len = (int64_t)n;
    k_clear_u8<<<stride_grid(len), kWG, 0, st>>>(len, sp);
    k_tie_mark<<<stride_grid(k), kWG, 0, st>>>(k, xs, ys, sp);
    const unsigned grid = (unsigned)((len + kWG * 16 - 1) / (kWG * 16));
    k_tie_compact<<<grid, kWG, 0, st>>>(n, sp, spid, slist, scnt);
    (void)succ;
    (void)onC;
}

void launch_tie_walk(int n, unsigned ns, const int* slist, const int* succ,
                     const unsigned char* sp, const unsigned char* onC, const int* spid, int* P,
                     unsigned k, int* xs, int* ys, hipStream_t st)
{
    if (ns) k_tie_walk<<<stride_grid(ns), kWG, 0, st>>>(n, ns, slist, succ, sp, onC, spid, P);
    if (k) k_tie_ends<<<stride_grid(k), kWG, 0, st>>>(k, xs, ys, onC, spid, nullptr);
    k_clear_u8<<<stride_grid(n), kWG, 0, st>>>(n, (unsigned char*)sp);
}

void launch_adjoint_scatter(int64_t m, const int* cyc, int64_t len, const double* g, double* grad,
                            hipStream_t st)
{
    k_fill_f64<<<stride_grid(m), kWG, 0, st>>>(m, grad, 0.0);
    if (len > 0) k_adjoint_scatter<<<stride_grid(len), kWG, 0, st>>>(len, cyc, g, grad);
}

void launch_w_from_f64(int64_t m, const double* w, long long* out, unsigned* bad, hipStream_t st)
{
    k_w_from_f64<<<stride_grid(m), kWG, 0, st>>>(m, w, out, bad);
}

void launch_fits64(int n, const long long* lo, const long long* hi, unsigned* bad, hipStream_t st)
{
    k_fits64<<<stride_grid(n), kWG, 0, st>>>(n, lo, hi, bad);
}

void launch_check_policy(int n, const int* row_ptr, const int* pi, unsigned* bad, hipStream_t st)
{
    k_check_policy<<<stride_grid(n), kWG, 0, st>>>(n, row_ptr, pi, bad);
}

void launch_ctl_clear(Ctl* ctl, unsigned what, hipStream_t st)
{
    k_ctl_clear<<<1, 64, 0, st>>>(ctl, what);
}

void launch_zero2(unsigned* a, unsigned* b, hipStream_t st)
{
    k_zero2<<<1, 64, 0, st>>>(a, b);
}

void launch_ctl_set(Ctl* ctl, int s, long long W, long long L, hipStream_t st)
{
    k_ctl_set<<<1, 64, 0, st>>>(ctl, s, W, L);
}

void launch_fill_u8(unsigned char* p, int64_t n, unsigned char v, hipStream_t st)
{
    if (n > 0) k_fill_u8<<<blocks_for(n), kWG, 0, st>>>(p, n, v);
}

void launch_fill_u32(unsigned* p, int64_t len, unsigned v, hipStream_t st)
{
    if (len > 0) k_fill_u32<<<stride_grid(len), kWG, 0, st>>>(len, p, v);
}

// ---------------------------------------------------------------------------
// host readback of a small control block
// ---------------------------------------------------------------------------
// A one-wave kernel copies the block into pinned, coherent host memory,
// fences, and then publishes a sequence number that the host spins on; this
// avoids a staged device-to-host copy and a stream synchronisation per read.
constexpr int kPostWords = 64;

__global__ void k_post(const unsigned* __restrict__ src, int words, unsigned* dst,
                       unsigned* seq_slot, unsigned seq)
{
    const int t = threadIdx.x;
    if (t < words) dst[t] = src[t];
    __threadfence_system();
    __syncthreads();
    if (t == 0) {
        __hip_atomic_store(seq_slot, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Folds the lanes of a control block into a snapshot and publishes it like
// k_post.
// lanes 0..kLanes-1 of the wave each hold one copy; fold over them
__device__ __forceinline__ unsigned long long lane_sum(unsigned long long x)
{
    for (int o = kLanes / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kLanes);
    return x;
}
__device__ __forceinline__ unsigned long long lane_max(unsigned long long x)
{
    for (int o = kLanes / 2; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(x, o, kLanes);
        x = y > x ? y : x;
    }
    return x;
}
__device__ __forceinline__ unsigned lane_or(unsigned x)
{
    for (int o = kLanes / 2; o > 0; o >>= 1) x |= __shfl_xor(x, o, kLanes);
    return x;
}

__global__ void k_post_ctl(const Ctl* __restrict__ c, CtlView* dst, unsigned* seq_slot,
                           unsigned seq)
{
    // one wave; thread l < kLanes loads lane l (the others load lane 0 and
    // take no part in the result)
    const int l = threadIdx.x < kLanes ? threadIdx.x : 0;
    const CtlLane& ln = c->lane[l];
    CtlView v;
    v.changed = lane_sum(ln.changed);
    v.tight = lane_sum(ln.tight);
    v.certain = lane_sum(ln.certain);
    v.nondec = lane_sum(ln.nondec);
    v.pedges = lane_sum(ln.pedges);
    v.ledges = lane_sum(ln.ledges);
    v.maxabsw = lane_max(ln.maxabsw);
    v.active = (unsigned)lane_sum(ln.active);
    v.active2 = (unsigned)lane_sum(ln.active2);
    v.got = (unsigned)lane_sum(ln.got);
    v.left = (unsigned)lane_sum(ln.left);
    v.err = lane_or(ln.err);
    v.cbroken = lane_or(ln.cbroken);
    v.overflow = lane_or(ln.overflow);
    v.bad = lane_or(ln.bad);
    v.wide32 = lane_or(ln.wide32);
    v.ncrit = (unsigned)lane_sum(ln.ncrit);
    for (int j = 0; j < 4; ++j) v.pjc[j] = (unsigned)lane_sum(ln.pjc[j]);
    if (threadIdx.x == 0) {
        v.W = c->W;
        v.L = c->L;
        v.s = c->s;
        v.ncyc = c->ncyc;
        v.rmode = c->rmode;
        v.rleft = c->rleft;
        v.rfront = c->rfront;
        v.rerr = c->rerr;
        v.rk = c->rk;
        v.jk = c->jk;
        v.jmode = c->jmode;
        v.jlast = c->jlast;
        v.jstall = c->jstall;
        v.xcnt = c->xcnt;
        v.scnt = c->scnt;
        v.clen = c->clen;
        v.ngiant = c->ngiant;
        *dst = v;
        __threadfence_system();
        __hip_atomic_store(seq_slot, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

namespace {
struct Mailbox {
    unsigned* host = nullptr;   // kPostWords data words, then the sequence word
    unsigned* dev = nullptr;    // the same memory as seen by the device
    unsigned seq = 0;
    bool stream_mode = false;
    bool init = false;
};
thread_local Mailbox tl_mb;

Mailbox& mailbox()
{
    Mailbox& mb = tl_mb;
    if (mb.init) return mb;
    mb.init = true;
    const char* env = getenv("OCM_HOST_SYNC");
    mb.stream_mode = env && env[0] == 's';
    if (mb.stream_mode) return mb;
    void* h = nullptr;
    hipError_t e = hipHostMalloc(&h, 4 * (kPostWords + 16),
                                 hipHostMallocMapped | hipHostMallocCoherent |
                                     hipHostMallocPortable);
    void* d = nullptr;
    if (e == hipSuccess) e = hipHostGetDevicePointer(&d, h, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        mb.stream_mode = true;
        return mb;
    }
    // kept for the life of the process (a few hundred bytes per thread)
    mb.host = (unsigned*)h;
    mb.dev = (unsigned*)d;
    __atomic_store_n(&mb.host[kPostWords], 0u, __ATOMIC_RELEASE);
    return mb;
}

// Spins until the post with sequence number `want` lands.
hipError_t wait_post(const Mailbox& mb, unsigned want, hipStream_t st)
{
    const unsigned* seq = mb.host + kPostWords;
    for (uint64_t i = 1;; ++i) {
        if (__atomic_load_n(seq, __ATOMIC_ACQUIRE) == want) return hipSuccess;
        if ((i & 1023) == 0) {
            // the stream may have failed or finished without the post landing
            const hipError_t e = hipStreamQuery(st);
            if (e == hipSuccess)
                return __atomic_load_n(seq, __ATOMIC_ACQUIRE) == want ? hipSuccess
                                                                      : hipErrorUnknown;
            if (e != hipErrorNotReady) return e;
        }
        __builtin_ia32_pause();
    }
}

}  // namespace

hipError_t host_read(const void* dsrc, void* hdst, size_t bytes, hipStream_t st)
{
    Mailbox& mb = mailbox();
    if (mb.stream_mode || bytes > 4 * kPostWords || (bytes & 3) != 0) {
        hipError_t e = hipMemcpyAsync(hdst, dsrc, bytes, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(st);
    }
    const unsigned want = ++mb.seq;
    k_post<<<1, 64, 0, st>>>((const unsigned*)dsrc, (int)(bytes / 4), mb.dev,
                             mb.dev + kPostWords, want);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = wait_post(mb, want, st);
    if (e != hipSuccess) return e;
    memcpy(hdst, mb.host, bytes);
    return hipSuccess;
}

hipError_t host_read_ctl_copy(const Ctl* ctl, CtlView* out, hipStream_t st)
{
    Ctl h;   // on the caller's stack: this path allocates nothing
    hipError_t e = hipMemcpyAsync(&h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) fold_lanes(h, *out);
    return e;
}

hipError_t host_read_ctl(const Ctl* ctl, CtlView* out, hipStream_t st)
{
    static_assert(sizeof(CtlView) <= 4 * kPostWords && sizeof(CtlView) % 4 == 0,
                  "the snapshot fits the mailbox");
    Mailbox& mb = mailbox();
    if (mb.stream_mode) return host_read_ctl_copy(ctl, out, st);
    const unsigned want = ++mb.seq;
    k_post_ctl<<<1, 64, 0, st>>>(ctl, (CtlView*)mb.dev, mb.dev + kPostWords, want);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = wait_post(mb, want, st);
    if (e != hipSuccess) return e;
    memcpy(out, mb.host, sizeof(CtlView));
    return hipSuccess;
}

}  // namespace ocm
