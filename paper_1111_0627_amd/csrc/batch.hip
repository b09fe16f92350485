// Batched exact optimal cycle mean: many independent graphs solved together.
//
// Section 3.3 runs the computation concurrently on all strongly connected
// components ("regions") of one graph, with a per-region lambda, a
// per-region minimum vote (Alg. 5) and per-region work flags that retire
// finished regions.  Here the regions are the graphs of a disjoint-union CSR:
// graph g owns vertices [vptr[g], vptr[g+1]) and edges [eptr[g], eptr[g+1]).
// Each graph follows exactly the rules of the single-graph solver, so its
// result (value, cycle, iteration count) equals a separate ocm_min call on
// it (Prop. 2.2 gives the optimum of the union as the minimum over graphs).
//
// Work distribution: vertex kernels run over a list of chunks (graph, first
// vertex) covering only the graphs in the phase at hand, so retired graphs
// cost nothing.  The chunk size and the lanes per vertex of the sweep are
// the batch schedule (chosen by the autotuner or given by the caller).
#include "ocm.h"

#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "device_util.h"
#include "kernels.h"

namespace ocm {
namespace b {

constexpr int kMinChunk = 512;   // smallest chunk the workspace is sized for

// per-graph modes
constexpr int kDone = 0;      // converged or failed
constexpr int kActive = 1;    // next: a sweep
constexpr int kFast = 2;      // next: values with the old cycle (fast path)
constexpr int kGeneral = 3;   // next: cycles, select, rebuild, values
constexpr int kTieList = 4;   // after the loop: tie left open by the quick tests

struct GArrays {              // device arrays with one entry per graph
    long long* W;
    long long* L;
    int* s;
    int* iter;
    int* mode;
    int* status;
    int* best;                // vote: rep of the best cycle so far
    unsigned* changed;
    unsigned* cbroken;
    unsigned* vrun;           // values: 1 while the graph is propagating
    // values: some vertex unfinished after the round / some vertex finished
    // in it, in three slots per graph ([4 g + slot]): round r reads slot
    // r % 3 (the previous round's, the init's for r = 0), writes slot
    // (r + 1) % 3 and clears slot (r + 2) % 3 for round r + 1
    unsigned* vact;
    unsigned* vprog;
    unsigned* ovf;
    int* fin;                 // values: ping-pong buffer holding the final entries
    unsigned char* have_c;
    unsigned long long* tight;
    unsigned long long* certain;
    unsigned long long* nondec;
    long long* vptr;          // G+1
    long long* eptr;          // G+1
    unsigned* ccnt;           // chunk counts / offsets scratch
    unsigned* coff;
    unsigned* ctot;
};

struct BCtl {
    unsigned nchunks;
    unsigned nactive, nfast, ngeneral, ndone;
    unsigned vrun_round[32];   // value phase: round r has a graph to advance
    unsigned vlast;            // value phase: slot / buffer parity of the last round's output
    unsigned nspans;           // rebuild: spans holding a rebuilt graph
    unsigned ncyc;
    unsigned overflow;
    unsigned xcnt;             // tie test: tight non-policy edges listed
    unsigned scnt;             // tie test: special vertices
    unsigned rounds_open;      // device-driven rebuild rounds of the iteration left unfinished
    unsigned wide32;           // some value left int32: sweeps gather V, not its int32 copy
    unsigned hop_act[34];      // hop phase: entries short of s after round r - 1 (r = 0: 1)
};

// Value-round entry of the loop: the sum D of (L * w - W) over the policy
// path from v to J, as two 32-bit words so that an entry takes 12 bytes
// (hop counts are not carried: they are needed only after the loop, which
// computes them once).  A sum that leaves int64 becomes kDOverflow, which
// every later sum keeps.
struct VJ {
    unsigned lo, hi;
    int J;
};

constexpr long long kDOverflow = (long long)(1ull << 63);

__device__ __forceinline__ long long vj_d(const VJ& q)
{
    return (long long)(((unsigned long long)q.hi << 32) | q.lo);
}

__device__ __forceinline__ VJ vj_make(long long d, int j)
{
    VJ q;
    q.lo = (unsigned)(unsigned long long)d;
    q.hi = (unsigned)((unsigned long long)d >> 32);
    q.J = j;
    return q;
}

__device__ __forceinline__ bool chunk_range(const int2* __restrict__ chunks, const unsigned* nch,
                                            const long long* __restrict__ vptr, int T, int& g,
                                            int64_t& v0, int64_t& v1)
{
    if (blockIdx.x >= *nch) return false;
    const int2 c = chunks[blockIdx.x];
    g = c.x;
    v0 = c.y;
    const int64_t end = vptr[g + 1];
    v1 = v0 + T < end ? v0 + T : end;
    return true;
}

// Grid-stride over the chunk list: workgroup b takes chunks b, b + grid, ...,
// so a launch needs no more workgroups than there are chunks to do, whatever
// the list's capacity.  f(g, v0, v1) runs once per chunk; its `return` skips
// to the next chunk.
constexpr unsigned kChunkGrid = 2048;

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2: when the grid is a multiple of 8, XCD x takes the x-th eighth of the
// list (consecutive chunks, i.e. the same few graphs), so a graph's gathered
// values stay in one L2 instead of being fetched by all eight.
template <typename F>
__device__ __forceinline__ void for_each_chunk(const int2* __restrict__ chunks, const unsigned* nch,
                                               const long long* __restrict__ vptr, int T, F&& f)
{
    const unsigned nc = *nch;
    unsigned lo = 0, hi = nc, first = blockIdx.x, step = gridDim.x;
    if ((gridDim.x & 7u) == 0u) {
        const unsigned x = blockIdx.x & 7u;
        lo = (unsigned)((unsigned long long)nc * x / 8u);
        hi = (unsigned)((unsigned long long)nc * (x + 1u) / 8u);
        first = lo + (blockIdx.x >> 3);
        step = gridDim.x >> 3;
    }
    for (unsigned ci = first; ci < hi; ci += step) {
        const int2 c = chunks[ci];
        const int g = c.x;
        const int64_t v0 = c.y;
        const int64_t end = vptr[g + 1];
        f(g, v0, v0 + T < end ? v0 + T : end);
    }
}

// ---------------------------------------------------------------------------
// chunk lists
// ---------------------------------------------------------------------------
// halt (nullable): while *halt is non-zero every count is 0 (the list is
// empty and the kernels that take it do nothing).
// Chunk count of graph g for the selection `want`: a mode, -1 = every graph
// not done, -2 = every graph.
__device__ __forceinline__ unsigned chunk_count(int g, const int* __restrict__ mode, int want,
                                                const long long* __restrict__ vptr, int T)
{
    const bool sel = want == -2 ? true : want == -1 ? mode[g] != kDone : mode[g] == want;
    const long long n = vptr[g + 1] - vptr[g];
    return sel ? (unsigned)((n + T - 1) / T) : 0u;
}

// The whole list in one workgroup when the batch is small enough
// (G <= kChunkListOne): each thread takes a run of consecutive graphs, a
// workgroup scan of the runs' chunk counts gives every run its offset, and
// the runs are written in order: the same list as k_chunk_count, a scan and
// k_chunk_fill, in one launch instead of five.
constexpr int kChunkListWG = 1024;
constexpr int kChunkListOne = 16 * kChunkListWG;

__global__ __launch_bounds__(kChunkListWG) void k_chunk_list(int G, const int* __restrict__ mode,
                                                             int want,
                                                             const long long* __restrict__ vptr,
                                                             int T, int2* __restrict__ chunks,
                                                             unsigned* nch, const unsigned* halt)
{
    __shared__ unsigned wsum[kChunkListWG / 64];
    constexpr int kPer = kChunkListOne / kChunkListWG;
    const int per = (G + kChunkListWG - 1) / kChunkListWG;   // <= kPer
    const int g0 = (int)threadIdx.x * per;
    const bool off = halt && *halt != 0u;
    unsigned cnt[kPer];
    unsigned mine = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int g = g0 + i;
        cnt[i] = !off && i < per && g < G ? chunk_count(g, mode, want, vptr, T) : 0u;
        mine += cnt[i];
    }
    const unsigned incl = wave_incl_scan(mine);
    if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = incl;
    __syncthreads();
    unsigned o = incl - mine, total = 0;
    for (int i = 0; i < kChunkListWG / 64; ++i) {
        if (i < (int)(threadIdx.x >> 6)) o += wsum[i];
        total += wsum[i];
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        if (cnt[i] == 0) continue;
        const int g = g0 + i;
        const long long v0 = vptr[g];
        for (unsigned j = 0; j < cnt[i]; ++j) chunks[o + j] = make_int2(g, (int)(v0 + (long long)j * T));
        o += cnt[i];
    }
    if (threadIdx.x == 0) *nch = total;
}

__global__ __launch_bounds__(kWG) void k_chunk_count(int G, const int* __restrict__ mode, int want,
                                                     const long long* __restrict__ vptr, int T,
                                                     unsigned* __restrict__ cnt,
                                                     const unsigned* halt)
{
    const bool off = halt && *halt != 0u;
    for (int g = blockIdx.x * kWG + threadIdx.x; g <= G; g += gridDim.x * kWG) {
        if (g == G || off) {
            cnt[g] = 0;
            continue;
        }
        cnt[g] = chunk_count(g, mode, want, vptr, T);
    }
}

__global__ __launch_bounds__(kWG) void k_chunk_fill(int G, const unsigned* __restrict__ cnt,
                                                    const unsigned* __restrict__ off,
                                                    const long long* __restrict__ vptr, int T,
                                                    int2* __restrict__ chunks, unsigned* nch)
{
    for (int g = blockIdx.x * kWG + threadIdx.x; g < G; g += gridDim.x * kWG) {
        const unsigned o = off[g], c = cnt[g];
        for (unsigned i = 0; i < c; ++i) chunks[o + i] = make_int2(g, (int)(vptr[g] + (long long)i * T));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *nch = off[G];
}

// ---------------------------------------------------------------------------
// validation of the disjoint union: every edge stays inside its graph
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_check_union(int G, const long long* __restrict__ vptr,
                                                     const long long* __restrict__ eptr,
                                                     const int* __restrict__ row_ptr,
                                                     const int* __restrict__ col,
                                                     const int2* __restrict__ chunks,
                                                     const unsigned* nch, int T,
                                                     unsigned* bad)
{
    for_each_chunk(chunks, nch, vptr, T, [&](int g, int64_t v0, int64_t v1) {
        unsigned err = 0;
        const long long lo = vptr[g], hi = vptr[g + 1];
        for (int64_t v = v0 + threadIdx.x; v < v1; v += kWG) {
            const int a = row_ptr[v], b = row_ptr[v + 1];
            if (v == lo && a != eptr[g]) err = 1;
            if (v + 1 == hi && b != eptr[g + 1]) err = 1;
            for (int e = a; e < b; ++e) {
                const int c = col[e];
                if (c < lo || c >= hi) err = 1;
            }
        }
        if (__ballot(err != 0) && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
    });
}

// ---------------------------------------------------------------------------
// sweep over the chunks of active graphs (SPFPassIter per region)
//
// A vertex whose edge changes also gets the edge's head in succ and its raw
// weight in wsel.  Outside a rebuild (which rewrites pi alone) both then hold
// col[pi] and w[pi] for every vertex: the value init after a rebuild writes
// them for the whole graph, the sweeps keep them, so the fast path's value
// init and the cycle init read them instead of one col and one w line per
// few rows.
// ---------------------------------------------------------------------------
template <int G, typename WT, bool TIE>
__global__ __launch_bounds__(kWG) void k_sweep(const int2* __restrict__ chunks,
                                               const unsigned* nch, int T, GArrays ga,
                                               const int* __restrict__ row_ptr,
                                               const int* __restrict__ col,
                                               const WT* __restrict__ w, int neg,
                                               const long long* __restrict__ V,
                                               int* __restrict__ pi,
                                               const unsigned char* __restrict__ onC,
                                               const int* __restrict__ hop,
                                               int* __restrict__ xs, int* __restrict__ ys,
                                               unsigned* xcnt, unsigned xcap,
                                               int* __restrict__ succ, WT* __restrict__ wsel)
{
    constexpr int VPB = kWG / G;
    for_each_chunk(chunks, nch, ga.vptr, T, [&](int g, int64_t v0, int64_t v1) {
        if (TIE && ga.status[g] != OCM_OK) return;
        const bool first = !TIE && ga.iter[g] == 0;
        const long long L = first ? 1 : ga.L[g];
        const long long W = first ? 0 : ga.W[g];
        const int lane = threadIdx.x & (G - 1);
        unsigned long long cnt = 0, certain = 0, nondec = 0;
        unsigned brk = 0;
        for (int64_t vb = v0; vb < v1; vb += VPB) {
            const int64_t v = vb + threadIdx.x / G;
            const bool live = v < v1;
            int beg = 0, end = 0, cur = -1;
            long long own = 0;
            if (live) {
                beg = row_ptr[v];
                end = row_ptr[v + 1];
                if (!first) own = V[v];
                if (TIE) cur = pi[v];
            }
            long long best = INT64_MAX;
            int bpos = INT32_MAX;
            for (int e = beg + lane; e < end; e += G) {
                const long long we = wval(w, e, neg);
                const long long key = first ? we : V[col[e]] + L * we - W;
                if (TIE) {
                    if (key == own && e != cur) {
                        cnt++;
                        const int y = col[e];
                        const bool sure = y == v || onC[v];
                        if (sure) certain++;
                        if (hop[y] >= hop[v]) {
                            nondec++;
                            // the short walk (few such edges: walked here,
                            // unless the graph is already known to tie)
                            if (succ && !sure && ga.certain[g] == 0) {
                                int x = y;
                                for (int st = 0; st < kShortWalk && x != (int)v; ++st) x = succ[x];
                                certain += x == (int)v;
                            }
                        }
                        if (xs) {   // list the tight non-policy edge (tie test)
                            const unsigned slot = atomicAdd(xcnt, 1u);
                            if (slot < xcap) {
                                xs[slot] = (int)v;
                                ys[slot] = col[e];
                            }
                        }
                    }
                } else if (key < best) {
                    best = key;
                    bpos = e;
                }
            }
            if (TIE) continue;
    #pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) {
                const long long ob = __shfl_xor(best, off, G);
                const int op = __shfl_xor(bpos, off, G);
                if (ob < best || (ob == best && op < bpos)) {
                    best = ob;
                    bpos = op;
                }
            }
            if (live && lane == 0 && (first || best < own)) {
                pi[v] = bpos;
                succ[v] = col[bpos];
                wsel[v] = w[bpos];
                cnt++;
                if (!first && onC[v]) brk = 1;
            }
        }
        cnt = block_sum_u64(cnt);
        if (TIE) {
            certain = block_sum_u64(certain);
            nondec = block_sum_u64(nondec);
            if (threadIdx.x == 0) {
                if (cnt) atomicAdd(&ga.tight[g], cnt);
                if (certain) atomicAdd(&ga.certain[g], certain);
                if (nondec) atomicAdd(&ga.nondec[g], nondec);
            }
        } else {
            const unsigned long long bb = block_sum_u64(brk);
            if (threadIdx.x == 0) {
                if (cnt) atomicAdd(&ga.changed[g], (unsigned)(cnt > 0xffffffffull ? 0xffffffffu : cnt));
                if (bb) atomicOr(&ga.cbroken[g], 1u);
            }
        }
    });
}

// The same sweep over vertex tiles: a workgroup takes its chunk 256 vertices
// at a time; their out-edges form one contiguous CSR range, streamed through
// LDS in batches of kBTileEdges (col and w loaded coalesced, the gathered V
// and the key computed per edge), then each thread walks its own vertex's
// keys in CSR order for the lowest-position minimum.  Same results as
// k_sweep (strict "<" in CSR order).  Batches of 1024 keys measured faster
// than 2048 or 1536 on the 4096-graph batch (more workgroups resident).
constexpr int kBTileEdges = 1024;

// A workgroup per tile (blockIdx.x -> chunk, tile of the chunk; the grid
// covers the list's capacity and idle workgroups leave at once), so that
// the dispatcher overlaps one tile's loads with another's (measured faster
// than a resident grid that walks its chunks' tiles in order).
//
// TIE: the tie scan after the loop instead (no policy change), with the
// counts, the short walk (succ non-null) and the edge list of k_sweep's
// tie form; graphs whose solve failed are skipped, and V is read in full
// (the small class writes no int32 copy).
template <typename WT, bool TIE>
__global__ __launch_bounds__(kWG) void k_sweep_tile(const int2* __restrict__ chunks,
                                                    const unsigned* nch, int T, GArrays ga,
                                                    const int* __restrict__ row_ptr,
                                                    const int* __restrict__ col,
                                                    const WT* __restrict__ w, int neg,
                                                    const long long* __restrict__ V,
                                                    int* __restrict__ pi,
                                                    const unsigned char* __restrict__ onC,
                                                    const int* __restrict__ V32, const BCtl* bc,
                                                    int* __restrict__ succ,
                                                    WT* __restrict__ wsel,
                                                    const int* __restrict__ hop,
                                                    int* __restrict__ xs, int* __restrict__ ys,
                                                    unsigned* xcnt, unsigned xcap)
{
    __shared__ int beg[kWG + 1];
    __shared__ long long key[kBTileEdges];
    constexpr int U = kBTileEdges / kWG;
    const int t = threadIdx.x;
    const unsigned per = (unsigned)((T + kWG - 1) / kWG);
    const unsigned ci = blockIdx.x / per;
    if (ci >= *nch) return;
    const int2 ch = chunks[ci];
    const int g = ch.x;
    if (TIE && ga.status[g] != OCM_OK) return;
    // every value written so far fits int32: gather the 4-byte copy
    const bool use32 = !TIE && bc->wide32 == 0u;
    unsigned long long cnt = 0, certain = 0, nondec = 0;
    unsigned brk = 0;
    // tie form: the tight non-policy edge e of vertex v
    auto tight_edge = [&](int64_t v, int e) {
        cnt++;
        const int y = col[e];
        const bool sure = y == v || onC[v];
        if (sure) certain++;
        if (hop[y] >= hop[v]) {
            nondec++;
            // the short walk (few such edges: walked here, unless the graph
            // is already known to tie)
            if (succ && !sure && ga.certain[g] == 0) {
                int x = y;
                for (int st = 0; st < kShortWalk && x != (int)v; ++st) x = succ[x];
                certain += x == (int)v;
            }
        }
        if (xs) {
            const unsigned slot = atomicAdd(xcnt, 1u);
            if (slot < xcap) {
                xs[slot] = (int)v;
                ys[slot] = y;
            }
        }
    };
    // the tile of nv <= kWG vertices from v0
    auto tile = [&](int64_t v0, int nv, bool first, long long L, long long W) {
        long long own = 0, best = INT64_MAX;
        int pos = INT32_MAX, cur = -1;
        if (t < nv) {
            beg[t] = row_ptr[v0 + t];
            if (!first) own = use32 ? (long long)V32[v0 + t] : V[v0 + t];
            if (TIE) cur = pi[v0 + t];
        }
        if (t == 0) beg[nv] = row_ptr[v0 + nv];
        __syncthreads();
        const int e0 = beg[0], e1 = beg[nv];
        const int mb = t < nv ? beg[t] : 0, me = t < nv ? beg[t + 1] : 0;
        for (int eb = e0; eb < e1; eb += kBTileEdges) {
            const int ne = e1 - eb < kBTileEdges ? e1 - eb : kBTileEdges;
            int c[U];
            WT wr[U];   // raw weights: half the registers of int64 ones for int32 w
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = t + u * kWG;
                c[u] = 0;
                wr[u] = 0;
                if (j < ne) {
                    c[u] = col[eb + j];
                    wr[u] = w[eb + j];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = t + u * kWG;
                if (j < ne) {
                    const long long wl = wval(&wr[u], 0, neg);
                    key[j] = first ? wl : (use32 ? (long long)V32[c[u]] : V[c[u]]) + L * wl - W;
                }
            }
            __syncthreads();
            const int lo = mb > eb ? mb : eb, hi = me < eb + ne ? me : eb + ne;
            const bool long_row = hi - lo > kLongRow;
            if (!long_row)
                for (int e = lo; e < hi; ++e) {
                    const long long k = key[e - eb];
                    if (TIE) {
                        if (k == own && e != cur) tight_edge(v0 + t, e);
                    } else if (k < best) {
                        best = k;
                        pos = e;
                    }
                }
            // the wave's long rows, one after the other, by all its lanes
            for (unsigned long long lm = __ballot(long_row); lm; lm &= lm - 1) {
                const int l = __ffsll((long long)lm) - 1;
                const int rlo = __shfl(lo, l, 64), rhi = __shfl(hi, l, 64);
                if (TIE) {
                    const long long rown = __shfl(own, l, 64);
                    const int rcur = __shfl(cur, l, 64);
                    const int64_t rv = v0 + (t & ~63) + l;
                    for (int e = rlo + (t & 63); e < rhi; e += 64)
                        if (key[e - eb] == rown && e != rcur) tight_edge(rv, e);
                    continue;
                }
                long long rb = INT64_MAX;
                int rp = INT32_MAX, rh = 0;
                for (int e = rlo + (t & 63); e < rhi; e += 64) {
                    const long long k = key[e - eb];
                    if (k < rb) {
                        rb = k;
                        rp = e;
                    }
                }
                wave_argmin<long long, false>(rb, rp, rh);
                if ((t & 63) == l && rb < best) {
                    best = rb;
                    pos = rp;
                }
            }
            __syncthreads();
        }
        if (!TIE && t < nv && pos != INT32_MAX && (first || best < own)) {
            pi[v0 + t] = pos;
            succ[v0 + t] = col[pos];
            wsel[v0 + t] = w[pos];
            cnt++;
            if (!first && onC[v0 + t]) brk = 1;
        }
    };
    const int64_t end = ga.vptr[g + 1];
    const int64_t c1 = ch.y + (int64_t)T < end ? ch.y + (int64_t)T : end;
    const int64_t v0 = ch.y + (int64_t)(blockIdx.x % per) * kWG;
    if (v0 >= c1) return;
    const bool first = !TIE && ga.iter[g] == 0;
    tile(v0, c1 - v0 < kWG ? (int)(c1 - v0) : kWG, first, first ? 1 : ga.L[g],
         first ? 0 : ga.W[g]);
    cnt = block_sum_u64(cnt);
    if (TIE) {
        certain = block_sum_u64(certain);
        nondec = block_sum_u64(nondec);
        if (threadIdx.x == 0) {
            if (cnt) atomicAdd(&ga.tight[g], cnt);
            if (certain) atomicAdd(&ga.certain[g], certain);
            if (nondec) atomicAdd(&ga.nondec[g], nondec);
        }
    } else {
        const unsigned long long bb = block_sum_u64(brk);
        if (threadIdx.x == 0) {
            if (cnt) atomicAdd(&ga.changed[g], (unsigned)(cnt > 0xffffffffull ? 0xffffffffu : cnt));
            if (bb) atomicOr(&ga.cbroken[g], 1u);
        }
    }
}

// After the sweep: converged graphs retire; the others take the fast path
// (C intact) or the general phases.
__global__ __launch_bounds__(kWG) void k_after_sweep(int G, GArrays ga, int max_iters,
                                                     BCtl* bc)
{
    unsigned na = 0, nf = 0, ng = 0;
    for (int g = blockIdx.x * kWG + threadIdx.x; g < G; g += gridDim.x * kWG) {
        if (ga.mode[g] != kActive) continue;
        const int it = ++ga.iter[g];
        const unsigned ch = ga.changed[g];
        ga.changed[g] = 0;
        const unsigned cb = ga.cbroken[g];
        ga.cbroken[g] = 0;
        if (it >= 2 && ch == 0) {
            ga.mode[g] = kDone;
            continue;
        }
        if (max_iters > 0 && it >= max_iters) {
            ga.mode[g] = kDone;
            ga.status[g] = OCM_E_NOT_CONVERGED;
            continue;
        }
        ++na;
        if (ga.have_c[g] && !cb) {
            ga.mode[g] = kFast;
            ++nf;
        } else {
            ga.mode[g] = kGeneral;
            ++ng;
        }
    }
    const unsigned long long a = block_sum_u64(na), f = block_sum_u64(nf), q = block_sum_u64(ng);
    if (threadIdx.x == 0) {
        if (a) atomicAdd(&bc->nactive, (unsigned)a);
        if (f) atomicAdd(&bc->nfast, (unsigned)f);
        if (q) atomicAdd(&bc->ngeneral, (unsigned)q);
    }
}

// ---------------------------------------------------------------------------
// values: pointer jumping toward each graph's source
// ---------------------------------------------------------------------------
// Value init.  SEL (fast path): each vertex's successor and edge weight come
// from succ and wsel, and the entry already spans two policy edges (succ
// and wsel of the successor are gathered); otherwise (after a rebuild) they
// come from pi, col and w, the entry spans one edge, and succ and wsel are
// written.  It also books the first round in slot 0: a graph none of
// whose vertices has an entry short of s is finished (vact stays clear).
template <typename WT, bool SEL>
__global__ __launch_bounds__(kWG) void k_val_init(const int2* __restrict__ chunks,
                                                  const unsigned* nch, int T, GArrays ga,
                                                  const int* __restrict__ col,
                                                  const int* __restrict__ pi,
                                                  const WT* __restrict__ w, int neg,
                                                  int* __restrict__ succ, WT* __restrict__ wsel,
                                                  VJ* __restrict__ Q, BCtl* bc)
{
    for_each_chunk(chunks, nch, ga.vptr, T, [&](int g, int64_t v0, int64_t v1) {
        const int s = ga.s[g];
        const long long W = ga.W[g], L = ga.L[g];
        unsigned act = 0;
        for (int64_t v = v0 + threadIdx.x; v < v1; v += kWG) {
            int t;
            long long we;
            if (SEL) {
                t = succ[v];
                we = wval(wsel, v, neg);
            } else {
                const int e = pi[v];
                const WT x = w[e];
                t = col[e];
                succ[v] = t;
                wsel[v] = x;
                we = wval(&x, 0, neg);
            }
            int j = v == s ? s : t;
            long long d = v == s ? 0 : L * we - W;
            if (SEL && j != s) {
                // two policy edges (the first jump round's work); each term
                // is below 2^62 in magnitude (the weight bound): no overflow
                d += L * wval(wsel, t, neg) - W;
                j = succ[t];
            }
            act |= j != s ? 1u : 0u;
            Q[v] = vj_make(d, j);
        }
        const unsigned long long a = block_sum_u64(act);
        if (threadIdx.x == 0) {
            ga.vrun[g] = 1;
            ga.ovf[g] = 0;
            if (a) {
                atomicOr(&ga.vact[4 * g], 1u);
                atomicOr(&bc->vrun_round[0], 1u);
            }
            atomicOr(&ga.vprog[4 * g], 1u);
        }
    });
}

// entries in flight per thread in a value round (batch4096: 16 measured
// fastest; 8, 12 and 24 slower, 32 spills)
constexpr int kValRoundU = 16;

// Value round r: first the previous round's booking (slot r % 3) of each
// graph: a graph with no unfinished vertex is finished (its entries stay in
// buffer r & 1), one whose previous round finished none while some remain
// never reaches s (fast path: C is no longer the only cycle; it falls back
// to the general phases, a general graph fails).  Every workgroup of the
// graph takes the same decision from the same slot.  The rest advance one
// jump and book slot (r + 1) % 3; the graph's first chunk clears slot
// (r + 2) % 3 for the next round.
__global__ __launch_bounds__(kWG) void k_val_round(const int2* __restrict__ chunks,
                                                   const unsigned* nch, int T, GArrays ga,
                                                   const VJ* __restrict__ Qin,
                                                   VJ* __restrict__ Qout, int want, int r,
                                                   BCtl* bc)
{
    if (bc->vrun_round[r] == 0) return;   // no graph of the phase left to advance
    if (blockIdx.x == 0 && threadIdx.x == 0) bc->vlast = (unsigned)r + 1u;
    const int si = r % 3, so = (r + 1) % 3, sc = (r + 2) % 3;
    unsigned any = 0;
    for_each_chunk(chunks, nch, ga.vptr, T, [&](int g, int64_t v0, int64_t v1) {
        // independent loads, issued together
        const unsigned run = ga.vrun[g];
        const unsigned pa = ga.vact[4 * g + si], pp = ga.vprog[4 * g + si];
        const int s = ga.s[g];
        const bool head = v0 == ga.vptr[g];
        if (threadIdx.x == 0 && head) {
            ga.vact[4 * g + sc] = 0;
            ga.vprog[4 * g + sc] = 0;
        }
        if (!run) return;   // finished or stalled graph: its entries stay put
        if (!pa || !pp) {
            if (threadIdx.x == 0) {
                ga.vrun[g] = 0;
                if (!pa) ga.fin[g] = r & 1;
                else if (want == kFast) ga.mode[g] = kGeneral;   // fall back
                else {
                    ga.mode[g] = kDone;
                    ga.status[g] = OCM_E_NOT_STRONGLY_CONNECTED;
                }
            }
            return;
        }
        unsigned act = 0, prog = 0;
        // kValRoundU entries in flight per thread: loads, then the dependent gathers
        constexpr int U = kValRoundU;
        for (int64_t vb = v0 + threadIdx.x; vb < v1; vb += U * kWG) {
            VJ q[U], rr[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t v = vb + u * kWG;
                if (v < v1) q[u] = Qin[v];
                else q[u].J = s;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (q[u].J != s) rr[u] = Qin[q[u].J];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t v = vb + u * kWG;
                if (v >= v1) continue;
                if (q[u].J != s) {
                    const long long a = vj_d(q[u]), b = vj_d(rr[u]);
                    long long d;
                    if (a == kDOverflow || b == kDOverflow || __builtin_add_overflow(a, b, &d))
                        d = kDOverflow;
                    q[u] = vj_make(d, rr[u].J);
                    if (q[u].J == s) prog = 1;
                    else act = 1;
                }
                Qout[v] = q[u];
            }
        }
        const unsigned long long a = block_sum_u64(act), p = block_sum_u64(prog);
        if (threadIdx.x == 0) {
            if (a) atomicOr(&ga.vact[4 * g + so], 1u);
            if (p) atomicOr(&ga.vprog[4 * g + so], 1u);
            any |= a ? 1u : 0u;
        }
    });
    if (threadIdx.x == 0 && any && r + 1 < 32) atomicOr(&bc->vrun_round[r + 1], 1u);
}

// After the last round: the same decision from the last round's booking
// (slot vlast % 3, buffer vlast & 1) for the graphs still running.
__global__ __launch_bounds__(kWG) void k_val_close(int G, GArrays ga, int want, const BCtl* bc,
                                                   const unsigned* halt)
{
    if (halt && *halt != 0u) return;
    const unsigned k = bc->vlast;
    for (int g = blockIdx.x * kWG + threadIdx.x; g < G; g += gridDim.x * kWG) {
        if (ga.mode[g] != want || !ga.vrun[g]) continue;
        const unsigned a = ga.vact[4 * g + k % 3u], p = ga.vprog[4 * g + k % 3u];
        if (!a) {
            ga.vrun[g] = 0;
            ga.fin[g] = (int)(k & 1u);
        } else if (!p) {
            ga.vrun[g] = 0;
            if (want == kFast) ga.mode[g] = kGeneral;
            else {
                ga.mode[g] = kDone;
                ga.status[g] = OCM_E_NOT_STRONGLY_CONNECTED;
            }
        }
    }
}

__global__ __launch_bounds__(kWG) void k_val_final(const int2* __restrict__ chunks,
                                                   const unsigned* nch, int T, GArrays ga,
                                                   int want, const VJ* __restrict__ Q0,
                                                   const VJ* __restrict__ Q1,
                                                   long long* __restrict__ V,
                                                   int* __restrict__ V32, BCtl* bc)
{
    for_each_chunk(chunks, nch, ga.vptr, T, [&](int g, int64_t v0, int64_t v1) {
        // mode[g] may be changed by another workgroup of this launch: decide once
        const int state = block_bcast(ga.mode[g] != want ? 0 : (ga.vrun[g] ? 1 : 2));
        // the phase's bookings are read: leave every slot clear for the next phase
        if (threadIdx.x < 3 && v0 == ga.vptr[g]) {
            ga.vact[4 * g + threadIdx.x] = 0;
            ga.vprog[4 * g + threadIdx.x] = 0;
        }
        if (state == 0) return;   // fell back or failed
        if (state == 1) {         // did not finish within the rounds
            if (threadIdx.x == 0) {
                ga.mode[g] = kDone;
                ga.status[g] = OCM_E_HIP;
            }
            return;
        }
        const VJ* __restrict__ Q = ga.fin[g] ? Q1 : Q0;
        unsigned bad = 0, big = 0;
        for (int64_t v = v0 + threadIdx.x; v < v1; v += kWG) {
            const long long d = vj_d(Q[v]);   // kDOverflow lies below -kValLimit
            V[v] = d;
            V32[v] = (int)d;
            if (d > kValLimit || d < -kValLimit) bad = 1;
            big |= d > INT32_MAX || d < INT32_MIN ? 1u : 0u;
        }
        const unsigned long long b = block_sum_u64(bad);
        const unsigned long long bg = block_sum_u64(big);
        if (threadIdx.x == 0) {
            if (b) {
                ga.mode[g] = kDone;
                ga.status[g] = OCM_E_OVERFLOW;
            }
            // sticky: from now on the sweeps gather the int64 values
            if (bg) atomicOr(&bc->wide32, 1u);
        }
    });
}

// Hops to the source after the loop (the policy edges from v to s, which
// the tie tests and the cycle listing use), by pointer jumping on entries
// (J in the high word, H in the low word).  Graphs that failed are skipped,
// and so are those of the small class (never in the loop, so have_c is
// clear), which wrote their hops themselves.
__device__ __forceinline__ bool hop_graph(const GArrays& ga, int g)
{
    return ga.status[g] == OCM_OK && ga.have_c[g];
}

__global__ __launch_bounds__(kWG) void k_hop_init(const int2* __restrict__ chunks,
                                                  const unsigned* nch, int T, GArrays ga,
                                                  const int* __restrict__ succ,
                                                  unsigned long long* __restrict__ P)
{
    for_each_chunk(chunks, nch, ga.vptr, T, [&](int g, int64_t v0, int64_t v1) {
        if (!hop_graph(ga, g)) return;
        const int s = ga.s[g];
        for (int64_t v = v0 + threadIdx.x; v < v1; v += kWG)
            P[v] = v == s ? (unsigned long long)(unsigned)s << 32
                          : ((unsigned long long)(unsigned)succ[v] << 32) | 1u;
    });
}

// running: some entry of the last round had not reached s (round 0: set
// by the host); act: this round's.
__global__ __launch_bounds__(kWG) void k_hop_round(const int2* __restrict__ chunks,
                                                   const unsigned* nch, int T, GArrays ga,
                                                   const unsigned long long* __restrict__ Pin,
                                                   unsigned long long* __restrict__ Pout,
                                                   const unsigned* running, unsigned* act_out)
{
    if (*running == 0) return;
    for_each_chunk(chunks, nch, ga.vptr, T, [&](int g, int64_t v0, int64_t v1) {
        if (!hop_graph(ga, g)) return;
        const unsigned s = (unsigned)ga.s[g];
        unsigned act = 0;
        constexpr int U = 8;
        for (int64_t vb = v0 + threadIdx.x; vb < v1; vb += U * kWG) {
            unsigned long long p[U], q[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t v = vb + u * kWG;
                p[u] = v < v1 ? Pin[v] : (unsigned long long)s << 32;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if ((unsigned)(p[u] >> 32) != s) q[u] = Pin[(unsigned)(p[u] >> 32)];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t v = vb + u * kWG;
                if (v >= v1) continue;
                if ((unsigned)(p[u] >> 32) != s) {
                    p[u] = (q[u] & 0xffffffff00000000ull) |
                           (unsigned)((unsigned)p[u] + (unsigned)q[u]);
                    act |= (unsigned)(p[u] >> 32) != s ? 1u : 0u;
                }
                Pout[v] = p[u];
            }
        }
        const unsigned long long a = block_sum_u64(act);
        if (threadIdx.x == 0 && a) atomicOr(act_out, 1u);
    });
}

// Round r reads P0 when r is even and writes the other buffer; a round
// whose running flag is clear writes nothing, so the entries are in the
// output of the last round that ran (P0 if none did).
__global__ __launch_bounds__(kWG) void k_hop_final(const int2* __restrict__ chunks,
                                                   const unsigned* nch, int T, GArrays ga,
                                                   const unsigned long long* __restrict__ P0,
                                                   const unsigned long long* __restrict__ P1,
                                                   const unsigned* hop_act, int R,
                                                   int* __restrict__ hop)
{
    int ran = 0;
    while (ran < R && hop_act[ran] != 0u) ++ran;
    const unsigned long long* __restrict__ P = ran == 0 ? P0 : ((ran - 1) & 1 ? P0 : P1);
    for_each_chunk(chunks, nch, ga.vptr, T, [&](int g, int64_t v0, int64_t v1) {
        if (!hop_graph(ga, g)) return;
        for (int64_t v = v0 + threadIdx.x; v < v1; v += kWG) hop[v] = (int)(unsigned)P[v];
    });
}

// The iteration's rebuild rounds did not all run (more than the captured
// number were needed): the host finishes them.
__global__ void k_rounds_open(BCtl* bc, const Ctl* ctl)
{
    if (threadIdx.x == 0) bc->rounds_open = ctl->rmode != 0u ? 1u : 0u;
}

// fast or general graph whose values are ready: back to sweeping
__global__ __launch_bounds__(kWG) void k_values_done(int G, GArrays ga, int want,
                                                     const unsigned* halt)
{
    if (halt && *halt != 0u) return;
    for (int g = blockIdx.x * kWG + threadIdx.x; g < G; g += gridDim.x * kWG) {
        if (ga.mode[g] != want) continue;
        ga.mode[g] = kActive;
        ga.have_c[g] = 1;
    }
}

// ---------------------------------------------------------------------------
// cycles of the policy graph (pointer jumping), per-cycle sums, vote
// ---------------------------------------------------------------------------
// succ holds col[pi] here (a sweep, never a rebuild, changed pi last)
__global__ __launch_bounds__(kWG) void k_pj_init(const int2* __restrict__ chunks,
                                                 const unsigned* nch, int T, GArrays ga,
                                                 const int* __restrict__ succ,
                                                 unsigned long long* __restrict__ P,
                                                 unsigned char* __restrict__ onc)
{
    for_each_chunk(chunks, nch, ga.vptr, T, [&](int g, int64_t v0, int64_t v1) {
        for (int64_t v = v0 + threadIdx.x; v < v1; v += kWG) {
            const int s = succ[v];
            P[v] = ((unsigned long long)(unsigned)s << 32) | (unsigned)v;
            onc[v] = 0;
        }
        if (threadIdx.x == 0) ga.best[g] = -1;
    });
}

// Rounds a graph of n vertices needs: ceil(log2 n) (2^K >= n covers every
// policy path and cycle in it).
__device__ __forceinline__ int graph_rounds(const long long* __restrict__ vptr, int g)
{
    const long long n = vptr[g + 1] - vptr[g];
    return n <= 1 ? 0 : 64 - __clzll((unsigned long long)(n - 1));
}

// Round k reads P[k & 1] and writes P[(k + 1) & 1]; a graph takes part only
// in its first graph_rounds rounds, so its entries end in P[rounds & 1].
__global__ __launch_bounds__(kWG) void k_pj_round(const int2* __restrict__ chunks,
                                                  const unsigned* nch, int T, GArrays ga, int k,
                                                  const unsigned long long* __restrict__ Pin,
                                                  unsigned long long* __restrict__ Pout)
{
    for_each_chunk(chunks, nch, ga.vptr, T, [&](int g, int64_t v0, int64_t v1) {
        if (k >= graph_rounds(ga.vptr, g)) return;
        constexpr int U = 8;   // entries in flight per thread
        for (int64_t vb = v0 + threadIdx.x; vb < v1; vb += U * kWG) {
            unsigned long long p[U], q[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t v = vb + u * kWG;
                p[u] = v < v1 ? Pin[v] : 0ull;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (vb + u * kWG < v1) q[u] = Pin[(int)(p[u] >> 32)];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t v = vb + u * kWG;
                if (v >= v1) continue;
                const unsigned m0 = (unsigned)p[u], m1 = (unsigned)q[u];
                Pout[v] = (q[u] & 0xffffffff00000000ull) | (m0 < m1 ? m0 : m1);
            }
        }
    });
}

__global__ __launch_bounds__(kWG) void k_pj_final(const int2* __restrict__ chunks,
                                                  const unsigned* nch, int T, GArrays ga,
                                                  const unsigned long long* __restrict__ P0,
                                                  const unsigned long long* __restrict__ P1,
                                                  int* __restrict__ rep,
                                                  unsigned char* __restrict__ onc)
{
    for_each_chunk(chunks, nch, ga.vptr, T, [&](int g, int64_t v0, int64_t v1) {
        const unsigned long long* __restrict__ P = graph_rounds(ga.vptr, g) & 1 ? P1 : P0;
        for (int64_t v = v0 + threadIdx.x; v < v1; v += kWG) {
            const int c = (int)(P[v] >> 32);
            rep[v] = (int)(unsigned)P[c];
            onc[c] = 1;
        }
    });
}

// cycle heads of general graphs: zero their sums and list (rep, graph)
__global__ __launch_bounds__(kWG) void k_cyc_zero(const int2* __restrict__ chunks,
                                                  const unsigned* nch, int T, GArrays ga,
                                                  const int* __restrict__ rep,
                                                  const unsigned char* __restrict__ onc,
                                                  long long* __restrict__ wsum,
                                                  unsigned* __restrict__ lcnt,
                                                  int2* __restrict__ heads, BCtl* bc)
{
    for_each_chunk(chunks, nch, ga.vptr, T, [&](int g, int64_t v0, int64_t v1) {
        for (int64_t vb = v0; vb < v1; vb += kWG) {
            const int64_t v = vb + threadIdx.x;
            const bool head = v < v1 && onc[v] && rep[v] == v;
            if (head) {
                wsum[v] = 0;
                lcnt[v] = 0;
            }
            const unsigned long long mask = __ballot(head);
            if (mask) {
                const unsigned lane = threadIdx.x & 63;
                const unsigned leader = (unsigned)__ffsll((long long)mask) - 1u;
                unsigned base = 0;
                if (lane == leader) base = atomicAdd(&bc->ncyc, (unsigned)__popcll(mask));
                base = __shfl(base, (int)leader, 64);
                if (head) heads[base + __popcll(mask & ((1ull << lane) - 1ull))] = make_int2((int)v, g);
            }
        }
    });
}

template <typename WT>
__global__ __launch_bounds__(kWG) void k_cyc_sum(const int2* __restrict__ chunks,
                                                 const unsigned* nch, int T, GArrays ga,
                                                 const int* __restrict__ rep,
                                                 const unsigned char* __restrict__ onc,
                                                 const int* __restrict__ pi,
                                                 const WT* __restrict__ w, int neg,
                                                 long long* __restrict__ wsum,
                                                 unsigned* __restrict__ lcnt)
{
    for_each_chunk(chunks, nch, ga.vptr, T, [&](int g, int64_t v0, int64_t v1) {
        for (int64_t v = v0 + threadIdx.x; v < v1; v += kWG) {
            if (!onc[v]) continue;
            const int r = rep[v];
            atomicAdd((unsigned long long*)&wsum[r], (unsigned long long)wval(w, pi[v], neg));
            atomicAdd(&lcnt[r], 1u);
        }
    });
}

// a < b in the order (W/L, rep)
__device__ __forceinline__ bool rep_less(int a, int b, const long long* __restrict__ wsum,
                                         const unsigned* __restrict__ lcnt)
{
    const __int128 x = (__int128)wsum[a] * (long long)lcnt[b];
    const __int128 y = (__int128)wsum[b] * (long long)lcnt[a];
    if (x != y) return x < y;
    return a < b;
}

// Region-specific minimum vote (Alg. 5) with the exact comparator: the
// final value is the minimum whatever the order of the votes.
__global__ __launch_bounds__(kWG) void k_vote(const int2* __restrict__ heads, const BCtl* bc,
                                              GArrays ga, const long long* __restrict__ wsum,
                                              const unsigned* __restrict__ lcnt)
{
    const unsigned nc = bc->ncyc;
    for (unsigned i = blockIdx.x * kWG + threadIdx.x; i < nc; i += gridDim.x * kWG) {
        const int2 h = heads[i];
        int cur = ga.best[h.y];
        while (cur < 0 || rep_less(h.x, cur, wsum, lcnt)) {
            const int prev = atomicCAS(&ga.best[h.y], cur, h.x);
            if (prev == cur) break;
            cur = prev;
        }
    }
}

__global__ __launch_bounds__(kWG) void k_set_lambda(int G, GArrays ga,
                                                    const long long* __restrict__ wsum,
                                                    const unsigned* __restrict__ lcnt)
{
    for (int g = blockIdx.x * kWG + threadIdx.x; g < G; g += gridDim.x * kWG) {
        if (ga.mode[g] != kGeneral) continue;
        const int r = ga.best[g];
        if (r < 0) {
            ga.mode[g] = kDone;
            ga.status[g] = OCM_E_HIP;
            continue;
        }
        ga.s[g] = r;
        ga.W[g] = wsum[r];
        ga.L[g] = (long long)lcnt[r];
    }
}

// ---------------------------------------------------------------------------
// rebuild: keep each graph's chosen component, list the rest
// ---------------------------------------------------------------------------
// Clears, in a bitmap, the bits of this wave's 64 consecutive vertices
// vb .. vb+63 whose lanes pass `cond` (one atomicAnd per touched word).
__device__ __forceinline__ void clear_wave_bits(unsigned* bits, int64_t vb, bool cond)
{
    const unsigned long long B = __ballot(cond);
    const int lane = threadIdx.x & 63;
    const int64_t w0 = vb >> 5;
    // the 64 vertices span at most three words; lane j < 3 handles word w0 + j
    if (lane < 3) {
        const int64_t j = w0 + lane;
        const int64_t lo = (j * 32 > vb ? j * 32 : vb) - vb;
        const int64_t hi = ((j + 1) * 32 < vb + 64 ? (j + 1) * 32 : vb + 64) - vb;
        if (lo < hi) {
            const unsigned long long span = hi - lo == 64 ? ~0ull : ((1ull << (hi - lo)) - 1ull);
            const unsigned m = (unsigned)(((B >> lo) & span) << ((vb + lo) & 31));
            if (m) atomicAnd(&bits[j], ~m);
        }
    }
}

// Rebuild init for the graphs in chunks (mode kGeneral): C's component keeps
// pi (layer 0), the rest is unattached (layer -1).  Both bitmaps start all
// ones (every other graph counts as attached); here every vertex leaves a0
// and every unattached one leaves a1, so round 1 sees the components as its
// frontier.  Counts go to cc's lanes (got = components, left = unattached).
__global__ __launch_bounds__(kWG) void k_conn_init(const int2* __restrict__ chunks,
                                                   const unsigned* nch, int T, GArrays ga,
                                                   const int* __restrict__ rep,
                                                   const unsigned char* __restrict__ onc,
                                                   int* __restrict__ layer,
                                                   unsigned char* __restrict__ onC,
                                                   unsigned* a1, unsigned* a0, Ctl* cc)
{
    for_each_chunk(chunks, nch, ga.vptr, T, [&](int g, int64_t v0, int64_t v1) {
        const int s = ga.s[g];
        unsigned long long ncomp = 0, nleft = 0;
        for (int64_t vb = v0 + (threadIdx.x & ~63); vb < v1; vb += kWG) {
            const int64_t v = vb + (threadIdx.x & 63);
            const bool live = v < v1;
            bool comp = false;
            if (live) {
                comp = rep[v] == s;
                if (layer) layer[v] = comp ? 0 : -1;
                onC[v] = (unsigned char)(comp && onc[v]);
                ncomp += comp;
                nleft += !comp;
            }
            clear_wave_bits(a0, vb, live);
            clear_wave_bits(a1, vb, live && !comp);
        }
        ncomp = block_sum_u64(ncomp);
        nleft = block_sum_u64(nleft);
        if (threadIdx.x == 0) {
            if (ncomp) atomicAdd(&my_lane(cc).got, (unsigned)ncomp);
            if (nleft) atomicAdd(&my_lane(cc).left, (unsigned)nleft);
        }
    });
}

// Graphs with a vertex that stays unattached (not in acur) are not strongly
// connected.  Device-driven rounds (ctl non-null): only after a round that
// attached nobody (rerr), on that round's bitmap (a0 / a1 by its parity).
__global__ __launch_bounds__(kWG) void k_conn_fail(int G, int n, const long long* __restrict__ vptr,
                                                   const unsigned* __restrict__ acur, GArrays ga,
                                                   const unsigned* __restrict__ a1 = nullptr,
                                                   const Ctl* ctl = nullptr)
{
    if (ctl) {
        if (!ctl->rerr) return;
        if (ctl->rk & 1u) acur = a1;
    }
    const int64_t words = ((int64_t)n + 31) / 32;
    for (int64_t w = (int64_t)blockIdx.x * kWG + threadIdx.x; w < words;
         w += (int64_t)gridDim.x * kWG) {
        const int64_t lo32 = w * 32;
        unsigned un = ~acur[w] & (lo32 + 32 <= n ? 0xffffffffu : (1u << (unsigned)(n - lo32)) - 1u);
        while (un) {
            const int u = (int)(lo32 + __ffs(un) - 1);
            un &= un - 1;
            int lo = 0, hi = G - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) / 2;
                if (vptr[mid] <= u) lo = mid;
                else hi = mid - 1;
            }
            ga.mode[lo] = kDone;
            ga.status[lo] = OCM_E_NOT_STRONGLY_CONNECTED;
        }
    }
}

// Flags the round-kernel spans (vertices [i * span_verts, (i + 1) *
// span_verts)) that hold a vertex of a listed chunk.
__global__ __launch_bounds__(kWG) void k_span_flag(const int2* __restrict__ chunks,
                                                   const unsigned* nch, int T, GArrays ga,
                                                   int64_t span_verts,
                                                   unsigned char* __restrict__ flags)
{
    for_each_chunk(chunks, nch, ga.vptr, T, [&](int g, int64_t v0, int64_t v1) {
        for (int64_t sp = v0 / span_verts + threadIdx.x; sp <= (v1 - 1) / span_verts; sp += kWG)
            flags[sp] = 1;
    });
}

// Lists the flagged spans in order (and clears the flags); one workgroup.
__global__ __launch_bounds__(kWG) void k_span_list(int64_t nall, unsigned char* __restrict__ flags,
                                                   int* __restrict__ spans, unsigned* nspans)
{
    __shared__ unsigned wsum[kWG / 64];
    unsigned base = 0;
    for (int64_t s0 = 0; s0 < nall; s0 += kWG) {
        const int64_t i = s0 + threadIdx.x;
        const bool f = i < nall && flags[i];
        if (i < nall && f) flags[i] = 0;
        const unsigned incl = wave_incl_scan(f ? 1u : 0u);
        if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = incl;
        __syncthreads();
        unsigned wbase = 0, tot = 0;
        for (int w = 0; w < kWG / 64; ++w) {
            if (w < (int)(threadIdx.x >> 6)) wbase += wsum[w];
            tot += wsum[w];
        }
        if (f) spans[base + wbase + incl - 1] = (int)i;
        base += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *nspans = base;
}

// ---------------------------------------------------------------------------
// results
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_cycle_list(const int2* __restrict__ chunks,
                                                    const unsigned* nch, int T, GArrays ga,
                                                    const long long* __restrict__ cptr,
                                                    const unsigned char* __restrict__ onC,
                                                    const int* __restrict__ pi,
                                                    const int* __restrict__ hop,
                                                    int* __restrict__ out)
{
    for_each_chunk(chunks, nch, ga.vptr, T, [&](int g, int64_t v0, int64_t v1) {
        if (ga.status[g] != OCM_OK) return;
        const int s = ga.s[g];
        const long long L = ga.L[g], base = cptr[g];
        for (int64_t v = v0 + threadIdx.x; v < v1; v += kWG) {
            if (!onC[v]) continue;
            const long long j = v == s ? 0 : L - (long long)hop[v];
            if (j >= 0 && j < L) out[base + j] = pi[v];
        }
    });
}

__global__ void k_bctl_clear(BCtl* bc)
{
    if (threadIdx.x == 0) {
        unsigned* p = (unsigned*)bc;
        for (unsigned i = 0; i < sizeof(BCtl) / sizeof(unsigned); ++i) p[i] = 0;
    }
}

// The tie list's edges whose graph is in mode kTieList, appended to xo / yo
// (their graph found by a binary search over vptr).
__global__ __launch_bounds__(kWG) void k_list_open(unsigned k, const int* __restrict__ xs,
                                                   const int* __restrict__ ys, int G,
                                                   const long long* __restrict__ vptr,
                                                   const int* __restrict__ mode,
                                                   int* __restrict__ xo, int* __restrict__ yo,
                                                   unsigned* cnt)
{
    for (unsigned i = blockIdx.x * kWG + threadIdx.x; i < k; i += gridDim.x * kWG) {
        const long long v = xs[i];
        int lo = 0, hi = G;   // vptr[lo] <= v < vptr[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (vptr[mid] <= v) lo = mid;
            else hi = mid;
        }
        if (mode[lo] != kTieList) continue;
        const unsigned slot = atomicAdd(cnt, 1u);
        xo[slot] = (int)v;
        yo[slot] = ys[i];
    }
}

__global__ void k_bctl_zero(unsigned* a, unsigned* b)
{
    if (threadIdx.x == 0) {
        *a = 0;
        if (b) *b = 0;
    }
}

__global__ __launch_bounds__(kWG) void k_graph_init(int G, GArrays ga)
{
    for (int g = blockIdx.x * kWG + threadIdx.x; g < G; g += gridDim.x * kWG) {
        ga.W[g] = 0;
        ga.L[g] = 1;
        ga.s[g] = -1;
        ga.iter[g] = 0;
        ga.mode[g] = kActive;
        ga.status[g] = OCM_OK;
        ga.best[g] = -1;
        ga.changed[g] = 0;
        ga.cbroken[g] = 0;
        ga.vrun[g] = 0;
        for (int k = 0; k < 4; ++k) {
            ga.vact[4 * g + k] = 0;
            ga.vprog[4 * g + k] = 0;
        }
        ga.ovf[g] = 0;
        ga.have_c[g] = 0;
        ga.tight[g] = 0;
        ga.certain[g] = 0;
        ga.nondec[g] = 0;
    }
}

__global__ __launch_bounds__(kWG) void k_fast_to_general(int G, GArrays ga)
{
    for (int g = blockIdx.x * kWG + threadIdx.x; g < G; g += gridDim.x * kWG)
        if (ga.mode[g] == kFast) ga.mode[g] = kGeneral;
}

// One graph of the union as a graph of its own: offsets, targets and policy
// rebased to local numbering (weights are used in place).
__global__ __launch_bounds__(kWG) void k_rebase(int n, int m, const int* __restrict__ row_ptr,
                                                const int* __restrict__ col,
                                                const int* __restrict__ pi, int voff, int eoff,
                                                int* __restrict__ rp_out, int* __restrict__ col_out,
                                                int* __restrict__ pi_out)
{
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i <= (int64_t)m;
         i += (int64_t)gridDim.x * kWG) {
        if (i <= n) rp_out[i] = row_ptr[i] - eoff;
        if (i < n) pi_out[i] = pi[i] - eoff;
        if (i < m) col_out[i] = col[i] - voff;
    }
}

__global__ __launch_bounds__(kWG) void k_tie_init(int G, GArrays ga)
{
    for (int g = blockIdx.x * kWG + threadIdx.x; g < G; g += gridDim.x * kWG) {
        ga.tight[g] = 0;
        ga.certain[g] = 0;
        ga.nondec[g] = 0;
    }
}

// ---------------------------------------------------------------------------
// The small-graph class: a graph of at most kSmallN vertices and kSmallM
// edges is solved whole by one workgroup, every per-vertex array in LDS
// (vertex ids local, 16 bits), its CSR read from global memory (it stays in
// L2 across the iterations).  The phases and rules are the single-graph
// solver's (R1-R10): first sweep, then per iteration the policy graph's
// cycles by pointer jumping, the minimum-mean select, the breadth-first
// rebuild rounds, values by pointer jumping and the improvement sweep.
// There is no fast path (it changes no result).  The graph's final policy,
// successors, values, hops and C flags go to the batch arrays, so the
// cycle listing and tie tests after the loop treat it like any other graph.
// ---------------------------------------------------------------------------
constexpr int kSmallN = 2048;
constexpr int kSmallM = 32768;
constexpr int kSmallWG = 512;
constexpr int kSmallVPT = kSmallN / kSmallWG;   // vertices per thread
constexpr int kSmallIterCap = 1 << 20;

struct SmallLds {
    long long V[kSmallN];       // values scaled by L
    int pi[kSmallN];            // policy: global edge positions
    short succ[kSmallN];        // local successor
    short rep[kSmallN];         // smallest vertex of the reached cycle
    short layer[kSmallN];       // rebuild round, -1 unattached
    unsigned char onc[kSmallN]; // on a policy cycle
    union {
        struct {
            short J[kSmallN];   // 2^k-th successor
            short M[kSmallN];   // minimum over the next 2^k vertices
        } cyc;
        struct {
            long long wsum[kSmallN];
            int lcnt[kSmallN];
        } sel;
        struct {
            long long D[kSmallN];   // sum of (L*w - W) over the first H policy edges
            short J[kSmallN];
            short H[kSmallN];
        } val;
    } u;
    unsigned long long red[kSmallWG / 64];
    long long cw[kSmallWG / 64], cl[kSmallWG / 64];
    int cr[kSmallWG / 64];
};

// Sum over the workgroup, returned to every thread.
__device__ __forceinline__ unsigned long long small_sum(unsigned long long x, SmallLds& S)
{
    x = wave_sum_u64(x);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) S.red[threadIdx.x >> 6] = x;
    __syncthreads();
    unsigned long long t = 0;
    for (int i = 0; i < kSmallWG / 64; ++i) t += S.red[i];
    return t;
}

// (a.W / a.L, a.r) < (b.W / b.L, b.r); r < 0: none.
__device__ __forceinline__ bool small_less(long long aw, long long al, int ar, long long bw,
                                           long long bl, int br)
{
    if (br < 0) return ar >= 0;
    if (ar < 0) return false;
    const __int128 x = (__int128)aw * bl, y = (__int128)bw * al;
    if (x != y) return x < y;
    return ar < br;
}

template <typename WT>
__global__ __launch_bounds__(kSmallWG) void k_small_solve(
    const int* __restrict__ list, int nlist, GArrays ga, const int* __restrict__ row_ptr,
    const int* __restrict__ col, const WT* __restrict__ w, int neg, int max_iters,
    int* __restrict__ pi_out, int* __restrict__ succ_out, long long* __restrict__ V_out,
    int* __restrict__ hop_out, unsigned char* __restrict__ onC_out)
{
    __shared__ SmallLds S;
    const int t = threadIdx.x;
    for (int li = blockIdx.x; li < nlist; li += gridDim.x) {
        const int g = list[li];
        const int v0 = (int)ga.vptr[g];
        const int n = (int)(ga.vptr[g + 1] - v0);
        // R1: the lowest-position minimum-weight out-edge
        for (int v = t; v < n; v += kSmallWG) {
            const int b = row_ptr[v0 + v], e1 = row_ptr[v0 + v + 1];
            long long best = 0;
            int arg = -1;
            for (int e = b; e < e1; ++e) {
                const long long x = wval(w, e, neg);
                if (arg < 0 || x < best) {
                    best = x;
                    arg = e;
                }
            }
            S.pi[v] = arg;
            S.succ[v] = (short)(col[arg] - v0);
        }
        int iter = 1, status = OCM_OK, s = 0;
        long long W = 0, L = 1;
        __syncthreads();
        for (;;) {
            if ((max_iters > 0 && iter >= max_iters) || iter >= kSmallIterCap) {
                status = OCM_E_NOT_CONVERGED;
                break;
            }
            // cycles: after K rounds (2^K >= n) J(v) lies on v's cycle and
            // M(J(v)) is that cycle's smallest vertex; the image of J is the
            // set of cycle vertices
            for (int v = t; v < n; v += kSmallWG) {
                S.u.cyc.J[v] = S.succ[v];
                S.u.cyc.M[v] = (short)v;
                S.onc[v] = 0;
            }
            __syncthreads();
            for (int span = 1; span < n; span <<= 1) {
                short nj[kSmallVPT], nm[kSmallVPT];
#pragma unroll
                for (int i = 0; i < kSmallVPT; ++i) {
                    const int v = t + i * kSmallWG;
                    if (v < n) {
                        const int j = S.u.cyc.J[v];
                        nj[i] = S.u.cyc.J[j];
                        const short a = S.u.cyc.M[v], b = S.u.cyc.M[j];
                        nm[i] = a < b ? a : b;
                    }
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < kSmallVPT; ++i) {
                    const int v = t + i * kSmallWG;
                    if (v < n) {
                        S.u.cyc.J[v] = nj[i];
                        S.u.cyc.M[v] = nm[i];
                    }
                }
                __syncthreads();
            }
            for (int v = t; v < n; v += kSmallWG) {
                const int x = S.u.cyc.J[v];
                S.onc[x] = 1;
                S.rep[v] = S.u.cyc.M[x];
            }
            __syncthreads();
            // select: per-cycle (W, L) keyed by the smallest vertex, then
            // the order (W / L, rep)
            for (int v = t; v < n; v += kSmallWG) {
                S.u.sel.wsum[v] = 0;
                S.u.sel.lcnt[v] = 0;
            }
            __syncthreads();
            for (int v = t; v < n; v += kSmallWG)
                if (S.onc[v]) {
                    atomicAdd((unsigned long long*)&S.u.sel.wsum[S.rep[v]],
                              (unsigned long long)wval(w, S.pi[v], neg));
                    atomicAdd(&S.u.sel.lcnt[S.rep[v]], 1);
                }
            __syncthreads();
            {
                long long bw = 0, bl = 1;
                int br = -1;
                for (int v = t; v < n; v += kSmallWG)
                    if (S.onc[v] && S.rep[v] == v &&
                        small_less(S.u.sel.wsum[v], S.u.sel.lcnt[v], v, bw, bl, br)) {
                        bw = S.u.sel.wsum[v];
                        bl = S.u.sel.lcnt[v];
                        br = v;
                    }
                for (int off = 32; off > 0; off >>= 1) {
                    const long long ow = __shfl_xor(bw, off, 64), ol = __shfl_xor(bl, off, 64);
                    const int orr = __shfl_xor(br, off, 64);
                    if (small_less(ow, ol, orr, bw, bl, br)) {
                        bw = ow;
                        bl = ol;
                        br = orr;
                    }
                }
                if ((t & 63) == 0) {
                    S.cw[t >> 6] = bw;
                    S.cl[t >> 6] = bl;
                    S.cr[t >> 6] = br;
                }
                __syncthreads();
                bw = S.cw[0];
                bl = S.cl[0];
                br = S.cr[0];
                for (int i = 1; i < kSmallWG / 64; ++i)
                    if (small_less(S.cw[i], S.cl[i], S.cr[i], bw, bl, br)) {
                        bw = S.cw[i];
                        bl = S.cl[i];
                        br = S.cr[i];
                    }
                s = br;
                W = bw;
                L = bl;
            }
            // rebuild (R5, R6): C's component keeps its edges; round k
            // attaches every other vertex with an out-edge into the vertices
            // attached before round k, by its lowest such edge.  A vertex
            // attached in round k is written at once: the others' test
            // (0 <= layer < k) ignores it either way.
            unsigned long long left = 0;
            for (int v = t; v < n; v += kSmallWG) {
                const bool keep = S.rep[v] == s;
                S.layer[v] = keep ? 0 : -1;
                left += !keep;
            }
            left = small_sum(left, S);
            for (int k = 1; left > 0; ++k) {
                unsigned long long got = 0;
                for (int v = t; v < n; v += kSmallWG) {
                    if (S.layer[v] != -1) continue;
                    const int b = row_ptr[v0 + v], e1 = row_ptr[v0 + v + 1];
                    for (int e = b; e < e1; ++e) {
                        const int x = col[e] - v0;
                        const int ly = S.layer[x];
                        if (ly >= 0 && ly < k) {
                            S.pi[v] = e;
                            S.succ[v] = (short)x;
                            S.layer[v] = (short)k;
                            ++got;
                            break;
                        }
                    }
                }
                got = small_sum(got, S);
                if (got == 0) break;
                left -= got;
            }
            if (left > 0) {
                status = OCM_E_NOT_STRONGLY_CONNECTED;
                break;
            }
            // values (R7) by pointer jumping toward s, one buffer: each
            // round reads into registers, then writes
            for (int v = t; v < n; v += kSmallWG) {
                if (v == s) {
                    S.u.val.D[v] = 0;
                    S.u.val.J[v] = (short)s;
                    S.u.val.H[v] = 0;
                } else {
                    S.u.val.D[v] = L * wval(w, S.pi[v], neg) - W;
                    S.u.val.J[v] = S.succ[v];
                    S.u.val.H[v] = 1;
                }
            }
            unsigned long long ovf = 0;
            bool stuck = false;
            for (int r = 0;; ++r) {
                // every vertex reaches s after the rebuild: ceil(log2 n) + 1
                // rounds suffice; the bound only guarantees an exit
                if (r > 32) {
                    stuck = true;
                    break;
                }
                __syncthreads();
                long long nd[kSmallVPT];
                short nj[kSmallVPT], nh[kSmallVPT];
                unsigned long long act = 0;
#pragma unroll
                for (int i = 0; i < kSmallVPT; ++i) {
                    const int v = t + i * kSmallWG;
                    nj[i] = -1;
                    if (v < n && S.u.val.J[v] != s) {
                        const int j = S.u.val.J[v];
                        long long d;
                        if (__builtin_add_overflow(S.u.val.D[v], S.u.val.D[j], &d)) {
                            d = 0;
                            ovf = 1;
                        }
                        nd[i] = d;
                        nj[i] = S.u.val.J[j];
                        nh[i] = (short)(S.u.val.H[v] + S.u.val.H[j]);
                    }
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < kSmallVPT; ++i) {
                    const int v = t + i * kSmallWG;
                    if (nj[i] >= 0) {
                        S.u.val.D[v] = nd[i];
                        S.u.val.J[v] = nj[i];
                        S.u.val.H[v] = nh[i];
                        act += nj[i] != s;
                    }
                }
                if (small_sum(act, S) == 0) break;
            }
            if (stuck) {
                status = OCM_E_NOT_STRONGLY_CONNECTED;
                break;
            }
            for (int v = t; v < n; v += kSmallWG) {
                const long long d = S.u.val.D[v];
                if (d > kValLimit || d < -kValLimit) ovf = 1;
                S.V[v] = d;
            }
            if (small_sum(ovf, S) != 0) {
                status = OCM_E_OVERFLOW;
                break;
            }
            // improvement sweep (R2): strict improvement, lowest position
            unsigned long long changed = 0;
            for (int v = t; v < n; v += kSmallWG) {
                const int b = row_ptr[v0 + v], e1 = row_ptr[v0 + v + 1];
                long long best = INT64_MAX;
                int arg = -1, bh = 0;
                for (int e = b; e < e1; ++e) {
                    const int x = col[e] - v0;
                    const long long key = S.V[x] + L * wval(w, e, neg) - W;
                    if (key < best) {
                        best = key;
                        arg = e;
                        bh = x;
                    }
                }
                if (best < S.V[v]) {
                    S.pi[v] = arg;
                    S.succ[v] = (short)bh;
                    ++changed;
                }
            }
            ++iter;
            if (small_sum(changed, S) == 0) break;
        }
        // the last value phase's results (the final sweep changed nothing)
        const bool ok = status == OCM_OK;
        for (int v = t; v < n; v += kSmallWG) {
            pi_out[v0 + v] = S.pi[v];
            succ_out[v0 + v] = v0 + S.succ[v];
            if (ok) {
                V_out[v0 + v] = S.V[v];
                hop_out[v0 + v] = S.u.val.H[v];
                onC_out[v0 + v] = (unsigned char)(S.onc[v] && S.rep[v] == s);
            }
        }
        if (t == 0) {
            ga.W[g] = W;
            ga.L[g] = L;
            ga.s[g] = v0 + s;
            ga.iter[g] = iter;
            ga.status[g] = status;
            ga.mode[g] = kDone;
        }
        __syncthreads();   // S is reused by the next graph
    }
}

}  // namespace b
}  // namespace ocm

// ===========================================================================
// host driver
// ===========================================================================
namespace {

using ocm::b::BCtl;
using ocm::b::GArrays;

ocm_status bfail(ocm_status s, const char* what)
{
    ocm::set_last_error(what);
    return s;
}

#define BHIP(expr)                                                                     \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            char b_[256];                                                              \
            snprintf(b_, sizeof b_, "%s: %s", #expr, hipGetErrorString(e_));           \
            return bfail(OCM_E_HIP, b_);                                               \
        }                                                                              \
    } while (0)

#define BTRY(expr)                                                                     \
    do {                                                                               \
        ocm_status s_ = (expr);                                                        \
        if (s_ != OCM_OK) return s_;                                                   \
    } while (0)

size_t bal(size_t x) { return (x + 255) & ~size_t(255); }

struct BWs {
    BCtl* bc;
    GArrays ga;
    int2* chunks;
    long long* cptr;     // G+1 cycle offsets
    long long* V;
    int* V32;            // int32 copy of V (used while every value fits)
    int* pi;
    int* succ;
    void* wsel;          // raw weight of each vertex's policy edge (WT)
    int* hop;
    ocm::b::VJ* Q[2];    // value rounds (the cycle and hop rounds alias them)
    int* rep;
    unsigned char* onc;
    unsigned char* onC;
    long long* wsum;
    unsigned* lcnt;
    int2* heads;
    unsigned* rdeg;
    unsigned* stot;
    int* rin_ptr;
    int* rin;
    void* rscratch;
    unsigned* abits[2];
    unsigned char* marks;
    unsigned char* marks2;      // device-driven rounds: the other round parity's marks
    unsigned char* span_flag;   // rebuild: spans holding a rebuilt graph (flags, then list)
    int* spans;
    unsigned* bad;
    int* small;          // graphs of the small class (solved one per workgroup in LDS)
    void* vctl;          // control block of the validation kernel
    void* sub;           // exact tie test of one graph: its rebased CSR, policy and
    size_t sub_bytes;    //   single-graph workspace (sized for the largest graph)
    size_t total;
};

// Bytes to solve the largest graph of the batch on its own (rebased CSR and
// policy, then ocm_min's workspace).
size_t sub_bytes_for(int64_t max_n, int64_t max_m)
{
    ocm_graph g{max_n, max_m, (const int32_t*)16, (const int32_t*)16, (const void*)16, OCM_W_I64};
    const size_t ws = ocm_workspace_size(&g, nullptr);
    return ws + 4 * (size_t)(max_n + 1) + 4 * (size_t)max_m + 8 * (size_t)max_n + 4 * 256;
}

BWs bcarve(void* base, int64_t G, int64_t n, int64_t m, size_t sub_bytes)
{
    const int T = ocm::b::kMinChunk;
    char* b = (char*)base;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        size_t o = off;
        off += bal(bytes);
        return b ? (void*)(b + o) : nullptr;
    };
    BWs w;
    const size_t Gs = (size_t)G, N = (size_t)n, M = (size_t)m;
    const size_t maxch = N / (size_t)T + Gs + 1;
    w.bc = (BCtl*)take(sizeof(BCtl));
    GArrays& a = w.ga;
    a.W = (long long*)take(8 * Gs);
    a.L = (long long*)take(8 * Gs);
    a.s = (int*)take(4 * Gs);
    a.iter = (int*)take(4 * Gs);
    a.mode = (int*)take(4 * Gs);
    a.status = (int*)take(4 * Gs);
    a.best = (int*)take(4 * Gs);
    a.changed = (unsigned*)take(4 * Gs);
    a.cbroken = (unsigned*)take(4 * Gs);
    a.vrun = (unsigned*)take(4 * Gs);
    a.vact = (unsigned*)take(16 * Gs);
    a.vprog = (unsigned*)take(16 * Gs);
    a.ovf = (unsigned*)take(4 * Gs);
    a.fin = (int*)take(4 * Gs);
    a.have_c = (unsigned char*)take(Gs);
    a.tight = (unsigned long long*)take(8 * Gs);
    a.certain = (unsigned long long*)take(8 * Gs);
    a.nondec = (unsigned long long*)take(8 * Gs);
    a.vptr = (long long*)take(8 * (Gs + 1));
    a.eptr = (long long*)take(8 * (Gs + 1));
    a.ccnt = (unsigned*)take(4 * (Gs + 1));
    a.coff = (unsigned*)take(4 * (Gs + 1));
    a.ctot = (unsigned*)take(4 * ((Gs + 1) / 2048 + 2));
    w.chunks = (int2*)take(8 * maxch);
    w.cptr = (long long*)take(8 * (Gs + 1));
    w.V = (long long*)take(8 * N);
    w.V32 = (int*)take(4 * N);
    w.pi = (int*)take(4 * N);
    w.succ = (int*)take(4 * N);
    w.wsel = take(8 * N);
    w.hop = (int*)take(4 * N);
    static_assert(sizeof(ocm::b::VJ) >= 8, "the 8-byte jump entries alias Q");
    w.Q[0] = (ocm::b::VJ*)take(sizeof(ocm::b::VJ) * N);
    w.Q[1] = (ocm::b::VJ*)take(sizeof(ocm::b::VJ) * N);
    w.rep = (int*)take(4 * N);
    w.onc = (unsigned char*)take(N);
    w.onC = (unsigned char*)take(N);
    w.wsum = (long long*)take(8 * N);
    w.lcnt = (unsigned*)take(4 * N);
    w.heads = (int2*)take(8 * N);
    w.rdeg = (unsigned*)take(4 * (N + 1));
    w.stot = (unsigned*)take(4 * ((N + 1) / 2048 + 2));
    w.rin_ptr = (int*)take(4 * (N + 1));
    w.rin = (int*)take(4 * M);
    w.rscratch = take(ocm::rev_scratch_bytes(n, m));
    w.abits[0] = (unsigned*)take(4 * ((N + 31) / 32 + 1));
    w.abits[1] = (unsigned*)take(4 * ((N + 31) / 32 + 1));
    w.marks = (unsigned char*)take(N + 16);
    w.marks2 = (unsigned char*)take(N + 16);
    const size_t nsp = (size_t)ocm::round_spans((int)n) + 1;
    w.span_flag = (unsigned char*)take(nsp);
    w.spans = (int*)take(4 * nsp);
    w.bad = (unsigned*)take(256);
    w.small = (int*)take(4 * Gs);
    w.vctl = take(sizeof(ocm::Ctl));
    w.sub = take(sub_bytes);
    w.sub_bytes = sub_bytes;
    w.total = off;
    return w;
}

}  // namespace

// Workspace of a batched call with G graphs over n vertices and m edges
// whose largest graph has at most max_n vertices and max_m edges (an upper
// bound of ocm_batched_workspace_size for every such batch).
size_t ocm::batched_ws_bound(int64_t G, int64_t n, int64_t m, int64_t max_n, int64_t max_m)
{
    return bcarve(nullptr, G, n, m, sub_bytes_for(max_n, max_m)).total;
}

namespace {

// The batch schedule: lanes per vertex in the sweeps and vertices per chunk.
struct Schedule {
    int lanes;
    int chunk;
};

int default_lanes(int64_t n, int64_t m)
{
    const double d = (double)m / (double)std::max<int64_t>(n, 1);
    int G = 1;
    while (G < 64 && G < d) G <<= 1;
    return G;
}

struct BCtx {
    int64_t G;
    int n, m;
    const int* row_ptr;
    const int* col;
    const void* w;
    int wtype, sw, neg;
    hipStream_t st;
    BWs ws;
    BCtl h;
    Schedule sch;
    ocm_profile* prof = nullptr;
    bool rev_built = false;
    bool tile_sweep = true;   // improvement sweeps over vertex tiles (else lanes per vertex)
    bool device_rounds = true;   // iterations after the first decide their rounds on the device
    int max_n = 1;
    int64_t loop_G = 0, loop_n = 0;   // graphs and vertices the loop solves (not the small class)
};

ocm_status bread(BCtx& c)
{
    BHIP(ocm::host_read(c.ws.bc, &c.h, sizeof(BCtl), c.st));
    return OCM_OK;
}

// workgroups of a chunked launch: enough for the largest chunk list, at
// most kChunkGrid (the kernels stride over the list)
unsigned chunk_grid(const BCtx& c)
{
    const unsigned most = (unsigned)(c.n / ocm::b::kMinChunk + c.G + 1);
    return most < ocm::b::kChunkGrid ? most : ocm::b::kChunkGrid;
}

unsigned chunk_grid(unsigned nch) { return nch < ocm::b::kChunkGrid ? nch : ocm::b::kChunkGrid; }

// Workgroups of `kernel` that are resident on the device at once, rounded
// down to a multiple of 8 (one per XCD slot): a grid-stride chunk kernel
// launched with at most this many runs in a single wave of workgroups, with
// no tail of late ones (2048 workgroups of a kernel that fits 6 per CU would
// run as 1536 plus a third-full second wave).
unsigned resident_grid(const void* kernel)
{
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, unsigned> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_pair(dev, kernel);
    const auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, ocm::kWG, 0) != hipSuccess ||
        per < 1)
        per = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 8;
    (void)hipGetLastError();
    unsigned g = (unsigned)(per * cus) & ~7u;
    if (g < 8) g = 8;
    cache[key] = g;
    return g;
}

// Grid of a chunk kernel: the chunk bound, at most one resident wave.
unsigned kgrid(unsigned most, const void* kernel)
{
    const unsigned r = resident_grid(kernel);
    return most < r ? most : r;
}

// Chunk list of the graphs in `want` (a mode, -1 = every graph not done,
// -2 = every graph), built on the device; kernels read the count from
// device memory, so nothing here waits for the host.
void enqueue_chunks(BCtx& c, int want, const unsigned* halt = nullptr)
{
    GArrays& a = c.ws.ga;
    const int T = c.sch.chunk;
    if (c.G <= ocm::b::kChunkListOne) {
        ocm::b::k_chunk_list<<<1, ocm::b::kChunkListWG, 0, c.st>>>((int)c.G, a.mode, want, a.vptr, T,
                                                                  c.ws.chunks, &c.ws.bc->nchunks,
                                                                  halt);
        return;
    }
    ocm::b::k_chunk_count<<<ocm::stride_grid(c.G + 1), ocm::kWG, 0, c.st>>>((int)c.G, a.mode, want,
                                                                          a.vptr, T, a.ccnt, halt);
    ocm::launch_exclusive_scan(c.G + 1, a.ccnt, a.coff, a.ctot, c.st);
    ocm::b::k_chunk_fill<<<ocm::stride_grid(c.G), ocm::kWG, 0, c.st>>>((int)c.G, a.ccnt, a.coff,
                                                                     a.vptr, T, c.ws.chunks,
                                                                     &c.ws.bc->nchunks);
}

ocm_status build_chunks(BCtx& c, int want, unsigned* nch_out)
{
    enqueue_chunks(c, want);
    BHIP(hipGetLastError());
    BTRY(bread(c));
    *nch_out = c.h.nchunks;
    return OCM_OK;
}

template <typename WT>
void launch_bsweep_t(BCtx& c, unsigned nch, bool tie, int* xs, int* ys, unsigned* xcnt,
                     unsigned xcap, bool walk)
{
    const WT* w = (const WT*)c.w;
    BWs& ws = c.ws;
    const int T = c.sch.chunk;
#define OCM_BSW(GG)                                                                              \
    case GG:                                                                                     \
        if (tie)                                                                                 \
            ocm::b::k_sweep<GG, WT, true><<<chunk_grid(nch), ocm::kWG, 0, c.st>>>(          \
                ws.chunks, &ws.bc->nchunks, T, ws.ga, c.row_ptr, c.col, w, c.neg, ws.V, ws.pi,   \
                ws.onC, ws.hop, xs, ys, xcnt, xcap, walk ? ws.succ : nullptr, nullptr);          \
        else                                                                                     \
            ocm::b::k_sweep<GG, WT, false><<<chunk_grid(nch), ocm::kWG, 0, c.st>>>(         \
                ws.chunks, &ws.bc->nchunks, T, ws.ga, c.row_ptr, c.col, w, c.neg, ws.V, ws.pi,   \
                ws.onC, ws.hop, nullptr, nullptr, nullptr, 0u, ws.succ, (WT*)ws.wsel);           \
        break;
    switch (c.sch.lanes) {
        OCM_BSW(1)
        OCM_BSW(2)
        OCM_BSW(4)
        OCM_BSW(8)
        OCM_BSW(16)
        OCM_BSW(32)
        OCM_BSW(64)
        default: break;
    }
#undef OCM_BSW
}

// xs / ys / xcnt (tie scans only, may be null): list the tight non-policy
// edges, at most xcap of them (xcnt counts all).  walk (tie scans only):
// also take the short walk from every tight edge that does not lower hop.
void launch_bsweep(BCtx& c, unsigned nch, bool tie, int* xs = nullptr, int* ys = nullptr,
                   unsigned* xcnt = nullptr, unsigned xcap = 0, bool walk = false)
{
    if (nch == 0) return;
    if (c.tile_sweep) {   // improvement sweeps and tie scans over vertex tiles
        BWs& ws = c.ws;
        const int T = c.sch.chunk;
        const unsigned per = (unsigned)((T + ocm::kWG - 1) / ocm::kWG);
        // one workgroup per tile: the list's capacity in tiles
        const unsigned one = (unsigned)(c.n / T + c.G + 1) * per;
#define OCM_BST(WT, TIE, SUCC, WSEL)                                                             \
    ocm::b::k_sweep_tile<WT, TIE><<<one, ocm::kWG, 0, c.st>>>(                                   \
        ws.chunks, &ws.bc->nchunks, T, ws.ga, c.row_ptr, c.col, (const WT*)c.w, c.neg, ws.V,     \
        ws.pi, ws.onC, ws.V32, ws.bc, SUCC, WSEL, ws.hop, xs, ys, xcnt, xcap)
        int* sc = !tie || walk ? ws.succ : nullptr;
        if (c.wtype == OCM_W_I64) {
            if (tie) OCM_BST(long long, true, sc, nullptr);
            else OCM_BST(long long, false, sc, (long long*)ws.wsel);
        } else {
            if (tie) OCM_BST(int, true, sc, nullptr);
            else OCM_BST(int, false, sc, (int*)ws.wsel);
        }
#undef OCM_BST
        return;
    }
    if (c.wtype == OCM_W_I64) launch_bsweep_t<long long>(c, nch, tie, xs, ys, xcnt, xcap, walk);
    else launch_bsweep_t<int>(c, nch, tie, xs, ys, xcnt, xcap, walk);
}


int jump_rounds(const BCtx& c)
{
    int K = 0;
    while ((int64_t(1) << K) < c.max_n) ++K;
    return K;
}

// Values for the graphs in mode `want` with a fixed number of rounds: every
// policy path has fewer than max_n edges, so K = ceil(log2 max_n) rounds
// finish every graph that reaches its source.  kFast graphs that stop
// progressing fall back to the general phases; kGeneral ones fail.
// halt (nullable): nothing runs while *halt is non-zero.
void enqueue_values(BCtx& c, int want, const unsigned* halt = nullptr)
{
    BWs& ws = c.ws;
    GArrays& a = ws.ga;
    const int T = c.sch.chunk;
    const unsigned mc = chunk_grid(c);
    enqueue_chunks(c, want, halt);
    // vrun_round and vlast (the init books round 0)
    ocm::launch_fill_u32(ws.bc->vrun_round, 33, 0u, c.st);
    // the fast path's graphs keep succ and wsel from their sweeps; the
    // general path's were rebuilt
    const bool sel = want == ocm::b::kFast;
#define OCM_BVI(WT, SEL)                                                                        \
    ocm::b::k_val_init<WT, SEL><<<mc, ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, T, a,     \
                                                          c.col, ws.pi, (const WT*)c.w, c.neg,  \
                                                          ws.succ, (WT*)ws.wsel, ws.Q[0], ws.bc)
    if (c.wtype == OCM_W_I64) {
        if (sel) OCM_BVI(long long, true);
        else OCM_BVI(long long, false);
    } else {
        if (sel) OCM_BVI(int, true);
        else OCM_BVI(int, false);
    }
#undef OCM_BVI
    const int R = jump_rounds(c);
    // one resident wave of round workgroups (its registers allow fewer than
    // the chunk grid)
    const unsigned vg = kgrid(chunk_grid(c), (const void*)ocm::b::k_val_round);
    for (int r = 0; r < R; ++r)
        ocm::b::k_val_round<<<vg, ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, T, a, ws.Q[r & 1],
                                                     ws.Q[(r + 1) & 1], want, r, ws.bc);
    ocm::b::k_val_close<<<ocm::stride_grid(c.G), ocm::kWG, 0, c.st>>>((int)c.G, a, want, ws.bc, halt);
    ocm::b::k_val_final<<<mc, ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, T, a, want, ws.Q[0],
                                                   ws.Q[1], ws.V, ws.V32, ws.bc);
    ocm::b::k_values_done<<<ocm::stride_grid(c.G), ocm::kWG, 0, c.st>>>((int)c.G, a, want, halt);
}

// Cycles, exact vote and the start of the rebuild for kGeneral graphs.
void enqueue_general_head(BCtx& c)
{
    BWs& ws = c.ws;
    GArrays& a = ws.ga;
    const int T = c.sch.chunk;
    const unsigned mc = chunk_grid(c);
    enqueue_chunks(c, ocm::b::kGeneral);
    auto* P0 = (unsigned long long*)ws.Q[0];
    auto* P1 = (unsigned long long*)ws.Q[1];
    const int K = jump_rounds(c);
    ocm::b::k_pj_init<<<mc, ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, T, a, ws.succ, P0,
                                                 ws.onc);
    for (int k = 0; k < K; ++k)
        ocm::b::k_pj_round<<<mc, ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, T, a, k,
                                                      k & 1 ? P1 : P0, k & 1 ? P0 : P1);
    ocm::b::k_pj_final<<<mc, ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, T, a, P0, P1, ws.rep,
                                                  ws.onc);
    ocm::b::k_bctl_zero<<<1, 64, 0, c.st>>>(&ws.bc->ncyc, nullptr);
    ocm::b::k_cyc_zero<<<mc, ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, T, a, ws.rep, ws.onc,
                                                  ws.wsum, ws.lcnt, ws.heads, ws.bc);
    if (c.wtype == OCM_W_I64)
        ocm::b::k_cyc_sum<long long><<<mc, ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, T, a,
                                                                ws.rep, ws.onc, ws.pi,
                                                                (const long long*)c.w, c.neg,
                                                                ws.wsum, ws.lcnt);
    else
        ocm::b::k_cyc_sum<int><<<mc, ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, T, a, ws.rep,
                                                          ws.onc, ws.pi, (const int*)c.w, c.neg,
                                                          ws.wsum, ws.lcnt);
    ocm::b::k_vote<<<2048, ocm::kWG, 0, c.st>>>(ws.heads, ws.bc, a, ws.wsum, ws.lcnt);
    ocm::b::k_set_lambda<<<ocm::stride_grid(c.G), ocm::kWG, 0, c.st>>>((int)c.G, a, ws.wsum,
                                                                     ws.lcnt);
    enqueue_chunks(c, ocm::b::kGeneral);   // graphs whose vote failed retired
    // rebuild init: counters and both bitmaps reset (all ones: graphs that
    // are not rebuilt count as attached)
    ocm::Ctl* cc = (ocm::Ctl*)ws.vctl;
    ocm::launch_ctl_clear(cc, ocm::kClrCount, c.st);
    const int64_t words = ((int64_t)c.n + 31) / 32;
    ocm::launch_fill_u32(ws.abits[0], words, 0xffffffffu, c.st);
    ocm::launch_fill_u32(ws.abits[1], words, 0xffffffffu, c.st);
    ocm::b::k_conn_init<<<mc, ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, T, a, ws.rep, ws.onc,
                                                   nullptr, ws.onC, ws.abits[1], ws.abits[0], cc);
    // the rounds visit only the spans that hold a rebuilt graph
    const int64_t span_verts = (int64_t)32 * ocm::kWG * ocm::round_wpt(c.n);
    ocm::b::k_span_flag<<<mc, ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, T, a, span_verts,
                                                   ws.span_flag);
    ocm::b::k_span_list<<<1, ocm::kWG, 0, c.st>>>(ocm::round_spans(c.n), ws.span_flag, ws.spans,
                                                  &ws.bc->nspans);
}

// One iteration up to the rebuild rounds: sweep, retire converged graphs,
// fast-path values, then cycles / vote / rebuild start for the others.
void enqueue_head(BCtx& c, int max_iters, bool fast_path)
{
    BWs& ws = c.ws;
    GArrays& a = ws.ga;
    enqueue_chunks(c, ocm::b::kActive);
    launch_bsweep(c, chunk_grid(c), false);
    ocm::b::k_bctl_zero<<<1, 64, 0, c.st>>>(&ws.bc->nactive, &ws.bc->nfast);
    ocm::b::k_bctl_zero<<<1, 64, 0, c.st>>>(&ws.bc->ngeneral, nullptr);
    ocm::b::k_after_sweep<<<ocm::stride_grid(c.G), ocm::kWG, 0, c.st>>>((int)c.G, a, max_iters,
                                                                      ws.bc);
    if (fast_path) enqueue_values(c, ocm::b::kFast);
    else ocm::b::k_fast_to_general<<<ocm::stride_grid(c.G), ocm::kWG, 0, c.st>>>((int)c.G, a);
    enqueue_general_head(c);
}

// Rebuild rounds over the union after k_conn_init (pull or push per round,
// as in ocm_min); reads the counts back, so it runs outside the graphs.
ocm_status host_connect(BCtx& c)
{
    BWs& ws = c.ws;
    GArrays& a = ws.ga;
    ocm::Ctl* cc = (ocm::Ctl*)ws.vctl;
    ocm::CtlView h;
    BHIP(ocm::host_read_ctl(cc, &h, c.st));
    unsigned left = h.left, front = h.got;
    int k = 0;
    while (left > 0) {
        ++k;
        const bool push = left >= (1u << 16) && (uint64_t)front * 2 < left;
        if (push && !c.rev_built) {
            ocm::launch_rev_build(c.n, c.m, c.row_ptr, c.col, ws.rdeg, ws.stot, ws.rin_ptr, ws.rin,
                                  ws.marks, ws.rscratch, c.st);
            c.rev_built = true;
        }
        const unsigned* acur = ws.abits[k & 1];
        unsigned* anext = ws.abits[(k + 1) & 1];
        ocm::launch_ctl_clear(cc, ocm::kClrCount, c.st);
        if (push) {
            ocm::launch_conn_mark(c.n, ws.rin_ptr, ws.rin, acur, anext, ws.marks, nullptr, ws.spans,
                                  &ws.bc->nspans, c.st);
            ocm::launch_conn_claim(k, c.n, c.row_ptr, c.col, acur, anext, ws.marks, ws.pi, nullptr,
                                   cc, nullptr, ws.spans, &ws.bc->nspans, nullptr, nullptr,
                                   nullptr, nullptr, c.st);
        } else {
            ocm::launch_conn_pull(k, c.n, c.row_ptr, c.col, acur, anext, nullptr, ws.pi, cc,
                                  nullptr, ws.spans, &ws.bc->nspans, nullptr, c.st);
        }
        BHIP(hipGetLastError());
        BHIP(ocm::host_read_ctl(cc, &h, c.st));
        const unsigned got = h.got;
        if (got == 0) {
            // the vertices still outside acur cannot reach their graph's cycle
            ocm::b::k_conn_fail<<<ocm::stride_grid((c.n + 31) / 32), ocm::kWG, 0, c.st>>>(
                (int)c.G, c.n, a.vptr, acur, a);
            BHIP(hipGetLastError());
            break;
        }
        left -= got;
        front = got;
    }
    return OCM_OK;
}

// Rebuild rounds decided on the device (as ocm_min's), over the whole union:
// graphs that are not rebuilt count as attached in both bitmaps.  Round k
// reads abits[k & 1] and completes abits[(k + 1) & 1]; the marks alternate
// the same way.  Pull only (policy 1) while no reverse CSR exists.
// rounds captured in each iteration (12 measured faster than 8 or 16)
constexpr int kLoopRounds = 12;
constexpr unsigned kBPushMin = 1u << 16;

void enqueue_rounds(BCtx& c, int k0, int k1)
{
    BWs& ws = c.ws;
    ocm::Ctl* cc = (ocm::Ctl*)ws.vctl;
    unsigned char* mk[2] = {ws.marks, ws.marks2};
    for (int k = k0; k <= k1; ++k)
        ocm::launch_round(k, c.n, c.row_ptr, c.col, ws.rin_ptr, ws.rin, ws.abits[k & 1],
                          ws.abits[(k + 1) & 1], mk[k & 1], mk[(k + 1) & 1], ws.pi, nullptr, cc,
                          &cc->lane[0].pedges, c.rev_built ? 0 : 1, kBPushMin, c.rev_built,
                          false, c.st);
}

// One whole iteration without a host read: sweep, retirement, fast-path
// values, cycles, vote, rebuild init, kLoopRounds device-driven rounds, the
// failure marks of a round that attached nobody, then the general graphs'
// values -- these only once the rounds are over (the host finishes them
// otherwise, flagged in rounds_open).
void enqueue_iteration(BCtx& c, int max_iters, bool fast_path)
{
    BWs& ws = c.ws;
    ocm::Ctl* cc = (ocm::Ctl*)ws.vctl;
    enqueue_head(c, max_iters, fast_path);
    ocm::launch_round_setup_dev(cc, c.rev_built ? 0 : 1, kBPushMin, c.st);
    enqueue_rounds(c, 1, kLoopRounds);
    ocm::b::k_conn_fail<<<ocm::stride_grid((c.n + 31) / 32), ocm::kWG, 0, c.st>>>(
        (int)c.G, c.n, ws.ga.vptr, ws.abits[0], ws.ga, ws.abits[1], cc);
    ocm::b::k_rounds_open<<<1, 64, 0, c.st>>>(ws.bc, cc);
    enqueue_values(c, ocm::b::kGeneral, &cc->rmode);
}

// Rounds left open by an iteration: queued in batches of 8 until the device
// says the rebuild is over, then the failure marks and the values.
ocm_status finish_rounds(BCtx& c)
{
    BWs& ws = c.ws;
    ocm::Ctl* cc = (ocm::Ctl*)ws.vctl;
    ocm::CtlView h;
    int k = kLoopRounds;
    for (;;) {
        enqueue_rounds(c, k + 1, k + 8);
        k += 8;
        BHIP(hipGetLastError());
        BHIP(ocm::host_read_ctl(cc, &h, c.st));
        if (h.rmode == 0) break;
        if (k > c.n + 8) return bfail(OCM_E_HIP, "rebuild rounds did not finish");
    }
    ocm::b::k_conn_fail<<<ocm::stride_grid((c.n + 31) / 32), ocm::kWG, 0, c.st>>>(
        (int)c.G, c.n, ws.ga.vptr, ws.abits[0], ws.ga, ws.abits[1], cc);
    enqueue_values(c, ocm::b::kGeneral);
    BHIP(hipGetLastError());
    return OCM_OK;
}

// The fixed parts of an iteration as captured hipGraphs: head and tail
// around the host-driven rounds of the first iteration, then whole
// iterations with device-driven rounds.
struct Loop {
    hipStream_t cs = nullptr;
    hipGraphExec_t head = nullptr, tail = nullptr, iter = nullptr;
    ~Loop()
    {
        if (head) (void)hipGraphExecDestroy(head);
        if (tail) (void)hipGraphExecDestroy(tail);
        if (iter) (void)hipGraphExecDestroy(iter);
        if (cs) (void)hipStreamDestroy(cs);
    }
};

template <typename F>
ocm_status capture(BCtx& c, Loop& lp, hipGraphExec_t* out, F&& body)
{
    hipStream_t user = c.st;
    c.st = lp.cs;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(lp.cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        body();
        e = hipStreamEndCapture(lp.cs, &g);
    }
    c.st = user;
    if (e != hipSuccess || !g) {
        (void)hipGetLastError();
        return bfail(OCM_E_HIP, "graph capture failed");
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return bfail(OCM_E_HIP, "graph instantiation failed");
    return OCM_OK;
}

// ---------------------------------------------------------------------------
// autotuner: lanes per vertex and chunk size, timed on the batch itself
// (one sweep plus two jump rounds per candidate) and cached per size class
// ---------------------------------------------------------------------------
struct TuneKey {
    int wtype, gbits, nbits, lanes0;
    bool operator<(const TuneKey& o) const
    {
        if (wtype != o.wtype) return wtype < o.wtype;
        if (gbits != o.gbits) return gbits < o.gbits;
        if (nbits != o.nbits) return nbits < o.nbits;
        return lanes0 < o.lanes0;
    }
};

std::mutex g_tune_mu;
std::map<TuneKey, Schedule> g_tune;
thread_local Schedule g_last_sched = {0, 0};
thread_local int g_last_tuned = 0;

int bits_of(int64_t x)
{
    int b = 0;
    while ((int64_t(1) << b) < x) ++b;
    return b;
}

ocm_status autotune(BCtx& c, Schedule* out, int* tuned)
{
    const int l0 = default_lanes(c.n, c.m);
    // the size class of the graphs the loop solves
    const TuneKey key{c.wtype, bits_of(c.loop_G), bits_of(c.loop_n / std::max<int64_t>(c.loop_G, 1)),
                      l0};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            *out = it->second;
            *tuned = 0;
            return OCM_OK;
        }
    }
    // the improvement sweeps run over vertex tiles, so lanes per vertex only
    // serve the tie scans after the loop: there they follow the mean degree
    std::vector<Schedule> cands;
    for (int l : {l0 / 2, l0, l0 * 2})
        if (l >= 1 && l <= 64 && (!c.tile_sweep || l == l0))
            for (int t : {512, 1024, 2048}) cands.push_back({l, t});
    hipEvent_t e0, e1;
    BHIP(hipEventCreate(&e0));
    BHIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    Schedule best = {l0, 1024};
    BWs& ws = c.ws;
    for (const Schedule& s : cands) {
        c.sch = s;
        enqueue_chunks(c, -2);
        float ms = 0.f;
        for (int rep = 0; rep < 2; ++rep) {
            BHIP(hipEventRecord(e0, c.st));
            launch_bsweep(c, chunk_grid(c), false);   // iteration 0: the first sweep
            auto* P0 = (unsigned long long*)ws.Q[0];
            auto* P1 = (unsigned long long*)ws.Q[1];
            const unsigned mc = chunk_grid(c);
            ocm::b::k_pj_init<<<mc, ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, s.chunk, ws.ga,
                                                         ws.succ, P0, ws.onc);
            ocm::b::k_pj_round<<<mc, ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, s.chunk, ws.ga,
                                                          0, P0, P1);
            ocm::b::k_pj_round<<<mc, ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, s.chunk, ws.ga,
                                                          1, P1, P0);
            BHIP(hipEventRecord(e1, c.st));
            BHIP(hipEventSynchronize(e1));
            float t = 0.f;
            BHIP(hipEventElapsedTime(&t, e0, e1));
            ms = rep == 0 ? t : std::min(ms, t);
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = s;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the timing sweeps touched per-graph counters: start clean
    ocm::b::k_graph_init<<<ocm::stride_grid(c.G), ocm::kWG, 0, c.st>>>((int)c.G, ws.ga);
    BHIP(hipGetLastError());
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = best;
    }
    *out = best;
    *tuned = 1;
    return OCM_OK;
}

long long bgcd(long long a, long long b)
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

// Size of the largest graph's own solve (see sub_bytes_for).
size_t batch_sub_bytes(int64_t G, const int64_t* vptr, const int64_t* eptr)
{
    int64_t mn = 1, mm = 1;
    for (int64_t g = 0; g < G; ++g) {
        mn = std::max<int64_t>(mn, vptr[g + 1] - vptr[g]);
        mm = std::max<int64_t>(mm, eptr[g + 1] - eptr[g]);
    }
    return sub_bytes_for(mn, mm);
}

ocm_status check_batch(int64_t G, const int64_t* vptr, const int64_t* eptr, const ocm_graph* u)
{
    if (G < 1 || !vptr || !eptr || !u) return bfail(OCM_E_INVALID_ARG, "null argument or G < 1");
    if (u->n < 1 || u->m < 1 || u->n >= (int64_t(1) << 31) - 1 || u->m >= (int64_t(1) << 31))
        return bfail(OCM_E_INVALID_ARG, "union sizes out of range");
    if (!u->row_ptr || !u->col || !u->w) return bfail(OCM_E_INVALID_ARG, "null graph array");
    if (u->wtype != OCM_W_I32 && u->wtype != OCM_W_I64) return bfail(OCM_E_INVALID_ARG, "bad wtype");
    if (vptr[0] != 0 || eptr[0] != 0 || vptr[G] != u->n || eptr[G] != u->m)
        return bfail(OCM_E_BAD_CSR, "vptr/eptr do not span the union");
    for (int64_t g = 0; g < G; ++g)
        if (vptr[g + 1] <= vptr[g] || eptr[g + 1] <= eptr[g])
            return bfail(OCM_E_BAD_CSR, "every graph needs at least one vertex and edge");
    return OCM_OK;
}

// Capacity of the first tie scan's edge list: its two arrays and the open
// graphs' copy (four arrays of int32) fit the two jump buffers (24 bytes per
// vertex).
unsigned tie_cap1(const BCtx& c)
{
    return (unsigned)std::min<int64_t>(int64_t(1) << 20, (int64_t)c.n);
}

// Exact uniqueness of the critical cycles of every graph flagged
// OCM_F_TIE_UNCHECKED, together: their tight non-policy edges (taken from the
// first tie scan's list when all of it fit, kx1 <= tie_cap1(c), else listed
// by one more tie scan over their chunks) each give two special vertices;
// each special vertex learns the next special vertex (or its graph's C) on
// its policy path, and the host looks for cycles in that small graph (one
// node c*_g per graph; no edge joins two graphs, so a cycle decides its own
// graph).  *listed = false when the edges do not fit the list (nothing
// decided).
ocm_status union_tie(BCtx& c, const int64_t* vptr, uint32_t* flags, unsigned kx1, bool* listed)
{
    BWs& ws = c.ws;
    GArrays& a = ws.ga;
    const int64_t G = c.G;
    *listed = false;
    std::vector<int> mode(G, ocm::b::kDone);
    for (int64_t g = 0; g < G; ++g)
        if (flags[g] & OCM_F_TIE_UNCHECKED) mode[g] = ocm::b::kTieList;
    BHIP(hipMemcpyAsync(a.mode, mode.data(), 4 * (size_t)G, hipMemcpyHostToDevice, c.st));
    ocm::b::k_bctl_zero<<<1, 64, 0, c.st>>>(&ws.bc->xcnt, &ws.bc->scnt);
    // lists in the (now free) jump buffers
    int* xs;
    int* ys;
    unsigned xcap;
    const unsigned cap1 = tie_cap1(c);
    if (kx1 <= cap1) {
        // the open graphs' share of the first list, behind it
        const int* xs1 = (const int*)ws.Q[0];
        xs = (int*)ws.Q[0] + 2 * (size_t)cap1;
        ys = xs + cap1;
        xcap = cap1;
        if (kx1)
            ocm::b::k_list_open<<<ocm::stride_grid(kx1), ocm::kWG, 0, c.st>>>(
                kx1, xs1, xs1 + cap1, (int)G, a.vptr, a.mode, xs, ys, &ws.bc->xcnt);
    } else {
        xcap = (unsigned)std::min<int64_t>(int64_t(1) << 20, 2 * (int64_t)c.n);
        xs = (int*)ws.Q[0];
        ys = xs + xcap;
        unsigned nch = 0;
        BTRY(build_chunks(c, ocm::b::kTieList, &nch));
        launch_bsweep(c, nch, true, xs, ys, &ws.bc->xcnt, xcap);
    }
    BHIP(hipGetLastError());
    BTRY(bread(c));
    const unsigned kx = c.h.xcnt;
    if (kx > xcap) return OCM_OK;
    // special vertices: endpoints of the listed edges (marks, rep, heads and
    // lcnt are free after the loop)
    unsigned char* sp = ws.marks;
    int* spid = ws.rep;
    int* slist = (int*)ws.heads;
    int* P = (int*)ws.lcnt;
    ocm::launch_tie_special(c.n, kx, xs, ys, ws.succ, ws.onC, sp, spid, slist, &ws.bc->scnt, c.st);
    BHIP(hipGetLastError());
    BTRY(bread(c));
    const unsigned ns = c.h.scnt;
    std::vector<int> hx(kx), hy(kx), hs(ns), hp(ns);
    if (kx) {
        BHIP(hipMemcpyAsync(hx.data(), xs, 4 * (size_t)kx, hipMemcpyDeviceToHost, c.st));
        BHIP(hipMemcpyAsync(hy.data(), ys, 4 * (size_t)kx, hipMemcpyDeviceToHost, c.st));
    }
    // the walk's own endpoint conversion is not used (xs / ys stay vertices)
    ocm::launch_tie_walk(c.n, ns, slist, ws.succ, sp, ws.onC, spid, P, 0, nullptr, nullptr, c.st);
    if (ns) {
        BHIP(hipMemcpyAsync(hs.data(), slist, 4 * (size_t)ns, hipMemcpyDeviceToHost, c.st));
        BHIP(hipMemcpyAsync(hp.data(), P, 4 * (size_t)ns, hipMemcpyDeviceToHost, c.st));
    }
    BHIP(hipStreamSynchronize(c.st));
    auto graph_of = [&](int v) {
        return (int64_t)(std::upper_bound(vptr, vptr + G + 1, (int64_t)v) - vptr) - 1;
    };
    std::map<int, int> id;   // special vertex -> index
    for (unsigned i = 0; i < ns; ++i) id[hs[i]] = (int)i;
    // nodes: special vertices 0..ns-1 (one on C stands for its graph's c*),
    // then c*_g = ns + g
    auto node = [&](int v) -> int64_t {
        const auto it = id.find(v);
        if (it == id.end()) return -1;
        const int i = it->second;
        return hp[i] == -2 ? (int64_t)ns + graph_of(v) : (int64_t)i;
    };
    const int64_t N = (int64_t)ns + G;
    std::vector<std::vector<int64_t>> adj(N);
    for (unsigned i = 0; i < ns; ++i) {
        if (hp[i] == -2) continue;
        if (hp[i] == -3) return bfail(OCM_E_HIP, "policy path does not reach the critical cycle");
        adj[i].push_back(hp[i] == -1 ? (int64_t)ns + graph_of(hs[i]) : node(hs[hp[i]]));
    }
    for (unsigned i = 0; i < kx; ++i) {
        const int64_t x = node(hx[i]), y = node(hy[i]);
        if (x < 0 || y < 0) return bfail(OCM_E_HIP, "tie list endpoint without a special index");
        adj[x].push_back(y);
    }
    // three-colour depth-first search; a back edge marks its graph
    std::vector<unsigned char> colr(N, 0);
    std::vector<unsigned char> tie(G, 0);
    std::vector<std::pair<int64_t, size_t>> st;
    auto graph_of_node = [&](int64_t x) { return x >= (int64_t)ns ? x - (int64_t)ns : graph_of(hs[x]); };
    for (int64_t r = 0; r < N; ++r) {
        if (colr[r]) continue;
        colr[r] = 1;
        st.push_back({r, 0});
        while (!st.empty()) {
            auto& top = st.back();
            if (top.second == adj[top.first].size()) {
                colr[top.first] = 2;
                st.pop_back();
                continue;
            }
            const int64_t u = adj[top.first][top.second++];
            if (colr[u] == 1) tie[graph_of_node(u)] = 1;
            else if (colr[u] == 0) {
                colr[u] = 1;
                st.push_back({u, 0});
            }
        }
    }
    for (int64_t g = 0; g < G; ++g)
        if (flags[g] & OCM_F_TIE_UNCHECKED)
            flags[g] = (flags[g] & ~(uint32_t)OCM_F_TIE_UNCHECKED) | (tie[g] ? OCM_F_TIE : 0u);
    *listed = true;
    return OCM_OK;
}

// Exact uniqueness of graph g's critical cycle: graph g rebased into the
// workspace's sub region and solved alone from its final policy; *f gets
// that solve's OCM_F_TIE / OCM_F_TIE_UNCHECKED.
ocm_status exact_tie(BCtx& c, int64_t g, const int64_t* vptr, const int64_t* eptr, long long W,
                     long long L, uint32_t* f)
{
    const int64_t v0 = vptr[g], e0 = eptr[g];
    const int n = (int)(vptr[g + 1] - v0), m = (int)(eptr[g + 1] - e0);
    char* b = (char*)c.ws.sub;
    int* rp = (int*)b;
    int* cl = (int*)(b + bal(4 * (size_t)(n + 1)));
    int* pol = (int*)((char*)cl + bal(4 * (size_t)m));
    int32_t* cyc = (int32_t*)((char*)pol + bal(4 * (size_t)n));
    char* ws = (char*)cyc + bal(4 * (size_t)n);
    const size_t ws_bytes = c.ws.sub_bytes - (size_t)(ws - b);
    ocm::b::k_rebase<<<ocm::stride_grid(m + 1), ocm::kWG, 0, c.st>>>(
        n, m, c.row_ptr + v0, c.col + e0, c.ws.pi + v0, (int)v0, (int)e0, rp, cl, pol);
    BHIP(hipGetLastError());
    ocm_graph sg{n, m, rp, cl, (const char*)c.w + (size_t)c.sw * (size_t)e0, c.wtype};
    ocm_options o;
    ocm_default_options(&o);
    o.validate = 0;
    o.init_policy = pol;
    ocm_result r;
    const ocm_status rc = (c.neg ? ocm_max : ocm_min)(&sg, &o, ws, ws_bytes, cyc, n, &r, c.st);
    if (rc != OCM_OK) return rc;
    // the same optimum (W, L), from the same policy
    if (r.W != (c.neg ? -W : W) || r.L != L) return bfail(OCM_E_HIP, "tie test solved another optimum");
    *f = r.flags & (OCM_F_TIE | OCM_F_TIE_UNCHECKED);
    return OCM_OK;
}

ocm_status solve_batched(int64_t G, const int64_t* vptr, const int64_t* eptr, const ocm_graph* u,
                         const ocm_options* o_in, void* wsp, size_t ws_bytes, int64_t* p,
                         int64_t* q, int64_t* cycle_ptr, int32_t* cycle_edges, int64_t cycle_cap,
                         int32_t* iters, uint32_t* flags, int32_t* status, void* stream, int neg)
{
    BTRY(check_batch(G, vptr, eptr, u));
    if (!p || !q || !cycle_ptr || !iters || !flags) return bfail(OCM_E_INVALID_ARG, "null output");
    ocm_options o;
    if (o_in) o = *o_in;
    else ocm_default_options(&o);
    if (o.init_policy) return bfail(OCM_E_INVALID_ARG, "warm start is not supported in batches");
    if (o.multichain) return bfail(OCM_E_INVALID_ARG, "multichain is not supported in batches");
    // a chunk's vertices are listed through an LDS buffer of kListItems
    if (o.tile != 0 && (o.tile < ocm::b::kMinChunk || o.tile > ocm::kListItems))
        return bfail(OCM_E_INVALID_ARG, "tile must be 0 or in [512, 4096]");
    BCtx c;
    c.G = G;
    c.n = (int)u->n;
    c.m = (int)u->m;
    c.row_ptr = u->row_ptr;
    c.col = u->col;
    c.w = u->w;
    c.wtype = u->wtype;
    c.sw = u->wtype == OCM_W_I64 ? 8 : 4;
    c.neg = neg;
    c.st = (hipStream_t)stream;
    c.sch.lanes = o.schedule > 0 ? o.schedule : default_lanes(u->n, u->m);
    c.tile_sweep = o.schedule <= 0;
    c.sch.chunk = 1024;
    if (!(c.sch.lanes == 1 || c.sch.lanes == 2 || c.sch.lanes == 4 || c.sch.lanes == 8 ||
          c.sch.lanes == 16 || c.sch.lanes == 32 || c.sch.lanes == 64))
        return bfail(OCM_E_INVALID_ARG, "schedule must be a power of two <= 64");
    for (int64_t g = 0; g < G; ++g) c.max_n = (int)std::max<int64_t>(c.max_n, vptr[g + 1] - vptr[g]);
    const size_t sub = batch_sub_bytes(G, vptr, eptr);
    c.ws = bcarve(nullptr, G, u->n, u->m, sub);
    if (!wsp || ws_bytes < c.ws.total) return bfail(OCM_E_WORKSPACE, "workspace missing or too small");
    c.ws = bcarve(wsp, G, u->n, u->m, sub);
    BWs& ws = c.ws;
    GArrays& a = ws.ga;

    ocm::b::k_bctl_clear<<<1, 64, 0, c.st>>>(ws.bc);
    ocm::launch_fill_u8(ws.span_flag, ocm::round_spans(c.n) + 1, 0, c.st);
    ocm::launch_fill_u8(ws.marks, (int64_t)c.n + 16, 0, c.st);
    ocm::launch_fill_u8(ws.marks2, (int64_t)c.n + 16, 0, c.st);
    BHIP(hipMemcpyAsync(a.vptr, vptr, 8 * (size_t)(G + 1), hipMemcpyHostToDevice, c.st));
    BHIP(hipMemcpyAsync(a.eptr, eptr, 8 * (size_t)(G + 1), hipMemcpyHostToDevice, c.st));
    ocm::b::k_graph_init<<<ocm::stride_grid(G), ocm::kWG, 0, c.st>>>((int)G, a);
    BHIP(hipGetLastError());

    // validation: the union's CSR, the weight bound, and edges inside graphs
    {
        ocm::Ctl* vctl = (ocm::Ctl*)ws.vctl;
        ocm::launch_ctl_clear(vctl, ocm::kClrAll | ocm::kClrCount | ocm::kClrChanged, c.st);
        ocm::launch_validate(c.n, c.m, c.row_ptr, c.col, c.w, c.wtype, o.validate != 0, vctl, c.st);
        ocm::CtlView hc;
        BHIP(ocm::host_read_ctl(vctl, &hc, c.st));
        if (hc.err & ocm::kErrBadCsr) return bfail(OCM_E_BAD_CSR, "malformed CSR");
        if (hc.err & ocm::kErrNoOut) return bfail(OCM_E_NO_OUT_EDGE, "a vertex has no out-edge");
        const unsigned __int128 bound = (unsigned __int128)2 * (unsigned)c.max_n * hc.maxabsw;
        if (bound >= ((unsigned __int128)1 << 62))
            return bfail(OCM_E_OVERFLOW, "weights too large for int64 values");
        if (o.validate) {
            unsigned nch = 0;
            BTRY(build_chunks(c, -1, &nch));
            ocm::b::k_bctl_zero<<<1, 64, 0, c.st>>>(&ws.bc->overflow, nullptr);
            ocm::b::k_check_union<<<chunk_grid(nch), ocm::kWG, 0, c.st>>>((int)G, a.vptr, a.eptr, c.row_ptr, c.col,
                                                              ws.chunks, &ws.bc->nchunks,
                                                              c.sch.chunk, &ws.bc->overflow);
            BHIP(hipGetLastError());
            BTRY(bread(c));
            if (c.h.overflow) return bfail(OCM_E_BAD_CSR, "an edge leaves its graph");
        }
    }

    // size classes: graphs of at most kSmallN vertices and kSmallM edges are
    // solved one per workgroup in LDS (OCM_BATCH_SMALL=0 sends them through
    // the loop too; same results), the others by the loop
    std::vector<int> small;
    {
        const char* se = getenv("OCM_BATCH_SMALL");
        const bool use_small = !(se && se[0] == '0');
        for (int64_t g = 0; g < G; ++g) {
            const int64_t ng = vptr[g + 1] - vptr[g];
            if (use_small && ng <= ocm::b::kSmallN && eptr[g + 1] - eptr[g] <= ocm::b::kSmallM) {
                small.push_back((int)g);
            } else {
                ++c.loop_G;
                c.loop_n += ng;
            }
        }
    }

    // schedule of the loop: given (lanes, tile), or autotuned and cached per
    // size class
    int tuned = 0;
    if ((o.schedule <= 0 || o.tile <= 0) && c.loop_G > 0) {
        Schedule t;
        BTRY(autotune(c, &t, &tuned));
        if (o.schedule <= 0) c.sch.lanes = t.lanes;
        if (o.tile <= 0) c.sch.chunk = t.chunk;
    }
    if (o.tile > 0) c.sch.chunk = o.tile;
    g_last_sched = {c.sch.lanes, c.sch.chunk};
    g_last_tuned = tuned;

    // the small class, before the loop (which then leaves them alone: they
    // are done)
    if (!small.empty()) {
        const int ns = (int)small.size();
        BHIP(hipMemcpyAsync(ws.small, small.data(), 4 * (size_t)ns, hipMemcpyHostToDevice, c.st));
        const void* kern = c.wtype == OCM_W_I64 ? (const void*)ocm::b::k_small_solve<long long>
                                                : (const void*)ocm::b::k_small_solve<int>;
        int per = 0, cus = 0, dev = 0;
        (void)hipGetDevice(&dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, ocm::b::kSmallWG, 0) != hipSuccess ||
            per < 1)
            per = 1;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus < 1)
            cus = 8;
        (void)hipGetLastError();
        const unsigned grid = (unsigned)std::min<int64_t>(ns, (int64_t)per * cus);
        if (c.wtype == OCM_W_I64)
            ocm::b::k_small_solve<long long><<<grid, ocm::b::kSmallWG, 0, c.st>>>(
                ws.small, ns, a, c.row_ptr, c.col, (const long long*)c.w, neg, o.max_iters, ws.pi,
                ws.succ, ws.V, ws.hop, ws.onC);
        else
            ocm::b::k_small_solve<int><<<grid, ocm::b::kSmallWG, 0, c.st>>>(
                ws.small, ns, a, c.row_ptr, c.col, (const int*)c.w, neg, o.max_iters, ws.pi,
                ws.succ, ws.V, ws.hop, ws.onC);
        BHIP(hipGetLastError());
    }

    // iterations: [head graph] -> host rebuild rounds -> [tail graph]
    const char* env = getenv("OCM_BATCH_GRAPH");
    const bool use_graph = !(env && env[0] == '0');
    Loop lp;
    if (use_graph) {
        BHIP(hipStreamCreate(&lp.cs));
        BTRY(capture(c, lp, &lp.head, [&] { enqueue_head(c, o.max_iters, o.fast_path != 0); }));
        BTRY(capture(c, lp, &lp.tail, [&] { enqueue_values(c, ocm::b::kGeneral); }));
    }
    // the first iteration (every graph rebuilds) with host-driven rounds,
    // which build the reverse CSR when push rounds pay; then whole
    // iterations with device-driven rounds, one host read each
    for (int guard = 0;; ++guard) {
        if (guard > (1 << 20)) return bfail(OCM_E_NOT_CONVERGED, "iteration guard");
        if (guard == 0 || !c.device_rounds) {
            if (use_graph) BHIP(hipGraphLaunch(lp.head, c.st));
            else enqueue_head(c, o.max_iters, o.fast_path != 0);
            BHIP(hipGetLastError());
            BTRY(bread(c));
            if (c.h.nactive == 0) break;   // every graph converged or failed
            BTRY(host_connect(c));
            if (use_graph) BHIP(hipGraphLaunch(lp.tail, c.st));
            else enqueue_values(c, ocm::b::kGeneral);
            BHIP(hipGetLastError());
            continue;
        }
        if (use_graph && !lp.iter)
            BTRY(capture(c, lp, &lp.iter, [&] { enqueue_iteration(c, o.max_iters, o.fast_path != 0); }));
        if (use_graph) BHIP(hipGraphLaunch(lp.iter, c.st));
        else enqueue_iteration(c, o.max_iters, o.fast_path != 0);
        BHIP(hipGetLastError());
        BTRY(bread(c));
        if (c.h.nactive == 0) break;
        if (c.h.rounds_open) BTRY(finish_rounds(c));
    }

    // hops to the source for every solved graph (the small class's are
    // recomputed, equal), then the per-graph results
    {
        unsigned nch = 0;
        BTRY(build_chunks(c, -2, &nch));
        if (nch > 0) {
            const int T = c.sch.chunk;
            const unsigned mc = chunk_grid(nch);
            auto* P0 = (unsigned long long*)ws.Q[0];
            auto* P1 = (unsigned long long*)ws.Q[1];
            const int R = jump_rounds(c);
            ocm::launch_fill_u32(ws.bc->hop_act, 34, 0u, c.st);
            ocm::launch_fill_u32(ws.bc->hop_act, 1, 1u, c.st);
            ocm::b::k_hop_init<<<mc, ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, T, a, ws.succ,
                                                          P0);
            for (int r = 0; r < R; ++r)
                ocm::b::k_hop_round<<<mc, ocm::kWG, 0, c.st>>>(
                    ws.chunks, &ws.bc->nchunks, T, a, r & 1 ? P1 : P0, r & 1 ? P0 : P1,
                    &ws.bc->hop_act[r], &ws.bc->hop_act[r + 1]);
            ocm::b::k_hop_final<<<mc, ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, T, a, P0,
                                                           P1, ws.bc->hop_act, R, ws.hop);
            BHIP(hipGetLastError());
        }
    }
    std::vector<long long> hW(G), hL(G);
    std::vector<int> hs(G), hit(G), hst(G);
    BHIP(hipMemcpyAsync(hW.data(), a.W, 8 * (size_t)G, hipMemcpyDeviceToHost, c.st));
    BHIP(hipMemcpyAsync(hL.data(), a.L, 8 * (size_t)G, hipMemcpyDeviceToHost, c.st));
    BHIP(hipMemcpyAsync(hs.data(), a.s, 4 * (size_t)G, hipMemcpyDeviceToHost, c.st));
    BHIP(hipMemcpyAsync(hit.data(), a.iter, 4 * (size_t)G, hipMemcpyDeviceToHost, c.st));
    BHIP(hipMemcpyAsync(hst.data(), a.status, 4 * (size_t)G, hipMemcpyDeviceToHost, c.st));
    BHIP(hipStreamSynchronize(c.st));
    std::vector<long long> cptr(G + 1, 0);
    ocm_status first_err = OCM_OK;
    for (int64_t g = 0; g < G; ++g) {
        const bool ok = hst[g] == OCM_OK;
        cptr[g + 1] = cptr[g] + (ok ? hL[g] : 0);
        if (!ok && first_err == OCM_OK) first_err = (ocm_status)hst[g];
        const long long W = hW[g], L = hL[g];
        const long long gg = ok ? bgcd(W, L) : 1;
        p[g] = ok ? (neg ? -W : W) / gg : 0;
        q[g] = ok ? L / gg : 0;
        iters[g] = hit[g];
        flags[g] = 0;
        if (status) status[g] = hst[g];
        cycle_ptr[g] = cptr[g];
    }
    cycle_ptr[G] = cptr[G];
    if (cycle_cap < cptr[G]) return bfail(OCM_E_CAPACITY, "cycle_cap smaller than the cycles");
    if (cptr[G] > 0 && !cycle_edges) return bfail(OCM_E_INVALID_ARG, "cycle_edges is null");
    BHIP(hipMemcpyAsync(ws.cptr, cptr.data(), 8 * (size_t)(G + 1), hipMemcpyHostToDevice, c.st));
    {
        // every graph; the kernels skip failed ones
        unsigned nch = 0;
        BTRY(build_chunks(c, -2, &nch));
        if (nch == 0) nch = 1;
        ocm::b::k_cycle_list<<<chunk_grid(nch), ocm::kWG, 0, c.st>>>(ws.chunks, &ws.bc->nchunks, c.sch.chunk, a,
                                                         ws.cptr, ws.onC, ws.pi, ws.hop, cycle_edges);
        if (o.tie_check) {
            ocm::b::k_tie_init<<<ocm::stride_grid(G), ocm::kWG, 0, c.st>>>((int)G, a);
            ocm::b::k_bctl_zero<<<1, 64, 0, c.st>>>(&ws.bc->xcnt, nullptr);
            const unsigned cap1 = tie_cap1(c);
            launch_bsweep(c, nch, true, (int*)ws.Q[0], (int*)ws.Q[0] + cap1, &ws.bc->xcnt, cap1, true);
            unsigned kx1 = 0;
            BHIP(hipMemcpyAsync(&kx1, &ws.bc->xcnt, 4, hipMemcpyDeviceToHost, c.st));
            std::vector<unsigned long long> ht(G), hc(G), hn(G);
            BHIP(hipMemcpyAsync(ht.data(), a.tight, 8 * (size_t)G, hipMemcpyDeviceToHost, c.st));
            BHIP(hipMemcpyAsync(hc.data(), a.certain, 8 * (size_t)G, hipMemcpyDeviceToHost, c.st));
            BHIP(hipMemcpyAsync(hn.data(), a.nondec, 8 * (size_t)G, hipMemcpyDeviceToHost, c.st));
            BHIP(hipStreamSynchronize(c.st));
            for (int64_t g = 0; g < G; ++g) {
                if (hst[g] != OCM_OK || ht[g] == 0) continue;
                flags[g] |= OCM_F_TIGHT_EDGES;
                if (hc[g]) flags[g] |= OCM_F_TIE;
                else if (hn[g]) flags[g] |= OCM_F_TIE_UNCHECKED;
            }
            // graphs the quick tests left open: the special-vertex test over
            // all of them at once; if their tight edges do not fit the list,
            // each is solved again on its own (warm started from its final
            // policy), whose full test decides
            bool open = false;
            for (int64_t g = 0; g < G; ++g) open |= (flags[g] & OCM_F_TIE_UNCHECKED) != 0;
            bool listed = false;
            if (open) BTRY(union_tie(c, vptr, flags, kx1, &listed));
            if (open && !listed)
                for (int64_t g = 0; g < G; ++g)
                    if (flags[g] & OCM_F_TIE_UNCHECKED) {
                        uint32_t f = 0;
                        BTRY(exact_tie(c, g, vptr, eptr, hW[g], hL[g], &f));
                        flags[g] = (flags[g] & ~(uint32_t)OCM_F_TIE_UNCHECKED) | f;
                    }
        } else {
            for (int64_t g = 0; g < G; ++g) flags[g] |= OCM_F_TIE_UNCHECKED;
        }
        BHIP(hipGetLastError());
    }
    BHIP(hipStreamSynchronize(c.st));
    if (first_err != OCM_OK) return bfail(first_err, "some graphs failed (see status)");
    return OCM_OK;
}

}  // namespace

extern "C" {

size_t ocm_batched_workspace_size(int64_t G, const int64_t* vptr, const int64_t* eptr,
                                  const ocm_graph* u, const ocm_options* o)
{
    (void)o;
    if (check_batch(G, vptr, eptr, u) != OCM_OK) return 0;
    return bcarve(nullptr, G, u->n, u->m, batch_sub_bytes(G, vptr, eptr)).total;
}

ocm_status ocm_min_batched(int64_t G, const int64_t* vptr, const int64_t* eptr, const ocm_graph* u,
                           const ocm_options* o, void* ws, size_t ws_bytes, int64_t* p, int64_t* q,
                           int64_t* cycle_ptr, int32_t* cycle_edges, int64_t cycle_cap,
                           int32_t* iters, uint32_t* flags, int32_t* status, void* stream)
{
    return solve_batched(G, vptr, eptr, u, o, ws, ws_bytes, p, q, cycle_ptr, cycle_edges, cycle_cap,
                         iters, flags, status, stream, 0);
}

ocm_status ocm_max_batched(int64_t G, const int64_t* vptr, const int64_t* eptr, const ocm_graph* u,
                           const ocm_options* o, void* ws, size_t ws_bytes, int64_t* p, int64_t* q,
                           int64_t* cycle_ptr, int32_t* cycle_edges, int64_t cycle_cap,
                           int32_t* iters, uint32_t* flags, int32_t* status, void* stream)
{
    return solve_batched(G, vptr, eptr, u, o, ws, ws_bytes, p, q, cycle_ptr, cycle_edges, cycle_cap,
                         iters, flags, status, stream, 1);
}

void ocm_batched_last_schedule(int32_t* lanes, int32_t* tile, int32_t* tuned)
{
    if (lanes) *lanes = g_last_sched.lanes;
    if (tile) *tile = g_last_sched.chunk;
    if (tuned) *tuned = g_last_tuned;
}

}  // extern "C"
