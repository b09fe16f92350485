// Multichain policy iteration on the device: the alternative to the rebuild
// of Alg. 2 in which every cycle of the policy graph keeps its own gain
// lambda_r = W_r / L_r (W_r, L_r: weight and length of the cycle whose
// smallest vertex is r).  A vertex takes the gain of the cycle its policy
// path reaches and a value scaled by that cycle's length: V(r) = 0, V(v) =
// V(succ v) + L_r * w(pi v) - W_r.  The edge v -> u offers the pair (gain of
// u, bias (V(u) + L_u * w - W_u) / L_u); the sweep moves v to the
// lowest-position edge with the lexicographically smallest pair when that
// pair is strictly below v's own (gain of v, V(v) / L_v).  Pairs are compared
// by int128 cross products.  The cycle phase and the per-cycle sums are the
// single-gain solver's; there are no rebuild rounds.
#include <climits>

#include "kernels.h"
#include "device_util.h"

namespace ocm {

namespace {

// Sign of (gw / gl, b / gl) - (hw / hl, c / hl) in lexicographic order; gl,
// hl > 0.
// Branch-free: both cross products are formed, then selected.
__device__ __forceinline__ int mc_cmp(long long gw, long long gl, long long b, long long hw,
                                      long long hl, long long c)
{
    const __int128 x = (__int128)gw * hl, y = (__int128)hw * gl;
    const __int128 p = (__int128)b * hl, q = (__int128)c * gl;
    const int sg = (int)(x > y) - (int)(x < y), sb = (int)(p > q) - (int)(p < q);
    return sg != 0 ? sg : sb;
}

template <typename WT>
__global__ __launch_bounds__(kWG) void k_mc_val_init(int n, const int* __restrict__ col,
                                                     const int* __restrict__ pi,
                                                     const WT* __restrict__ w, int neg,
                                                     const int* __restrict__ rep,
                                                     const unsigned char* __restrict__ onc,
                                                     const long long* __restrict__ wsum,
                                                     const unsigned* __restrict__ lcnt,
                                                     int* __restrict__ succ, int have_succ,
                                                     Jmp* __restrict__ Q, Ctl* ctl)
{
    unsigned long long act = 0;
    constexpr int U = 4;   // independent vertices in flight per thread
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t vb = (int64_t)blockIdx.x * kWG + threadIdx.x; vb < n; vb += U * stride) {
        int e[U], t[U], r[U];
        bool root[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t v = vb + u * stride;
            e[u] = v < n ? pi[v] : 0;
            r[u] = v < n ? rep[v] : 0;
            root[u] = v < n && onc[v] && r[u] == v;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t v = vb + u * stride;
            if (v >= n) continue;
            t[u] = have_succ ? succ[v] : col[e[u]];
            if (!have_succ) succ[v] = t[u];
            Jmp q;
            if (root[u]) {
                q.D = 0;
                q.J = ~(int)v;
                q.H = 0;
            } else {
                // |L_r * w - W_r| <= 2 n max|w| < 2^62 (validated)
                q.D = (long long)lcnt[r[u]] * wval(w, e[u], neg) - wsum[r[u]];
                q.J = t[u];
                q.H = 1;
                act += 1;
            }
            Q[v] = q;
        }
    }
    act = block_sum_u64(act);
    if (threadIdx.x == 0 && act) atomicAdd(&my_lane(ctl).active, (unsigned)act);
}

// One jump round: an unfinished entry (J >= 0) takes the entry of the vertex
// it points at; a root's entry (J < 0, D = 0, H = 0) finishes it.
__global__ __launch_bounds__(kWG) void k_mc_round_dev(int n, int r, const Jmp* __restrict__ Qin,
                                                      Jmp* __restrict__ Qout, Ctl* ctl)
{
    if (!jump_round_is(ctl, r)) return;
    constexpr int U = 4;
    unsigned long long act = 0;
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t v0 = (int64_t)blockIdx.x * kWG + threadIdx.x; v0 < n; v0 += U * stride) {
        Jmp q[U], p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t v = v0 + u * stride;
            q[u].J = -1;
            if (v < n) q[u] = Qin[v];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (q[u].J >= 0) p[u] = Qin[q[u].J];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t v = v0 + u * stride;
            if (v >= n) continue;
            if (q[u].J >= 0) {
                q[u] = jmp_combine(q[u], p[u]);
                act += q[u].J >= 0;
            }
            Qout[v] = q[u];
        }
    }
    act = block_sum_u64(act);
    if (threadIdx.x != 0) return;
    unsigned long long tot;
    if (!last_arrival(ctl, arrival_word(act, 0), &tot)) return;
    const unsigned now = (unsigned)tot;
    ctl->jk = (unsigned)r;
    if (now == 0) {
        ctl->jmode = 0;
    } else if (now == ctl->jlast) {
        ctl->jstall = 1;   // no entry finished: cannot happen on a policy graph
        ctl->jmode = 0;
    } else {
        ctl->jlast = now;
    }
}

__global__ __launch_bounds__(kWG) void k_mc_final_dev(int n, Jmp* __restrict__ Q0,
                                                      Jmp* __restrict__ Q1,
                                                      long long* __restrict__ V,
                                                      int* __restrict__ hop, Ctl* ctl)
{
    if (ctl->jmode != 0 || ctl->jstall || !ctl->jgate) return;
    Jmp* Q = (ctl->jk & 1) ? Q1 : Q0;
    const int v = blockIdx.x * kWG + threadIdx.x;
    unsigned bad = 0;
    if (v < n) {
        Jmp q = Q[v];
        bad = (q.H & kHopOverflow) || q.D > kValLimit || q.D < -kValLimit;
        q.J = ~q.J;
        q.H &= ~kHopOverflow;
        V[v] = q.D;
        hop[v] = (int)q.H;
        Q[v] = q;
    }
    if (__ballot(bad != 0) && (threadIdx.x & 63) == 0) atomicOr(&my_lane(ctl).overflow, 1u);
}

// G lanes per vertex; each lane walks positions e0 + lane, e0 + lane + G, ...
// so a strict compare keeps its lowest position among equal pairs, and the
// lanes' bests merge with ties to the lower position.
template <typename WT, int G, bool TIE>
__global__ __launch_bounds__(kWG) void k_mc_sweep(McArgs a, const WT* __restrict__ w)
{
    constexpr int VPB = kWG / G;
    const int lane = threadIdx.x & (G - 1);
    const int64_t stride = (int64_t)gridDim.x * VPB;
    unsigned long long cnt = 0, certain = 0, nondec = 0, changed = 0;
    // every thread of the workgroup runs the same passes (the shuffles)
    for (int64_t vb = (int64_t)xcd_block(blockIdx.x, gridDim.x) * VPB; vb < a.n; vb += stride) {
        const int64_t v = vb + threadIdx.x / G;
        long long bw = 0, bl = 1, bb = 0;
        int pos = INT_MAX, bh = 0;
        long long ow = 0, ol = 1, od = 0;
        int cur = -1;
        if (v < a.n) {
            const int e0 = a.row_ptr[v], e1 = a.row_ptr[v + 1];
            const Jmp own = a.R[v];
            ow = a.wsum[own.J];
            ol = (long long)a.lcnt[own.J];
            od = own.D;
            cur = a.pi[v];
            const bool opt = !TIE || (__int128)ow * a.L == (__int128)a.W * ol;
            const bool on_c = TIE && a.onC[v];
            // giant rows are left to k_mc_giant_part / k_mc_giant_merge
            const bool giant = a.giant.ngiant > 0 && e1 - e0 > kGiantRow;
            for (int e = opt && !giant ? e0 + lane : e1; e < e1; e += G) {
                const int u = a.col[e];
                const Jmp ru = a.R[u];
                const long long gw = a.wsum[ru.J], gl = (long long)a.lcnt[ru.J];
                const long long nb = ru.D + gl * wval(w, e, a.neg) - gw;
                const int c = mc_cmp(gw, gl, nb, ow, ol, od);
                if (!TIE && (pos == INT_MAX || mc_cmp(gw, gl, nb, bw, bl, bb) < 0)) {
                    bw = gw;
                    bl = gl;
                    bb = nb;
                    pos = e;
                    bh = u;
                }
                const bool tight = c == 0 && e != cur;
                if (tight) {
                    ++cnt;
                    if (TIE) {
                        if (u == v || on_c) ++certain;
                        if ((int)ru.H >= (int)own.H) ++nondec;
                    }
                }
                if (TIE && a.xs) {   // one counter atomic per wave and step
                    const unsigned slot = wave_append(tight, a.xcnt);
                    if (tight && slot < a.xcap) {
                        a.xs[slot] = (int)v;
                        a.ys[slot] = u;
                    }
                }
            }
        }
        if (TIE) continue;
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
            const long long xw = __shfl_xor(bw, off, 64), xl = __shfl_xor(bl, off, 64);
            const long long xb = __shfl_xor(bb, off, 64);
            const int xp = __shfl_xor(pos, off, 64), xh = __shfl_xor(bh, off, 64);
            if (xp == INT_MAX) continue;
            const int c = pos == INT_MAX ? -1 : mc_cmp(xw, xl, xb, bw, bl, bb);
            if (c < 0 || (c == 0 && xp < pos)) {
                bw = xw;
                bl = xl;
                bb = xb;
                pos = xp;
                bh = xh;
            }
        }
        if (lane == 0 && v < a.n && pos != INT_MAX && mc_cmp(bw, bl, bb, ow, ol, od) < 0) {
            a.pi[v] = pos;
            a.succ[v] = bh;
            ++changed;
        }
    }
    unsigned long long sums[4] = {cnt, certain, nondec, changed};
    block_sums_u64(sums);
    if (threadIdx.x == 0) {
        CtlLane& ln = my_lane(a.ctl);
        if (sums[0]) atomicAdd(&ln.tight, sums[0]);
        if (sums[1]) atomicAdd(&ln.certain, sums[1]);
        if (sums[2]) atomicAdd(&ln.nondec, sums[2]);
        if (sums[3]) atomicAdd(&ln.changed, sums[3]);
    }
}

// Giant rows of the multichain sweep: one workgroup per chunk keeps the
// chunk's smallest pair at its lowest position (and, for the tie scan, the
// counts and the list), then one thread per row merges its chunks in
// position order and applies the strict-improvement rule.
struct alignas(16) McPart {
    long long gw, gl, nb;   // the chunk's best pair: gain W / L and bias numerator
    int pos, head;          // its lowest position (INT_MAX: none) and head
};
static_assert(sizeof(McPart) == 32, "one 32-byte slot per chunk");

template <typename WT, bool TIE>
__global__ __launch_bounds__(kWG) void k_mc_giant_part(McArgs a, const WT* __restrict__ w)
{
    __shared__ McPart sp[kWG / 64];
    const GiantTab& g = a.giant;
    McPart* parts = (McPart*)g.parts;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    unsigned long long cnt = 0, certain = 0, nondec = 0;
    for (int c = blockIdx.x; c < g.nchunks; c += gridDim.x) {
        const int v = g.cv[c];
        const Jmp own = a.R[v];
        const long long ow = a.wsum[own.J], ol = (long long)a.lcnt[own.J], od = own.D;
        const int cur = a.pi[v];
        const bool opt = !TIE || (__int128)ow * a.L == (__int128)a.W * ol;
        const bool on_c = TIE && a.onC[v];
        long long bw = 0, bl = 1, bb = 0;
        int pos = INT_MAX, bh = 0;
        for (int e = opt ? g.cs[c] + t : g.ce[c]; e < g.ce[c]; e += kWG) {
            const int u = a.col[e];
            const Jmp ru = a.R[u];
            const long long gw = a.wsum[ru.J], gl = (long long)a.lcnt[ru.J];
            const long long nb = ru.D + gl * wval(w, e, a.neg) - gw;
            if (!TIE && (pos == INT_MAX || mc_cmp(gw, gl, nb, bw, bl, bb) < 0)) {
                bw = gw;
                bl = gl;
                bb = nb;
                pos = e;
                bh = u;
            }
            const bool tight = e != cur && mc_cmp(gw, gl, nb, ow, ol, od) == 0;
            if (tight) {
                ++cnt;
                if (TIE) {
                    if (u == v || on_c) ++certain;
                    if ((int)ru.H >= (int)own.H) ++nondec;
                }
            }
            if (TIE && a.xs) {
                const unsigned slot = wave_append(tight, a.xcnt);
                if (tight && slot < a.xcap) {
                    a.xs[slot] = v;
                    a.ys[slot] = u;
                }
            }
        }
        if (TIE) continue;
        for (int off = 32; off > 0; off >>= 1) {
            const long long xw = __shfl_xor(bw, off, 64), xl = __shfl_xor(bl, off, 64);
            const long long xb = __shfl_xor(bb, off, 64);
            const int xp = __shfl_xor(pos, off, 64), xh = __shfl_xor(bh, off, 64);
            if (xp == INT_MAX) continue;
            const int k = pos == INT_MAX ? -1 : mc_cmp(xw, xl, xb, bw, bl, bb);
            if (k < 0 || (k == 0 && xp < pos)) {
                bw = xw;
                bl = xl;
                bb = xb;
                pos = xp;
                bh = xh;
            }
        }
        if (lane == 0) sp[wave] = McPart{bw, bl, bb, pos, bh};
        __syncthreads();
        if (t == 0) {
            // the best wave by index: a record assigned under this condition
            // lost its head in the generated code (its position was taken)
            int bi = 0;
            for (int i = 1; i < kWG / 64; ++i) {
                if (sp[i].pos == INT_MAX) continue;
                const int k = sp[bi].pos == INT_MAX
                                  ? -1
                                  : mc_cmp(sp[i].gw, sp[i].gl, sp[i].nb, sp[bi].gw, sp[bi].gl,
                                           sp[bi].nb);
                if (k < 0 || (k == 0 && sp[i].pos < sp[bi].pos)) bi = i;
            }
            parts[c] = sp[bi];
        }
        __syncthreads();   // sp is reused by the next chunk
    }
    unsigned long long sums[3] = {cnt, certain, nondec};
    block_sums_u64(sums);
    if (t == 0) {
        CtlLane& ln = my_lane(a.ctl);
        if (sums[0]) atomicAdd(&ln.tight, sums[0]);
        if (sums[1]) atomicAdd(&ln.certain, sums[1]);
        if (sums[2]) atomicAdd(&ln.nondec, sums[2]);
    }
}

__global__ __launch_bounds__(kWG) void k_mc_giant_merge(McArgs a)
{
    const GiantTab& g = a.giant;
    const McPart* parts = (const McPart*)g.parts;
    unsigned long long changed = 0;
    for (int i = blockIdx.x * kWG + threadIdx.x; i < g.ngiant; i += gridDim.x * kWG) {
        const int v = g.gv[i];
        // the best chunk by index (position order: strict keeps the lowest);
        // see k_mc_giant_part for why not a running record
        int bi = -1;
        for (int c = g.gc0[i]; c < g.gc1[i]; ++c) {
            if (parts[c].pos == INT_MAX) continue;
            if (bi < 0 || mc_cmp(parts[c].gw, parts[c].gl, parts[c].nb, parts[bi].gw, parts[bi].gl,
                                 parts[bi].nb) < 0)
                bi = c;
        }
        if (bi < 0) continue;
        const McPart b = parts[bi];
        const Jmp own = a.R[v];
        if (mc_cmp(b.gw, b.gl, b.nb, a.wsum[own.J], (long long)a.lcnt[own.J], own.D) < 0) {
            a.pi[v] = b.pos;
            a.succ[v] = b.head;
            ++changed;
        }
    }
    changed = block_sum_u64(changed);
    if (threadIdx.x == 0 && changed) atomicAdd(&my_lane(a.ctl).changed, changed);
}

__global__ __launch_bounds__(kWG) void k_mc_ncrit(const int* __restrict__ cyc_list,
                                                  const long long* __restrict__ wsum,
                                                  const unsigned* __restrict__ lcnt, long long W,
                                                  long long L, Ctl* ctl)
{
    const unsigned nc = ctl->ncyc;
    unsigned long long k = 0;
    for (unsigned i = blockIdx.x * kWG + threadIdx.x; i < nc; i += gridDim.x * kWG) {
        const int r = cyc_list[i];
        k += (__int128)wsum[r] * L == (__int128)W * (long long)lcnt[r];
    }
    k = block_sum_u64(k);
    if (threadIdx.x == 0 && k) atomicAdd(&my_lane(ctl).ncrit, (unsigned)k);
}

__global__ __launch_bounds__(kWG) void k_mc_mark_c(int n, const int* __restrict__ rep,
                                                   const unsigned char* __restrict__ onc, int s,
                                                   unsigned char* __restrict__ onC)
{
    const int v = blockIdx.x * kWG + threadIdx.x;
    if (v < n) onC[v] = onc[v] && rep[v] == s;
}

template <typename WT, int G>
void mc_sweep_g(const McArgs& a, const WT* w, bool tie, hipStream_t st)
{
    constexpr int VPB = kWG / G;
    int64_t g = (a.n + VPB - 1) / VPB;
    if (g > 16384) g = 16384;
    if (g >= 8) g &= ~int64_t(7);
    const unsigned grid = (unsigned)(g < 1 ? 1 : g);
    if (tie) k_mc_sweep<WT, G, true><<<grid, kWG, 0, st>>>(a, w);
    else k_mc_sweep<WT, G, false><<<grid, kWG, 0, st>>>(a, w);
}

template <typename WT>
void mc_sweep_t(const McArgs& a, const WT* w, int G, bool tie, hipStream_t st)
{
    switch (G) {
    case 1: mc_sweep_g<WT, 1>(a, w, tie, st); break;
    case 2: mc_sweep_g<WT, 2>(a, w, tie, st); break;
    case 4: mc_sweep_g<WT, 4>(a, w, tie, st); break;
    case 8: mc_sweep_g<WT, 8>(a, w, tie, st); break;
    case 16: mc_sweep_g<WT, 16>(a, w, tie, st); break;
    case 32: mc_sweep_g<WT, 32>(a, w, tie, st); break;
    default: mc_sweep_g<WT, 64>(a, w, tie, st); break;
    }
}

}  // namespace

void launch_mc_val_init(int n, const int* col, const int* pi, const void* w, int wtype, int neg,
                        const int* rep, const unsigned char* onc, const long long* wsum,
                        const unsigned* lcnt, int* succ, bool have_succ, Jmp* Q, Ctl* ctl,
                        hipStream_t st)
{
    if (wtype == kWI64)
        k_mc_val_init<long long><<<stride_grid(n), kWG, 0, st>>>(
            n, col, pi, (const long long*)w, neg, rep, onc, wsum, lcnt, succ, have_succ ? 1 : 0,
            Q, ctl);
    else
        k_mc_val_init<int><<<stride_grid(n), kWG, 0, st>>>(n, col, pi, (const int*)w, neg, rep,
                                                           onc, wsum, lcnt, succ,
                                                           have_succ ? 1 : 0, Q, ctl);
}

void launch_mc_round_dev(int n, int r, const Jmp* Qin, Jmp* Qout, Ctl* ctl, hipStream_t st)
{
    k_mc_round_dev<<<stride_grid(n), kWG, 0, st>>>(n, r, Qin, Qout, ctl);
}

void launch_mc_final_dev(int n, Jmp* Q0, Jmp* Q1, long long* V, int* hop, Ctl* ctl,
                         hipStream_t st)
{
    k_mc_final_dev<<<blocks_for(n), kWG, 0, st>>>(n, Q0, Q1, V, hop, ctl);
}

template <typename WT>
void mc_giant(const McArgs& a, const WT* w, bool tie, hipStream_t st)
{
    if (a.giant.ngiant <= 0) return;
    const unsigned grid = a.giant.nchunks < 2048 ? (unsigned)a.giant.nchunks : 2048u;
    if (tie) {
        k_mc_giant_part<WT, true><<<grid, kWG, 0, st>>>(a, w);
    } else {
        k_mc_giant_part<WT, false><<<grid, kWG, 0, st>>>(a, w);
        k_mc_giant_merge<<<blocks_for(a.giant.ngiant), kWG, 0, st>>>(a);
    }
}

void launch_mc_sweep(const McArgs& a, const void* w, int wtype, int G, bool tie, hipStream_t st)
{
    if (wtype == kWI64) {
        mc_sweep_t(a, (const long long*)w, G, tie, st);
        mc_giant(a, (const long long*)w, tie, st);
    } else {
        mc_sweep_t(a, (const int*)w, G, tie, st);
        mc_giant(a, (const int*)w, tie, st);
    }
}

void launch_mc_ncrit(const int* cyc_list, const long long* wsum, const unsigned* lcnt, long long W,
                     long long L, Ctl* ctl, hipStream_t st)
{
    k_mc_ncrit<<<kSelectParts, kWG, 0, st>>>(cyc_list, wsum, lcnt, W, L, ctl);
}

void launch_mc_mark_c(int n, const int* rep, const unsigned char* onc, int s, unsigned char* onC,
                      hipStream_t st)
{
    k_mc_mark_c<<<blocks_for(n), kWG, 0, st>>>(n, rep, onc, s, onC);
}

}  // namespace ocm
