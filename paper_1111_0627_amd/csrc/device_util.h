// Device helpers shared by the kernel files: wave and workgroup reductions,
// LDS-buffered list appends, XCD-aware block mapping.
#pragma once

#include "kernels.h"

namespace ocm {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the 8 XCDs; remapping the block
// index gives every XCD one contiguous slice of the vertex range, so the
// gathers of neighbouring vertices hit that XCD's own L2.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

template <typename WT>
__device__ __forceinline__ int64_t wval(const WT* w, int64_t e, int neg)
{
    int64_t x = (int64_t)w[e];
    return neg ? -x : x;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long x)
{
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long y = __shfl_xor(x, off, 64);
        x = y > x ? y : x;
    }
    return x;
}

// Sum over the workgroup; the result is valid in thread 0.  Counters are
// reduced per workgroup so a launch issues one global atomic per block, not
// one per wave (same-address atomics serialise in the L2).
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long x)
{
    __shared__ unsigned long long part[kWG / 64];
    x = wave_sum_u64(x);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
    __syncthreads();
    unsigned long long t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kWG / 64; ++i) t += part[i];
    return t;
}

// N sums over the workgroup in one pass (two barriers); the results are
// valid in thread 0.
template <int N>
__device__ __forceinline__ void block_sums_u64(unsigned long long (&x)[N])
{
    __shared__ unsigned long long part[kWG / 64][N];
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = wave_sum_u64(x[i]);
    __syncthreads();   // part may still be read by an earlier call
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < N; ++i) part[threadIdx.x >> 6][i] = x[i];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < N; ++i) {
            unsigned long long t = 0;
            for (int w = 0; w < kWG / 64; ++w) t += part[w][i];
            x[i] = t;
        }
}

__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long x)
{
    __shared__ unsigned long long part[kWG / 64];
    x = wave_max_u64(x);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
    __syncthreads();
    unsigned long long t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kWG / 64; ++i) t = part[i] > t ? part[i] : t;
    return t;
}

// Thread 0's value, seen by the whole workgroup (for early exits that must be
// uniform while other workgroups may change the value being read).  All
// threads call it.
__device__ __forceinline__ int block_bcast(int x)
{
    __shared__ int v;
    __syncthreads();
    if (threadIdx.x == 0) v = x;
    __syncthreads();
    return v;
}

// Workgroup-buffered list append: items go to an LDS buffer first and the
// block reserves its slice of the global list with one atomic at the end.
struct BlockList {
    int* buf;          // LDS, capacity kListItems
    unsigned* n;       // LDS counter
};

__device__ __forceinline__ void blist_push(BlockList& b, bool want, int item)
{
    const unsigned long long mask = __ballot(want);
    if (!mask) return;
    const unsigned lane = threadIdx.x & 63;
    const unsigned leader = (unsigned)__ffsll((long long)mask) - 1u;
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(b.n, (unsigned)__popcll(mask));
    base = __shfl(base, (int)leader, 64);
    if (want) b.buf[base + __popcll(mask & ((1ull << lane) - 1ull))] = item;
}

__device__ __forceinline__ void blist_flush(BlockList& b, int* out, unsigned* out_cnt)
{
    __shared__ unsigned base;
    __syncthreads();
    const unsigned cnt = *b.n;
    if (threadIdx.x == 0) base = cnt ? atomicAdd(out_cnt, cnt) : 0u;
    __syncthreads();
    for (unsigned j = threadIdx.x; j < cnt; j += kWG) out[base + j] = b.buf[j];
}

__device__ __forceinline__ unsigned wave_incl_scan(unsigned x)
{
    const int lane = threadIdx.x & 63;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// How the sweeps read the values V (value mode VM):
//   0  int64 values;
//   1  int128 values in two int64 arrays, lo and hi: value = hi * 2^64 +
//      (unsigned) lo (the fallback once a value leaves int64);
//   2  an int32 copy, written by the value phase when every value fits
//      int32 (half the gathered bytes; the keys are still formed in int64).
// ValT<VM>::type is the type keys are compared in.
template <int VM>
struct ValT {
    using type = long long;
};
template <>
struct ValT<1> {
    using type = __int128;
};

template <int VM>
__device__ __forceinline__ typename ValT<VM>::type load_val(const long long* __restrict__ lo,
                                                            const long long* __restrict__ hi,
                                                            const int* __restrict__ v32, int64_t i)
{
    if constexpr (VM == 1)
        return (__int128)(((unsigned __int128)(unsigned long long)hi[i] << 64) |
                          (unsigned long long)lo[i]);
    else if constexpr (VM == 2)
        return (long long)v32[i];
    else
        return lo[i];
}

template <typename KT>
__device__ __forceinline__ KT val_max()
{
    if constexpr (sizeof(KT) == 16)
        return (KT)(~((unsigned __int128)1 << 127));
    else
        return (KT)INT64_MAX;
}

// |x| as unsigned, defined for INT64_MIN too.
__device__ __forceinline__ unsigned long long uabs64(int64_t x)
{
    return x < 0 ? (unsigned long long)(-(x + 1)) + 1ull : (unsigned long long)x;
}

// Appends `want` lanes' items to a global list with one atomic per wave.
// Returns this lane's slot (valid only when want is true).
__device__ __forceinline__ unsigned wave_append(bool want, unsigned* counter)
{
    unsigned long long mask = __ballot(want);
    unsigned lane = threadIdx.x & 63;
    unsigned before = __popcll(mask & ((1ull << lane) - 1ull));
    unsigned total = __popcll(mask);
    unsigned leader = mask ? (unsigned)__ffsll((long long)mask) - 1u : 0u;
    unsigned base = 0;
    if (want && lane == leader) base = atomicAdd(counter, total);
    base = __shfl(base, (int)leader, 64);
    return base + before;
}

// ---------------------------------------------------------------------------
// Device-driven rounds (rebuild, values, cycles): the host queues several
// rounds ahead; a round kernel runs only while the control block says its
// round is next, and the last of its workgroups to finish books the round.
// Each workgroup's thread 0 arrives with one 64-bit atomic adding
// (1 << 48) + (flag << 32) + count, so its counts travel with the arrival
// and no fence is needed.  Arrivals are counted per lane first (same-address
// atomics serialise), then per lane.  Counts must sum below 2^32, flags
// below 2^16.
// ---------------------------------------------------------------------------
constexpr unsigned long long kArrive = 1ull << 48;

__device__ __forceinline__ unsigned long long arrival_word(unsigned long long count, unsigned flag)
{
    return count + ((unsigned long long)flag << 32);
}

// True for the grid's last arrival, which gets the summed word (arrival
// counts removed) in *total and leaves the counters at zero.
__device__ __forceinline__ bool last_arrival(Ctl* c, unsigned long long word,
                                             unsigned long long* total)
{
    const unsigned lane = blockIdx.x & (kLanes - 1);
    const unsigned in_lane = (gridDim.x - lane + kLanes - 1) / kLanes;
    const unsigned lanes = gridDim.x < (unsigned)kLanes ? gridDim.x : (unsigned)kLanes;
    const unsigned long long lp = atomicAdd(&c->lane[lane].rpack, word + kArrive);
    if ((unsigned)(lp >> 48) != in_lane - 1) return false;
    __hip_atomic_store(&c->lane[lane].rpack, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long lane_sum = lp + word + kArrive - (unsigned long long)in_lane * kArrive;
    const unsigned long long tp = atomicAdd(&c->rpack, lane_sum + kArrive);
    if ((unsigned)(tp >> 48) != lanes - 1) return false;
    __hip_atomic_store(&c->rpack, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *total = tp - (unsigned long long)(lanes - 1) * kArrive + lane_sum;
    return true;
}

// Is round r of the device-driven jump rounds the next one?
__device__ __forceinline__ bool jump_round_is(const Ctl* c, int r)
{
    return c->jk + 1 == (unsigned)r && c->jmode == 1u;
}

// Jump entries: q followed by r (sums add, hops add; bit 31 of H flags an
// int64 overflow of the sum).
__device__ __forceinline__ Jmp jmp_combine(Jmp q, const Jmp& r)
{
    long long d;
    if (__builtin_add_overflow(q.D, r.D, &d)) {
        d = 0;
        q.H |= kHopOverflow;
    }
    q.D = d;
    q.J = r.J;
    q.H = ((q.H & ~kHopOverflow) + (r.H & ~kHopOverflow)) | ((q.H | r.H) & kHopOverflow);
    return q;
}

// Rows with more than kLongRow keys in a batch are walked by the vertex's
// whole wave (64 lanes striding over the keys, then a wave minimum with
// ties to the lower position) instead of by its own thread alone: a hub's
// row then costs its length / 64 steps, not its length, while rows of
// ordinary degree keep the one-thread walk.
constexpr int kLongRow = 32;

template <typename KT>
__device__ __forceinline__ KT shfl_kt(KT x, int src)
{
    if constexpr (sizeof(KT) == 16) {
        const unsigned long long lo = __shfl((unsigned long long)x, src, 64);
        const long long hi = __shfl((long long)(x >> 64), src, 64);
        return (KT)(((unsigned __int128)(unsigned long long)hi << 64) | lo);
    } else {
        return __shfl(x, src, 64);
    }
}

template <typename KT>
__device__ __forceinline__ KT shfl_xor_kt(KT x, int off)
{
    if constexpr (sizeof(KT) == 16) {
        const unsigned long long lo = __shfl_xor((unsigned long long)x, off, 64);
        const long long hi = __shfl_xor((long long)(x >> 64), off, 64);
        return (KT)(((unsigned __int128)(unsigned long long)hi << 64) | lo);
    } else {
        return __shfl_xor(x, off, 64);
    }
}

// Minimum key over the wave, ties to the lower position; every lane gets it
// (with the head when H is set).
template <typename KT, bool H>
__device__ __forceinline__ void wave_argmin(KT& k, int& p, int& h)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const KT ok = shfl_xor_kt(k, off);
        const int op = __shfl_xor(p, off, 64);
        const int oh = H ? __shfl_xor(h, off, 64) : 0;
        if (ok < k || (ok == k && op < p)) {
            k = ok;
            p = op;
            if (H) h = oh;
        }
    }
}

}  // namespace ocm
