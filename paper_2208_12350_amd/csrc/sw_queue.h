// sw_queue.h -- work-queue kernels over the sweep shapes (gfx950).
//
// A queue kernel is compiled for one bin shape (precision, W, R), one
// direction (forward sweep, or reverse sweep when REV) and one score source
// (column words when COL, table lookups otherwise), and aligns
// the work items [meta[lo_idx], meta[hi_idx]) of that bin: every wavefront
// takes the next item with one atomic increment of the bin's queue head and
// sweeps it, until the range is exhausted.
//   * plain mode launches it with one wavefront per item (the grid is sized
//     from the item count the host reads back);
//   * persistent mode launches it, for every bin, with as many workgroups as
//     the device holds at once (capped by what the batch could need), without
//     reading anything back; items of a bin come longest first.
// Every wavefront leaves the loop once the head passes the end of the range,
// so the grid always drains.  Range bounds, item fields and pair ids are
// checked against the array capacities: a violated invariant sets an error
// flag and the work is skipped rather than indexed.
#pragma once

#include <type_traits>

#include "sw_sweep.h"

namespace sw {

// The work-queue loop of one wavefront: claim items of the launch's range
// and sweep each with `sweep(first, count)`.
template <int kPPW, class Sweep>
__device__ __forceinline__ void queue_loop(const KParams& P, int lane, int lo, int hi, int n_pairs, Sweep&& sweep,
                                           int head_idx = -1) {
    if (head_idx < 0) head_idx = P.head_idx;
    // The loop has no lane-divergent branch: every lane takes part in the
    // fetch (only lane 0 adds 1, so each wavefront claims exactly one item
    // whether or not the lanes' atomics are merged), and the item index is
    // lane 0's return value.  A lane-0-only atomic inside this loop was
    // lowered into an inner loop that re-entered without the fetch.
    for (;;) {
        const int mine = atomicAdd(&P.meta[head_idx], lane == 0 ? 1 : 0);
        const int it = __builtin_amdgcn_readlane(mine, 0);
        if (it >= hi - lo) break;
        const WorkItem* wp = P.items + lo + it;
        const int first = __builtin_amdgcn_readfirstlane(__atomic_load_n(&wp->first, __ATOMIC_RELAXED));
        const int count = __builtin_amdgcn_readfirstlane((int)__atomic_load_n(&wp->count, __ATOMIC_RELAXED));
        const bool valid = first >= 0 && count >= 1 && count <= kPPW && first + count <= n_pairs;
        if (valid) {
            wave_lds_sync();
            sweep(first, count);
        } else {
            atomicOr(&P.flags[kFlagInternal], 1);
        }
    }
}

// The item range of the launch, read first: a launch for an empty bin (the
// host does not know which bins are empty) costs its workgroups two loads
// and an exit.  Returns false when there is nothing to do.
__device__ __forceinline__ bool launch_range(const KParams& P, int tid, int& lo, int& hi) {
    lo = __atomic_load_n(&P.meta[P.lo_idx], __ATOMIC_RELAXED);
    hi = __atomic_load_n(&P.meta[P.hi_idx], __ATOMIC_RELAXED);
    lo = __builtin_amdgcn_readfirstlane(lo);
    hi = __builtin_amdgcn_readfirstlane(hi);
    if (lo == hi) return false;
    if (lo < 0 || hi > P.max_items || lo > hi) {
        if (tid == 0) atomicOr(&P.flags[kFlagInternal], 1);
        return false;
    }
    return true;
}

// Body of a queue kernel whose sweeps stream the reference in tiles of C
// steps.
template <int PREC, int W, int R, bool REV, bool COL, int C>
__device__ __forceinline__ void queue_body(const KParams& P, SchemeLds& L, uint16_t* wbufs) {
    constexpr int kPPW = (64 / W) * (PREC == 16 ? 2 : 1);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    int lo, hi;
    if (!launch_range(P, tid, lo, hi)) return;
    const int n_pairs = __builtin_amdgcn_readfirstlane(*P.n_dev);
    load_schemes(L, P, tid);
    __syncthreads();
    uint16_t* wbuf = wbufs + wave * kWaveBuf;
    queue_loop<kPPW>(P, lane, lo, hi, n_pairs, [&](int first, int count) {
        if constexpr (COL)
            sweep_i16_col<W, R, REV, C>(P, L, wbuf, first, count, lane);
        else if constexpr (PREC == 16)
            sweep_i16<W, R, REV, C>(P, L, wbuf, first, count, lane);
        else
            sweep_i32<W, R, REV, C>(P, L, wbuf, first, count, lane);
    });
}

template <int W, int R, bool REV, int C>
__device__ __forceinline__ void ptab_body(const KParams& P, PtabLds& L, uint16_t* wbufs) {
    constexpr int kPPW = (64 / W) * 2;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    int lo, hi;
    if (!launch_range(P, tid, lo, hi)) return;
    if (P.ptab_sid < 0 || P.ptab_sid >= SW_MAX_SCHEMES || P.ptab_dim < 2 || P.ptab_dim > kPtabMaxDim) {
        if (tid == 0) atomicOr(&P.flags[kFlagInternal], 1);
        return;
    }
    const int n_pairs = __builtin_amdgcn_readfirstlane(*P.n_dev);
    load_ptab(L, P, tid);
    __syncthreads();
    uint16_t* wbuf = wbufs + wave * kWaveBuf;
    queue_loop<kPPW>(P, lane, lo, hi, n_pairs, [&](int first, int count) {
        sweep_i16_ptab<W, R, REV, C>(P, L, wbuf, first, count, lane);
    });
}

// Queue kernels with the default tile width (kChunk steps) ...
template <int PREC, int W, int R, bool REV, bool COL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void sw_queue_kernel(KParams P) {
    __shared__ __attribute__((aligned(16))) SchemeLds L;
    __shared__ uint16_t wbufs[kWavesPerBlock * kWaveBuf];
    queue_body<PREC, W, R, REV, COL, kChunk>(P, L, wbufs);
}

// ... and with a tile of C steps (kept apart so that the default kernels keep
// their names in profiles).
template <int PREC, int W, int R, bool REV, bool COL, int C>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void sw_queue_chunk_kernel(KParams P) {
    __shared__ __attribute__((aligned(16))) SchemeLds L;
    __shared__ uint16_t wbufs[kWavesPerBlock * kWaveBuf];
    queue_body<PREC, W, R, REV, COL, C>(P, L, wbufs);
}

// Packed int16 shapes with the pair table of one scheme (sweep_i16_ptab).
template <int W, int R, bool REV>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void sw_ptab_kernel(KParams P) {
    __shared__ __attribute__((aligned(16))) PtabLds L;
    __shared__ uint16_t wbufs[kWavesPerBlock * kWaveBuf];
    ptab_body<W, R, REV, kChunk>(P, L, wbufs);
}

template <int W, int R, bool REV, int C>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void sw_ptab_chunk_kernel(KParams P) {
    __shared__ __attribute__((aligned(16))) PtabLds L;
    __shared__ uint16_t wbufs[kWavesPerBlock * kWaveBuf];
    ptab_body<W, R, REV, C>(P, L, wbufs);
}

// Forward sweep of a database search with the query profile
// (sweep_i16_qprof): every pair of the launch aligns queries[0 ..
// P.qprof_n) with scheme P.ptab_sid.  The workgroup builds the profile of
// its lanes' rows in LDS before it takes items.
template <int W, int R>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void sw_qprof_kernel(KParams P) {
    constexpr int RD = (R + 3) / 4;
    constexpr int kRowBytes = W * RD * 4;
    constexpr int kPPW = (64 / W) * 2;
    __shared__ __attribute__((aligned(16))) uint8_t prof[kPtabMaxDim * kRowBytes];
    __shared__ int32_t gopen[SW_MAX_SCHEMES], gext[SW_MAX_SCHEMES];
    __shared__ uint16_t wbufs[kWavesPerBlock * kWaveBuf];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    int lo, hi;
    if (!launch_range(P, tid, lo, hi)) return;
    const int D = P.ptab_dim, sid = P.ptab_sid, n = P.qprof_n;
    if (!P.qprof || sid < 0 || sid >= SW_MAX_SCHEMES || D < 2 || D > kPtabMaxDim || n < 1 || n > W * R) {
        if (tid == 0) atomicOr(&P.flags[kFlagInternal], 1);
        return;
    }
    const int A = D - 1;
    const int o = P.gap_open[sid];
    const int8_t* mat = P.mats + sid * kMatBytes;   // [b][a] = M[a][b]
    bool bad = false;
    for (int idx = tid; idx < D * kRowBytes; idx += kBlock) {
        const int b = idx / kRowBytes, rem = idx % kRowBytes;
        const int l = rem / (RD * 4), r = rem % (RD * 4);
        const int i = l * R + r;
        int v = 0;
        if (b < A && r < R && i < n) {
            const int a = P.queries[i];
            bad |= a >= A;
            v = a < A ? mat[b * kMatDim + a] + o : 0;
        }
        prof[idx] = (uint8_t)v;
    }
    if (bad && P.validate) atomicOr(&P.flags[kFlagBadResidue], 1);
    if (tid < SW_MAX_SCHEMES) {
        gopen[tid] = P.gap_open[tid];
        gext[tid] = P.gap_extend[tid];
    }
    const int n_pairs = __builtin_amdgcn_readfirstlane(*P.n_dev);
    __syncthreads();
    uint16_t* wbuf = wbufs + wave * kWaveBuf;
    queue_loop<kPPW>(P, lane, lo, hi, n_pairs, [&](int first, int count) {
        sweep_i16_qprof<W, R>(P, gopen, gext, prof, wbuf, first, count, lane);
    });
}

// ---- family kernels ----------------------------------------------------------
// A family kernel serves a run of shapes of one precision and lane width
// (rows per lane Rs..., largest first): it drains the queue of member k's
// bin (P.fam_bins[k]; -1: not launched), then member k+1's, each with the
// sweep compiled for that member.  One launch per pass thus takes the items
// of every member bin, and a wavefront whose bin runs dry moves on to the
// next instead of idling until the launch ends.  The members follow one
// another (no loop around them), so each member's loop-invariant values are
// live only while it runs and the register allocation is about that of the
// largest member.
template <int PREC, int W, int R, bool REV, int VAR, int C, class Lds>
__device__ __forceinline__ void family_member(const KParams& P, Lds& L, uint16_t* wbuf, int lane, int bin,
                                              int n_pairs) {
    constexpr int kPPW = (64 / W) * (PREC == 16 ? 2 : 1);
    if (bin < 0) return;
    const int lo_i = VAR == kVarCol ? kMetaItemFirst + bin : kMetaItemSplit + bin;
    const int hi_i = VAR == kVarCol ? kMetaItemSplit + bin : kMetaItemFirst + bin + 1;
    const int lo = __builtin_amdgcn_readfirstlane(__atomic_load_n(&P.meta[lo_i], __ATOMIC_RELAXED));
    const int hi = __builtin_amdgcn_readfirstlane(__atomic_load_n(&P.meta[hi_i], __ATOMIC_RELAXED));
    if (lo >= hi) return;
    if (lo < 0 || hi > P.max_items) {
        atomicOr(&P.flags[kFlagInternal], 1);
        return;
    }
    queue_loop<kPPW>(P, lane, lo, hi, n_pairs, [&](int first, int count) {
        if constexpr (VAR == kVarPtab)
            sweep_i16_ptab<W, R, REV, C>(P, L, wbuf, first, count, lane);
        else if constexpr (VAR == kVarCol)
            sweep_i16_col<W, R, REV, C>(P, L, wbuf, first, count, lane);
        else if constexpr (PREC == 16)
            sweep_i16<W, R, REV, C>(P, L, wbuf, first, count, lane);
        else
            sweep_i32<W, R, REV, C>(P, L, wbuf, first, count, lane);
    }, (VAR == kVarCol ? kMetaColHeads : kMetaHeads) + bin);
}

template <int... Rs>
constexpr int family_size() { return (int)sizeof...(Rs); }

template <int PREC, int W, bool REV, int VAR, int WPE, int C, int... Rs>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WPE))) void sw_family_kernel(KParams P) {
    static_assert(sizeof...(Rs) <= kFamilyMax, "family too large");
    using Lds = typename std::conditional<VAR == kVarPtab, PtabLds, SchemeLds>::type;
    __shared__ __attribute__((aligned(16))) Lds L;
    __shared__ uint16_t wbufs[kWavesPerBlock * kWaveBuf];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if constexpr (VAR == kVarPtab) {
        if (P.ptab_sid < 0 || P.ptab_sid >= SW_MAX_SCHEMES || P.ptab_dim < 2 || P.ptab_dim > kPtabMaxDim) {
            if (tid == 0) atomicOr(&P.flags[kFlagInternal], 1);
            return;
        }
        load_ptab(L, P, tid);
    } else {
        load_schemes(L, P, tid);
    }
    const int n_pairs = __builtin_amdgcn_readfirstlane(*P.n_dev);
    __syncthreads();
    uint16_t* wbuf = wbufs + wave * kWaveBuf;
    int k = 0;
    ((family_member<PREC, W, Rs, REV, VAR, C, Lds>(P, L, wbuf, lane, P.fam_bins[k++], n_pairs)), ...);
}

// Register budgets and tiles of a family's kernels: CW wavefronts per SIMD
// for its column-word kernel, PW and the reference tile PC for its
// pair-table kernel (the table-lookup kernel keeps 2 and kChunk).
// Measured: the 9..16-row 16-lane and 11..16-row 32-lane column-word
// families run dna_large 2.5% faster at 3 (a few spilled registers).  Their
// pair-table families ran protein 4% slower at 3, and the 32-lane one no
// faster at 3 with tiles of 64 steps (168 registers, 3 spilled).
#define SW_FAMILY16(W, CW, PW, PC, ...)                                                                       \
    {16, W, family_size<__VA_ARGS__>(), {__VA_ARGS__},                                                        \
     {{&sw_family_kernel<16, W, false, kVarTable, 2, kChunk, __VA_ARGS__>,                                    \
       &sw_family_kernel<16, W, true, kVarTable, 2, kChunk, __VA_ARGS__>},                                    \
      {&sw_family_kernel<16, W, false, kVarCol, CW, kChunk, __VA_ARGS__>,                                     \
       &sw_family_kernel<16, W, true, kVarCol, CW, kChunk, __VA_ARGS__>},                                     \
      {&sw_family_kernel<16, W, false, kVarPtab, PW, PC, __VA_ARGS__>,                                        \
       &sw_family_kernel<16, W, true, kVarPtab, PW, PC, __VA_ARGS__>}},                                       \
     {2, CW, PW}, {kChunk, kChunk, PC}}

// Per tile width (index 0: kChunk, 1: kChunkNarrow) and score source
// (kVarTable, kVarCol, kVarPtab): the forward and reverse kernels, null
// where a shape has no such variant.
struct KernelEntry { int prec, W, R; QueueFn k[2][kNumVars][2]; };

}  // namespace sw

