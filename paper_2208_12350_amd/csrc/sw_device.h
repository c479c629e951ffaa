// sw_device.h -- device-side helpers shared by the gfx950 sweep kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_internal.h"

namespace sw {

template <int W>
__device__ __forceinline__ int shift_in_group(int x, int fill = 0) {
    // Lane l receives lane l-1's value; the first lane of each W-lane group
    // receives `fill`.  row_shr:1 shifts within 16-lane rows, wave_shr:1
    // across the whole wavefront; with bound_ctrl off, a lane with no source
    // keeps the `old` operand.  32-lane groups take the wave shift and
    // select `fill` for lane 32 (its source, lane 31, belongs to the other
    // group).
    if constexpr (W == 16) {
        return __builtin_amdgcn_update_dpp(fill, x, 0x111, 0xF, 0xF, false);
    } else if constexpr (W == 32) {
        const int y = __builtin_amdgcn_update_dpp(fill, x, 0x138, 0xF, 0xF, false);
        return (__lane_id() & 31) ? y : fill;
    } else {
        static_assert(W == 64, "W must be 16, 32 or 64");
        return __builtin_amdgcn_update_dpp(fill, x, 0x138, 0xF, 0xF, false);
    }
}

// shift_in_group with a zero fill: bound_ctrl writes the zero, so no fill
// register has to be set up.
template <int W>
__device__ __forceinline__ int shift_in_group_zero(int x) {
    if constexpr (W == 16) {
        return __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, true);
    } else if constexpr (W == 32) {
        const int y = __builtin_amdgcn_update_dpp(0, x, 0x138, 0xF, 0xF, true);
        return (__lane_id() & 31) ? y : 0;
    } else {
        static_assert(W == 64, "W must be 16, 32 or 64");
        return __builtin_amdgcn_update_dpp(0, x, 0x138, 0xF, 0xF, true);
    }
}

__device__ __forceinline__ int sat_sub(int x, int y) {
    // max(x - y, 0) for x >= 0, y >= 0
    return (int)__builtin_elementwise_sub_sat((unsigned)x, (unsigned)y);
}

__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }

// A gap cost as one 16-bit half of a packed operand.  Packed values never
// exceed 0x7BFF, so subtracting any cost of at least 0x7C00 saturates to 0,
// the same as subtracting the true cost: clamping at 0x7FFF keeps every
// result exact, while a cost of 65536 or more would otherwise be truncated
// and spill into the other pair's half.
__device__ __forceinline__ uint32_t cost16(int c) { return (uint32_t)(c < 0x7FFF ? c : 0x7FFF); }

struct PairJob {
    int64_t qbase, rbase;
    int n, m, dir, sid;
    int fwd_score, fwd_qe, fwd_re;
};

// The sub-problem of one pair for this sweep.  Pair ids come from the
// planning arrays; any id or length outside its documented range is an
// internal error, flagged and turned into an empty job.
// Extent of the reverse sweep of a pair whose forward pass found best score
// S > 0 ending at (qe, re): rows n = qe + 1 and columns m = re + 1 of the
// reversed prefixes, cut to the part that can hold a cell of score S.
// Every such cell (p, q) closes an alignment of score S that spans exactly p
// query and q reference residues (the forward end is the row-major-first
// maximum, so no S-scoring alignment from it ends earlier).  Such an
// alignment has at most min(p, q) aligned pairs, each scoring at most Mx,
// and at least |p - q| gap residues, which cost at least
// o + (k - 1) e for k of them when o >= e (k o when o < e).  So q - p is at
// most the largest k whose cost fits in Mx p - S, and likewise p - q.
// Cells right of or below the cut are never needed by those inside it, so
// the cut leaves every value inside, and the first S cell, unchanged.
__device__ __forceinline__ int gap_room(int64_t slack, int o, int e) {
    // largest number of gap residues whose least cost is at most `slack`
    if (o <= 0 || e < 0) return SW_MAX_REF;   // no bound
    if (slack < (int64_t)o) return 0;
    const int64_t k = o < e ? slack / o : (e == 0 ? (int64_t)SW_MAX_REF : 1 + (slack - o) / e);
    return k < (int64_t)SW_MAX_REF ? (int)k : SW_MAX_REF;
}
__device__ __forceinline__ void reverse_extent(int S, int Mx, int o, int e, int& n, int& m) {
    const int mq = n + gap_room((int64_t)Mx * n - S, o, e);
    if (m > mq) m = mq;
    const int np = m + gap_room((int64_t)Mx * m - S, o, e);
    if (n > np) n = np;
}

__device__ __forceinline__ PairJob load_job(const KParams& P, int pair, int reverse) {
    PairJob J;
    J.dir = 1; J.n = 0; J.m = 0; J.qbase = 0; J.rbase = 0; J.sid = 0;
    J.fwd_score = 0; J.fwd_qe = -1; J.fwd_re = -1;
    if (pair < 0) return J;
    if (pair >= *P.n_dev) {
        atomicOr(&P.flags[kFlagInternal], 1);
        return J;
    }
    J.sid = P.scheme_id ? (int)P.scheme_id[pair] : 0;
    const int64_t q0 = P.q_beg[pair], q1 = P.q_end[pair];
    const int64_t r0 = P.r_beg[pair], r1 = P.r_end[pair];
    if (!reverse) {
        J.qbase = q0; J.rbase = r0;
        J.n = (int)(q1 - q0); J.m = (int)(r1 - r0);
    } else {
        const sw_result f = P.out[pair];
        J.fwd_score = f.score; J.fwd_qe = f.q_end; J.fwd_re = f.r_end;
        if (f.score > 0) {
            J.n = f.q_end + 1; J.m = f.r_end + 1;
            J.qbase = q0 + f.q_end; J.rbase = r0 + f.r_end;
            J.dir = -1;
            if (J.sid < SW_MAX_SCHEMES)
                reverse_extent(f.score, P.max_score[J.sid], P.gap_open[J.sid], P.gap_extend[J.sid], J.n, J.m);
        }
    }
    if (J.n < 0 || J.n > SW_MAX_QUERY || J.m < 0 || J.m > SW_MAX_REF || J.sid >= SW_MAX_SCHEMES) {
        atomicOr(&P.flags[kFlagInternal], 1);
        J.n = 0; J.m = 0; J.sid = 0; J.fwd_score = 0;
    }
    return J;
}

// Wave-scope ordering of LDS traffic: every lane's earlier LDS accesses are
// complete and visible before any lane's later ones (the wavefront executes
// in lock-step, so no workgroup barrier is needed).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Reference columns are streamed through LDS in chunks of C sweep steps
// (the tile width; kChunk unless a kernel is compiled for another).  While
// a chunk is swept, lanes read columns t0-W+1 .. t0+C+1 (the loop reads two
// steps ahead), so a group's buffer holds at least C+W+2 entries: entry x is
// column t0-W+x.  Each lane prefetches kPerLane entries of the next chunk
// into registers, so a narrower tile costs fewer registers and more chunk
// boundaries.  (kChunk and kChunkNarrow are in sw_internal.h.)

template <int W, int C = kChunk>
struct RefStager {
    static constexpr int kPerLane = (C + W + 2 + W - 1) / W;
    static constexpr int kBuf = kPerLane * W;
    int raw[kPerLane];

    // Issue the loads of the chunk starting at sweep step t0.  Addresses are
    // clamped into the pair's reference so that the loads are unconditional
    // and stay in flight while the previous chunk is swept.
    __device__ __forceinline__ void load(const uint8_t* refs, const PairJob& J, const void* dummy,
                                         int t0, int l) {
#pragma unroll
        for (int k = 0; k < kPerLane; ++k) {
            int j = t0 - W + l + k * W;
            j = j < 0 ? 0 : (j >= J.m ? J.m - 1 : j);
            const uint8_t* p = J.m > 0 ? refs + J.rbase + (int64_t)J.dir * j
                                       : reinterpret_cast<const uint8_t*>(dummy);
            raw[k] = *p;
        }
    }
    // Write the chunk into the group's LDS buffer as matrix row offsets,
    // replacing out-of-range columns and invalid residues by the padding code.
    __device__ __forceinline__ void store(uint16_t* buf, const PairJob& J, int A, int t0, int l,
                                          bool& bad) const {
        const int sbase = J.sid * kMatBytes;
#pragma unroll
        for (int k = 0; k < kPerLane; ++k) {
            const int j = t0 - W + l + k * W;
            int b = raw[k];
            const bool inside = j >= 0 && j < J.m;
            bad |= inside && b >= A;
            b = (inside && b < A) ? b : kPad;
            buf[l + k * W] = (uint16_t)(sbase + b * kMatDim);
        }
    }
    // Pair-table path: write the chunk as byte offsets 2 b of the reference
    // residues into a pair-table row; out-of-range columns and invalid
    // residues get the padding code D - 1 (whose entries are 0, a score of -o).
    __device__ __forceinline__ void store_ptab(uint16_t* buf, const PairJob& J, int A, int D, int t0, int l,
                                               bool& bad) const {
#pragma unroll
        for (int k = 0; k < kPerLane; ++k) {
            const int j = t0 - W + l + k * W;
            const int b = raw[k];
            const bool inside = j >= 0 && j < J.m;
            bad |= inside && b >= A;
            buf[l + k * W] = (uint16_t)(2 * ((inside && b < A) ? b : D - 1));
        }
    }
    // Query-profile path: write the chunk as byte offsets b * row_bytes of
    // the reference residues' profile rows; out-of-range columns and invalid
    // residues get the padding code D - 1 (a row of zeros, a score of -o).
    __device__ __forceinline__ void store_qprof(uint16_t* buf, const PairJob& J, int A, int D, int row_bytes, int t0,
                                                int l, bool& bad) const {
#pragma unroll
        for (int k = 0; k < kPerLane; ++k) {
            const int j = t0 - W + l + k * W;
            const int b = raw[k];
            const bool inside = j >= 0 && j < J.m;
            bad |= inside && b >= A;
            buf[l + k * W] = (uint16_t)(row_bytes * ((inside && b < A) ? b : D - 1));
        }
    }
    // Small-alphabet path: write the chunk as column words (bytes M[a][b] + o
    // for a = 0..3); out-of-range columns and invalid residues get word 0,
    // i.e. a score of -o for every row.
    __device__ __forceinline__ void store_col(uint32_t* buf, const PairJob& J, int A, const uint32_t* colw,
                                              int t0, int l, bool& bad) const {
#pragma unroll
        for (int k = 0; k < kPerLane; ++k) {
            const int j = t0 - W + l + k * W;
            const int b = raw[k];
            const bool inside = j >= 0 && j < J.m;
            bad |= inside && b >= A;
            buf[l + k * W] = (inside && b < A) ? colw[b] : 0u;
        }
    }
};

// Per-block copy of the scoring schemes: substitution tables, column words
// of the small-alphabet path and gap costs.
struct SchemeLds {
    int8_t mat[SW_MAX_SCHEMES * kMatBytes];
    uint32_t colw[SW_MAX_SCHEMES][kMatDim];
    int32_t alphabet[SW_MAX_SCHEMES];
    int32_t gap_open[SW_MAX_SCHEMES];
    int32_t gap_extend[SW_MAX_SCHEMES];
    int32_t col_ok[SW_MAX_SCHEMES];
};

// Per-block copy for the pair-table sweep: the pair table of scheme
// P.ptab_sid (D^3 16-bit entries) and the gap costs of every scheme.
struct PtabLds {
    uint16_t tab[kPtabBytes / 2];
    int32_t alphabet[SW_MAX_SCHEMES];
    int32_t gap_open[SW_MAX_SCHEMES];
    int32_t gap_extend[SW_MAX_SCHEMES];
};

__device__ __forceinline__ void load_ptab(PtabLds& S, const KParams& P, int tid) {
    const int D = P.ptab_dim;
    const int words = (D > 0 && D <= kPtabMaxDim) ? (D * D * D + 1) / 2 : 0;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(P.mats + kPtabOffset);
    for (int k = tid; k < words; k += kBlock) reinterpret_cast<uint32_t*>(S.tab)[k] = src[k];
    if (tid < SW_MAX_SCHEMES) {
        S.alphabet[tid] = P.alphabet[tid];
        S.gap_open[tid] = P.gap_open[tid];
        S.gap_extend[tid] = P.gap_extend[tid];
    }
}

__device__ __forceinline__ void load_schemes(SchemeLds& S, const KParams& P, int tid) {
    for (int k = tid; k < SW_MAX_SCHEMES * kMatBytes / 4; k += kBlock)
        reinterpret_cast<int32_t*>(S.mat)[k] = reinterpret_cast<const int32_t*>(P.mats)[k];
    for (int k = tid; k < SW_MAX_SCHEMES * kMatDim; k += kBlock)
        (&S.colw[0][0])[k] = reinterpret_cast<const uint32_t*>(P.mats + SW_MAX_SCHEMES * kMatBytes)[k];
    if (tid < SW_MAX_SCHEMES) {
        S.col_ok[tid] = P.col_ok[tid];
        S.alphabet[tid] = P.alphabet[tid];
        S.gap_open[tid] = P.gap_open[tid];
        S.gap_extend[tid] = P.gap_extend[tid];
    }
}

}  // namespace sw
