// sw_sweep.h -- the forward/reverse sweep of one wavefront work item (gfx950).
//
// Hot path: the forward and reverse sweeps of the affine-gap Smith-Waterman
// (Gotoh) recurrences of Section II-B-1 / Fig. 2, batched over many
// independent query/reference pairs.
//
// Mapping onto CDNA4 (one pair per lane group, anti-diagonal sweep):
//   * A wavefront (64 lanes) is split into 64/W groups of W lanes (W = 16 or
//     64).  Each group owns one pair.  Lane l of a group owns query rows
//     l*R .. l*R+R-1 in registers (H, E and the row's running best), so a
//     group covers W*R >= n rows in a single sweep.
//   * At step t lane l computes column j = t - l for its R rows, i.e. the
//     group sweeps anti-diagonals of lane-blocks.  The value a lane needs from
//     the row above its block (H and F of the last row of lane l-1 at
//     column j) was produced by lane l-1 one step earlier and arrives through
//     a DPP row/wave shift -- the same mechanism for every lane, with no
//     divergent first-lane path (the lesson of Section V-A).  Lane 0 of a
//     group receives zeros, the matrix's top boundary.
//   * The reference of each group is staged in LDS as pre-scaled row offsets
//     into the LDS substitution matrix, so one LDS byte read per cell gives
//     M[a_i][b_j].  Columns left of 0 (ramp-up) and right of m (ramp-down)
//     read a padding code whose score is -1.
//   * No per-step barrier or warp vote: a wavefront runs in lock-step
//     (Section V-B), and shared state is initialised once, by the lanes that
//     use it (Section V-C).
//
// Exactness of the padding: E and F are carried clamped at zero
// (E* = max(E, 0)), which leaves H unchanged because H takes a max with 0.  A
// padded cell (row >= n or column >= m or < 0) scores at most
// max(diag - 1, E, F) where diag <= S and E, F <= S - o, so with o >= 1 it is
// strictly below the pair's best S and never changes S or its first cell;
// real cells never depend on padded ones (they lie below or to the right).
//
// Packed int16 variant (sweep_i16):
// Same anti-diagonal lane-group sweep as the int32 kernel, but every 32-bit
// register carries two independent pairs: pair A in the low 16 bits and pair
// B in the high 16 bits, so one packed VALU instruction (v_pk_*_i16/u16)
// advances two cells.  A W-lane group therefore aligns two pairs, and the
// host pairs them up from the same length bin (similar query and reference
// lengths, so little padding).
//
// Range: the host routes a pair here only when min(n, m) * max_score fits
// in 15 bits, which bounds every H, E, F and H + M[a][b] of the pair (and of
// its reverse sweep, whose values never exceed the forward maximum).  E, F
// and H - o are carried saturated at 0 (v_pk_sub_u16 with clamp), exactly as
// the int32 kernel clamps them, so the packed arithmetic is exact.
//
// Row best per lane is tracked as a 32-bit key (H << 16) | (kColMax - j):
// an unsigned max keeps the largest H and, among equal H, the smallest
// column j -- the row-major-first maximum within a row.
#pragma once

#include "sw_device.h"
#include "sw_internal.h"

namespace sw {

// LDS reference buffer of one wavefront, sized for the widest layout
// (four 16-lane groups with two packed pairs each).
constexpr int kWaveBuf = 4 * 2 * RefStager<16>::kBuf;
// One sweep (forward or reverse per P.reverse) of the wave item
// order[first .. first+count), one pair per W-lane group, int32 arithmetic.
template <int W, int R>
__device__ __forceinline__ void sweep_i32(const KParams& P, const SchemeLds& S, uint16_t* wbuf,
                                          int first, int count, int lane) {
    constexpr int G = 64 / W;
    using Stager = RefStager<W>;
    const int reverse = P.reverse;
    const int g = lane / W;
    const int l = lane % W;

    const int pair = g < count ? P.order[first + g] : -1;
    const PairJob J = load_job(P, pair, reverse);

    // wave-uniform step count: longest reference in the wavefront + ramp
    int mmax = J.m;
    for (int off = 32; off > 0; off >>= 1) mmax = imax(mmax, __shfl_xor(mmax, off));
    const int steps = __builtin_amdgcn_readfirstlane(mmax > 0 ? mmax + W - 1 : 0);

    uint16_t* buf = wbuf + g * Stager::kBuf;
    Stager stage;
    stage.load(P.refs, J, P.order, 0, l);

    // query rows of this lane (padding code below the query end)
    int a[R];
    {
        int raw[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int i = l * R + r;
            i = i < J.n ? i : (J.n > 0 ? J.n - 1 : 0);
            const uint8_t* p = J.n > 0 ? P.queries + J.qbase + (int64_t)J.dir * i
                                       : reinterpret_cast<const uint8_t*>(P.order);
            raw[r] = *p;
        }
        const int A = S.alphabet[J.sid];
        bool bad = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool inside = l * R + r < J.n;
            bad |= inside && raw[r] >= A;
            a[r] = (inside && raw[r] < A) ? raw[r] : kPad;
        }
        stage.store(buf, J, A, 0, l, bad);
        if (bad && P.validate) atomicOr(&P.flags[kFlagBadResidue], 1);
    }
    const int A = S.alphabet[J.sid];
    const int go = S.gap_open[J.sid];
    const int ge = S.gap_extend[J.sid];
    wave_lds_sync();

    int H[R], E[R], Hm[R], best[R], bj[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { H[r] = 0; E[r] = 0; Hm[r] = 0; best[r] = 0; bj[r] = -1; }
    int Hlast = 0, Flast = 0, Hup_prev = 0;
    const uint16_t* rbl = buf + W - l;   // rbl[tt] = column t0 + tt - l

    // software pipeline: scores of the current step and the matrix row of
    // the next step are read one step ahead
    int sc[R];
    int bb_next = rbl[1];
    {
        const int bb0 = rbl[0];
#pragma unroll
        for (int r = 0; r < R; ++r) sc[r] = S.mat[bb0 + a[r]];
    }
    bool bad = false;
    int j = -l;
    for (int t0 = 0; t0 < steps; t0 += kChunk) {
        const bool more = t0 + kChunk < steps;
        if (more) stage.load(P.refs, J, P.order, t0 + kChunk, l);
        const int tn = __builtin_amdgcn_readfirstlane(steps - t0 < kChunk ? steps - t0 : kChunk);
        for (int tt = 0; tt < tn; ++tt) {
            const int bb2 = rbl[tt + 2];
            int sn[R];
#pragma unroll
            for (int r = 0; r < R; ++r) sn[r] = S.mat[bb_next + a[r]];
            const int Hup = shift_in_group<W>(Hlast);
            const int Fup = shift_in_group<W>(Flast);
            int diag = Hup_prev;
            Hup_prev = Hup;
            int Hmu = sat_sub(Hup, go);
            int F = Fup;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int en = imax(E[r] - ge, Hm[r]);
                F = imax(F - ge, Hmu);
                const int h = imax(imax(diag + sc[r], en), F);
                diag = H[r];
                H[r] = h;
                E[r] = en;
                Hm[r] = sat_sub(h, go);
                Hmu = Hm[r];
                if (h > best[r]) { best[r] = h; bj[r] = j; }
            }
            Hlast = H[R - 1];
            Flast = F;
#pragma unroll
            for (int r = 0; r < R; ++r) sc[r] = sn[r];
            bb_next = bb2;
            ++j;
        }
        if (more) {
            wave_lds_sync();
            stage.store(buf, J, A, t0 + kChunk, l, bad);
            wave_lds_sync();
            // the two look-ahead reads of the next chunk's first steps were
            // taken from the old buffer; the new buffer holds the same
            // columns at entries W-l+0 and W-l+1, so re-read them
            bb_next = rbl[1];
            const int bb0 = rbl[0];
#pragma unroll
            for (int r = 0; r < R; ++r) sc[r] = S.mat[bb0 + a[r]];
        }
    }
    if (bad && P.validate) atomicOr(&P.flags[kFlagBadResidue], 1);

    // best of this lane in row-major order, then of the group
    int lb = 0, li = -1, lj = -1;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (best[r] > lb) { lb = best[r]; li = l * R + r; lj = bj[r]; }
    for (int off = 1; off < W; off <<= 1) {
        const int ob = __shfl_xor(lb, off);
        const int oi = __shfl_xor(li, off);
        const int oj = __shfl_xor(lj, off);
        if (ob > lb || (ob == lb && oi < li)) { lb = ob; li = oi; lj = oj; }
    }
    if (l == 0 && pair >= 0) {
        if (!reverse) {
            sw_result res;
            if (lb > 0) { res.score = lb; res.q_start = -1; res.q_end = li; res.r_start = -1; res.r_end = lj; }
            else { res.score = 0; res.q_start = res.q_end = res.r_start = res.r_end = -1; }
            P.out[pair] = res;
        } else if (J.fwd_score > 0) {
            if (lb != J.fwd_score) {
                atomicOr(&P.flags[kFlagReverseMismatch], 1);
            } else {
                P.out[pair].q_start = J.fwd_qe - li;
                P.out[pair].r_start = J.fwd_re - lj;
            }
        }
    }
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

// Columns are encoded as kColMax - j in the low half of a key; j ranges over
// -(W-1) .. SW_MAX_REF + W - 2, so kColMax - j stays within 0..65535.
constexpr int kColMax = 65535 - 64;

__device__ __forceinline__ uint32_t u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ u16x2 pk(uint32_t v) { return __builtin_bit_cast(u16x2, v); }

// max(x - y, 0) per 16-bit half, for non-negative halves
__device__ __forceinline__ u16x2 pk_sat_sub(u16x2 x, u16x2 y) { return __builtin_elementwise_sub_sat(x, y); }
__device__ __forceinline__ u16x2 pk_max_u(u16x2 x, u16x2 y) { return __builtin_elementwise_max(x, y); }
__device__ __forceinline__ u16x2 pk_max_s(u16x2 x, u16x2 y) {
    return __builtin_bit_cast(u16x2, __builtin_elementwise_max(__builtin_bit_cast(s16x2, x),
                                                               __builtin_bit_cast(s16x2, y)));
}

// Scores of one step for both pairs: low half M[aA][bA], high half M[aB][bB],
// each sign-extended to 16 bits.
__device__ __forceinline__ u16x2 load_scores(const int8_t* mat, int addrA, int addrB) {
    s16x2 s;
    s.x = (short)mat[addrA];
    s.y = (short)mat[addrB];
    return __builtin_bit_cast(u16x2, s);
}

// One sweep of the wave item order[first .. first+count), two pairs per
// W-lane group packed into int16 halves.
template <int W, int R>
__device__ __forceinline__ void sweep_i16(const KParams& P, const SchemeLds& S, uint16_t* wbuf,
                                          int first, int count, int lane) {
    constexpr int G = 64 / W;
    using Stager = RefStager<W>;
    const int reverse = P.reverse;
    const int g = lane / W;
    const int l = lane % W;

    const int slot = g * 2;
    const int pairA = slot < count ? P.order[first + slot] : -1;
    const int pairB = slot + 1 < count ? P.order[first + slot + 1] : -1;
    const PairJob JA = load_job(P, pairA, reverse);
    const PairJob JB = load_job(P, pairB, reverse);

    int mmax = imax(JA.m, JB.m);
    for (int off = 32; off > 0; off >>= 1) mmax = imax(mmax, __shfl_xor(mmax, off));
    const int steps = __builtin_amdgcn_readfirstlane(mmax > 0 ? mmax + W - 1 : 0);

    uint16_t* bufA = wbuf + (g * 2) * Stager::kBuf;
    uint16_t* bufB = bufA + Stager::kBuf;
    Stager stA, stB;
    stA.load(P.refs, JA, P.order, 0, l);
    stB.load(P.refs, JB, P.order, 0, l);

    // query rows: residue codes of A (low half) and B (high half)
    uint32_t apk[R];
    {
        int rawA[R], rawB[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = l * R + r;
            const int iA = i < JA.n ? i : (JA.n > 0 ? JA.n - 1 : 0);
            const int iB = i < JB.n ? i : (JB.n > 0 ? JB.n - 1 : 0);
            const uint8_t* pA = JA.n > 0 ? P.queries + JA.qbase + (int64_t)JA.dir * iA
                                         : reinterpret_cast<const uint8_t*>(P.order);
            const uint8_t* pB = JB.n > 0 ? P.queries + JB.qbase + (int64_t)JB.dir * iB
                                         : reinterpret_cast<const uint8_t*>(P.order);
            rawA[r] = *pA;
            rawB[r] = *pB;
        }
        const int AA = S.alphabet[JA.sid], AB = S.alphabet[JB.sid];
        bool bad = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = l * R + r;
            const bool inA = i < JA.n, inB = i < JB.n;
            bad |= (inA && rawA[r] >= AA) || (inB && rawB[r] >= AB);
            const uint32_t a = (inA && rawA[r] < AA) ? rawA[r] : kPad;
            const uint32_t b = (inB && rawB[r] < AB) ? rawB[r] : kPad;
            apk[r] = a | (b << 16);
        }
        stA.store(bufA, JA, AA, 0, l, bad);
        stB.store(bufB, JB, AB, 0, l, bad);
        if (bad && P.validate) atomicOr(&P.flags[kFlagBadResidue], 1);
    }
    const int AA = S.alphabet[JA.sid], AB = S.alphabet[JB.sid];
    const u16x2 go2 = pk((uint32_t)S.gap_open[JA.sid] | ((uint32_t)S.gap_open[JB.sid] << 16));
    const u16x2 ge2 = pk((uint32_t)S.gap_extend[JA.sid] | ((uint32_t)S.gap_extend[JB.sid] << 16));
    wave_lds_sync();

    u16x2 H[R], E[R], Hm[R];
    uint32_t kA[R], kB[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        H[r] = pk(0u); E[r] = pk(0u); Hm[r] = pk(0u); kA[r] = 0u; kB[r] = 0u;
    }
    uint32_t Hlast = 0, Flast = 0, Hup_prev = 0;
    const uint16_t* rblA = bufA + W - l;
    const uint16_t* rblB = bufB + W - l;

    u16x2 sc[R];
    int bbA_next = rblA[1], bbB_next = rblB[1];
    {
        const int a0 = rblA[0], b0 = rblB[0];
#pragma unroll
        for (int r = 0; r < R; ++r) sc[r] = load_scores(S.mat, a0 + (int)(apk[r] & 0xFFFF), b0 + (int)(apk[r] >> 16));
    }
    bool bad = false;
    uint32_t jc = (uint32_t)(kColMax + l);   // kColMax - j with j = t - l
    for (int t0 = 0; t0 < steps; t0 += kChunk) {
        const bool more = t0 + kChunk < steps;
        if (more) {
            stA.load(P.refs, JA, P.order, t0 + kChunk, l);
            stB.load(P.refs, JB, P.order, t0 + kChunk, l);
        }
        const int tn = __builtin_amdgcn_readfirstlane(steps - t0 < kChunk ? steps - t0 : kChunk);
        for (int tt = 0; tt < tn; ++tt) {
            const int bbA2 = rblA[tt + 2];
            const int bbB2 = rblB[tt + 2];
            u16x2 sn[R];
#pragma unroll
            for (int r = 0; r < R; ++r)
                sn[r] = load_scores(S.mat, bbA_next + (int)(apk[r] & 0xFFFF), bbB_next + (int)(apk[r] >> 16));
            const u16x2 Hup = pk((uint32_t)shift_in_group<W>((int)Hlast));
            const u16x2 Fup = pk((uint32_t)shift_in_group<W>((int)Flast));
            u16x2 diag = pk(Hup_prev);
            Hup_prev = u32(Hup);
            u16x2 Hmu = pk_sat_sub(Hup, go2);
            u16x2 F = Fup;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const u16x2 en = pk_max_u(pk_sat_sub(E[r], ge2), Hm[r]);
                F = pk_max_u(pk_sat_sub(F, ge2), Hmu);
                const u16x2 h = pk_max_s(pk_max_s(diag + sc[r], en), F);
                diag = H[r];
                H[r] = h;
                E[r] = en;
                Hm[r] = pk_sat_sub(h, go2);
                Hmu = Hm[r];
                const uint32_t hv = u32(h);
                const uint32_t keyA = (hv << 16) | jc;
                const uint32_t keyB = (hv & 0xFFFF0000u) | jc;
                kA[r] = kA[r] > keyA ? kA[r] : keyA;
                kB[r] = kB[r] > keyB ? kB[r] : keyB;
            }
            Hlast = u32(H[R - 1]);
            Flast = u32(F);
#pragma unroll
            for (int r = 0; r < R; ++r) sc[r] = sn[r];
            bbA_next = bbA2;
            bbB_next = bbB2;
            --jc;
        }
        if (more) {
            wave_lds_sync();
            stA.store(bufA, JA, AA, t0 + kChunk, l, bad);
            stB.store(bufB, JB, AB, t0 + kChunk, l, bad);
            wave_lds_sync();
            bbA_next = rblA[1];
            bbB_next = rblB[1];
            const int a0 = rblA[0], b0 = rblB[0];
#pragma unroll
            for (int r = 0; r < R; ++r)
                sc[r] = load_scores(S.mat, a0 + (int)(apk[r] & 0xFFFF), b0 + (int)(apk[r] >> 16));
        }
    }
    if (bad && P.validate) atomicOr(&P.flags[kFlagBadResidue], 1);

    // per pair: best of this lane in row-major order, then of the group
    int lb[2] = {0, 0}, li[2] = {-1, -1}, lj[2] = {-1, -1};
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int hA = (int)(kA[r] >> 16), hB = (int)(kB[r] >> 16);
        if (hA > lb[0]) { lb[0] = hA; li[0] = l * R + r; lj[0] = kColMax - (int)(kA[r] & 0xFFFF); }
        if (hB > lb[1]) { lb[1] = hB; li[1] = l * R + r; lj[1] = kColMax - (int)(kB[r] & 0xFFFF); }
    }
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        for (int off = 1; off < W; off <<= 1) {
            const int ob = __shfl_xor(lb[p], off);
            const int oi = __shfl_xor(li[p], off);
            const int oj = __shfl_xor(lj[p], off);
            if (ob > lb[p] || (ob == lb[p] && oi < li[p])) { lb[p] = ob; li[p] = oi; lj[p] = oj; }
        }
    }
    if (l == 0) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int pair = p == 0 ? pairA : pairB;
            const PairJob& J = p == 0 ? JA : JB;
            if (pair < 0) continue;
            if (!reverse) {
                sw_result res;
                if (lb[p] > 0) { res.score = lb[p]; res.q_start = -1; res.q_end = li[p]; res.r_start = -1; res.r_end = lj[p]; }
                else { res.score = 0; res.q_start = res.q_end = res.r_start = res.r_end = -1; }
                P.out[pair] = res;
            } else if (J.fwd_score > 0) {
                if (lb[p] != J.fwd_score) {
                    atomicOr(&P.flags[kFlagReverseMismatch], 1);
                } else {
                    P.out[pair].q_start = J.fwd_qe - li[p];
                    P.out[pair].r_start = J.fwd_re - lj[p];
                }
            }
        }
    }
}

}  // namespace sw
