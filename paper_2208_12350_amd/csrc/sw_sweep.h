// sw_sweep.h -- the forward/reverse sweep of one wavefront work item (gfx950).
//
// Hot path: the forward and reverse sweeps of the affine-gap Smith-Waterman
// (Gotoh) recurrences of Section II-B-1 / Fig. 2, batched over many
// independent query/reference pairs.
//
// Mapping onto CDNA4 (one pair per lane group, anti-diagonal sweep):
//   * A wavefront (64 lanes) is split into 64/W groups of W lanes (W = 16,
//     32 or 64).  Each group owns one pair.  Lane l of a group owns query rows
//     l*R .. l*R+R-1 in registers (H, E and the row's running best), so a
//     group covers W*R >= n rows in a single sweep.
//   * At step t lane l computes column j = t - l for its R rows, i.e. the
//     group sweeps anti-diagonals of lane-blocks.  The value a lane needs from
//     the row above its block (H and F of the last row of lane l-1 at
//     column j) was produced by lane l-1 one step earlier and arrives through
//     a DPP row/wave shift -- the same mechanism for every lane, with no
//     divergent first-lane path (the lesson of Section VI-A).  Lane 0 of a
//     group receives zeros, the matrix's top boundary.
//   * The reference of each group is staged in LDS as pre-scaled row offsets
//     into the LDS substitution matrix, so one LDS byte read per cell gives
//     M[a_i][b_j].  Columns left of 0 (ramp-up) and right of m (ramp-down)
//     read a padding code whose score is -1.
//   * No per-step barrier or warp vote: a wavefront runs in lock-step
//     (Section VI-B), and shared state is initialised once, by the lanes that
//     use it (Section VI-C).
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
// Biased values: every H, E and F of the packed path is stored plus a bias
// K = kI16Bias (1024), so "zero" is K.  All stored values then lie in
// [K, 0x7BFF]: bit patterns of positive normal half-precision numbers, whose
// numeric order is their integer order.  A three-way maximum of two packed
// halves is therefore one v_pk_maximum3_f16 on the raw patterns (it never
// rounds: it returns one of its inputs).  The clamps E* = max(E, 0) and
// F* = max(F, 0) become a third operand K of that maximum, and with E, F >= K
// the clamp of H at zero comes for free: H = max3(diag + M[a][b], E, F).
// diag + M[a][b] may fall below K (a mismatch next to a zero cell), even
// into the denormal range, but it is then below E >= K and never selected.
//
// Range: the host routes a pair here only when min(n, m) * max_score <=
// kI16Limit, which keeps K + H + max_score <= 0x7BFF for every cell of the
// pair (and of its reverse sweep, whose values never exceed the forward
// maximum), and when m <= kI16MaxRef, which keeps the column field of the
// keys below to 15 bits.
//
// Row best: rows r (even) and r+1 of a lane share one 32-bit key per pair,
// (H << 16) | (rowbit << 15) | (kColMax - j) with rowbit = 1 for row r.  An
// unsigned max (v_max3_u32 over both rows) keeps the largest H, then the
// upper row, then the smallest column j: the row-major-first maximum of the
// two rows.
#pragma once

#include "sw_device.h"
#include "sw_internal.h"

namespace sw {

// LDS reference buffer of one wavefront (in 16-bit entries), sized for the
// widest layout (four 16-lane groups with two packed pairs each) of 32-bit
// column words.
constexpr int kWaveBuf = 2 * 4 * 2 * RefStager<16>::kBuf;
// One sweep (forward, or reverse when REV) of the wave item
// order[first .. first+count), one pair per W-lane group, int32 arithmetic.
template <int W, int R, bool REV, int C = kChunk>
__device__ __forceinline__ void sweep_i32(const KParams& P, const SchemeLds& S, uint16_t* wbuf,
                                          int first, int count, int lane) {
    constexpr int G = 64 / W;
    using Stager = RefStager<W, C>;
    constexpr int reverse = REV ? 1 : 0;
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

    // E[r] holds E of row r at the column the lane sweeps next: it is
    // advanced right after that row's H is computed, so H - o is never kept
    int H[R], E[R], best[R], bj[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { H[r] = 0; E[r] = 0; best[r] = 0; bj[r] = -1; }
    int Hlast = 0, Flast = 0, Hup_prev = 0;
    const uint16_t* rbl = buf + W - l;   // rbl[tt] = column t0 + tt - l

    // software pipeline: a row's score for the next step is read as soon as
    // its score for this step is used, and the matrix row offset of the
    // next step one step before that
    int sc[R];
    int bb_next = rbl[1];
    {
        const int bb0 = rbl[0];
#pragma unroll
        for (int r = 0; r < R; ++r) sc[r] = S.mat[bb0 + a[r]];
    }
    bool bad = false;
    int j = -l;
    for (int t0 = 0; t0 < steps; t0 += C) {
        const bool more = t0 + C < steps;
        if (more) stage.load(P.refs, J, P.order, t0 + C, l);
        const int tn = __builtin_amdgcn_readfirstlane(steps - t0 < C ? steps - t0 : C);
        for (int tt = 0; tt < tn; ++tt) {
            const int bb2 = rbl[tt + 2];
            const int Hup = shift_in_group<W>(Hlast);
            const int Fup = shift_in_group<W>(Flast);
            int diag = Hup_prev;
            Hup_prev = Hup;
            int Hmu = sat_sub(Hup, go);
            int F = Fup;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                F = imax(F - ge, Hmu);
                const int h = imax(imax(diag + sc[r], E[r]), F);
                sc[r] = S.mat[bb_next + a[r]];
                diag = H[r];
                H[r] = h;
                Hmu = sat_sub(h, go);
                E[r] = imax(E[r] - ge, Hmu);
                if (h > best[r]) { best[r] = h; bj[r] = j; }
            }
            Hlast = H[R - 1];
            Flast = F;
            bb_next = bb2;
            ++j;
        }
        if (more) {
            wave_lds_sync();
            stage.store(buf, J, A, t0 + C, l, bad);
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
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// Columns are encoded as kColMax - j in the low 15 bits of a key; j ranges
// over -(W-1) .. kI16MaxRef + W - 2 for groups of up to 256 lanes, so
// kColMax - j stays within 0..32767.
constexpr int kColMax = 32767 - 255;
static_assert(kI16MaxRef + 256 - 2 <= kColMax, "column field of the keys overflows");

__device__ __forceinline__ uint32_t u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ u16x2 pk(uint32_t v) { return __builtin_bit_cast(u16x2, v); }

// max(x - y, 0) per 16-bit half
__device__ __forceinline__ u16x2 pk_sat_sub(u16x2 x, u16x2 y) { return __builtin_elementwise_sub_sat(x, y); }
// max of three per 16-bit half, for halves that are positive normal
// half-precision patterns (see above); one v_pk_maximum3_f16
__device__ __forceinline__ u16x2 pk_max3(u16x2 x, u16x2 y, u16x2 z) {
    const f16x2 a = __builtin_bit_cast(f16x2, x), b = __builtin_bit_cast(f16x2, y), c = __builtin_bit_cast(f16x2, z);
    return __builtin_bit_cast(u16x2, __builtin_elementwise_maximum(__builtin_elementwise_maximum(a, b), c));
}
__device__ __forceinline__ uint32_t umax3(uint32_t a, uint32_t b, uint32_t c) {
    const uint32_t m = a > b ? a : b;
    return m > c ? m : c;
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
template <int W, int R, bool REV, int C = kChunk>
__device__ __forceinline__ void sweep_i16(const KParams& P, const SchemeLds& S, uint16_t* wbuf,
                                          int first, int count, int lane) {
    using Stager = RefStager<W, C>;
    constexpr int reverse = REV ? 1 : 0;
    constexpr int RP = (R + 1) / 2;                 // row pairs per lane
    constexpr uint32_t K = kI16Bias;
    constexpr uint32_t K2 = K | (K << 16);
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
    const u16x2 go2 = pk(cost16(S.gap_open[JA.sid]) | (cost16(S.gap_open[JB.sid]) << 16));
    const u16x2 ge2 = pk(cost16(S.gap_extend[JA.sid]) | (cost16(S.gap_extend[JB.sid]) << 16));
    const u16x2 zero = pk(K2);
    wave_lds_sync();

    // H[r], E[r] (biased): H of row r at the last column swept, E of row r
    // at the next column (advanced right after the row's H, so H - o is
    // never kept).  kA/kB: keys of row pairs.
    u16x2 H[R], E[R];
    uint32_t kA[RP], kB[RP];
#pragma unroll
    for (int r = 0; r < R; ++r) { H[r] = zero; E[r] = zero; }
#pragma unroll
    for (int p = 0; p < RP; ++p) { kA[p] = 0u; kB[p] = 0u; }
    uint32_t Hlast = K2, Flast = K2, Hup_prev = K2;
    const uint16_t* rblA = bufA + W - l;
    const uint16_t* rblB = bufB + W - l;

    // software pipeline: a row's score for the next step is read as soon as
    // its score for this step is used, and the matrix row offset of the
    // next step one step before that
    u16x2 sc[R];
    int bbA_next = rblA[1], bbB_next = rblB[1];
    {
        const int a0 = rblA[0], b0 = rblB[0];
#pragma unroll
        for (int r = 0; r < R; ++r) sc[r] = load_scores(S.mat, a0 + (int)(apk[r] & 0xFFFF), b0 + (int)(apk[r] >> 16));
    }
    bool bad = false;
    uint32_t jc = (uint32_t)(kColMax + l);   // kColMax - j with j = t - l
    for (int t0 = 0; t0 < steps; t0 += C) {
        const bool more = t0 + C < steps;
        if (more) {
            stA.load(P.refs, JA, P.order, t0 + C, l);
            stB.load(P.refs, JB, P.order, t0 + C, l);
        }
        const int tn = __builtin_amdgcn_readfirstlane(steps - t0 < C ? steps - t0 : C);
        for (int tt = 0; tt < tn; ++tt) {
            const int bbA2 = rblA[tt + 2];
            const int bbB2 = rblB[tt + 2];
            const u16x2 Hup = pk((uint32_t)shift_in_group<W>((int)Hlast, (int)K2));
            // F above the group is 0 (K); a zero fill gives the same F below
            // because of the max with K
            const u16x2 Fup = pk((uint32_t)shift_in_group_zero<W>((int)Flast));
            u16x2 diag = pk(Hup_prev);
            Hup_prev = u32(Hup);
            u16x2 Hmu = pk_sat_sub(Hup, go2);
            u16x2 F = Fup;
            const uint32_t jc1 = jc | 0x8000u;   // upper row of a pair wins ties
            uint32_t keyA0 = 0, keyB0 = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                F = pk_max3(pk_sat_sub(F, ge2), Hmu, zero);
                const u16x2 h = pk_max3(diag + sc[r], E[r], F);
                sc[r] = load_scores(S.mat, bbA_next + (int)(apk[r] & 0xFFFF), bbB_next + (int)(apk[r] >> 16));
                diag = H[r];
                H[r] = h;
                Hmu = pk_sat_sub(h, go2);
                E[r] = pk_max3(pk_sat_sub(E[r], ge2), Hmu, zero);
                const uint32_t hv = u32(h);
                if ((r & 1) == 0) {
                    keyA0 = (hv << 16) | jc1;
                    keyB0 = (hv & 0xFFFF0000u) | jc1;
                    if (r == R - 1) {
                        kA[r / 2] = kA[r / 2] > keyA0 ? kA[r / 2] : keyA0;
                        kB[r / 2] = kB[r / 2] > keyB0 ? kB[r / 2] : keyB0;
                    }
                } else {
                    kA[r / 2] = umax3(kA[r / 2], keyA0, (hv << 16) | jc);
                    kB[r / 2] = umax3(kB[r / 2], keyB0, (hv & 0xFFFF0000u) | jc);
                }
            }
            Hlast = u32(H[R - 1]);
            Flast = u32(F);
            bbA_next = bbA2;
            bbB_next = bbB2;
            --jc;
        }
        if (more) {
            wave_lds_sync();
            stA.store(bufA, JA, AA, t0 + C, l, bad);
            stB.store(bufB, JB, AB, t0 + C, l, bad);
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
    // (scores unbiased; a best of 0 leaves the coordinates at -1)
    int lb[2] = {0, 0}, li[2] = {-1, -1}, lj[2] = {-1, -1};
#pragma unroll
    for (int p = 0; p < RP; ++p) {
        const uint32_t ks[2] = {kA[p], kB[p]};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int h = (int)(ks[q] >> 16) - (int)K;
            const int row = l * R + 2 * p + ((ks[q] & 0x8000u) ? 0 : 1);
            if (h > lb[q]) { lb[q] = h; li[q] = row; lj[q] = kColMax - (int)(ks[q] & 0x7FFFu); }
        }
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

// Small-alphabet ("column word") variant of sweep_i16, for wave items whose
// pairs all use schemes with at most four residues whose scores plus the gap
// open cost fit a byte.  The staged reference holds, per column b, one
// 32-bit word with bytes M[a][b] + o for a = 0..3, so a row's score is one
// v_perm_b32 of the two pairs' column words with a per-row selector (the
// query residues), instead of two address computations and two LDS reads.
// The selector takes a zero byte for rows past the query end, and padding
// columns hold word 0: both score -o <= -1, as the padding code does.
//
// The score arrives biased by +o, so each row keeps Hm = H - o (biased by K;
// exact because o <= K) instead of H:  H(i-1,j-1) + M = Hm(i-1,j-1) + (M + o).
// Hm is what E and F need anyway, and what the lane exchange carries, so
// the row update is  F = max3(F - e, Hm_up, K);  h = max3(Hm_diag + s', E, F);
// Hm = h - o;  E = max3(E - e, Hm, K);  keys from h.  The top boundary is
// Hm = K - o, F = K.
template <int W, int R, bool REV, int C = kChunk>
__device__ __forceinline__ void sweep_i16_col(const KParams& P, const SchemeLds& S, uint16_t* wbuf,
                                              int first, int count, int lane) {
    using Stager = RefStager<W, C>;
    constexpr int reverse = REV ? 1 : 0;
    constexpr int RP = (R + 1) / 2;
    constexpr uint32_t K = kI16Bias;
    constexpr uint32_t K2 = K | (K << 16);
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

    // 32-bit column words: the wave buffer holds twice as many bytes
    uint32_t* bufA = reinterpret_cast<uint32_t*>(wbuf) + (g * 2) * Stager::kBuf;
    uint32_t* bufB = bufA + Stager::kBuf;
    Stager stA, stB;
    stA.load(P.refs, JA, P.order, 0, l);
    stB.load(P.refs, JB, P.order, 0, l);

    // per-row selectors: byte 0 picks pair A's score from its column word
    // (bytes 0..3 of the perm input), byte 2 pair B's (bytes 4..7); bytes 1
    // and 3 are zero (selector 0x0C), as is a row past the query end
    uint32_t sel[R];
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
            const uint32_t a = (inA && rawA[r] < AA) ? (uint32_t)rawA[r] : 0x0Cu;
            const uint32_t b = (inB && rawB[r] < AB) ? (uint32_t)(4 + rawB[r]) : 0x0Cu;
            sel[r] = a | 0x0C00u | (b << 16) | 0x0C000000u;
        }
        stA.store_col(bufA, JA, AA, S.colw[JA.sid], 0, l, bad);
        stB.store_col(bufB, JB, AB, S.colw[JB.sid], 0, l, bad);
        if (bad && P.validate) atomicOr(&P.flags[kFlagBadResidue], 1);
    }
    const int AA = S.alphabet[JA.sid], AB = S.alphabet[JB.sid];
    const uint32_t goA = (uint32_t)S.gap_open[JA.sid], goB = (uint32_t)S.gap_open[JB.sid];
    const u16x2 go2 = pk(goA | (goB << 16));
    const u16x2 ge2 = pk(cost16(S.gap_extend[JA.sid]) | (cost16(S.gap_extend[JB.sid]) << 16));
    const u16x2 zero = pk(K2);
    const uint32_t hm_top = (K - goA) | ((K - goB) << 16);   // Hm of the zero boundary
    wave_lds_sync();

    // Hm[r]: H - o of row r at the last column swept; E[r]: E of row r at the
    // next column; kA/kB: keys of row pairs (from H itself)
    u16x2 Hm[R], E[R];
    uint32_t kA[RP], kB[RP];
#pragma unroll
    for (int r = 0; r < R; ++r) { Hm[r] = pk(hm_top); E[r] = zero; }
#pragma unroll
    for (int p = 0; p < RP; ++p) { kA[p] = 0u; kB[p] = 0u; }
    uint32_t Hlast = hm_top, Flast = K2, Hup_prev = hm_top;
    const uint32_t* rblA = bufA + W - l;
    const uint32_t* rblB = bufB + W - l;

    // Column words of even steps live in (a0, b0), of odd steps in (a1, b1);
    // a step reloads its pair with the words two steps ahead as soon as its
    // rows are done, so the steps are unrolled by two and no register
    // rotates.
    bool bad = false;
    uint32_t jc = (uint32_t)(kColMax + l);
    auto step = [&](uint32_t& ca, uint32_t& cb, int ahead) {
        const u16x2 Hmu0 = pk((uint32_t)shift_in_group<W>((int)Hlast, (int)hm_top));
        // F above the group is 0 (K); a zero fill gives the same F below
        // because of the max with K
        const u16x2 Fup = pk((uint32_t)shift_in_group_zero<W>((int)Flast));
        u16x2 diag = pk(Hup_prev);
        Hup_prev = u32(Hmu0);
        u16x2 Hmu = Hmu0;
        u16x2 F = Fup;
        const uint32_t jc1 = jc | 0x8000u;
        uint32_t keyA0 = 0, keyB0 = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            F = pk_max3(pk_sat_sub(F, ge2), Hmu, zero);
            const u16x2 sc = pk(__builtin_amdgcn_perm(cb, ca, sel[r]));
            const u16x2 h = pk_max3(diag + sc, E[r], F);
            diag = Hm[r];
            Hmu = h - go2;
            Hm[r] = Hmu;
            E[r] = pk_max3(pk_sat_sub(E[r], ge2), Hmu, zero);
            const uint32_t hv = u32(h);
            if ((r & 1) == 0) {
                keyA0 = (hv << 16) | jc1;
                keyB0 = (hv & 0xFFFF0000u) | jc1;
                if (r == R - 1) {
                    kA[r / 2] = kA[r / 2] > keyA0 ? kA[r / 2] : keyA0;
                    kB[r / 2] = kB[r / 2] > keyB0 ? kB[r / 2] : keyB0;
                }
            } else {
                kA[r / 2] = umax3(kA[r / 2], keyA0, (hv << 16) | jc);
                kB[r / 2] = umax3(kB[r / 2], keyB0, (hv & 0xFFFF0000u) | jc);
            }
        }
        ca = rblA[ahead];
        cb = rblB[ahead];
        Hlast = u32(Hm[R - 1]);
        Flast = u32(F);
        --jc;
    };
    for (int t0 = 0; t0 < steps; t0 += C) {
        const bool more = t0 + C < steps;
        if (more) {
            stA.load(P.refs, JA, P.order, t0 + C, l);
            stB.load(P.refs, JB, P.order, t0 + C, l);
        }
        const int tn = __builtin_amdgcn_readfirstlane(steps - t0 < C ? steps - t0 : C);
        uint32_t a0 = rblA[0], b0 = rblB[0], a1 = rblA[1], b1 = rblB[1];
        int tt = 0;
        for (; tt + 1 < tn; tt += 2) {
            step(a0, b0, tt + 2);
            step(a1, b1, tt + 3);
        }
        if (tt < tn) step(a0, b0, tt + 2);
        if (more) {
            wave_lds_sync();
            stA.store_col(bufA, JA, AA, S.colw[JA.sid], t0 + C, l, bad);
            stB.store_col(bufB, JB, AB, S.colw[JB.sid], t0 + C, l, bad);
            wave_lds_sync();
        }
    }
    if (bad && P.validate) atomicOr(&P.flags[kFlagBadResidue], 1);

    int lb[2] = {0, 0}, li[2] = {-1, -1}, lj[2] = {-1, -1};
#pragma unroll
    for (int p = 0; p < RP; ++p) {
        const uint32_t ks[2] = {kA[p], kB[p]};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int h = (int)(ks[q] >> 16) - (int)K;
            const int row = l * R + 2 * p + ((ks[q] & 0x8000u) ? 0 : 1);
            if (h > lb[q]) { lb[q] = h; li[q] = row; lj[q] = kColMax - (int)(ks[q] & 0x7FFFu); }
        }
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

// Pair-table variant of sweep_i16, for wave items whose pairs all use the
// one scheme of the call whose pair table sits in LDS (alphabets of up to 24
// residues whose scores plus the gap open cost fit a byte, o <= K).  Entry
// [(x D + y) D + b] of the table holds the bytes M[x][b] + o and M[y][b] + o
// for two consecutive query rows with residues x, y (D = alphabet + 1; code
// D - 1 pads rows past the query end and columns outside the reference with
// 0, a score of -o <= -1, as the padding code does).  A lane's row pair p
// therefore reads both of its scores for one column with a single 16-bit LDS
// load at rc[p] + 2 b, where rc[p] is a per-row-pair constant: one address
// add and one load per two rows and pair, against two adds and two loads per
// row in the byte-table form; one v_perm_b32 per row then places pair A's
// score in the low half and pair B's in the high half.
//
// Scores arrive biased by +o, so rows keep Hm = H - o as in sweep_i16_col.
// A row pair's scores of the next step are loaded as soon as the pair has
// used the current ones; the column offsets they need are read from the
// staged reference two steps ahead.
template <int W, int R, bool REV, int C = kChunk>
__device__ __forceinline__ void sweep_i16_ptab(const KParams& P, const PtabLds& S, uint16_t* wbuf,
                                               int first, int count, int lane) {
    using Stager = RefStager<W, C>;
    constexpr int reverse = REV ? 1 : 0;
    constexpr int RP = (R + 1) / 2;
    constexpr uint32_t K = kI16Bias;
    constexpr uint32_t K2 = K | (K << 16);
    const int g = lane / W;
    const int l = lane % W;
    const int D = P.ptab_dim;
    const int tsid = P.ptab_sid >= 0 && P.ptab_sid < SW_MAX_SCHEMES ? P.ptab_sid : 0;
    const uint8_t* tab = reinterpret_cast<const uint8_t*>(S.tab);

    const int slot = g * 2;
    const int pairA = slot < count ? P.order[first + slot] : -1;
    const int pairB = slot + 1 < count ? P.order[first + slot + 1] : -1;
    PairJob JA = load_job(P, pairA, reverse);
    PairJob JB = load_job(P, pairB, reverse);
    // every pair of a pair-table item uses the table's scheme; anything else
    // is an internal error, swept as an empty pair
    if (pairA >= 0 && JA.sid != P.ptab_sid) {
        atomicOr(&P.flags[kFlagInternal], 1);
        JA.n = JA.m = 0; JA.fwd_score = 0; JA.sid = tsid;
    }
    if (pairB >= 0 && JB.sid != P.ptab_sid) {
        atomicOr(&P.flags[kFlagInternal], 1);
        JB.n = JB.m = 0; JB.fwd_score = 0; JB.sid = tsid;
    }

    int mmax = imax(JA.m, JB.m);
    for (int off = 32; off > 0; off >>= 1) mmax = imax(mmax, __shfl_xor(mmax, off));
    const int steps = __builtin_amdgcn_readfirstlane(mmax > 0 ? mmax + W - 1 : 0);

    uint16_t* bufA = wbuf + (g * 2) * Stager::kBuf;
    uint16_t* bufB = bufA + Stager::kBuf;
    Stager stA, stB;
    stA.load(P.refs, JA, P.order, 0, l);
    stB.load(P.refs, JB, P.order, 0, l);

    // per row pair: byte offsets of its table rows, ((x D + y) D) * 2, for
    // pair A (low half) and pair B (high half); both are below 2 D^3 <= 2^15
    const int A = S.alphabet[tsid];
    uint32_t rc[RP];
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
        bool bad = false;
        int xA[2 * RP], xB[2 * RP];
#pragma unroll
        for (int r = 0; r < 2 * RP; ++r) {
            const int i = l * R + r;
            const bool inA = r < R && i < JA.n, inB = r < R && i < JB.n;
            const int ra = r < R ? rawA[r] : 0, rb = r < R ? rawB[r] : 0;
            bad |= (inA && ra >= A) || (inB && rb >= A);
            xA[r] = (inA && ra < A) ? ra : D - 1;
            xB[r] = (inB && rb < A) ? rb : D - 1;
        }
#pragma unroll
        for (int p = 0; p < RP; ++p)
            rc[p] = (uint32_t)((xA[2 * p] * D + xA[2 * p + 1]) * D * 2) |
                    ((uint32_t)((xB[2 * p] * D + xB[2 * p + 1]) * D * 2) << 16);
        stA.store_ptab(bufA, JA, A, D, 0, l, bad);
        stB.store_ptab(bufB, JB, A, D, 0, l, bad);
        if (bad && P.validate) atomicOr(&P.flags[kFlagBadResidue], 1);
    }
    const uint32_t goA = (uint32_t)S.gap_open[JA.sid], goB = (uint32_t)S.gap_open[JB.sid];
    const u16x2 go2 = pk(goA | (goB << 16));
    const u16x2 ge2 = pk(cost16(S.gap_extend[JA.sid]) | (cost16(S.gap_extend[JB.sid]) << 16));
    const u16x2 zero = pk(K2);
    const uint32_t hm_top = (K - goA) | ((K - goB) << 16);   // Hm of the zero boundary
    wave_lds_sync();

    u16x2 Hm[R], E[R];
    uint32_t kA[RP], kB[RP];
#pragma unroll
    for (int r = 0; r < R; ++r) { Hm[r] = pk(hm_top); E[r] = zero; }
#pragma unroll
    for (int p = 0; p < RP; ++p) { kA[p] = 0u; kB[p] = 0u; }
    uint32_t Hlast = hm_top, Flast = K2, Hup_prev = hm_top;
    const uint16_t* rblA = bufA + W - l;
    const uint16_t* rblB = bufB + W - l;

    // uA/uB[p]: row pair p's scores (bytes) of the current step, pair A's
    // two rows and pair B's.  Column offsets of even steps live in (xa0, xb0), of odd
    // steps in (xa1, xb1).  A step first reloads its own offsets with those
    // two steps ahead (its scores are already loaded), then, row pair by row
    // pair, uses the scores and loads the next step's with the other
    // offsets.  Steps are unrolled by two, so no register rotates.
    // Up to 14 rows per lane pairs A and B keep their scores in separate
    // registers (one v_perm_b32 per row reads both); above that the two
    // loads fill the halves of one register, which costs one more v_perm_b32
    // per row pair but keeps the kernel within 256 registers, i.e. two
    // wavefronts per SIMD instead of one.
    constexpr bool kSplit = R <= 14;
    uint32_t uA[RP], uB[kSplit ? RP : 1];
    auto load_pair = [&](int p, uint32_t ca, uint32_t cb) {
        const uint32_t a = *reinterpret_cast<const uint16_t*>(tab + (rc[p] & 0xFFFFu) + ca);
        const uint32_t b = *reinterpret_cast<const uint16_t*>(tab + (rc[p] >> 16) + cb);
        if constexpr (kSplit) {
            uA[p] = a;
            uB[p] = b;
        } else {
            uA[p] = __builtin_amdgcn_perm(b, a, 0x05040100u);
        }
    };
    bool bad = false;
    uint32_t jc = (uint32_t)(kColMax + l);
    auto step = [&](uint32_t& xa, uint32_t& xb, uint32_t na, uint32_t nb, int ahead) {
        xa = rblA[ahead];
        xb = rblB[ahead];
        const u16x2 Hmu0 = pk((uint32_t)shift_in_group<W>((int)Hlast, (int)hm_top));
        // F above the group is 0 (K); a zero fill gives the same F below
        // because of the max with K
        const u16x2 Fup = pk((uint32_t)shift_in_group_zero<W>((int)Flast));
        u16x2 diag = pk(Hup_prev);
        Hup_prev = u32(Hmu0);
        u16x2 Hmu = Hmu0;
        u16x2 F = Fup;
        const uint32_t jc1 = jc | 0x8000u;
        uint32_t keyA0 = 0, keyB0 = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int p = r / 2;
            F = pk_max3(pk_sat_sub(F, ge2), Hmu, zero);
            u16x2 sc;
            if constexpr (kSplit)
                sc = pk(__builtin_amdgcn_perm(uB[p], uA[p], (r & 1) ? 0x0C050C01u : 0x0C040C00u));
            else
                sc = pk(__builtin_amdgcn_perm(uA[p], uA[p], (r & 1) ? 0x0C030C01u : 0x0C020C00u));
            const u16x2 h = pk_max3(diag + sc, E[r], F);
            diag = Hm[r];
            Hmu = h - go2;
            Hm[r] = Hmu;
            E[r] = pk_max3(pk_sat_sub(E[r], ge2), Hmu, zero);
            const uint32_t hv = u32(h);
            if ((r & 1) == 0) {
                keyA0 = (hv << 16) | jc1;
                keyB0 = (hv & 0xFFFF0000u) | jc1;
                if (r == R - 1) {
                    kA[p] = kA[p] > keyA0 ? kA[p] : keyA0;
                    kB[p] = kB[p] > keyB0 ? kB[p] : keyB0;
                }
            } else {
                kA[p] = umax3(kA[p], keyA0, (hv << 16) | jc);
                kB[p] = umax3(kB[p], keyB0, (hv & 0xFFFF0000u) | jc);
            }
            if ((r & 1) == 1 || r == R - 1) load_pair(p, na, nb);
        }
        Hlast = u32(Hm[R - 1]);
        Flast = u32(F);
        --jc;
    };
    for (int t0 = 0; t0 < steps; t0 += C) {
        const bool more = t0 + C < steps;
        if (more) {
            stA.load(P.refs, JA, P.order, t0 + C, l);
            stB.load(P.refs, JB, P.order, t0 + C, l);
        }
        const int tn = __builtin_amdgcn_readfirstlane(steps - t0 < C ? steps - t0 : C);
        uint32_t xa0 = rblA[0], xb0 = rblB[0], xa1 = rblA[1], xb1 = rblB[1];
#pragma unroll
        for (int p = 0; p < RP; ++p) load_pair(p, xa0, xb0);
        int tt = 0;
        for (; tt + 1 < tn; tt += 2) {
            step(xa0, xb0, xa1, xb1, tt + 2);
            step(xa1, xb1, xa0, xb0, tt + 3);
        }
        if (tt < tn) step(xa0, xb0, xa1, xb1, tt + 2);
        if (more) {
            wave_lds_sync();
            stA.store_ptab(bufA, JA, A, D, t0 + C, l, bad);
            stB.store_ptab(bufB, JB, A, D, t0 + C, l, bad);
            wave_lds_sync();
        }
    }
    if (bad && P.validate) atomicOr(&P.flags[kFlagBadResidue], 1);

    int lb[2] = {0, 0}, li[2] = {-1, -1}, lj[2] = {-1, -1};
#pragma unroll
    for (int p = 0; p < RP; ++p) {
        const uint32_t ks[2] = {kA[p], kB[p]};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int h = (int)(ks[q] >> 16) - (int)K;
            const int row = l * R + 2 * p + ((ks[q] & 0x8000u) ? 0 : 1);
            if (h > lb[q]) { lb[q] = h; li[q] = row; lj[q] = kColMax - (int)(ks[q] & 0x7FFFu); }
        }
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

// Query-profile variant of the forward sweep, for a database search: every
// pair of the call aligns the same query, whose profile the workgroup builds
// in LDS once: byte ((b W + l) Rp + r) is M[a_i][b] + o for row i = l R + r
// of lane l (0 past the query end, and for the padding code b = D - 1), with
// Rp = R rounded up to whole dwords.  A lane reads its R rows' scores for
// one reference residue as Rp/4 consecutive dwords at one address (one add
// per pair and step), and one v_perm_b32 per row places pair A's score in
// the low half and pair B's in the high half.  Scores arrive biased by +o
// and rows keep Hm = H - o, as in sweep_i16_col.  The profile stands for
// the pair table (at most 24 residues, scores plus o a byte, o <= K), whose
// two loads and two adds per row pair it replaces.
template <int W, int R, int C = kChunk>
__device__ __forceinline__ void sweep_i16_qprof(const KParams& P, const int32_t* gap_open, const int32_t* gap_extend,
                                                const uint8_t* prof, uint16_t* wbuf, int first, int count,
                                                int lane) {
    using Stager = RefStager<W, C>;
    constexpr int RP = (R + 1) / 2;
    constexpr int RD = (R + 3) / 4;                 // profile dwords per lane and residue
    constexpr uint32_t K = kI16Bias;
    constexpr uint32_t K2 = K | (K << 16);
    const int g = lane / W;
    const int l = lane % W;
    const int D = P.ptab_dim;
    const int A = D - 1;

    const int slot = g * 2;
    const int pairA = slot < count ? P.order[first + slot] : -1;
    const int pairB = slot + 1 < count ? P.order[first + slot + 1] : -1;
    PairJob JA = load_job(P, pairA, 0);
    PairJob JB = load_job(P, pairB, 0);
    // every pair aligns the profiled query with the profile's scheme
    if (pairA >= 0 && (JA.sid != P.ptab_sid || JA.n != P.qprof_n)) {
        atomicOr(&P.flags[kFlagInternal], 1);
        JA.n = JA.m = 0; JA.sid = P.ptab_sid;
    }
    if (pairB >= 0 && (JB.sid != P.ptab_sid || JB.n != P.qprof_n)) {
        atomicOr(&P.flags[kFlagInternal], 1);
        JB.n = JB.m = 0; JB.sid = P.ptab_sid;
    }

    int mmax = imax(JA.m, JB.m);
    for (int off = 32; off > 0; off >>= 1) mmax = imax(mmax, __shfl_xor(mmax, off));
    const int steps = __builtin_amdgcn_readfirstlane(mmax > 0 ? mmax + W - 1 : 0);

    uint16_t* bufA = wbuf + (g * 2) * Stager::kBuf;
    uint16_t* bufB = bufA + Stager::kBuf;
    Stager stA, stB;
    stA.load(P.refs, JA, P.order, 0, l);
    stB.load(P.refs, JB, P.order, 0, l);
    constexpr int kRowBytes = W * RD * 4;           // profile bytes per residue
    bool bad = false;
    stA.store_qprof(bufA, JA, A, D, kRowBytes, 0, l, bad);
    stB.store_qprof(bufB, JB, A, D, kRowBytes, 0, l, bad);
    if (bad && P.validate) atomicOr(&P.flags[kFlagBadResidue], 1);
    const uint8_t* lprof = prof + l * RD * 4;       // this lane's rows of residue 0
    const int sid = JA.sid < SW_MAX_SCHEMES ? JA.sid : 0;
    const uint32_t go = (uint32_t)gap_open[sid];
    const u16x2 go2 = pk(go | (go << 16));
    const uint32_t ge = cost16(gap_extend[sid]);
    const u16x2 ge2 = pk(ge | (ge << 16));
    const u16x2 zero = pk(K2);
    const uint32_t hm_top = (K - go) | ((K - go) << 16);
    wave_lds_sync();

    u16x2 Hm[R], E[R];
    uint32_t kA[RP], kB[RP];
#pragma unroll
    for (int r = 0; r < R; ++r) { Hm[r] = pk(hm_top); E[r] = zero; }
#pragma unroll
    for (int p = 0; p < RP; ++p) { kA[p] = 0u; kB[p] = 0u; }
    uint32_t Hlast = hm_top, Flast = K2, Hup_prev = hm_top;
    const uint16_t* rblA = bufA + W - l;
    const uint16_t* rblB = bufB + W - l;

    // dA/dB: the lane's scores (bytes) of the current step for pairs A and
    // B, four rows per dword; reloaded for the next step dword by dword as
    // soon as its rows are done.  Column offsets as in sweep_i16_ptab.
    uint32_t dA[RD], dB[RD];
    uint32_t jc = (uint32_t)(kColMax + l);
    auto step = [&](uint32_t& xa, uint32_t& xb, uint32_t na, uint32_t nb, int ahead) {
        xa = rblA[ahead];
        xb = rblB[ahead];
        const u16x2 Hmu0 = pk((uint32_t)shift_in_group<W>((int)Hlast, (int)hm_top));
        const u16x2 Fup = pk((uint32_t)shift_in_group_zero<W>((int)Flast));
        u16x2 diag = pk(Hup_prev);
        Hup_prev = u32(Hmu0);
        u16x2 Hmu = Hmu0;
        u16x2 F = Fup;
        const uint32_t jc1 = jc | 0x8000u;
        uint32_t keyA0 = 0, keyB0 = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int p = r / 2;
            F = pk_max3(pk_sat_sub(F, ge2), Hmu, zero);
            const uint32_t sel = (uint32_t)(r % 4) | 0x0C00u | ((uint32_t)(4 + r % 4) << 16) | 0x0C000000u;
            const u16x2 sc = pk(__builtin_amdgcn_perm(dB[r / 4], dA[r / 4], sel));
            const u16x2 h = pk_max3(diag + sc, E[r], F);
            diag = Hm[r];
            Hmu = h - go2;
            Hm[r] = Hmu;
            E[r] = pk_max3(pk_sat_sub(E[r], ge2), Hmu, zero);
            const uint32_t hv = u32(h);
            if ((r & 1) == 0) {
                keyA0 = (hv << 16) | jc1;
                keyB0 = (hv & 0xFFFF0000u) | jc1;
                if (r == R - 1) {
                    kA[p] = kA[p] > keyA0 ? kA[p] : keyA0;
                    kB[p] = kB[p] > keyB0 ? kB[p] : keyB0;
                }
            } else {
                kA[p] = umax3(kA[p], keyA0, (hv << 16) | jc);
                kB[p] = umax3(kB[p], keyB0, (hv & 0xFFFF0000u) | jc);
            }
            if (r % 4 == 3 || r == R - 1) {
                dA[r / 4] = *reinterpret_cast<const uint32_t*>(lprof + na + 4 * (r / 4));
                dB[r / 4] = *reinterpret_cast<const uint32_t*>(lprof + nb + 4 * (r / 4));
            }
        }
        Hlast = u32(Hm[R - 1]);
        Flast = u32(F);
        --jc;
    };
    for (int t0 = 0; t0 < steps; t0 += C) {
        const bool more = t0 + C < steps;
        if (more) {
            stA.load(P.refs, JA, P.order, t0 + C, l);
            stB.load(P.refs, JB, P.order, t0 + C, l);
        }
        const int tn = __builtin_amdgcn_readfirstlane(steps - t0 < C ? steps - t0 : C);
        uint32_t xa0 = rblA[0], xb0 = rblB[0], xa1 = rblA[1], xb1 = rblB[1];
#pragma unroll
        for (int k = 0; k < RD; ++k) {
            dA[k] = *reinterpret_cast<const uint32_t*>(lprof + xa0 + 4 * k);
            dB[k] = *reinterpret_cast<const uint32_t*>(lprof + xb0 + 4 * k);
        }
        int tt = 0;
        for (; tt + 1 < tn; tt += 2) {
            step(xa0, xb0, xa1, xb1, tt + 2);
            step(xa1, xb1, xa0, xb0, tt + 3);
        }
        if (tt < tn) step(xa0, xb0, xa1, xb1, tt + 2);
        if (more) {
            wave_lds_sync();
            stA.store_qprof(bufA, JA, A, D, kRowBytes, t0 + C, l, bad);
            stB.store_qprof(bufB, JB, A, D, kRowBytes, t0 + C, l, bad);
            wave_lds_sync();
        }
    }
    if (bad && P.validate) atomicOr(&P.flags[kFlagBadResidue], 1);

    int lb[2] = {0, 0}, li[2] = {-1, -1}, lj[2] = {-1, -1};
#pragma unroll
    for (int p = 0; p < RP; ++p) {
        const uint32_t ks[2] = {kA[p], kB[p]};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int h = (int)(ks[q] >> 16) - (int)K;
            const int row = l * R + 2 * p + ((ks[q] & 0x8000u) ? 0 : 1);
            if (h > lb[q]) { lb[q] = h; li[q] = row; lj[q] = kColMax - (int)(ks[q] & 0x7FFFu); }
        }
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
            if (pair < 0) continue;
            sw_result res;
            if (lb[p] > 0) { res.score = lb[p]; res.q_start = -1; res.q_end = li[p]; res.r_start = -1; res.r_end = lj[p]; }
            else { res.score = 0; res.q_start = res.q_end = res.r_start = res.r_end = -1; }
            P.out[pair] = res;
        }
    }
}

}  // namespace sw
