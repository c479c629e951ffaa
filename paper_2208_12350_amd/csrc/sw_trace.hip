// sw_trace.hip -- alignment paths on gfx950: the traceback of Fig. 2(c),
// recovered inside each pair's result box.
//
// The score path gives, per pair, S and the box a[q_start..q_end] x
// b[r_start..r_end].  Every S-scoring alignment that ends at the box's last
// cell and stays in the box starts at its first cell (a later start would
// contradict the latest-start rule of the reverse sweep), so the path is a
// traceback of the box's own local Gotoh matrices from its last cell.  Two
// steps, per chunk of pairs:
//
//   1. Path sweep: the box is swept like the forward pass (W-lane groups, R
//      rows per lane, anti-diagonal steps with DPP lane shifts; two pairs
//      per group packed in biased int16 halves when S fits, else one pair
//      in int32), and every cell leaves 4 flags in a device record:
//        D   H is not the diagonal value
//        N   H is not F (with D set: H comes from E, a reference residue
//            over a gap; with D clear: from the diagonal)
//        FX  F does not open here (F != H(i-1, j) - o: it extends)
//        EX  E does not open in the next column (E(i, j+1) != H(i, j) - o:
//            it extends); computed where E(i, j+1) is, and read by the walk
//            when a gap move has brought it to (i, j)
//      Step t of lane l holds rows l*R .. l*R+R-1 of column t - l (R a
//      multiple of 4) in R/2 bytes: one dword per 8 rows, whose bytes are
//      the D, N, FX and EX bits of those rows (bit k: row 8j+k), and for
//      R % 8 == 4 a 16-bit tail for the last 4 rows (FX bits 0-3, D 4-7,
//      EX 8-11, N 12-15).  Records are laid out in blocks of kStage steps:
//      block b of lane l is the 4R bytes at (b * W + l) * 4R, step t = 8b + s
//      at byte s * R/2.  The sweep stages a block's steps in LDS and writes
//      it out as full 16-byte chunks per lane (a pair's block of all W lanes
//      is one contiguous W * 4R bytes); the walk moves mostly along one
//      lane's steps, so one block read serves up to 8 of its steps.
//      The flags are computed without compares.  In the packed sweeps every
//      value stays below 0x8000, so for x >= y the wrapping 16-bit
//      difference y - x has bit 15 set exactly when x != y: one packed
//      subtract gives a flag for both pairs, one v_perm_b32 gathers the top
//      bytes of two such differences (four flags, one per byte, in bit 7),
//      and a shift and a bitfield insert push them into the row's bit of
//      four byte-wide flag streams.  The int32 sweep takes min(x ^ y, 1).
//   2. Walk: one thread per pair follows the bits back from the box's last
//      cell, taking as H's source the diagonal, else F, else E (the first
//      that equals H) and opening a gap over extending it, and writes the path as
//      runs (length << 4) | op with the SAM codes 7 '=', 8 'X', 1 'I', 2 'D'.
//
// E and F are carried clamped at zero, as in the score sweeps; a clamped
// value only differs on cells whose H is 0, which no path visits (every
// prefix of an optimal path scores above 0).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_device.h"
#include "sw_internal.h"
#include "sw_sweep.h"

namespace sw {

// The box of one pair as a forward sub-problem; an empty job for a pair
// without an alignment, and an internal error for a box outside its pair or
// taller than `max_rows`.
__device__ __forceinline__ PairJob box_job(const KParams& P, int pair, int max_rows) {
    PairJob J;
    J.dir = 1; J.n = 0; J.m = 0; J.qbase = 0; J.rbase = 0; J.sid = 0;
    J.fwd_score = 0; J.fwd_qe = -1; J.fwd_re = -1;
    if (pair < 0) return J;
    if (pair >= *P.n_dev) {
        atomicOr(&P.flags[kFlagInternal], 1);
        return J;
    }
    const sw_result r = P.out[pair];
    if (r.score <= 0) return J;
    const int64_t q0 = P.q_beg[pair], q1 = P.q_end[pair];
    const int64_t r0 = P.r_beg[pair], r1 = P.r_end[pair];
    const int sid = P.scheme_id ? (int)P.scheme_id[pair] : 0;
    const bool ok = r.q_start >= 0 && r.q_start <= r.q_end && r.q_end < q1 - q0 && r.r_start >= 0 &&
                    r.r_start <= r.r_end && r.r_end < r1 - r0 && r.q_end - r.q_start < max_rows &&
                    r.r_end - r.r_start < SW_MAX_REF && sid < SW_MAX_SCHEMES;
    if (!ok) {
        atomicOr(&P.flags[kFlagInternal], 1);
        return J;
    }
    J.sid = sid;
    J.n = r.q_end - r.q_start + 1;
    J.m = r.r_end - r.r_start + 1;
    J.qbase = q0 + r.q_start;
    J.rbase = r0 + r.r_start;
    J.fwd_score = r.score;
    return J;
}

// Record staging of one wavefront: the current block (kStage steps) of each
// of its PPW pairs, in LDS in the record layout (pair p's block is W lanes x
// 4R bytes, lane-major), so that a complete block is copied out with
// 16-byte loads and stores.  A lane's step is R/2 bytes: R/8 dwords of 8
// rows, and for R % 8 == 4 a 16-bit tail of 4 rows.  In LDS a lane's 4R
// bytes start every kStride dwords: R, plus 4 when R/4 is even.  All lanes
// write the same step offset at once, so a stride of R dwords with R/4 even
// would start every lane in one of R = 8: 4, 16: 2, 32: 1 bank group; an odd
// number of 16-byte units spreads the lanes over 8 groups of 4 banks, and
// keeps every lane's block 16-byte aligned for the copy out.
template <int W, int R, int PPW>
struct RecordStage {
    static_assert(R % 4 == 0 && R >= 4 && R <= 32, "a lane's step is whole 16-bit units of 4 rows");
    static constexpr int NW = R / 8;                    // whole dwords per lane and step
    static constexpr int kStride = R + ((R / 4) % 2 == 0 ? 4 : 0);   // dwords per lane and block in LDS
    static constexpr int kDwords = PPW * W * kStride;   // per wavefront
    uint32_t* lds;

    __device__ __forceinline__ void put(int p, int l, int t, const uint32_t* v, uint32_t tail) const {
        const int byte = (p * W + l) * kStride * 4 + (t & (kStage - 1)) * (R / 2);
        if constexpr (R % 8 == 0) {
            uint32_t* d = lds + byte / 4;
#pragma unroll
            for (int k = 0; k < NW; ++k) d[k] = v[k];
        } else {
            // R/2 = 4k + 2 bytes: only 16-bit alignment is guaranteed
            uint16_t* d = reinterpret_cast<uint16_t*>(lds) + byte / 2;
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                d[2 * k] = (uint16_t)v[k];
                d[2 * k + 1] = (uint16_t)(v[k] >> 16);
            }
            d[2 * NW] = (uint16_t)tail;
        }
    }
    // Bit (c0 / 64) * PPW + p of the result: this lane's chunk of pair p in
    // the copy round starting at chunk c0 lies in a lane with rows of the
    // pair's box (n_rows rows).  Taken once per wave item, OR-ed over p.
    static_assert((W * R / 4 + 63) / 64 * PPW <= 32, "one bit per copy round and pair");
    __device__ __forceinline__ static uint32_t row_bits(int p, int n_rows, int lane) {
        uint32_t m = 0;
        const int qlim = (n_rows + R - 1) / R;
#pragma unroll
        for (int c0 = 0; c0 < W * R / 4; c0 += 64)
            m |= ((c0 + lane) / (R / 4) < qlim ? 1u : 0u) << ((c0 / 64) * PPW + p);
        return m;
    }
    // Copy block b of every pair of the wavefront (W * R dwords each) to its
    // record, 16 bytes per lane at a time: chunk c of a pair is 16-byte unit
    // c % (R/4) of lane c / (R/4), copy round k takes chunks 64k .. 64k+63.
    // rec_of(p) and steps_of(p) give pair p's record (nullptr: none) and
    // sweep steps.  Up to 8 chunks per lane are read from LDS before the
    // first store, so their round trips overlap.
    // A lane's part of the block is left unwritten when it holds no cell of
    // the pair's box: the lane's rows all lie past the box (its bit in
    // `rows` is clear, see row_bits), or the block's steps all come before
    // the lane's first column (step q).  The walk never reads such a part
    // (it reads a lane's block only for a step of a box cell, and the block
    // before it only for a later such step).
    static constexpr int kRounds = (W * R / 4 + 63) / 64;
    __device__ __forceinline__ uint4 chunk(int p, int k, int lane) const {
        int c = 64 * k + lane;
        c = c < W * R / 4 ? c : W * R / 4 - 1;   // lanes past the block read its last chunk
        return *reinterpret_cast<const uint4*>(lds + p * W * kStride + c / (R / 4) * kStride + 4 * (c % (R / 4)));
    }
    __device__ __forceinline__ void store(int p, int k, uint32_t* rec, int b, int lane, uint32_t rows,
                                          const uint4& v) const {
        const int c = 64 * k + lane;
        const int q = c / (R / 4);
        const bool cell = ((rows >> (k * PPW + p)) & 1u) && kStage * b + kStage > q;
        if ((W * R / 4 >= 64 * k + 64 || c < W * R / 4) && cell)
            *reinterpret_cast<uint4*>(rec + (int64_t)b * W * R + 4 * c) = v;
    }
    template <typename RecOf, typename StepsOf>
    __device__ __forceinline__ void flush(int t, int lane, uint32_t rows, RecOf rec_of, StepsOf steps_of) const {
        const int b = t / kStage;
        if constexpr (PPW * kRounds <= 8) {
            uint4 v[PPW][kRounds];
#pragma unroll
            for (int p = 0; p < PPW; ++p)
#pragma unroll
                for (int k = 0; k < kRounds; ++k) v[p][k] = chunk(p, k, lane);
#pragma unroll
            for (int p = 0; p < PPW; ++p) {
                uint32_t* rp = rec_of(p);
                if (rp && (t & ~(kStage - 1)) < steps_of(p))
#pragma unroll
                    for (int k = 0; k < kRounds; ++k) store(p, k, rp, b, lane, rows, v[p][k]);
            }
        } else {
#pragma unroll
            for (int p = 0; p < PPW; ++p) {
                constexpr int KB = kRounds < 8 ? kRounds : 8;
#pragma unroll
                for (int k0 = 0; k0 < kRounds; k0 += KB) {
                    uint4 v[KB];
#pragma unroll
                    for (int k = 0; k < KB; ++k) v[k] = chunk(p, k0 + k, lane);
                    uint32_t* rp = rec_of(p);
                    if (rp && (t & ~(kStage - 1)) < steps_of(p))
#pragma unroll
                        for (int k = 0; k < KB; ++k) store(p, k0 + k, rp, b, lane, rows, v[k]);
                }
            }
        }
    }
};

__device__ __forceinline__ uint32_t* readlane_ptr(uint32_t* p, int lane) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), lane);
    return reinterpret_cast<uint32_t*>(((uint64_t)hi << 32) | lo);
}

// 1 if x != 0, else 0: one v_min_u32.  Written as an instruction because
// the compiler otherwise turns min(x, 1) into a compare and a select (two
// instructions with a wait state between them).
__device__ __forceinline__ uint32_t ne01(uint32_t x) {
    uint32_t r;
    asm("v_min_u32 %0, 1, %1" : "=v"(r) : "v"(x));
    return r;
}

// Push four flags (bit 7 of each byte of p) into four byte-wide flag
// streams: each byte of acc moves down one bit and takes the new flag on top,
// so after 8 rows bit k of a byte is row k's flag.  The bits below bit 7 of
// p are dropped, and a bit that moves into the byte below lands in its bit
// 7, which the insert overwrites.  One shift and one v_bfi_b32, written as
// an instruction because the compiler otherwise splits the masks over three.
__device__ __forceinline__ uint32_t flag_push(uint32_t acc, uint32_t p) {
    uint32_t r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "s"(0x80808080u), "v"(p), "v"(acc >> 1));
    return r;
}
// Top bytes of two packed wrapping differences: bytes 1 and 3 of x (pair A,
// pair B) become bytes 0 and 2, those of y bytes 1 and 3.
__device__ __forceinline__ uint32_t flag_gather(uint32_t x, uint32_t y) {
    return __builtin_amdgcn_perm(y, x, 0x07030501u);
}

// Path sweep of the wave item order[first .. first+count), one pair per
// W-lane group, int32.
template <int W, int R>
__device__ __forceinline__ void sweep_trace(const KParams& P, const TraceArgs& T, const SchemeLds& S,
                                            uint16_t* wbuf, uint32_t* stg, int first, int count, int lane) {
    constexpr int NW = (R + 7) / 8;   // dwords of 8 rows (the last one half used when R % 8 == 4)
    constexpr int G = 64 / W;
    const RecordStage<W, R, G> rs{stg};
    using Stager = RefStager<W>;
    const int g = lane / W;
    const int l = lane % W;

    const int pair = g < count ? P.order[first + g] : -1;
    PairJob J = box_job(P, pair, W * R);
    uint32_t* rec = nullptr;
    if (J.m > 0) {
        const int64_t off = T.rec_off[pair] - (int64_t)T.chunk * T.chunk_bytes;
        const int64_t bytes = trace_record_bytes(W, R, J.m);
        if (off < 0 || off + bytes > T.ws_bytes || (off & 15) != 0) {
            atomicOr(&P.flags[kFlagInternal], 1);
            J.n = 0; J.m = 0;
        } else {
            rec = reinterpret_cast<uint32_t*>(T.ws + off);
        }
    }
    const int my_steps = J.m > 0 ? J.m + W - 1 : 0;
    uint32_t rowbits = 0;   // flush chunks in lanes with box rows
#pragma unroll
    for (int p = 0; p < G; ++p) rowbits |= rs.row_bits(p, __builtin_amdgcn_readlane(J.n, p * W), lane);
    int mmax = J.m;
    for (int off = 32; off > 0; off >>= 1) mmax = imax(mmax, __shfl_xor(mmax, off));
    const int steps = __builtin_amdgcn_readfirstlane(mmax > 0 ? mmax + W - 1 : 0);

    uint16_t* buf = wbuf + g * Stager::kBuf;
    Stager stage;
    stage.load(P.refs, J, P.order, 0, l);
    const int A = S.alphabet[J.sid];
    int a[R];
    {
        int raw[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int i = l * R + r;
            i = i < J.n ? i : (J.n > 0 ? J.n - 1 : 0);
            const uint8_t* p = J.n > 0 ? P.queries + J.qbase + i : reinterpret_cast<const uint8_t*>(P.order);
            raw[r] = *p;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = (l * R + r < J.n && raw[r] < A) ? raw[r] : kPad;
    }
    bool bad = false;   // residues were checked by the score passes
    stage.store(buf, J, A, 0, l, bad);
    const int go = S.gap_open[J.sid];
    const int ge = S.gap_extend[J.sid];
    wave_lds_sync();

    int H[R], E[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { H[r] = 0; E[r] = 0; }
    int Hlast = 0, Flast = 0, Hup_prev = 0;
    const uint16_t* rbl = buf + W - l;   // rbl[tt] = column t0 + tt - l
    int sc[R];
    int bb_next = rbl[1];
    {
        const int bb0 = rbl[0];
#pragma unroll
        for (int r = 0; r < R; ++r) sc[r] = S.mat[bb0 + a[r]];
    }
    for (int t0 = 0; t0 < steps; t0 += kChunk) {
        const bool more = t0 + kChunk < steps;
        if (more) stage.load(P.refs, J, P.order, t0 + kChunk, l);
        const int tn = __builtin_amdgcn_readfirstlane(steps - t0 < kChunk ? steps - t0 : kChunk);
        for (int tt = 0; tt < tn; ++tt) {
            const int bb2 = rbl[tt + 2];
            const int Hup = shift_in_group<W>(Hlast);
            const int Fup = shift_in_group<W>(Flast);
            int diag = Hup_prev;
            Hup_prev = Hup;
            int Hmu = sat_sub(Hup, go);
            int F = Fup;
            uint32_t wv[NW];
#pragma unroll
            for (int k = 0; k < NW; ++k) wv[k] = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                F = imax(F - ge, Hmu);
                const int d = diag + sc[r];
                const int h = imax(imax(d, E[r]), F);
                const uint32_t nd = ne01((uint32_t)(h ^ d));
                const uint32_t nf = ne01((uint32_t)(h ^ F));
                const uint32_t fx = ne01((uint32_t)(F - Hmu));
                sc[r] = S.mat[bb_next + a[r]];
                diag = H[r];
                H[r] = h;
                Hmu = sat_sub(h, go);
                E[r] = imax(E[r] - ge, Hmu);
                const uint32_t ex = ne01((uint32_t)(E[r] - Hmu));   // for the next column
                if (r < R / 8 * 8)
                    wv[r / 8] |= (nd | (nf << 8) | (fx << 16) | (ex << 24)) << (r % 8);
                else
                    wv[r / 8] |= (fx | (nd << 4) | (ex << 8) | (nf << 12)) << (r % 8);
            }
            Hlast = H[R - 1];
            Flast = F;
            bb_next = bb2;
            const int t = t0 + tt;
            rs.put(g, l, t, wv, wv[NW - 1]);
            if ((t & (kStage - 1)) == kStage - 1 || t == steps - 1) {
                wave_lds_sync();
                rs.flush(t, lane, rowbits, [&](int p) { return readlane_ptr(rec, p * W); },
                         [&](int p) { return __builtin_amdgcn_readlane(my_steps, p * W); });
                wave_lds_sync();
            }
        }
        if (more) {
            wave_lds_sync();
            stage.store(buf, J, A, t0 + kChunk, l, bad);
            wave_lds_sync();
            bb_next = rbl[1];
            const int bb0 = rbl[0];
#pragma unroll
            for (int r = 0; r < R; ++r) sc[r] = S.mat[bb0 + a[r]];
        }
    }
}

// Record of one pair of the packed path sweep: its byte offset in the
// workspace, checked against the chunk; nullptr for no job.
__device__ __forceinline__ uint32_t* trace_record(const KParams& P, const TraceArgs& T, int pair, PairJob& J, int W,
                                                  int R) {
    if (J.m <= 0) return nullptr;
    const int64_t off = T.rec_off[pair] - (int64_t)T.chunk * T.chunk_bytes;
    const int64_t bytes = trace_record_bytes(W, R, J.m);
    if (off < 0 || off + bytes > T.ws_bytes || (off & 15) != 0) {
        atomicOr(&P.flags[kFlagInternal], 1);
        J.n = 0; J.m = 0;
        return nullptr;
    }
    return reinterpret_cast<uint32_t*>(T.ws + off);
}

// Path sweep of the wave item, two pairs per W-lane group packed in int16
// halves (pair A low, pair B high), biased by kI16Bias as in the packed
// score sweep: a pair runs here when S <= kI16Limit, which bounds every
// value of its box.  The 4-bit codes of rows 4q..4q+3 of both pairs build up
// in one register (pair A in the low half); two v_perm_b32 split each
// 8 rows into pair A's and pair B's record dword.
template <int W, int R>
__device__ __forceinline__ void sweep_trace_i16(const KParams& P, const TraceArgs& T, const SchemeLds& S,
                                                uint16_t* wbuf, uint32_t* stg, int first, int count, int lane) {
    constexpr int NW = R / 8;   // whole dwords of 8 rows per pair; R % 8 == 4 adds a 16-bit tail
    constexpr int G = 64 / W;
    const RecordStage<W, R, 2 * G> rs{stg};
    constexpr uint32_t K = kI16Bias;
    constexpr uint32_t K2 = K | (K << 16);
    using Stager = RefStager<W>;
    const int g = lane / W;
    const int l = lane % W;

    const int slot = g * 2;
    const int pairA = slot < count ? P.order[first + slot] : -1;
    const int pairB = slot + 1 < count ? P.order[first + slot + 1] : -1;
    PairJob JA = box_job(P, pairA, W * R);
    PairJob JB = box_job(P, pairB, W * R);
    uint32_t* recA = trace_record(P, T, pairA, JA, W, R);
    uint32_t* recB = trace_record(P, T, pairB, JB, W, R);
    const int stepsA = JA.m > 0 ? JA.m + W - 1 : 0;
    const int stepsB = JB.m > 0 ? JB.m + W - 1 : 0;
    uint32_t rowbits = 0;   // flush chunks in lanes with box rows (pairs A, B of each group)
#pragma unroll
    for (int p = 0; p < 2 * G; ++p)
        rowbits |= rs.row_bits(p, __builtin_amdgcn_readlane((p & 1) ? JB.n : JA.n, (p / 2) * W), lane);
    int mmax = imax(JA.m, JB.m);
    for (int off = 32; off > 0; off >>= 1) mmax = imax(mmax, __shfl_xor(mmax, off));
    const int steps = __builtin_amdgcn_readfirstlane(mmax > 0 ? mmax + W - 1 : 0);

    uint16_t* bufA = wbuf + (g * 2) * Stager::kBuf;
    uint16_t* bufB = bufA + Stager::kBuf;
    Stager stA, stB;
    stA.load(P.refs, JA, P.order, 0, l);
    stB.load(P.refs, JB, P.order, 0, l);
    const int AA = S.alphabet[JA.sid], AB = S.alphabet[JB.sid];
    uint32_t apk[R];
    {
        int rawA[R], rawB[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = l * R + r;
            const int iA = i < JA.n ? i : (JA.n > 0 ? JA.n - 1 : 0);
            const int iB = i < JB.n ? i : (JB.n > 0 ? JB.n - 1 : 0);
            const uint8_t* pA = JA.n > 0 ? P.queries + JA.qbase + iA : reinterpret_cast<const uint8_t*>(P.order);
            const uint8_t* pB = JB.n > 0 ? P.queries + JB.qbase + iB : reinterpret_cast<const uint8_t*>(P.order);
            rawA[r] = *pA;
            rawB[r] = *pB;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = l * R + r;
            const uint32_t a = (i < JA.n && rawA[r] < AA) ? rawA[r] : kPad;
            const uint32_t b = (i < JB.n && rawB[r] < AB) ? rawB[r] : kPad;
            apk[r] = a | (b << 16);
        }
    }
    bool bad = false;   // residues were checked by the score passes
    stA.store(bufA, JA, AA, 0, l, bad);
    stB.store(bufB, JB, AB, 0, l, bad);
    const u16x2 go2 = pk(cost16(S.gap_open[JA.sid]) | (cost16(S.gap_open[JB.sid]) << 16));
    const u16x2 ge2 = pk(cost16(S.gap_extend[JA.sid]) | (cost16(S.gap_extend[JB.sid]) << 16));
    const u16x2 zero = pk(K2);
    wave_lds_sync();

    // H0/H1[r]: H of row r at the last column swept (even steps read H0 and
    // write H1, odd steps the reverse, so that no register is copied per
    // row, as in the column-word form); E[r]: E of row r at the next column
    u16x2 H0[R], H1[R], E[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { H0[r] = zero; E[r] = zero; }
    uint32_t Hlast = K2, Flast = K2, Hup_prev = K2;
    const uint16_t* rblA = bufA + W - l;
    const uint16_t* rblB = bufB + W - l;
    u16x2 sc[R];
    int bbA_next = rblA[1], bbB_next = rblB[1];
    {
        const int a0 = rblA[0], b0 = rblB[0];
#pragma unroll
        for (int r = 0; r < R; ++r) sc[r] = load_scores(S.mat, a0 + (int)(apk[r] & 0xFFFF), b0 + (int)(apk[r] >> 16));
    }
    auto step = [&](u16x2 (&Ho)[R], u16x2 (&Hn)[R], int t0, int tt) {
        const int bbA2 = rblA[tt + 2];
        const int bbB2 = rblB[tt + 2];
        const u16x2 Hup = pk((uint32_t)shift_in_group<W>((int)Hlast, (int)K2));
        const u16x2 Fup = pk((uint32_t)shift_in_group_zero<W>((int)Flast));
        u16x2 diag = pk(Hup_prev);
        Hup_prev = u32(Hup);
        u16x2 Hmu = pk_sat_sub(Hup, go2);
        u16x2 F = Fup;
        uint32_t acc[2 * NW + 2];   // per 8 rows: D, N streams and FX, EX streams
#pragma unroll
        for (int r = 0; r < R; ++r) {
            F = pk_max3(pk_sat_sub(F, ge2), Hmu, zero);
            const u16x2 d = diag + sc[r];
            const u16x2 h = pk_max3(d, E[r], F);
            const uint32_t p1 = flag_gather(u32(d - h), u32(F - h));
            const uint32_t xf = u32(Hmu - F);
            sc[r] = load_scores(S.mat, bbA_next + (int)(apk[r] & 0xFFFF), bbB_next + (int)(apk[r] >> 16));
            diag = Ho[r];
            Hn[r] = h;
            Hmu = pk_sat_sub(h, go2);
            E[r] = pk_max3(pk_sat_sub(E[r], ge2), Hmu, zero);
            const uint32_t p2 = flag_gather(xf, u32(Hmu - E[r]));
            uint32_t& a1 = acc[2 * (r / 8)];
            uint32_t& a2 = acc[2 * (r / 8) + 1];
            a1 = r % 8 == 0 ? p1 : flag_push(a1, p1);
            a2 = r % 8 == 0 ? p2 : flag_push(a2, p2);
        }
        Hlast = u32(Hn[R - 1]);
        Flast = u32(F);
        bbA_next = bbA2;
        bbB_next = bbB2;
        // a stream pair (D, N of A and B; FX, EX of A and B) per 8 rows
        // becomes one dword per pair; the last 4 rows of R % 8 == 4 sit in
        // bits 4-7 of their stream bytes and become the 16-bit tails
        uint32_t va[NW + 1], vb[NW + 1];
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            va[k] = __builtin_amdgcn_perm(acc[2 * k + 1], acc[2 * k], 0x05040100u);
            vb[k] = __builtin_amdgcn_perm(acc[2 * k + 1], acc[2 * k], 0x07060302u);
        }
        uint32_t tail = 0;
        if constexpr (R % 8 == 4)
            tail = (acc[2 * NW] & 0xF0F0F0F0u) | ((acc[2 * NW + 1] >> 4) & 0x0F0F0F0Fu);
        const int t = t0 + tt;
        rs.put(2 * g, l, t, va, tail);
        rs.put(2 * g + 1, l, t, vb, tail >> 16);
        if ((t & (kStage - 1)) == kStage - 1 || t == steps - 1) {
            wave_lds_sync();
            rs.flush(t, lane, rowbits, [&](int p) { return readlane_ptr((p & 1) ? recB : recA, (p / 2) * W); },
                     [&](int p) { return __builtin_amdgcn_readlane((p & 1) ? stepsB : stepsA, (p / 2) * W); });
            wave_lds_sync();
        }
    };
    for (int t0 = 0; t0 < steps; t0 += kChunk) {
        const bool more = t0 + kChunk < steps;
        if (more) {
            stA.load(P.refs, JA, P.order, t0 + kChunk, l);
            stB.load(P.refs, JB, P.order, t0 + kChunk, l);
        }
        const int tn = __builtin_amdgcn_readfirstlane(steps - t0 < kChunk ? steps - t0 : kChunk);
        int tt = 0;
        for (; tt + 1 < tn; tt += 2) {
            step(H0, H1, t0, tt);
            step(H1, H0, t0, tt + 1);
        }
        static_assert(kChunk % 2 == 0, "every chunk but the last ends on an odd step");
        if (tt < tn) {
            // an odd chunk (only the last one) ends in H1
            step(H0, H1, t0, tt);
#pragma unroll
            for (int r = 0; r < R; ++r) H0[r] = H1[r];
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
}

// Small-alphabet ("column word") form of sweep_trace_i16, for wave items
// whose pairs all use schemes with at most four residues whose scores plus
// the gap open cost fit a byte.  The reference is staged as one 32-bit word
// per column holding M[a][b] + o for a = 0..3, so a row's score is one
// v_perm_b32 of the two pairs' words with the row's selector; rows past the
// box and padding columns read a zero byte, i.e. a score of -o <= -1, as
// the padding code does in the table form.  Each row keeps Hm = H - o:
// H(i-1, j-1) + M = Hm(i-1, j-1) + (M + o), and Hm is what E, F, the lane
// exchange and the E-extends test need.  Every H, E and F, and therefore
// every record bit, equals the table form's.
template <int W, int R>
__device__ __forceinline__ void sweep_trace_i16_col(const KParams& P, const TraceArgs& T, const SchemeLds& S,
                                                    uint16_t* wbuf, uint32_t* stg, int first, int count,
                                                    int lane) {
    constexpr int NW = R / 8;
    constexpr int G = 64 / W;
    const RecordStage<W, R, 2 * G> rs{stg};
    constexpr uint32_t K = kI16Bias;
    constexpr uint32_t K2 = K | (K << 16);
    using Stager = RefStager<W>;
    const int g = lane / W;
    const int l = lane % W;

    const int slot = g * 2;
    const int pairA = slot < count ? P.order[first + slot] : -1;
    const int pairB = slot + 1 < count ? P.order[first + slot + 1] : -1;
    PairJob JA = box_job(P, pairA, W * R);
    PairJob JB = box_job(P, pairB, W * R);
    uint32_t* recA = trace_record(P, T, pairA, JA, W, R);
    uint32_t* recB = trace_record(P, T, pairB, JB, W, R);
    const int stepsA = JA.m > 0 ? JA.m + W - 1 : 0;
    const int stepsB = JB.m > 0 ? JB.m + W - 1 : 0;
    uint32_t rowbits = 0;   // flush chunks in lanes with box rows (pairs A, B of each group)
#pragma unroll
    for (int p = 0; p < 2 * G; ++p)
        rowbits |= rs.row_bits(p, __builtin_amdgcn_readlane((p & 1) ? JB.n : JA.n, (p / 2) * W), lane);
    int mmax = imax(JA.m, JB.m);
    for (int off = 32; off > 0; off >>= 1) mmax = imax(mmax, __shfl_xor(mmax, off));
    const int steps = __builtin_amdgcn_readfirstlane(mmax > 0 ? mmax + W - 1 : 0);

    // 32-bit column words: the wave buffer holds twice as many bytes
    uint32_t* bufA = reinterpret_cast<uint32_t*>(wbuf) + (g * 2) * Stager::kBuf;
    uint32_t* bufB = bufA + Stager::kBuf;
    Stager stA, stB;
    stA.load(P.refs, JA, P.order, 0, l);
    stB.load(P.refs, JB, P.order, 0, l);
    const int AA = S.alphabet[JA.sid], AB = S.alphabet[JB.sid];
    // per-row selectors: byte 0 picks pair A's score from its column word
    // (bytes 0..3 of the perm input), byte 2 pair B's (bytes 4..7); bytes 1
    // and 3, and a row past the box, select zero (0x0C)
    uint32_t sel[R];
    {
        int rawA[R], rawB[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = l * R + r;
            const int iA = i < JA.n ? i : (JA.n > 0 ? JA.n - 1 : 0);
            const int iB = i < JB.n ? i : (JB.n > 0 ? JB.n - 1 : 0);
            const uint8_t* pA = JA.n > 0 ? P.queries + JA.qbase + iA : reinterpret_cast<const uint8_t*>(P.order);
            const uint8_t* pB = JB.n > 0 ? P.queries + JB.qbase + iB : reinterpret_cast<const uint8_t*>(P.order);
            rawA[r] = *pA;
            rawB[r] = *pB;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = l * R + r;
            const uint32_t a = (i < JA.n && rawA[r] < AA) ? (uint32_t)rawA[r] : 0x0Cu;
            const uint32_t b = (i < JB.n && rawB[r] < AB) ? (uint32_t)(4 + rawB[r]) : 0x0Cu;
            sel[r] = a | 0x0C00u | (b << 16) | 0x0C000000u;
        }
    }
    bool bad = false;   // residues were checked by the score passes
    stA.store_col(bufA, JA, AA, S.colw[JA.sid], 0, l, bad);
    stB.store_col(bufB, JB, AB, S.colw[JB.sid], 0, l, bad);
    const uint32_t goA = (uint32_t)S.gap_open[JA.sid], goB = (uint32_t)S.gap_open[JB.sid];
    const u16x2 go2 = pk(goA | (goB << 16));
    const u16x2 ge2 = pk(cost16(S.gap_extend[JA.sid]) | (cost16(S.gap_extend[JB.sid]) << 16));
    const u16x2 zero = pk(K2);
    const uint32_t hm_top = (K - goA) | ((K - goB) << 16);   // Hm of the zero boundary
    wave_lds_sync();

    // Hm0/Hm1[r]: H - o of row r at the last column swept (even steps read
    // Hm0 and write Hm1, odd steps the reverse: a row's old value is still
    // needed as the next row's diagonal after its new one is computed, so one
    // array would cost a register copy per row); E[r]: E of row r at the
    // next column
    u16x2 Hm0[R], Hm1[R], E[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { Hm0[r] = pk(hm_top); E[r] = zero; }
    uint32_t Hlast = hm_top, Flast = K2, Hup_prev = hm_top;
    const uint32_t* rblA = bufA + W - l;   // rblA[tt] = column word of step t0 + tt
    const uint32_t* rblB = bufB + W - l;
    // step t of the chunk: Ho holds the last column's Hm, Hn receives this
    // one's; (ca, cb) are this step's column words, the next step's are
    // read into (na, nb)
    auto step = [&](u16x2 (&Ho)[R], u16x2 (&Hn)[R], uint32_t ca, uint32_t cb, uint32_t& na, uint32_t& nb,
                    int t0, int tt) {
        na = rblA[tt + 1];
        nb = rblB[tt + 1];
        const u16x2 Hmu0 = pk((uint32_t)shift_in_group<W>((int)Hlast, (int)hm_top));
        // F above the group is 0 (K); a zero fill gives the same F below
        // because of the max with K
        const u16x2 Fup = pk((uint32_t)shift_in_group_zero<W>((int)Flast));
        u16x2 diag = pk(Hup_prev);
        Hup_prev = u32(Hmu0);
        u16x2 Hmu = Hmu0;
        u16x2 F = Fup;
        uint32_t acc[2 * NW + 2];   // per 8 rows: D, N streams and FX, EX streams
#pragma unroll
        for (int r = 0; r < R; ++r) {
            F = pk_max3(pk_sat_sub(F, ge2), Hmu, zero);
            const u16x2 d = diag + pk(__builtin_amdgcn_perm(cb, ca, sel[r]));
            const u16x2 h = pk_max3(d, E[r], F);
            const uint32_t p1 = flag_gather(u32(d - h), u32(F - h));
            const uint32_t xf = u32(Hmu - F);
            diag = Ho[r];
            Hmu = h - go2;
            Hn[r] = Hmu;
            E[r] = pk_max3(pk_sat_sub(E[r], ge2), Hmu, zero);
            const uint32_t p2 = flag_gather(xf, u32(Hmu - E[r]));
            uint32_t& a1 = acc[2 * (r / 8)];
            uint32_t& a2 = acc[2 * (r / 8) + 1];
            a1 = r % 8 == 0 ? p1 : flag_push(a1, p1);
            a2 = r % 8 == 0 ? p2 : flag_push(a2, p2);
        }
        Hlast = u32(Hn[R - 1]);
        Flast = u32(F);
        // a stream pair (D, N of A and B; FX, EX of A and B) per 8 rows
        // becomes one dword per pair; the last 4 rows of R % 8 == 4 sit in
        // bits 4-7 of their stream bytes and become the 16-bit tails
        uint32_t va[NW + 1], vb[NW + 1];
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            va[k] = __builtin_amdgcn_perm(acc[2 * k + 1], acc[2 * k], 0x05040100u);
            vb[k] = __builtin_amdgcn_perm(acc[2 * k + 1], acc[2 * k], 0x07060302u);
        }
        uint32_t tail = 0;
        if constexpr (R % 8 == 4)
            tail = (acc[2 * NW] & 0xF0F0F0F0u) | ((acc[2 * NW + 1] >> 4) & 0x0F0F0F0Fu);
        const int t = t0 + tt;
        rs.put(2 * g, l, t, va, tail);
        rs.put(2 * g + 1, l, t, vb, tail >> 16);
        if ((t & (kStage - 1)) == kStage - 1 || t == steps - 1) {
            wave_lds_sync();
            rs.flush(t, lane, rowbits, [&](int p) { return readlane_ptr((p & 1) ? recB : recA, (p / 2) * W); },
                     [&](int p) { return __builtin_amdgcn_readlane((p & 1) ? stepsB : stepsA, (p / 2) * W); });
            wave_lds_sync();
        }
    };
    uint32_t cA0 = rblA[0], cB0 = rblB[0], cA1 = 0, cB1 = 0;
    for (int t0 = 0; t0 < steps; t0 += kChunk) {
        const bool more = t0 + kChunk < steps;
        if (more) {
            stA.load(P.refs, JA, P.order, t0 + kChunk, l);
            stB.load(P.refs, JB, P.order, t0 + kChunk, l);
        }
        const int tn = __builtin_amdgcn_readfirstlane(steps - t0 < kChunk ? steps - t0 : kChunk);
        int tt = 0;
        for (; tt + 1 < tn; tt += 2) {
            step(Hm0, Hm1, cA0, cB0, cA1, cB1, t0, tt);
            step(Hm1, Hm0, cA1, cB1, cA0, cB0, t0, tt + 1);
        }
        static_assert(kChunk % 2 == 0, "every chunk but the last ends on an odd step");
        if (tt < tn) {
            // an odd chunk (only the last one) ends in Hm1
            step(Hm0, Hm1, cA0, cB0, cA1, cB1, t0, tt);
#pragma unroll
            for (int r = 0; r < R; ++r) Hm0[r] = Hm1[r];
        }
        if (more) {
            wave_lds_sync();
            stA.store_col(bufA, JA, AA, S.colw[JA.sid], t0 + kChunk, l, bad);
            stB.store_col(bufB, JB, AB, S.colw[JB.sid], t0 + kChunk, l, bad);
            wave_lds_sync();
            cA0 = rblA[0];
            cB0 = rblB[0];
        }
    }
}

// LDS reference buffer of one wavefront (16-bit entries): four 16-lane
// groups of two packed pairs, the widest layout.
constexpr int kTraceWaveBuf = 8 * RefStager<16>::kBuf;
// and of its column-word form (32-bit entries)
constexpr int kTraceWaveBufCol = 2 * kTraceWaveBuf;

// Work-queue kernel of one path-sweep shape (same fetch loop as the score
// sweeps' queue kernels).
template <int PREC, int W, int R, bool COL>
__global__ __launch_bounds__(kBlock) void sw_trace_kernel(KParams P, TraceArgs T) {
    constexpr int kPPW = (64 / W) * (PREC == 16 ? 2 : 1);
    constexpr int kStageDwords = RecordStage<W, R, kPPW>::kDwords;
    constexpr int kWaveBuf = COL ? kTraceWaveBufCol : kTraceWaveBuf;
    __shared__ __attribute__((aligned(16))) SchemeLds L;
    __shared__ __attribute__((aligned(16))) uint16_t wbufs[kWavesPerBlock * kWaveBuf];
    __shared__ __attribute__((aligned(16))) uint32_t stages[kWavesPerBlock * kStageDwords];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    int lo = __atomic_load_n(&P.meta[P.lo_idx], __ATOMIC_RELAXED);
    int hi = __atomic_load_n(&P.meta[P.hi_idx], __ATOMIC_RELAXED);
    lo = __builtin_amdgcn_readfirstlane(lo);
    hi = __builtin_amdgcn_readfirstlane(hi);
    if (lo == hi) return;
    if (lo < 0 || hi > P.max_items || lo > hi) {
        if (tid == 0) atomicOr(&P.flags[kFlagInternal], 1);
        return;
    }
    const int n_pairs = __builtin_amdgcn_readfirstlane(*P.n_dev);
    load_schemes(L, P, tid);
    __syncthreads();
    uint16_t* wbuf = wbufs + wave * kWaveBuf;
    for (;;) {
        const int mine = atomicAdd(&P.meta[P.head_idx], lane == 0 ? 1 : 0);
        const int it = __builtin_amdgcn_readlane(mine, 0);
        if (it >= hi - lo) break;
        const WorkItem* wp = P.items + lo + it;
        const int first = __builtin_amdgcn_readfirstlane(__atomic_load_n(&wp->first, __ATOMIC_RELAXED));
        const int count = __builtin_amdgcn_readfirstlane((int)__atomic_load_n(&wp->count, __ATOMIC_RELAXED));
        const bool valid = first >= 0 && count >= 1 && count <= kPPW && first + count <= n_pairs;
        if (valid) {
            wave_lds_sync();
            if constexpr (PREC == 16 && COL)
                sweep_trace_i16_col<W, R>(P, T, L, wbuf, stages + wave * kStageDwords, first, count, lane);
            else if constexpr (PREC == 16)
                sweep_trace_i16<W, R>(P, T, L, wbuf, stages + wave * kStageDwords, first, count, lane);
            else
                sweep_trace<W, R>(P, T, L, wbuf, stages + wave * kStageDwords, first, count, lane);
        } else {
            atomicOr(&P.flags[kFlagInternal], 1);
        }
    }
}

// ---- box-sweep families -----------------------------------------------------
// One launch per lane width: the kernel drains the queue of member k's bin
// (P.fam_bins[k]; -1: not launched), then member k+1's, each with the box
// sweep compiled for that shape, as the score sweeps' family kernels do.
// The LDS record stage is sized for the largest member.
template <int PREC, int W, int R, bool COL>
__device__ __forceinline__ void trace_member(const KParams& P, const TraceArgs& T, SchemeLds& L, uint16_t* wbuf,
                                             uint32_t* stage, int lane, int bin, int n_pairs) {
    constexpr int kPPW = (64 / W) * (PREC == 16 ? 2 : 1);
    if (bin < 0) return;
    const int lo_i = COL ? kMetaItemFirst + bin : kMetaItemSplit + bin;
    const int hi_i = COL ? kMetaItemSplit + bin : kMetaItemFirst + bin + 1;
    const int lo = __builtin_amdgcn_readfirstlane(__atomic_load_n(&P.meta[lo_i], __ATOMIC_RELAXED));
    const int hi = __builtin_amdgcn_readfirstlane(__atomic_load_n(&P.meta[hi_i], __ATOMIC_RELAXED));
    if (lo >= hi) return;
    if (lo < 0 || hi > P.max_items) {
        atomicOr(&P.flags[kFlagInternal], 1);
        return;
    }
    const int head = (COL ? kMetaColHeads : kMetaHeads) + bin;
    for (;;) {
        const int mine = atomicAdd(&P.meta[head], lane == 0 ? 1 : 0);
        const int it = __builtin_amdgcn_readlane(mine, 0);
        if (it >= hi - lo) break;
        const WorkItem* wp = P.items + lo + it;
        const int first = __builtin_amdgcn_readfirstlane(__atomic_load_n(&wp->first, __ATOMIC_RELAXED));
        const int count = __builtin_amdgcn_readfirstlane((int)__atomic_load_n(&wp->count, __ATOMIC_RELAXED));
        const bool valid = first >= 0 && count >= 1 && count <= kPPW && first + count <= n_pairs;
        if (valid) {
            wave_lds_sync();
            if constexpr (PREC == 16 && COL)
                sweep_trace_i16_col<W, R>(P, T, L, wbuf, stage, first, count, lane);
            else if constexpr (PREC == 16)
                sweep_trace_i16<W, R>(P, T, L, wbuf, stage, first, count, lane);
            else
                sweep_trace<W, R>(P, T, L, wbuf, stage, first, count, lane);
        } else {
            atomicOr(&P.flags[kFlagInternal], 1);
        }
    }
}

template <int... Rs>
constexpr int max_rows() {
    int m = 0;
    for (int r : {Rs...}) m = r > m ? r : m;
    return m;
}

template <int PREC, int W, bool COL, int... Rs>
__global__ __launch_bounds__(kBlock) void sw_trace_family_kernel(KParams P, TraceArgs T) {
    constexpr int kPPW = (64 / W) * (PREC == 16 ? 2 : 1);
    constexpr int kStageDwords = RecordStage<W, max_rows<Rs...>(), kPPW>::kDwords;
    constexpr int kWaveBuf = COL ? kTraceWaveBufCol : kTraceWaveBuf;
    static_assert(sizeof...(Rs) <= kFamilyMax, "family too large");
    __shared__ __attribute__((aligned(16))) SchemeLds L;
    __shared__ __attribute__((aligned(16))) uint16_t wbufs[kWavesPerBlock * kWaveBuf];
    __shared__ __attribute__((aligned(16))) uint32_t stages[kWavesPerBlock * kStageDwords];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int n_pairs = __builtin_amdgcn_readfirstlane(*P.n_dev);
    load_schemes(L, P, tid);
    __syncthreads();
    uint16_t* wbuf = wbufs + wave * kWaveBuf;
    uint32_t* stage = stages + wave * kStageDwords;
    int k = 0;
    ((trace_member<PREC, W, Rs, COL>(P, T, L, wbuf, stage, lane, P.fam_bins[k++], n_pairs)), ...);
}

#define SW_TRACE_SHAPES(X, P)                                                                          \
    X(P, 16, 4) X(P, 16, 8) X(P, 16, 12) X(P, 16, 16) X(P, 32, 12) X(P, 32, 16) X(P, 64, 12) X(P, 64, 16) \
    X(P, 64, 20) X(P, 64, 24) X(P, 64, 28) X(P, 64, 32)

namespace {
struct TraceEntry { int prec, W, R; TraceFn fn, col; };
#define SW_TRACE_ENTRY16(P, W, R) {P, W, R, &sw_trace_kernel<P, W, R, false>, &sw_trace_kernel<P, W, R, true>},
#define SW_TRACE_ENTRY32(P, W, R) {P, W, R, &sw_trace_kernel<P, W, R, false>, nullptr},
const TraceEntry kTraceKernels[] = {SW_TRACE_SHAPES(SW_TRACE_ENTRY16, 16) SW_TRACE_SHAPES(SW_TRACE_ENTRY32, 32)};
#undef SW_TRACE_ENTRY16
#undef SW_TRACE_ENTRY32
constexpr int kNumTrace = sizeof(kTraceKernels) / sizeof(kTraceKernels[0]);
ShapeDesc g_trace_shapes[kNumTrace];
}  // namespace

const ShapeDesc* trace_shapes(int* n) {
    for (int k = 0; k < kNumTrace; ++k)
        g_trace_shapes[k] = {kTraceKernels[k].prec, kTraceKernels[k].W, kTraceKernels[k].R};
    *n = kNumTrace;
    return g_trace_shapes;
}

namespace {
// Box-sweep families, largest rows first (the order of KParams::fam_bins).
const TraceFamily kTraceFamilies[] = {
    {16, 16, 4, {16, 12, 8, 4}, &sw_trace_family_kernel<16, 16, false, 16, 12, 8, 4>,
     &sw_trace_family_kernel<16, 16, true, 16, 12, 8, 4>},
    {16, 32, 2, {16, 12}, &sw_trace_family_kernel<16, 32, false, 16, 12>, &sw_trace_family_kernel<16, 32, true, 16, 12>},
    {16, 64, 6, {32, 28, 24, 20, 16, 12}, &sw_trace_family_kernel<16, 64, false, 32, 28, 24, 20, 16, 12>,
     &sw_trace_family_kernel<16, 64, true, 32, 28, 24, 20, 16, 12>},
};
}  // namespace

const TraceFamily* trace_family(int prec, int W, int R) {
    for (const TraceFamily& f : kTraceFamilies)
        if (f.prec == prec && f.W == W)
            for (int k = 0; k < f.n; ++k)
                if (f.rows[k] == R) return &f;
    return nullptr;
}

TraceFn trace_kernel(int prec, int W, int R, bool col) {
    for (int k = 0; k < kNumTrace; ++k)
        if (kTraceKernels[k].prec == prec && kTraceKernels[k].W == W && kTraceKernels[k].R == R)
            return col ? kTraceKernels[k].col : kTraceKernels[k].fn;
    return nullptr;
}

// Path-sweep bin of a pair: packed int16 when its score allows, by box rows.
__device__ __forceinline__ int trace_bin(const TraceArgs& T, int score, int rows) {
    const int sel = score <= T.i16_limit ? 0 : 1;
    return T.lut[sel * kLutRows + (rows - 1) / 16];
}

// ---- record sizes and offsets ----------------------------------------------
constexpr int kScanThreads = 1024;

__device__ __forceinline__ long long wave_scan64(long long v, int lane) {
    for (int off = 1; off < 64; off <<= 1) {
        const long long u = __shfl_up(v, off);
        if (lane >= off) v += u;
    }
    return v;
}

// Exclusive scan within one block of kScanThreads values; returns the
// block total through *total.
__device__ __forceinline__ long long block_exclusive_scan(long long v, long long* total) {
    __shared__ long long wave_tot[kScanThreads / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const long long incl = wave_scan64(v, lane);
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    long long before = 0, all = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
        const long long x = wave_tot[w];
        before += w < wave ? x : 0;
        all += x;
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

// Record size of every pair (0 without an alignment), scanned per block:
// rec_off[i] = offset within the block, block_sums[b] = the block's total.
// Also counts the box cells.
__global__ __launch_bounds__(kScanThreads) void sw_trace_size_kernel(KParams P, TraceArgs T, int64_t* rec_off,
                                                                     int64_t* block_sums,
                                                                     unsigned long long* counters) {
    const int64_t n = *P.n_dev;
    const int64_t i = (int64_t)blockIdx.x * kScanThreads + threadIdx.x;
    long long bytes = 0;
    unsigned long long cells = 0;
    if (i < n) {
        const sw_result r = P.out[i];
        if (r.score > 0) {
            const int64_t nq = P.q_end[i] - P.q_beg[i], nr = P.r_end[i] - P.r_beg[i];
            const int rows = r.q_end - r.q_start + 1, cols = r.r_end - r.r_start + 1;
            if (r.q_start < 0 || rows < 1 || r.q_end >= nq || rows > SW_MAX_QUERY || r.r_start < 0 || cols < 1 ||
                r.r_end >= nr || cols > SW_MAX_REF) {
                atomicOr(&P.flags[kFlagInternal], 1);
            } else {
                const int b = trace_bin(T, r.score, rows);
                if (b < 0 || b >= T.n_bins || T.bins[b].W * T.bins[b].R < rows) {
                    atomicOr(&P.flags[kFlagInternal], 1);
                } else {
                    bytes = trace_record_bytes(T.bins[b].W, T.bins[b].R, cols);
                    bytes = (bytes + 15) & ~15ll;
                    cells = (unsigned long long)rows * (unsigned long long)cols;
                }
            }
        }
    }
    long long total;
    const long long ex = block_exclusive_scan(bytes, &total);
    if (i <= n) rec_off[i] = ex;
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
    // box cells of the block
    __shared__ unsigned long long s_cells;
    if (threadIdx.x == 0) s_cells = 0;
    __syncthreads();
    if (cells) atomicAdd(&s_cells, cells);
    __syncthreads();
    if (threadIdx.x == 0 && s_cells) atomicAdd(&counters[kCtrTraceCells], s_cells);
}

// Exclusive scan of the block totals in place (one block); block_sums[nb]
// receives the grand total.
__global__ __launch_bounds__(kScanThreads) void sw_trace_scan_sums_kernel(int64_t* block_sums, int64_t nb) {
    long long carry = 0;
    for (int64_t base = 0; base < nb; base += kScanThreads) {
        const int64_t k = base + threadIdx.x;
        const long long v = k < nb ? block_sums[k] : 0;
        long long total;
        const long long ex = block_exclusive_scan(v, &total);
        if (k < nb) block_sums[k] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) block_sums[nb] = carry;
}

// rec_off[i] += the offset of its block; rec_off[n] = the total.
__global__ __launch_bounds__(kScanThreads) void sw_trace_add_kernel(const KParams P, int64_t* rec_off,
                                                                    const int64_t* block_sums, int64_t nb) {
    const int64_t n = *P.n_dev;
    const int64_t i = (int64_t)blockIdx.x * kScanThreads + threadIdx.x;
    if (i < n) rec_off[i] += block_sums[blockIdx.x];
    if (i == n) rec_off[n] = block_sums[nb];
}

int64_t trace_scan_blocks(int64_t cap) { return (cap + 1 + kScanThreads - 1) / kScanThreads; }

hipError_t launch_trace_sizes(const KParams& P, const TraceArgs& T, int64_t cap, int64_t* rec_off,
                              int64_t* block_sums, unsigned long long* counters, hipStream_t s) {
    const int64_t nb = trace_scan_blocks(cap);
    hipLaunchKernelGGL(sw_trace_size_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, P, T, rec_off,
                       block_sums, counters);
    hipLaunchKernelGGL(sw_trace_scan_sums_kernel, dim3(1), dim3(kScanThreads), 0, s, block_sums, nb);
    hipLaunchKernelGGL(sw_trace_add_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, P, rec_off,
                       (const int64_t*)block_sums, nb);
    return hipGetLastError();
}

// ---- planning of one chunk ---------------------------------------------------
// Keys as in the score passes' classification: (bin, reference-length
// bucket, longest first); pairs outside the chunk or without an alignment
// get the trivial key.
__global__ void sw_trace_classify_kernel(KParams P, TraceArgs T, int32_t* keys, int32_t* hist,
                                         unsigned long long* counters, int32_t* path_len) {
    __shared__ unsigned long long s_cells[kMaxBins];
    __shared__ uint32_t s_pairs[kMaxBins];
    __shared__ int32_t s_trivial;
    if (threadIdx.x < kMaxBins) { s_cells[threadIdx.x] = 0; s_pairs[threadIdx.x] = 0; }
    if (threadIdx.x == 0) s_trivial = 0;
    __syncthreads();
    const int64_t n = *P.n_dev;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        int key = kTrivialKey;
        const sw_result r = P.out[i];
        if (r.score <= 0 && T.chunk == 0) path_len[i] = 0;   // no alignment, no path
        if (r.score > 0 && T.rec_off[i] / T.chunk_bytes == T.chunk) {
            const int rows = r.q_end - r.q_start + 1, cols = r.r_end - r.r_start + 1;
            // sizes were validated when the records were laid out
            if (rows >= 1 && rows <= SW_MAX_QUERY && cols >= 1 && cols <= SW_MAX_REF) {
                const int b = trace_bin(T, r.score, rows);
                if (b >= 0 && b < T.n_bins) {
                    // pairs of column-path schemes first (the bin's
                    // column-word kernel takes them; the host enables the
                    // column path only when every scheme of the call has it)
                    const int sid = P.scheme_id ? (int)P.scheme_id[i] : 0;
                    const int col = (T.bins[b].col && sid < SW_MAX_SCHEMES && P.col_ok[sid]) ? 1 : 0;
                    key = b * kMBuckets + (col ? 0 : kMHalf) + (kMHalf - 1 - m_bucket(cols));
                    atomicAdd(&s_cells[b], (unsigned long long)rows * (unsigned long long)cols);
                    atomicAdd(&s_pairs[b], 1u);
                }
            }
        }
        if (key == kTrivialKey) atomicAdd(&s_trivial, 1);
        else atomicAdd(&hist[key], 1);
        keys[i] = key;
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_trivial) atomicAdd(&hist[kTrivialKey], s_trivial);
    if (threadIdx.x < kMaxBins && s_pairs[threadIdx.x]) {
        atomicAdd(&counters[kCtrTraceBinCells + threadIdx.x], s_cells[threadIdx.x]);
        atomicAdd(&counters[kCtrTraceBinPairs + threadIdx.x], (unsigned long long)s_pairs[threadIdx.x]);
    }
}

hipError_t launch_trace_classify(const KParams& P, const TraceArgs& T, int64_t cap, int32_t* keys,
                                 int32_t* hist, unsigned long long* counters, int32_t* path_len, hipStream_t s) {
    if (cap <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((cap + 255) / 256);
    hipLaunchKernelGGL(sw_trace_classify_kernel, dim3(blocks), dim3(256), 0, s, P, T, keys, hist, counters,
                       path_len);
    return hipGetLastError();
}

// ---- walk ------------------------------------------------------------------------
// One thread per pair of the chunk.  Runs are written from the end of the
// pair's output room backwards while the path is followed back, then moved
// to its start.  A path that leaves its box or does not end at the box's
// first cell is an internal error; one that needs more runs than its room
// sets kFlagPathRoom.  Either way the pair's run count becomes -1.
// dwords per thread: two record blocks of up to 32 dwords, padded against
// bank conflicts
constexpr int kWalkSlot = 65;

// The 16 residues around a position, read as one aligned 16-byte load (an
// aligned 16-byte block never crosses a page, so it is readable whenever
// the residue itself is); a walk moves backwards through each sequence, so
// one load serves up to 16 of its steps.
__device__ __forceinline__ uint32_t window_at(const uint8_t* seq, int x, uintptr_t& base, uint32_t& w0, uint32_t& w1,
                                              uint32_t& w2, uint32_t& w3) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(seq + x);
    const uintptr_t b = a & ~(uintptr_t)15;
    if (b != base) {
        const uint4 v = *reinterpret_cast<const uint4*>(b);
        w0 = v.x; w1 = v.y; w2 = v.z; w3 = v.w;
        base = b;
    }
    const uint32_t o = (uint32_t)(a - b);
    const uint32_t w = o < 8 ? (o < 4 ? w0 : w1) : (o < 12 ? w2 : w3);
    return (w >> (8 * (o & 3))) & 0xFFu;
}

// Walk of pair i (whose record is in the current chunk).
__device__ __forceinline__ void walk_pair(const KParams& P, const TraceArgs& T, int i, const int64_t* path_off,
                                          uint32_t* path, int32_t* path_len, uint32_t* slot) {
    const sw_result r = P.out[i];
    const int64_t off = T.rec_off[i];
    const int rows = r.q_end - r.q_start + 1, cols = r.r_end - r.r_start + 1;
    const int b = (r.score > 0 && rows >= 1 && rows <= SW_MAX_QUERY) ? trace_bin(T, r.score, rows) : -1;
    const int64_t beg = path_off[i], end = path_off[i + 1];
    if (b < 0 || b >= T.n_bins || cols < 1 || end < beg) {
        atomicOr(&P.flags[end < beg ? kFlagPathRoom : kFlagInternal], 1);
        path_len[i] = -1;
        return;
    }
    const int W = T.bins[b].W, R = T.bins[b].R;
    const int64_t rel = off - (int64_t)T.chunk * T.chunk_bytes;
    if (W * R < rows || R > 32 || (R & 3) != 0 || rel < 0 || rel + trace_record_bytes(W, R, cols) > T.ws_bytes) {
        atomicOr(&P.flags[kFlagInternal], 1);
        path_len[i] = -1;
        return;
    }
    const uint32_t* rec = reinterpret_cast<const uint32_t*>(T.ws + rel);
    // `slot` (this thread's LDS copy) holds the record blocks of steps
    // [8 c_tb, 8 c_tb + 8) and, when c_tb >= 1, [8 c_tb - 8, 8 c_tb) of lane
    // c_lane: a walk only moves to the same or earlier steps, so the second
    // block is the next one it needs in that lane.  Both are fetched in one
    // round trip, every 16-byte load issued before the first is waited for.
    int c_lane = -1, c_tb = -1;
    const uint8_t* qa = P.queries + P.q_beg[i] + r.q_start;
    const uint8_t* rb = P.refs + P.r_beg[i] + r.r_start;
    uintptr_t qbase = ~(uintptr_t)0, rbase = ~(uintptr_t)0;
    uint32_t q0 = 0, q1 = 0, q2 = 0, q3 = 0, r0 = 0, r1 = 0, r2 = 0, r3 = 0;
    const int64_t room = end - beg;
    int x = rows - 1, y = cols - 1;
    int state = 0;   // 0 = H, 1 = F (query gap), 2 = E (reference gap), 3 = E moved, choice pending
    int64_t k = 0;   // runs written
    uint32_t op = 0, len = 0;
    int err = 0;     // 1 internal, 2 room
    const int64_t limit = 2 * ((int64_t)rows + cols) + 2;
    bool done = false;
    for (int64_t it = 0; it < limit && !err; ++it) {
        const int lane = x / R, rr = x - lane * R;
        const int t = y + lane;
        const int tb = t / kStage;
        if (lane != c_lane || tb > c_tb || tb < c_tb - 1) {
            const int nq = R / 4;   // 16-byte pieces per block (R <= 32)
            const uint4* src0 = reinterpret_cast<const uint4*>(rec + ((int64_t)tb * W + lane) * R);
            const uint4* src1 = reinterpret_cast<const uint4*>(rec + ((int64_t)(tb - 1) * W + lane) * R);
            const bool two = tb >= 1;
            uint4 v0[8], v1[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (q < nq) v0[q] = src0[q];
                if (q < nq && two) v1[q] = src1[q];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (q < nq) {
                    slot[4 * q] = v0[q].x; slot[4 * q + 1] = v0[q].y;
                    slot[4 * q + 2] = v0[q].z; slot[4 * q + 3] = v0[q].w;
                }
                if (q < nq && two) {
                    slot[R + 4 * q] = v1[q].x; slot[R + 4 * q + 1] = v1[q].y;
                    slot[R + 4 * q + 2] = v1[q].z; slot[R + 4 * q + 3] = v1[q].w;
                }
            }
            c_lane = lane;
            c_tb = tb;
        }
        // the step's R/2 bytes: a dword of D, N, FX, EX bytes per 8 rows,
        // then for R % 8 == 4 the 16-bit tail (FX, D, EX, N nibbles)
        const uint16_t* st = reinterpret_cast<const uint16_t*>(slot + (c_tb - tb) * R) + (t % kStage) * (R / 4);
        const int j = rr >> 3, kk = rr & 7;
        uint32_t fd, fn, ffx, fex;
        if (j < (R >> 3)) {
            const uint32_t v = ((uint32_t)st[2 * j] | ((uint32_t)st[2 * j + 1] << 16)) >> kk;
            fd = v & 1u; fn = (v >> 8) & 1u; ffx = (v >> 16) & 1u; fex = (v >> 24) & 1u;
        } else {
            const uint32_t v = (uint32_t)st[2 * j] >> kk;
            ffx = v & 1u; fd = (v >> 4) & 1u; fex = (v >> 8) & 1u; fn = (v >> 12) & 1u;
        }
        // a gap move from (x, y+1) left E's choice there open: this cell's
        // record holds whether E(x, y+1) extends E(x, y)
        if (state == 3) state = fex ? 2 : 0;
        uint32_t o;
        if (state == 0) {
            if (fd) { state = fn ? 2 : 1; continue; }
            o = window_at(qa, x, qbase, q0, q1, q2, q3) == window_at(rb, y, rbase, r0, r1, r2, r3) ? 7u : 8u;
            --x; --y;
        } else if (state == 1) {
            o = 1u;
            state = ffx ? 1 : 0;
            --x;
        } else {
            o = 2u;
            state = 3;
            --y;
        }
        if (o == op) {
            ++len;
        } else {
            if (len) {
                if (k >= room) { err = 2; break; }
                path[end - 1 - k] = (len << 4) | op;
                ++k;
            }
            op = o;
            len = 1;
        }
        if (x < 0 || y < 0) {
            // the first column of the path must be the box's first cell
            done = x == -1 && y == -1 && state == 0 && (o == 7u || o == 8u);
            if (!done) err = 1;
            break;
        }
    }
    if (!err && !done) err = 1;
    if (!err) {
        if (k >= room) err = 2;
        else {
            path[end - 1 - k] = (len << 4) | op;
            ++k;
        }
    }
    if (err) {
        atomicOr(&P.flags[err == 2 ? kFlagPathRoom : kFlagInternal], 1);
        path_len[i] = -1;
        return;
    }
    // runs sit at path[end-k .. end) in order; move them to the room's start
    for (int64_t q = 0; q < k; ++q) path[beg + q] = path[end - k + q];
    path_len[i] = (int32_t)k;
}

// One bin's walks: its pairs are order[meta[bin first] .. meta[next bin first]).
// A of each wavefront's lanes walk a pair each (the others return at once):
// a wavefront waits for every record block any of its walks misses, so long
// walks run few to a wavefront.
template <int A>
__global__ __launch_bounds__(256) void sw_trace_walk_kernel(KParams P, TraceArgs T, int bin, const int64_t* path_off,
                                                            uint32_t* path, int32_t* path_len) {
    __shared__ uint32_t cache[4 * A * kWalkSlot];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lo = P.meta[kMetaBinFirst + bin], hi = P.meta[kMetaBinFirst + bin + 1];
    if (lo < 0 || lo > hi || hi > P.n_pairs) {
        if (threadIdx.x == 0) atomicOr(&P.flags[kFlagInternal], 1);
        return;
    }
    if (lane >= A) return;
    uint32_t* slot = cache + (wave * A + lane) * kWalkSlot;
    const int n = *P.n_dev;
    const int stride = (int)gridDim.x * 4 * A;
    for (int k = lo + ((int)blockIdx.x * 4 + wave) * A + lane; k < hi; k += stride) {
        const int i = P.order[k];
        if (i < 0 || i >= n) {
            atomicOr(&P.flags[kFlagInternal], 1);
            continue;
        }
        walk_pair(P, T, i, path_off, path, path_len, slot);
    }
}

hipError_t launch_trace_walk(const KParams& P, const TraceArgs& T, int bin, int blocks, int active,
                             const int64_t* path_off, uint32_t* path, int32_t* path_len, hipStream_t s) {
    const dim3 grid(blocks > 0 ? blocks : 1);
    switch (active) {
        case 4: hipLaunchKernelGGL(sw_trace_walk_kernel<4>, grid, dim3(256), 0, s, P, T, bin, path_off, path, path_len); break;
        case 8: hipLaunchKernelGGL(sw_trace_walk_kernel<8>, grid, dim3(256), 0, s, P, T, bin, path_off, path, path_len); break;
        case 16: hipLaunchKernelGGL(sw_trace_walk_kernel<16>, grid, dim3(256), 0, s, P, T, bin, path_off, path, path_len); break;
        case 32: hipLaunchKernelGGL(sw_trace_walk_kernel<32>, grid, dim3(256), 0, s, P, T, bin, path_off, path, path_len); break;
        default: hipLaunchKernelGGL(sw_trace_walk_kernel<64>, grid, dim3(256), 0, s, P, T, bin, path_off, path, path_len);
    }
    return hipGetLastError();
}

}  // namespace sw
