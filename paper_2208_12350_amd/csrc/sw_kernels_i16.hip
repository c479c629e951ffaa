// sw_kernels_i16.hip -- packed 16-bit sweep kernel of libswalign (gfx950).
//
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
#include "sw_device.h"
#include "sw_internal.h"

namespace sw {

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

template <int W, int R>
__global__ __launch_bounds__(kBlock) void sw_pass_i16(KParams P, int first, int count,
                                                      int reverse) {
    constexpr int G = 64 / W;
    using Stager = RefStager<W>;
    __shared__ __attribute__((aligned(16))) SchemeLds S;
    __shared__ uint16_t refbuf[kWavesPerBlock * G * 2 * Stager::kBuf];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int g = lane / W;
    const int l = lane % W;

    load_schemes(S, P, tid);

    const int slot = ((blockIdx.x * kWavesPerBlock + wave) * G + g) * 2;
    const int pairA = slot < count ? P.order[first + slot] : -1;
    const int pairB = slot + 1 < count ? P.order[first + slot + 1] : -1;
    const PairJob JA = load_job(P, pairA, reverse);
    const PairJob JB = load_job(P, pairB, reverse);

    int mmax = imax(JA.m, JB.m);
    for (int off = 32; off > 0; off >>= 1) mmax = imax(mmax, __shfl_xor(mmax, off));
    const int steps = __builtin_amdgcn_readfirstlane(mmax > 0 ? mmax + W - 1 : 0);

    uint16_t* bufA = refbuf + ((wave * G + g) * 2) * Stager::kBuf;
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
        __syncthreads();   // scheme tables
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

template <int W, int R>
static constexpr PassFn pass_i16() { return &sw_pass_i16<W, R>; }

static const ShapeEntry kShapesI16[] = {
    {16, 16, 2, pass_i16<16, 2>()},   {16, 16, 4, pass_i16<16, 4>()},
    {16, 16, 6, pass_i16<16, 6>()},   {16, 16, 8, pass_i16<16, 8>()},
    {16, 16, 10, pass_i16<16, 10>()}, {16, 16, 12, pass_i16<16, 12>()},
    {16, 16, 14, pass_i16<16, 14>()}, {16, 16, 16, pass_i16<16, 16>()},
    {16, 64, 6, pass_i16<64, 6>()},   {16, 64, 8, pass_i16<64, 8>()},
    {16, 64, 10, pass_i16<64, 10>()}, {16, 64, 12, pass_i16<64, 12>()},
    {16, 64, 14, pass_i16<64, 14>()}, {16, 64, 16, pass_i16<64, 16>()},
    {16, 64, 20, pass_i16<64, 20>()}, {16, 64, 24, pass_i16<64, 24>()},
    {16, 64, 28, pass_i16<64, 28>()}, {16, 64, 32, pass_i16<64, 32>()},
};

const ShapeEntry* shapes_i16(int* n) {
    *n = (int)(sizeof(kShapesI16) / sizeof(kShapesI16[0]));
    return kShapesI16;
}

}  // namespace sw
