// sw_coop.h -- cooperative sweep: one pair group spread over the four
// wavefronts of a workgroup (gfx950).
//
// For long queries the critical path of a pair is its sweep on one lane
// group: m + W - 1 steps of R rows each.  A single 64-lane wavefront needs
// R = 32 rows per lane for a 2048-residue query; here the four wavefronts of
// a workgroup form one group of W = 256 lanes (R <= 8 rows per lane), which
// cuts each pair's latency by about four at the price of a longer ramp
// (W - 1 steps) and one workgroup barrier per step.
//
// Arithmetic, padding, biased packed int16 values and row-pair keys are
// those of sweep_i16 (sw_sweep.h): two pairs per group, pair A in the low
// halves, pair B in the high halves.  What changes is the exchange at the
// wavefront boundaries: lane 0 of wavefront w > 0 takes the H and F of lane
// 63 of wavefront w - 1 from the previous step through LDS (double-buffered
// by step parity) instead of the DPP fill, and every step ends with a
// workgroup barrier, so the value a wavefront reads at step t was written at
// step t - 1 and is overwritten no earlier than step t + 1.  All waves run
// the same number of steps and chunks (the step count depends only on the
// pair lengths, which every lane loads), so every barrier is reached by the
// whole workgroup.
#pragma once

#include "sw_sweep.h"

namespace sw {

constexpr int kCoopW = 64 * kWavesPerBlock;   // lanes of a cooperative group

struct CoopLds {
    uint16_t ref[2 * RefStager<kCoopW>::kBuf];   // staged columns of pairs A and B
    uint32_t xh[2][kWavesPerBlock];               // [step parity][wave]: lane 63's H
    uint32_t xf[2][kWavesPerBlock];               //                      and F
    int32_t res[kWavesPerBlock][2][3];            // per wave and pair: best, row, column
    int32_t item;
};

template <int R, bool REV>
__device__ __forceinline__ void sweep_coop(const KParams& P, const SchemeLds& S, CoopLds& C, int first,
                                           int count, int tid) {
    constexpr int W = kCoopW;
    using Stager = RefStager<W>;
    constexpr int reverse = REV ? 1 : 0;
    constexpr int RP = (R + 1) / 2;
    constexpr uint32_t K = kI16Bias;
    constexpr uint32_t K2 = K | (K << 16);
    const int l = tid;               // lane within the group
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    const int pairA = count > 0 ? P.order[first] : -1;
    const int pairB = count > 1 ? P.order[first + 1] : -1;
    const PairJob JA = load_job(P, pairA, reverse);
    const PairJob JB = load_job(P, pairB, reverse);
    const int mmax = imax(JA.m, JB.m);
    const int steps = __builtin_amdgcn_readfirstlane(mmax > 0 ? mmax + W - 1 : 0);

    uint16_t* bufA = C.ref;
    uint16_t* bufB = C.ref + Stager::kBuf;
    Stager stA, stB;
    stA.load(P.refs, JA, P.order, 0, l);
    stB.load(P.refs, JB, P.order, 0, l);

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
    if (wave == 0) {
        // "previous step" values of every wave's last lane: the matrix's
        // padding columns, biased zero (all lanes of wave 0 store the same
        // values, so there is no lane-divergent branch)
        C.xh[1][lane & (kWavesPerBlock - 1)] = K2;
        C.xf[1][lane & (kWavesPerBlock - 1)] = K2;
    }
    const int AA = S.alphabet[JA.sid], AB = S.alphabet[JB.sid];
    const u16x2 go2 = pk(cost16(S.gap_open[JA.sid]) | (cost16(S.gap_open[JB.sid]) << 16));
    const u16x2 ge2 = pk(cost16(S.gap_extend[JA.sid]) | (cost16(S.gap_extend[JB.sid]) << 16));
    const u16x2 zero = pk(K2);
    __syncthreads();

    u16x2 H[R], E[R];
    uint32_t kA[RP], kB[RP];
#pragma unroll
    for (int r = 0; r < R; ++r) { H[r] = zero; E[r] = zero; }
#pragma unroll
    for (int p = 0; p < RP; ++p) { kA[p] = 0u; kB[p] = 0u; }
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
    bool bad = false;
    uint32_t jc = (uint32_t)(kColMax + l);
    int parity = 0;
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
            // lane 0 of wave w > 0: the previous step's values of lane 63 of
            // wave w - 1; lane 0 of wave 0: the matrix top boundary
            const uint32_t inH = wave > 0 ? C.xh[parity ^ 1][wave - 1] : K2;
            const uint32_t inF = wave > 0 ? C.xf[parity ^ 1][wave - 1] : K2;
            const u16x2 Hup = pk((uint32_t)__builtin_amdgcn_update_dpp((int)inH, (int)Hlast, 0x138, 0xF, 0xF, false));
            const u16x2 Fup = pk((uint32_t)__builtin_amdgcn_update_dpp((int)inF, (int)Flast, 0x138, 0xF, 0xF, false));
            u16x2 diag = pk(Hup_prev);
            Hup_prev = u32(Hup);
            u16x2 Hmu = pk_sat_sub(Hup, go2);
            u16x2 F = Fup;
            const uint32_t jc1 = jc | 0x8000u;
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
            // lane 63's values for the next wavefront, stored by every lane
            // (same value, same address: no lane-divergent branch)
            C.xh[parity][wave] = __builtin_amdgcn_readlane(Hlast, 63);
            C.xf[parity][wave] = __builtin_amdgcn_readlane(Flast, 63);
            parity ^= 1;
            bbA_next = bbA2;
            bbB_next = bbB2;
            --jc;
            __syncthreads();
        }
        if (more) {
            stA.store(bufA, JA, AA, t0 + kChunk, l, bad);
            stB.store(bufB, JB, AB, t0 + kChunk, l, bad);
            __syncthreads();
            bbA_next = rblA[1];
            bbB_next = rblB[1];
            const int a0 = rblA[0], b0 = rblB[0];
#pragma unroll
            for (int r = 0; r < R; ++r)
                sc[r] = load_scores(S.mat, a0 + (int)(apk[r] & 0xFFFF), b0 + (int)(apk[r] >> 16));
        }
    }
    if (bad && P.validate) atomicOr(&P.flags[kFlagBadResidue], 1);

    // best of this lane in row-major order, then of the wave, then across
    // waves (lower waves hold lower rows)
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
        for (int off = 1; off < 64; off <<= 1) {
            const int ob = __shfl_xor(lb[p], off);
            const int oi = __shfl_xor(li[p], off);
            const int oj = __shfl_xor(lj[p], off);
            if (ob > lb[p] || (ob == lb[p] && oi < li[p])) { lb[p] = ob; li[p] = oi; lj[p] = oj; }
        }
        // after the butterfly every lane holds the wave's best
        C.res[wave][p][0] = lb[p];
        C.res[wave][p][1] = li[p];
        C.res[wave][p][2] = lj[p];
    }
    __syncthreads();
    // wave 0 combines; all its lanes compute and store the same values
    if (wave == 0) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            int b = 0, bi = -1, bj = -1;
            for (int w = 0; w < kWavesPerBlock; ++w) {
                const int ob = C.res[w][p][0], oi = C.res[w][p][1], oj = C.res[w][p][2];
                if (ob > b || (ob == b && ob > 0 && oi < bi)) { b = ob; bi = oi; bj = oj; }
            }
            const int pair = p == 0 ? pairA : pairB;
            const PairJob& J = p == 0 ? JA : JB;
            if (pair < 0) continue;
            if (!reverse) {
                sw_result res;
                if (b > 0) { res.score = b; res.q_start = -1; res.q_end = bi; res.r_start = -1; res.r_end = bj; }
                else { res.score = 0; res.q_start = res.q_end = res.r_start = res.r_end = -1; }
                P.out[pair] = res;
            } else if (J.fwd_score > 0) {
                if (b != J.fwd_score) {
                    atomicOr(&P.flags[kFlagReverseMismatch], 1);
                } else {
                    P.out[pair].q_start = J.fwd_qe - bi;
                    P.out[pair].r_start = J.fwd_re - bj;
                }
            }
        }
    }
}

// Work-queue kernel of the cooperative shapes: every workgroup claims one
// two-pair item at a time (wave 0 fetches, LDS broadcasts) until the bin's
// range is exhausted.
template <int R, bool REV>
__global__ __launch_bounds__(kBlock) void sw_coop_kernel(KParams P) {
    __shared__ __attribute__((aligned(16))) SchemeLds L;
    __shared__ __attribute__((aligned(16))) CoopLds C;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
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
    for (;;) {
        // wave 0 claims the next item (every lane takes part in the atomic,
        // only lane 0 adds); every lane of wave 0 writes the same value
        if (wave == 0) {
            const int mine = atomicAdd(&P.meta[P.head_idx], lane == 0 ? 1 : 0);
            C.item = __builtin_amdgcn_readlane(mine, 0);
        }
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(C.item);
        __syncthreads();
        if (it >= hi - lo) break;
        const WorkItem* wp = P.items + lo + it;
        const int first = __builtin_amdgcn_readfirstlane(__atomic_load_n(&wp->first, __ATOMIC_RELAXED));
        const int count = __builtin_amdgcn_readfirstlane((int)__atomic_load_n(&wp->count, __ATOMIC_RELAXED));
        const bool valid = first >= 0 && count >= 1 && count <= 2 && first + count <= n_pairs;
        if (valid) {
            sweep_coop<R, REV>(P, L, C, first, count, tid);
        } else {
            atomicOr(&P.flags[kFlagInternal], 1);
        }
    }
}

}  // namespace sw
