// sw_queue_i16_w64.hip -- queue kernels of the packed int16 sweep shapes with
// 64-lane groups, 9..20 rows per lane (queries up to 1280 residues): table-lookup, column-word, pair-table and (forward only) query-profile
// kernels, forward and reverse.
#include "sw_queue.h"

namespace sw {

extern const KernelEntry kI16W64Kernels[];
extern const int kNumI16W64Kernels;

#define SW_ENTRY(W, R) \
    {16, W, R, {{{&sw_queue_kernel<16, W, R, false, false>, &sw_queue_kernel<16, W, R, true, false>}, \
                 {&sw_queue_kernel<16, W, R, false, true>, &sw_queue_kernel<16, W, R, true, true>}, \
                 {&sw_ptab_kernel<W, R, false>, &sw_ptab_kernel<W, R, true>}, \
                 {&sw_qprof_kernel<W, R>, nullptr}}, \
                {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}}}},
const KernelEntry kI16W64Kernels[] = {
    SW_ENTRY(64, 9) SW_ENTRY(64, 10) SW_ENTRY(64, 11) SW_ENTRY(64, 12) SW_ENTRY(64, 13) SW_ENTRY(64, 14)
    SW_ENTRY(64, 15) SW_ENTRY(64, 16) SW_ENTRY(64, 17) SW_ENTRY(64, 18) SW_ENTRY(64, 19) SW_ENTRY(64, 20)
};
#undef SW_ENTRY
const int kNumI16W64Kernels = sizeof(kI16W64Kernels) / sizeof(kI16W64Kernels[0]);

// One launch per pass and score source serves every shape of this file.
extern const FamilyEntry kI16W64Family;
const FamilyEntry kI16W64Family = SW_FAMILY16(64, 2, 2, kChunk, 20, 19, 18, 17, 16, 15, 14, 13, 12, 11, 10, 9);

}  // namespace sw
