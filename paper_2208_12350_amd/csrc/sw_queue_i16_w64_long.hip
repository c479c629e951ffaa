// sw_queue_i16_w64_long.hip -- queue kernels of the packed int16 sweep shapes with
// 64-lane groups, 21..32 rows per lane (queries of 1281..2048 residues): table-lookup, column-word, pair-table and (forward only) query-profile
// kernels, forward and reverse.
#include "sw_queue.h"

namespace sw {

extern const KernelEntry kI16W64LongKernels[];
extern const int kNumI16W64LongKernels;

#define SW_ENTRY(W, R) \
    {16, W, R, {{{&sw_queue_kernel<16, W, R, false, false>, &sw_queue_kernel<16, W, R, true, false>}, \
                 {&sw_queue_kernel<16, W, R, false, true>, &sw_queue_kernel<16, W, R, true, true>}, \
                 {&sw_ptab_kernel<W, R, false>, &sw_ptab_kernel<W, R, true>}, \
                 {&sw_qprof_kernel<W, R>, nullptr}}, \
                {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}}}},
const KernelEntry kI16W64LongKernels[] = {
    SW_ENTRY(64, 21) SW_ENTRY(64, 22) SW_ENTRY(64, 23) SW_ENTRY(64, 24) SW_ENTRY(64, 25) SW_ENTRY(64, 26)
    SW_ENTRY(64, 27) SW_ENTRY(64, 28) SW_ENTRY(64, 29) SW_ENTRY(64, 30) SW_ENTRY(64, 31) SW_ENTRY(64, 32)
};
#undef SW_ENTRY
const int kNumI16W64LongKernels = sizeof(kI16W64LongKernels) / sizeof(kI16W64LongKernels[0]);

// One launch per pass and score source serves every shape of this file.
extern const FamilyEntry kI16W64LongFamily;
const FamilyEntry kI16W64LongFamily = SW_FAMILY16(64, 2, 2, kChunk, 32, 31, 30, 29, 28, 27, 26, 25, 24, 23, 22, 21);

}  // namespace sw
