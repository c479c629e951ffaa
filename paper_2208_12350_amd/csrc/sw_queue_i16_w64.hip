// sw_queue_i16_w64.hip -- queue kernels of the packed int16 sweep shapes with
// 64-lane groups, 9..32 rows per lane (queries up to 2048 residues).

#include "sw_queue.h"

namespace sw {

extern const KernelEntry kI16W64Kernels[];
extern const int kNumI16W64Kernels;

#define SW_ENTRY(W, R) \
    {16, W, R, &sw_queue_kernel<16, W, R, false, false>, &sw_queue_kernel<16, W, R, true, false>, \
     &sw_queue_kernel<16, W, R, false, true>, &sw_queue_kernel<16, W, R, true, true>},
const KernelEntry kI16W64Kernels[] = {
    SW_ENTRY(64, 9) SW_ENTRY(64, 10) SW_ENTRY(64, 11) SW_ENTRY(64, 12) SW_ENTRY(64, 13) SW_ENTRY(64, 14)
    SW_ENTRY(64, 15) SW_ENTRY(64, 16) SW_ENTRY(64, 17) SW_ENTRY(64, 18) SW_ENTRY(64, 19) SW_ENTRY(64, 20)
    SW_ENTRY(64, 21) SW_ENTRY(64, 22) SW_ENTRY(64, 23) SW_ENTRY(64, 24) SW_ENTRY(64, 25) SW_ENTRY(64, 26)
    SW_ENTRY(64, 27) SW_ENTRY(64, 28) SW_ENTRY(64, 29) SW_ENTRY(64, 30) SW_ENTRY(64, 31) SW_ENTRY(64, 32)
};
#undef SW_ENTRY
const int kNumI16W64Kernels = sizeof(kI16W64Kernels) / sizeof(kI16W64Kernels[0]);

}  // namespace sw
