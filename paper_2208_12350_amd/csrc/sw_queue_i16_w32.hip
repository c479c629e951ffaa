// sw_queue_i16_w32.hip -- queue kernels of the packed int16 sweep shapes with
// 32-lane groups, 5..16 rows per lane (queries up to 512 residues).

#include "sw_queue.h"

namespace sw {

extern const KernelEntry kI16W32Kernels[];
extern const int kNumI16W32Kernels;

#define SW_ENTRY(W, R) \
    {16, W, R, &sw_queue_kernel<16, W, R, false, false>, &sw_queue_kernel<16, W, R, true, false>, \
     &sw_queue_kernel<16, W, R, false, true>, &sw_queue_kernel<16, W, R, true, true>, \
     &sw_ptab_kernel<W, R, false>, &sw_ptab_kernel<W, R, true>},
const KernelEntry kI16W32Kernels[] = {
    SW_ENTRY(32, 5) SW_ENTRY(32, 6) SW_ENTRY(32, 7) SW_ENTRY(32, 8) SW_ENTRY(32, 9) SW_ENTRY(32, 10)
    SW_ENTRY(32, 11) SW_ENTRY(32, 12) SW_ENTRY(32, 13) SW_ENTRY(32, 14) SW_ENTRY(32, 15) SW_ENTRY(32, 16)
};
#undef SW_ENTRY
const int kNumI16W32Kernels = sizeof(kI16W32Kernels) / sizeof(kI16W32Kernels[0]);

}  // namespace sw
