// sw_queue_i16.hip -- queue kernels of the packed int16 sweep shapes.
#include "sw_queue.h"

namespace sw {

extern const KernelEntry kI16Kernels[];
extern const int kNumI16Kernels;

#define SW_ENTRY(W, R) {16, W, R, &sw_queue_kernel<16, W, R>},
const KernelEntry kI16Kernels[] = {
    SW_ENTRY(16, 2) SW_ENTRY(16, 4) SW_ENTRY(16, 6) SW_ENTRY(16, 8) SW_ENTRY(16, 10)
    SW_ENTRY(16, 12) SW_ENTRY(16, 14) SW_ENTRY(16, 16)
    SW_ENTRY(64, 6) SW_ENTRY(64, 8) SW_ENTRY(64, 10) SW_ENTRY(64, 12) SW_ENTRY(64, 14)
    SW_ENTRY(64, 16) SW_ENTRY(64, 20) SW_ENTRY(64, 24) SW_ENTRY(64, 28) SW_ENTRY(64, 32)
};
#undef SW_ENTRY
const int kNumI16Kernels = sizeof(kI16Kernels) / sizeof(kI16Kernels[0]);

}  // namespace sw
