// sw_queue_i16_w256.hip -- queue kernels of the cooperative packed int16
// shapes: 256-lane groups (a workgroup's four wavefronts), 3..8 rows per
// lane (queries up to 2048 residues).
#include "sw_coop.h"
#include "sw_queue.h"

namespace sw {

extern const KernelEntry kI16W256Kernels[];
extern const int kNumI16W256Kernels;

#define SW_ENTRY(R) \
    {16, kCoopW, R, {{{&sw_coop_kernel<R, false>, &sw_coop_kernel<R, true>}, {nullptr, nullptr}, {nullptr, nullptr}, \
                      {nullptr, nullptr}}, \
                     {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}}}},
const KernelEntry kI16W256Kernels[] = {
    SW_ENTRY(3) SW_ENTRY(4) SW_ENTRY(5) SW_ENTRY(6) SW_ENTRY(7) SW_ENTRY(8)
};
#undef SW_ENTRY
const int kNumI16W256Kernels = sizeof(kI16W256Kernels) / sizeof(kI16W256Kernels[0]);

}  // namespace sw
