// sw_queue_i32.hip -- queue kernels of the int32 sweep shapes, and the
// registry of every compiled shape.
#include "sw_queue.h"

namespace sw {

#define SW_ENTRY(W, R) {32, W, R, &sw_queue_kernel<32, W, R>},
static const KernelEntry kI32Kernels[] = {
    SW_ENTRY(16, 2) SW_ENTRY(16, 4) SW_ENTRY(16, 6) SW_ENTRY(16, 8) SW_ENTRY(16, 10)
    SW_ENTRY(16, 12) SW_ENTRY(16, 14) SW_ENTRY(16, 16)
    SW_ENTRY(64, 6) SW_ENTRY(64, 8) SW_ENTRY(64, 10) SW_ENTRY(64, 12) SW_ENTRY(64, 14)
    SW_ENTRY(64, 16) SW_ENTRY(64, 20) SW_ENTRY(64, 24) SW_ENTRY(64, 28) SW_ENTRY(64, 32)
};
#undef SW_ENTRY

extern const KernelEntry kI16Kernels[];
extern const int kNumI16Kernels;

static ShapeDesc g_shapes[64];
static int g_nshapes = 0;

const ShapeDesc* compiled_shapes(int* n) {
    if (g_nshapes == 0) {
        for (int k = 0; k < kNumI16Kernels; ++k)
            g_shapes[g_nshapes++] = {kI16Kernels[k].prec, kI16Kernels[k].W, kI16Kernels[k].R};
        for (const KernelEntry& e : kI32Kernels) g_shapes[g_nshapes++] = {e.prec, e.W, e.R};
    }
    *n = g_nshapes;
    return g_shapes;
}

QueueFn shape_kernel(int prec, int W, int R) {
    if (prec == 16) {
        for (int k = 0; k < kNumI16Kernels; ++k)
            if (kI16Kernels[k].W == W && kI16Kernels[k].R == R) return kI16Kernels[k].fn;
    } else {
        for (const KernelEntry& e : kI32Kernels)
            if (e.W == W && e.R == R) return e.fn;
    }
    return nullptr;
}

}  // namespace sw
