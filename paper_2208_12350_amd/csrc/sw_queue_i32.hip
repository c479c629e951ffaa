// sw_queue_i32.hip -- queue kernels of the int32 sweep shapes (the exact
// fallback for pairs whose scores may not fit 16 bits), and the registry of
// every compiled shape.
#include "sw_queue.h"

namespace sw {

#define SW_ENTRY(W, R) \
    {32, W, R, {{{&sw_queue_kernel<32, W, R, false, false>, &sw_queue_kernel<32, W, R, true, false>}, \
                 {nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}}, \
                {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}}}},
static const KernelEntry kI32Kernels[] = {
    SW_ENTRY(16, 2) SW_ENTRY(16, 4) SW_ENTRY(16, 6) SW_ENTRY(16, 8) SW_ENTRY(16, 10)
    SW_ENTRY(16, 12) SW_ENTRY(16, 14) SW_ENTRY(16, 16)
    SW_ENTRY(64, 6) SW_ENTRY(64, 8) SW_ENTRY(64, 10) SW_ENTRY(64, 12) SW_ENTRY(64, 14)
    SW_ENTRY(64, 16) SW_ENTRY(64, 20) SW_ENTRY(64, 24) SW_ENTRY(64, 28) SW_ENTRY(64, 32)
};
#undef SW_ENTRY

extern const KernelEntry kI16W16Kernels[];
extern const int kNumI16W16Kernels;
extern const KernelEntry kI16W16bKernels[];
extern const int kNumI16W16bKernels;
extern const KernelEntry kI16W32Kernels[];
extern const int kNumI16W32Kernels;
extern const KernelEntry kI16W32bKernels[];
extern const int kNumI16W32bKernels;
extern const KernelEntry kI16W64Kernels[];
extern const int kNumI16W64Kernels;
extern const KernelEntry kI16W64LongKernels[];
extern const int kNumI16W64LongKernels;
extern const KernelEntry kI16W256Kernels[];
extern const int kNumI16W256Kernels;
extern const FamilyEntry kI16W16Family;
extern const FamilyEntry kI16W16bFamily;
extern const FamilyEntry kI16W32Family;
extern const FamilyEntry kI16W32bFamily;
extern const FamilyEntry kI16W64Family;
extern const FamilyEntry kI16W64LongFamily;

namespace {

struct Table { const KernelEntry* e; int n; };

Table table(int k) {
    switch (k) {
        case 0: return {kI16W16Kernels, kNumI16W16Kernels};
        case 1: return {kI16W16bKernels, kNumI16W16bKernels};
        case 2: return {kI16W32Kernels, kNumI16W32Kernels};
        case 3: return {kI16W32bKernels, kNumI16W32bKernels};
        case 4: return {kI16W64Kernels, kNumI16W64Kernels};
        case 5: return {kI16W64LongKernels, kNumI16W64LongKernels};
        case 6: return {kI16W256Kernels, kNumI16W256Kernels};
        default: return {kI32Kernels, (int)(sizeof(kI32Kernels) / sizeof(kI32Kernels[0]))};
    }
}

constexpr int kTables = 8;
ShapeDesc g_shapes[kMaxBins];
int g_nshapes = 0;

}  // namespace

const ShapeDesc* compiled_shapes(int* n) {
    if (g_nshapes == 0) {
        for (int t = 0; t < kTables; ++t) {
            const Table tb = table(t);
            for (int k = 0; k < tb.n && g_nshapes < kMaxBins; ++k)
                g_shapes[g_nshapes++] = {tb.e[k].prec, tb.e[k].W, tb.e[k].R};
        }
    }
    *n = g_nshapes;
    return g_shapes;
}

const FamilyEntry* shape_family(int prec, int W, int R) {
    const FamilyEntry* fams[] = {&kI16W16Family, &kI16W16bFamily, &kI16W32Family,
                                 &kI16W32bFamily, &kI16W64Family, &kI16W64LongFamily};
    for (const FamilyEntry* f : fams)
        if (f->prec == prec && f->W == W)
            for (int k = 0; k < f->n; ++k)
                if (f->rows[k] == R) return f;
    return nullptr;
}

QueueFn shape_kernel(int prec, int W, int R, bool reverse, int var, bool narrow) {
    if (var < 0 || var >= kNumVars) return nullptr;
    for (int t = 0; t < kTables; ++t) {
        const Table tb = table(t);
        for (int k = 0; k < tb.n; ++k)
            if (tb.e[k].prec == prec && tb.e[k].W == W && tb.e[k].R == R)
                return tb.e[k].k[narrow ? 1 : 0][var][reverse ? 1 : 0];
    }
    return nullptr;
}

}  // namespace sw
