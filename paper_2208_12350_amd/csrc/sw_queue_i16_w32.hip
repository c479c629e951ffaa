// sw_queue_i16_w32.hip -- queue kernels of the packed int16 sweep shapes with
// 32-lane groups, 5..10 rows per lane (queries up to 320 residues): table-lookup, column-word, pair-table and (forward only) query-profile
// kernels, forward and reverse, each with the default tile of kChunk
// reference steps and the narrow tile of kChunkNarrow.
#include "sw_queue.h"

namespace sw {

extern const KernelEntry kI16W32Kernels[];
extern const int kNumI16W32Kernels;

#define SW_ENTRY(W, R) \
    {16, W, R, {{{&sw_queue_kernel<16, W, R, false, false>, &sw_queue_kernel<16, W, R, true, false>}, \
                 {&sw_queue_kernel<16, W, R, false, true>, &sw_queue_kernel<16, W, R, true, true>}, \
                 {&sw_ptab_kernel<W, R, false>, &sw_ptab_kernel<W, R, true>}, \
                 {&sw_qprof_kernel<W, R>, nullptr}}, \
                {{&sw_queue_chunk_kernel<16, W, R, false, false, kChunkNarrow>, \
                  &sw_queue_chunk_kernel<16, W, R, true, false, kChunkNarrow>}, \
                 {&sw_queue_chunk_kernel<16, W, R, false, true, kChunkNarrow>, \
                  &sw_queue_chunk_kernel<16, W, R, true, true, kChunkNarrow>}, \
                 {&sw_ptab_chunk_kernel<W, R, false, kChunkNarrow>, &sw_ptab_chunk_kernel<W, R, true, kChunkNarrow>}, \
                 {nullptr, nullptr}}}},
const KernelEntry kI16W32Kernels[] = {
    SW_ENTRY(32, 5) SW_ENTRY(32, 6) SW_ENTRY(32, 7) SW_ENTRY(32, 8) SW_ENTRY(32, 9) SW_ENTRY(32, 10)
};
#undef SW_ENTRY
const int kNumI16W32Kernels = sizeof(kI16W32Kernels) / sizeof(kI16W32Kernels[0]);

// One launch per pass and score source serves every shape of this file.
extern const FamilyEntry kI16W32Family;
const FamilyEntry kI16W32Family = SW_FAMILY16(32, 2, 2, kChunk, 10, 9, 8, 7, 6, 5);

}  // namespace sw
