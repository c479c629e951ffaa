// sw_queue_i16_w16b.hip -- queue kernels of the packed int16 sweep shapes with
// 16-lane groups, 9..16 rows per lane (queries of 129..256 residues): table-lookup, column-word, pair-table and (forward only) query-profile
// kernels, forward and reverse, each with the default tile of kChunk
// reference steps and the narrow tile of kChunkNarrow.
#include "sw_queue.h"

namespace sw {

extern const KernelEntry kI16W16bKernels[];
extern const int kNumI16W16bKernels;

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
const KernelEntry kI16W16bKernels[] = {
    SW_ENTRY(16, 9) SW_ENTRY(16, 10) SW_ENTRY(16, 11) SW_ENTRY(16, 12) SW_ENTRY(16, 13) SW_ENTRY(16, 14)
    SW_ENTRY(16, 15) SW_ENTRY(16, 16)
};
#undef SW_ENTRY
const int kNumI16W16bKernels = sizeof(kI16W16bKernels) / sizeof(kI16W16bKernels[0]);

// One launch per pass and score source serves every shape of this file.
extern const FamilyEntry kI16W16bFamily;
const FamilyEntry kI16W16bFamily = SW_FAMILY16(16, 3, 2, kChunk, 16, 15, 14, 13, 12, 11, 10, 9);

}  // namespace sw
