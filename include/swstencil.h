/*
 * swstencil.h -- C ABI of the grid diffusion library (libswstencil.so,
 * built for AMD Instinct MI355X / gfx950).
 *
 * The paper's second application (Section II-C) diffuses virus and
 * inflammatory signal over a 2-D grid of lung tissue, each grid point
 * spreading to its neighbours every step; Section VI-D shows that removing
 * the grid's boundary checks and instead padding the grid with a border of
 * zero points made that code faster.  This library provides one explicit
 * diffusion step of a float32 field, with and without that padding:
 *
 *     c'[y][x] = (1 - D) * c[y][x] + (D / 8) * sum of c over the 8 neighbours
 *
 * where neighbours outside the grid contribute 0 (the value a zero border
 * gives).  D is the diffusion fraction, 0 <= D <= 1.
 *
 * Padded layout: a grid of nx x ny points is stored as (ny + 2) rows of
 * `pitch` floats (pitch >= nx + 2); point (x, y) is at row y + 1, column
 * x + 1, and the border rows and columns hold 0 (sw_pad_grid writes them).
 * Unpadded layout: ny rows of nx floats.
 *
 * All pointers are DEVICE pointers owned by the caller; `src` and `dst` must
 * not overlap.  `stream` is a hipStream_t passed as void* (NULL = the null
 * stream); calls only enqueue work.  Return 0, or -1 for a bad argument
 * (null pointer, nx or ny < 1, pitch too small, D outside [0, 1]), or -4
 * when a HIP launch fails.
 */
#ifndef SWSTENCIL_H
#define SWSTENCIL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One diffusion step on the padded layout: reads the nx x ny interior of
 * `src` and its zero border (no bounds checks), writes the interior of
 * `dst` (its border is left as it is).  With pitch a multiple of 4 and both
 * pointers 16-byte aligned, each lane handles 4 columns (16-byte accesses);
 * the results are the same either way. */
int sw_diffuse_padded(const float* src, float* dst, int32_t nx, int32_t ny, int32_t pitch, float D,
                      void* stream);

/* The same step on the unpadded layout: every neighbour read is checked
 * against the grid bounds and reads as 0 outside.  With nx a multiple of 4
 * and both pointers 16-byte aligned, each lane handles 4 columns. */
int sw_diffuse_checked(const float* src, float* dst, int32_t nx, int32_t ny, float D, void* stream);

/* Copy an unpadded nx x ny grid into the padded layout, writing the zero
 * border (the whole (ny + 2) x pitch array is written). */
int sw_pad_grid(const float* grid, float* padded, int32_t nx, int32_t ny, int32_t pitch, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SWSTENCIL_H */
