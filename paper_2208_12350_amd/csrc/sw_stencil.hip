// sw_stencil.hip -- one diffusion step of a float32 grid on gfx950, with a
// zero-padded grid or with bounds checks (include/swstencil.h).
//
// The grid diffusion of the paper's second application (Section II-C):
// every point keeps (1 - D) of its value and receives D/8 of each of its 8
// neighbours'; points outside the grid count as 0.  Section V-D found that
// the boundary checks cost a fifth of the run time there, and that a border
// of zero points removes them.  Both forms are built here from one step
// function that differs only in how a neighbour is read, so they compute
// bit-identical results and their times compare the bounds logic alone.
//
// Mapping (HBM-bound: 8 bytes per point, about 10 VALU operations):
//   * a wavefront owns a strip of 62 output columns and 64 output rows;
//     lane l holds column strip*62 + l - 1 (lanes 0 and 63 only supply the
//     strip's left and right neighbour columns);
//   * it slides down its rows with three rows in registers, so every value
//     is read from memory once per strip (plus 2 halo rows per 64 and 2 halo
//     columns per 62), loading 8 rows ahead so that a wavefront keeps 8
//     loads in flight; left and right neighbours come from the adjacent
//     lanes through DPP wave shifts, not from memory;
//   * the horizontal triple sum of a row, (left + centre) + right, is formed
//     once when the row is loaded and reused for the two output rows next to
//     it, so a point costs one load, two lane shifts, seven adds and one
//     multiply-add.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swstencil.h"

namespace {

constexpr int kStrip = 62;   // output columns per wavefront
constexpr int kRows = 64;    // output rows per wavefront

__device__ __forceinline__ float lane_left(float v) {   // value of lane l-1 (0 for lane 0)
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_right(float v) {  // value of lane l+1 (0 for lane 63)
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}

// Reads the value of grid point (x, y); x, y may be one outside the grid.
struct PaddedGrid {
    const float* g;
    int pitch;
    int ncols;   // readable columns of a padded row
    __device__ __forceinline__ float at(int x, int y) const {
        // padded coordinates (x + 1, y + 1); columns past the row's end
        // (lanes beyond the last strip) are clamped and never stored
        const int xp = x + 1 < ncols ? x + 1 : ncols - 1;
        return g[(int64_t)(y + 1) * pitch + xp];
    }
};

struct CheckedGrid {
    const float* g;
    int nx, ny;
    __device__ __forceinline__ float at(int x, int y) const {
        return (x >= 0 && x < nx && y >= 0 && y < ny) ? g[(int64_t)y * nx + x] : 0.0f;
    }
};

template <class Grid, class Store>
__device__ __forceinline__ void diffuse_strip(const Grid& src, const Store& store, int nx, int ny, float keep,
                                              float share) {
    const int lane = threadIdx.x & 63;
    const int wave = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int strips = (nx + kStrip - 1) / kStrip;
    const int strip = wave % strips;
    const int y0 = (wave / strips) * kRows;
    if (y0 >= ny) return;
    const int y1 = y0 + kRows < ny ? y0 + kRows : ny;
    const int x = strip * kStrip + lane - 1;
    const bool out_lane = lane >= 1 && lane <= kStrip && x < nx;

    // rows y-1 and y, with their triple sums and side neighbours
    float up = src.at(x, y0 - 1);
    float h_up = (lane_left(up) + up) + lane_right(up);
    float mid = src.at(x, y0);
    float l_mid = lane_left(mid), r_mid = lane_right(mid);
    float h_mid = (l_mid + mid) + r_mid;
    // rows are loaded kAhead at a time, so that many loads of a wavefront
    // are in flight together (a row past the grid reads the last border
    // row, or 0, and is never used)
    constexpr int kAhead = 8;
    for (int y = y0; y < y1; y += kAhead) {
        float next[kAhead];
#pragma unroll
        for (int k = 0; k < kAhead; ++k) next[k] = src.at(x, y + 1 + k < ny ? y + 1 + k : ny);
#pragma unroll
        for (int k = 0; k < kAhead; ++k) {
            if (y + k >= y1) break;
            const float down = next[k];
            const float l_down = lane_left(down), r_down = lane_right(down);
            const float h_down = (l_down + down) + r_down;
            const float nbrs = (h_up + h_down) + (l_mid + r_mid);
            const float v = fmaf(share, nbrs, keep * mid);
            if (out_lane) store(x, y + k, v);
            h_up = h_mid;
            mid = down; l_mid = l_down; r_mid = r_down; h_mid = h_down;
        }
    }
}

struct PaddedStore {
    float* g;
    int pitch;
    __device__ __forceinline__ void operator()(int x, int y, float v) const { g[(int64_t)(y + 1) * pitch + x + 1] = v; }
};
struct PlainStore {
    float* g;
    int nx;
    __device__ __forceinline__ void operator()(int x, int y, float v) const { g[(int64_t)y * nx + x] = v; }
};

__global__ __launch_bounds__(256) void diffuse_padded_kernel(const float* src, float* dst, int nx, int ny, int pitch,
                                                             float keep, float share) {
    diffuse_strip(PaddedGrid{src, pitch, pitch}, PaddedStore{dst, pitch}, nx, ny, keep, share);
}

__global__ __launch_bounds__(256) void diffuse_checked_kernel(const float* src, float* dst, int nx, int ny,
                                                              float keep, float share) {
    diffuse_strip(CheckedGrid{src, nx, ny}, PlainStore{dst, nx}, nx, ny, keep, share);
}

__global__ void pad_grid_kernel(const float* grid, float* padded, int nx, int ny, int pitch) {
    const int64_t total = (int64_t)(ny + 2) * pitch;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int yp = (int)(i / pitch), xp = (int)(i % pitch);
        padded[i] = (yp >= 1 && yp <= ny && xp >= 1 && xp <= nx) ? grid[(int64_t)(yp - 1) * nx + xp - 1] : 0.0f;
    }
}

unsigned waves_blocks(int nx, int ny) {
    const int64_t strips = (nx + kStrip - 1) / kStrip;
    const int64_t waves = strips * ((ny + kRows - 1) / kRows);
    return (unsigned)((waves + 3) / 4);
}

bool bad_args(const void* a, const void* b, int nx, int ny, float D) {
    return !a || !b || nx < 1 || ny < 1 || !(D >= 0.0f && D <= 1.0f) || (int64_t)nx * ny > ((int64_t)1 << 40);
}

}  // namespace

extern "C" {

int sw_diffuse_padded(const float* src, float* dst, int32_t nx, int32_t ny, int32_t pitch, float D, void* stream) {
    if (bad_args(src, dst, nx, ny, D) || pitch < nx + 2) return -1;
    hipLaunchKernelGGL(diffuse_padded_kernel, dim3(waves_blocks(nx, ny)), dim3(256), 0, (hipStream_t)stream, src, dst,
                       nx, ny, pitch, 1.0f - D, D / 8.0f);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int sw_diffuse_checked(const float* src, float* dst, int32_t nx, int32_t ny, float D, void* stream) {
    if (bad_args(src, dst, nx, ny, D)) return -1;
    hipLaunchKernelGGL(diffuse_checked_kernel, dim3(waves_blocks(nx, ny)), dim3(256), 0, (hipStream_t)stream, src,
                       dst, nx, ny, 1.0f - D, D / 8.0f);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int sw_pad_grid(const float* grid, float* padded, int32_t nx, int32_t ny, int32_t pitch, void* stream) {
    if (!grid || !padded || nx < 1 || ny < 1 || pitch < nx + 2) return -1;
    const int64_t total = (int64_t)(ny + 2) * pitch;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(pad_grid_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, grid, padded, nx,
                       ny, pitch);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // extern "C"
