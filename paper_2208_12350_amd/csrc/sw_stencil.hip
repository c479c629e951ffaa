// sw_stencil.hip -- one diffusion step of a float32 grid on gfx950, with a
// zero-padded grid or with bounds checks (include/swstencil.h).
//
// The grid diffusion of the paper's second application (Section II-C):
// every point keeps (1 - D) of its value and receives D/8 of each of its 8
// neighbours'; points outside the grid count as 0.  Section VI-D found that
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
//     multiply-add;
//   * on 16-byte aligned rows (a padded pitch, or an unpadded width, that is
//     a multiple of 4 floats) each lane holds 4 columns instead
//     (diffuse_strip4), so a wavefront reads and writes 1 KiB per
//     instruction.
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

// The 4-columns-per-lane form (one 16-byte load per lane and row, 1 KiB per
// wavefront instruction).  Lane l of strip s holds the aligned group of
// columns x0 = kSpan * s + 4 l - kOff .. x0 + 3; lanes 0 and 63 supply the
// strip's halo and the outputs are the kSpan columns with local index
// 4 l + k in [kOff, kOff + kSpan).  On the padded grid the group starts one
// column left of an aligned padded column (kOff = 1, 252 outputs of 256
// columns); on the unpadded grid whole groups are the halo (kOff = 4, 248
// outputs).  Every output is formed by the same expression, in the same
// order, as in diffuse_strip, so all forms give bit-identical grids.
//
// Memory behaviour, chosen by timing repeated steps (each reading the grid
// the previous one wrote) on 2500^2 .. 16384^2 grids; the thresholds are
// the 256 MB last-level cache (MALL):
//   * source and destination fit in it together: ordinary loads and stores,
//     8 rows per wavefront, so the next step reads from cache;
//   * the source fits in twice its size: ordinary loads (halo rows and
//     columns that neighbouring strips share hit in cache), nontemporal
//     stores, 8 rows per wavefront;
//   * larger: nontemporal loads and stores, 16 rows per wavefront, 16 rows
//     in flight;
//   * consecutive blocks go to the 8 XCDs in turn, so block b runs tile
//     (b mod 8) * (blocks / 8) + b / 8: each XCD's L2 holds one contiguous
//     band of strips and rows, and strips that share a halo share an L2.
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <bool STREAM>
__device__ __forceinline__ f32x4 load4(const float* p) {
    const f32x4* q = reinterpret_cast<const f32x4*>(p);
    if constexpr (STREAM) return __builtin_nontemporal_load(q);
    else return *q;
}

struct PaddedRows4 {
    static constexpr int kSpan = 252, kOff = 1;
    const float* g;
    int pitch;
    template <bool STREAM>
    __device__ __forceinline__ f32x4 load(int x0, int y) const {
        // padded row y + 1, padded columns x0 + 1 .. x0 + 4; a group past the
        // row's end (spare lanes of the last strip) is clamped and feeds no
        // stored output
        const int c = x0 + 1 + 4 <= pitch ? x0 + 1 : pitch - 4;
        return load4<STREAM>(g + (int64_t)(y + 1) * pitch + c);
    }
    // the zero border is in memory: nothing to fix
    __device__ __forceinline__ f32x4 fix(f32x4 q, int, int) const { return q; }
};
struct CheckedRows4 {
    static constexpr int kSpan = 248, kOff = 4;
    const float* g;
    int nx, ny;   // nx is a multiple of 4, so a group is wholly in or out
    template <bool STREAM>
    __device__ __forceinline__ f32x4 load(int x0, int y) const {
        // an unconditional load of the nearest group inside the grid (one a
        // neighbouring lane or row reads anyway), so that every load of a
        // wavefront stays in flight; fix() applies the bounds test when the
        // row is used
        const int yc = y < 0 ? 0 : (y >= ny ? ny - 1 : y);
        const int xc = x0 < 0 ? 0 : (x0 >= nx ? nx - 4 : x0);
        return load4<STREAM>(g + (int64_t)yc * nx + xc);
    }
    __device__ __forceinline__ f32x4 fix(f32x4 q, int x0, int y) const {
        return (y >= 0 && y < ny && x0 >= 0 && x0 < nx) ? q : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    }
};
struct PaddedStore4 {
    float* g;
    int pitch;
    __device__ __forceinline__ float* at(int x0, int y) const { return g + (int64_t)(y + 1) * pitch + x0 + 1; }
};
struct PlainStore4 {
    float* g;
    int nx;
    __device__ __forceinline__ float* at(int x0, int y) const { return g + (int64_t)y * nx + x0; }
};

template <int AHEAD, bool STREAM, bool STREAM_OUT, class Rows, class Store>
__device__ __forceinline__ void diffuse_strip4(const Rows& src, const Store& dst, int nx, int ny, int rows,
                                               float keep, float share) {
    constexpr int kSpan = Rows::kSpan, kOff = Rows::kOff;
    const int per_xcd = (int)gridDim.x / 8;   // gridDim.x is a multiple of 8
    const int tile = ((int)blockIdx.x % 8) * per_xcd + (int)blockIdx.x / 8;
    const int lane = threadIdx.x & 63;
    const int wave = tile * 4 + (int)(threadIdx.x >> 6);
    const int strips = (nx + kSpan - 1) / kSpan;
    const int strip = wave % strips;
    const int y0 = (wave / strips) * rows;
    if (y0 >= ny) return;
    const int y1 = y0 + rows < ny ? y0 + rows : ny;
    const int x0 = strip * kSpan + 4 * lane - kOff;
    bool out[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = 4 * lane + k >= kOff && 4 * lane + k < kOff + kSpan && x0 + k < nx;
    const bool full = out[0] && out[3];
    // a row's values, side neighbours and horizontal triple sums
    struct Row { float v[4], l[4], r[4], h[4]; };
    auto prep = [&](const f32x4 q) {
        Row w;
        w.v[0] = q.x; w.v[1] = q.y; w.v[2] = q.z; w.v[3] = q.w;
        const float from_left = lane_left(w.v[3]), from_right = lane_right(w.v[0]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            w.l[k] = k > 0 ? w.v[k - 1] : from_left;
            w.r[k] = k < 3 ? w.v[k + 1] : from_right;
            w.h[k] = (w.l[k] + w.v[k]) + w.r[k];
        }
        return w;
    };
    Row up = prep(src.fix(src.template load<STREAM>(x0, y0 - 1), x0, y0 - 1));
    Row mid = prep(src.fix(src.template load<STREAM>(x0, y0), x0, y0));
    for (int y = y0; y < y1; y += AHEAD) {
        f32x4 next[AHEAD];
#pragma unroll
        for (int k = 0; k < AHEAD; ++k) next[k] = src.template load<STREAM>(x0, y + 1 + k < ny ? y + 1 + k : ny);
#pragma unroll
        for (int k = 0; k < AHEAD; ++k) {
            if (y + k >= y1) break;
            const Row down = prep(src.fix(next[k], x0, y + 1 + k));
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float nbrs = (up.h[e] + down.h[e]) + (mid.l[e] + mid.r[e]);
                v[e] = fmaf(share, nbrs, keep * mid.v[e]);
            }
            float* d = dst.at(x0, y + k);
            if (full) {
                const f32x4 o = {v[0], v[1], v[2], v[3]};
                if constexpr (STREAM_OUT) __builtin_nontemporal_store(o, reinterpret_cast<f32x4*>(d));
                else *reinterpret_cast<f32x4*>(d) = o;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (out[e]) d[e] = v[e];
            }
            up = mid;
            mid = down;
        }
    }
}

constexpr int64_t kCacheBytes = (int64_t)256 << 20;
constexpr int kRowsCached = 8, kRowsStream = 16;

template <int AHEAD, bool STREAM, bool STREAM_OUT>
__global__ __launch_bounds__(256) void diffuse_padded4_kernel(const float* src, float* dst, int nx, int ny, int pitch,
                                                              int rows, float keep, float share) {
    diffuse_strip4<AHEAD, STREAM, STREAM_OUT>(PaddedRows4{src, pitch}, PaddedStore4{dst, pitch}, nx, ny, rows, keep,
                                              share);
}

template <int AHEAD, bool STREAM, bool STREAM_OUT>
__global__ __launch_bounds__(256) void diffuse_checked4_kernel(const float* src, float* dst, int nx, int ny, int rows,
                                                               float keep, float share) {
    diffuse_strip4<AHEAD, STREAM, STREAM_OUT>(CheckedRows4{src, nx, ny}, PlainStore4{dst, nx}, nx, ny, rows, keep,
                                              share);
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

unsigned waves_blocks(int nx, int ny, int span, int rows = kRows) {
    const int64_t strips = (nx + span - 1) / span;
    const int64_t waves = strips * ((ny + rows - 1) / rows);
    return (unsigned)((waves + 3) / 4);
}

// blocks of the 4-column kernels: a multiple of 8 (the XCD-grouped order)
unsigned blocks4(int nx, int ny, int span, int rows) { return (waves_blocks(nx, ny, span, rows) + 7) / 8 * 8; }

bool aligned16(const void* a, const void* b) { return ((uintptr_t)a | (uintptr_t)b) % 16 == 0; }

bool bad_args(const void* a, const void* b, int nx, int ny, float D) {
    return !a || !b || nx < 1 || ny < 1 || !(D >= 0.0f && D <= 1.0f) || (int64_t)nx * ny > ((int64_t)1 << 40);
}

// Launches the 4-column kernel of the memory regime that an array of
// `bytes` bytes falls in.
template <template <int, bool, bool> class K, class... Args>
void launch4(int64_t bytes, int nx, int ny, int span, hipStream_t st, Args... args) {
    if (2 * bytes <= kCacheBytes)
        K<8, false, false>::launch(blocks4(nx, ny, span, kRowsCached), st, kRowsCached, args...);
    else if (bytes <= 2 * kCacheBytes)
        K<8, false, true>::launch(blocks4(nx, ny, span, kRowsCached), st, kRowsCached, args...);
    else
        K<16, true, true>::launch(blocks4(nx, ny, span, kRowsStream), st, kRowsStream, args...);
}

template <int A, bool S, bool SO>
struct Padded4 {
    static void launch(unsigned blocks, hipStream_t st, int rows, const float* src, float* dst, int nx, int ny,
                       int pitch, float keep, float share) {
        hipLaunchKernelGGL((diffuse_padded4_kernel<A, S, SO>), dim3(blocks), dim3(256), 0, st, src, dst, nx, ny, pitch,
                           rows, keep, share);
    }
};
template <int A, bool S, bool SO>
struct Checked4 {
    static void launch(unsigned blocks, hipStream_t st, int rows, const float* src, float* dst, int nx, int ny,
                       float keep, float share) {
        hipLaunchKernelGGL((diffuse_checked4_kernel<A, S, SO>), dim3(blocks), dim3(256), 0, st, src, dst, nx, ny,
                           rows, keep, share);
    }
};

}  // namespace

extern "C" {

int sw_diffuse_padded(const float* src, float* dst, int32_t nx, int32_t ny, int32_t pitch, float D, void* stream) {
    if (bad_args(src, dst, nx, ny, D) || pitch < nx + 2) return -1;
    const hipStream_t st = (hipStream_t)stream;
    const float keep = 1.0f - D, share = D / 8.0f;
    if (pitch % 4 != 0 || !aligned16(src, dst))
        hipLaunchKernelGGL(diffuse_padded_kernel, dim3(waves_blocks(nx, ny, kStrip)), dim3(256), 0, st, src, dst, nx,
                           ny, pitch, keep, share);
    else
        launch4<Padded4>((int64_t)(ny + 2) * pitch * 4, nx, ny, PaddedRows4::kSpan, st, src, dst, nx, ny, pitch, keep,
                         share);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int sw_diffuse_checked(const float* src, float* dst, int32_t nx, int32_t ny, float D, void* stream) {
    if (bad_args(src, dst, nx, ny, D)) return -1;
    const hipStream_t st = (hipStream_t)stream;
    const float keep = 1.0f - D, share = D / 8.0f;
    if (nx % 4 != 0 || !aligned16(src, dst))
        hipLaunchKernelGGL(diffuse_checked_kernel, dim3(waves_blocks(nx, ny, kStrip)), dim3(256), 0, st, src, dst, nx,
                           ny, keep, share);
    else
        launch4<Checked4>((int64_t)ny * nx * 4, nx, ny, CheckedRows4::kSpan, st, src, dst, nx, ny, keep, share);
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
