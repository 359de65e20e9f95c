// megs_internal.hpp -- shared device types and launch declarations of libmegs (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "megs.h"

namespace megs {

// 3DGS rasteriser conventions (the paper builds on them without restating them).
constexpr float kDilation = 0.3f;          // px^2 added to the 2D covariance diagonal
constexpr float kAlphaMin = 1.0f / 255.0f; // fragments below are skipped
constexpr float kAlphaMax = 0.99f;         // alpha clamp
constexpr float kTMin = 1e-4f;             // stop before transmittance drops below
constexpr float kFovClamp = 1.3f;          // Jacobian direction clamp, x half field of view
constexpr double kMaxCoord = 1e7;          // guard on |u|, |v| and the radius
constexpr float kLog2e = 1.4426950408889634f;

constexpr int kWave = 64;

// Per-view constants, device resident (uploaded once per forward or graph).
struct ViewInfo {
    float R[9];
    float t[3];
    float fx, fy, cx, cy, znear;
    float bg[3];
    float campos[3];   // camera centre -R^T t
    float limx, limy;  // Jacobian clamp bounds on x/z and y/z
    int32_t width, height, tiles_x, tiles_y;
    int64_t tile_off;  // first global tile id of the view
    int64_t pix_off;   // first pixel (over all views) of the view
};

struct SceneDev {
    int64_t n;
    int32_t k;
    int32_t dt_geom, dt_color, dt_amp;
    const void *pos, *logscale, *quat, *op_logit, *pmask_logit;
    const void *base, *axis, *sharp, *amp, *lmask_logit;
};

struct GradDev {
    float *pos, *logscale, *quat, *op_logit, *pmask_logit;
    float *base, *axis, *sharp, *amp, *lmask_logit;
};

// Record planes written by the projection (record r = view * n + i).
struct Records {
    double2* mean;      // pixel-space mean
    float4* conic_o;    // conic a, b, c and effective opacity
    float4* rgbd;       // colour and camera depth
    int32_t* radius;    // -1 when culled
    uint32_t* ntiles;   // tiles of the rectangle the footprint ellipse reaches
    uint32_t* dkey;     // depth sort key: float bits of depth, 0xffffffff when no tiles
    float* cutoff;      // k of the footprint ellipse q(d) = d' conic d <= k (with margin)
};

__device__ __forceinline__ float load_elem(const void* p, int dt, int64_t idx) {
    if (dt == MEGS_F32) return static_cast<const float*>(p)[idx];
    if (dt == MEGS_F16) return __half2float(static_cast<const __half*>(p)[idx]);
    uint32_t bits = static_cast<uint32_t>(static_cast<const uint16_t*>(p)[idx]) << 16;
    return __uint_as_float(bits);
}

// Tile rectangle [x0, x1] x [y0, y1] (inclusive tile indices) of pixel bounds floor(u) -/+ r,
// clipped to the image. Returns the number of tiles (0 when outside the image).
__device__ __forceinline__ uint32_t tile_rect(double u, double v, int32_t r, const ViewInfo& vw, int tile,
                                              int& x0, int& x1, int& y0, int& y1) {
    double fu = floor(u), fv = floor(v);
    double xl = fu - r, xh = fu + r, yl = fv - r, yh = fv + r;
    if (xh < 0.0 || yh < 0.0 || xl > vw.width - 1 || yl > vw.height - 1) return 0u;
    int ixl = xl < 0.0 ? 0 : static_cast<int>(xl);
    int iyl = yl < 0.0 ? 0 : static_cast<int>(yl);
    int ixh = xh > vw.width - 1 ? vw.width - 1 : static_cast<int>(xh);
    int iyh = yh > vw.height - 1 ? vw.height - 1 : static_cast<int>(yh);
    x0 = ixl / tile; x1 = ixh / tile; y0 = iyl / tile; y1 = iyh / tile;
    return static_cast<uint32_t>((x1 - x0 + 1) * (y1 - y0 + 1));
}

// Does the ellipse {p : (p - m)' C (p - m) <= k} (C = [[a, b], [b, c]] positive definite) reach
// the box [X0, X1] x [Y0, Y1] of a tile's pixel centres? The minimum of the convex quadratic over
// the box is 0 when the mean lies inside, else it is attained on an edge, where the 1D minimiser
// along the edge is clamped to the edge's extent. Plain FP64 +, *, / in a fixed order, so any
// IEEE implementation takes the same decision from the same inputs.
__device__ __forceinline__ bool tile_reached(double u, double v, double a, double b, double c, double k,
                                             double X0, double X1, double Y0, double Y1) {
    if (u >= X0 && u <= X1 && v >= Y0 && v <= Y1) return true;
    double best = INFINITY;
    for (int e = 0; e < 4; ++e) {
        double dx, dy;
        if (e < 2) {
            dx = (e == 0 ? X0 : X1) - u;
            const double lo = Y0 - v, hi = Y1 - v;
            dy = -(b * dx) / c;
            dy = dy < lo ? lo : (dy > hi ? hi : dy);
        } else {
            dy = (e == 2 ? Y0 : Y1) - v;
            const double lo = X0 - u, hi = X1 - u;
            dx = -(b * dy) / a;
            dx = dx < lo ? lo : (dx > hi ? hi : dx);
        }
        const double t1 = (a * dx) * dx;
        const double t2 = ((2.0 * b) * dx) * dy;
        const double t3 = (c * dy) * dy;
        const double q = (t1 + t2) + t3;
        best = q < best ? q : best;
    }
    return best <= k;
}

// Pixel-centre box of tile (tx, ty) of view vw.
__device__ __forceinline__ void tile_box(const ViewInfo& vw, int tile, int tx, int ty, double& X0, double& X1,
                                         double& Y0, double& Y1) {
    const int xe = (tx + 1) * tile < vw.width ? (tx + 1) * tile : vw.width;
    const int ye = (ty + 1) * tile < vw.height ? (ty + 1) * tile : vw.height;
    X0 = tx * tile + 0.5;
    X1 = xe - 0.5;
    Y0 = ty * tile + 0.5;
    Y1 = ye - 0.5;
}

// View of a global tile id: linear scan of the (few) view tile offsets.
__device__ __forceinline__ int view_of_tile(const ViewInfo* views, int nv, int64_t t) {
    int v = 0;
    while (v + 1 < nv && views[v + 1].tile_off <= t) ++v;
    return v;
}

// ---- per-stage profiling (api.hip): brackets a stage's launches with HIP events ----
struct StageTimer {
    StageTimer(int stage, hipStream_t stream);
    ~StageTimer();
    int stage;
    hipStream_t stream;
    void* start;
};

// ---- launch wrappers (one per kernel family; all enqueue on `stream`) ----

hipError_t launch_project(const SceneDev& sc, const ViewInfo* views, int nv, int tile, const Records& rec,
                          hipStream_t stream);
hipError_t launch_project_bwd(const SceneDev& sc, const ViewInfo* views, int nv, const float* grad2d,
                              const GradDev& g, hipStream_t stream);

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t stream);
hipError_t launch_iota(uint32_t* p, int64_t count, hipStream_t stream);

// Exclusive scan of x[idx[i]] (idx may be null) for i < n (n given on host), writing out[i];
// total written to *total (device). scratch: scan_scratch_bytes(n).
size_t scan_scratch_bytes(int64_t n);
hipError_t launch_scan(const uint32_t* x, const uint32_t* idx, int64_t n, uint32_t* out, uint32_t* total,
                       void* scratch, hipStream_t stream);

// Stable LSD radix sort of (key, value) pairs on bits [begin_bit, end_bit). The element count is
// read on device from *d_count (capped at max_count). Sorted output ends in keys/vals when
// the return flag `in_alt` is false, else in keys_alt/vals_alt.
size_t radix_scratch_bytes(int64_t max_count);
hipError_t launch_radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                                 const uint32_t* d_count, int64_t max_count, int begin_bit, int end_bit,
                                 void* scratch, hipStream_t stream, bool* in_alt);
hipError_t launch_radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                                 const uint32_t* d_count, int64_t max_count, int begin_bit, int end_bit,
                                 void* scratch, hipStream_t stream, bool* in_alt);

// Key emission: for every record (in `order`, or index order when order is null) write its
// tiles' keys at offsets[pos]. Two-stage: u32 global tile ids; one-stage: u64 tile|depth keys.
hipError_t launch_emit(const Records& rec, const ViewInfo* views, int nv, int64_t n, int tile,
                       const uint32_t* order, const uint32_t* offsets, int64_t n_records,
                       uint32_t* tile_keys, uint64_t* keys64, uint32_t* vals, int64_t capacity,
                       int32_t* status, hipStream_t stream);
hipError_t launch_ranges_u32(const uint32_t* tile_keys, const uint32_t* d_count, int64_t max_count,
                             uint2* ranges, hipStream_t stream);
hipError_t launch_ranges_u64(const uint64_t* keys, const uint32_t* d_count, int64_t max_count,
                             uint2* ranges, hipStream_t stream);
hipError_t launch_clamp_count(const uint32_t* total, int64_t capacity, uint32_t* count, int32_t* status,
                              hipStream_t stream);

struct BlendArgs {
    const ViewInfo* views;
    int nv;
    int64_t n_tiles;
    const double2* mean;
    const float4* conic_o;
    const float4* rgbd;
    const uint32_t* vals;
    const uint2* ranges;
    float* image;
    float* T_final;
    uint32_t* last;
    const float* dl;      // backward only
    float* grad2d;        // backward only, [NR][9]
    uint32_t* queue;      // persistent mode work counter (null: one workgroup per tile)
    unsigned long long* stats;  // forward fragment counters [blended, evaluated] (null: not counted)
    float* importance;          // forward: per-Gaussian sum of blending weights (null: not computed)
    int64_t n;                  // Gaussians per view (record r of view v is Gaussian r - v n)
};
hipError_t launch_blend_fwd(const BlendArgs& a, int tile, int batch, bool persistent, hipStream_t stream);
hipError_t launch_blend_bwd(const BlendArgs& a, int tile, int batch, bool persistent, hipStream_t stream);

// pruning steps (prune.hip)
size_t select_scratch_bytes(int64_t n);
hipError_t launch_select_topk(const float* score, int64_t n, int64_t kappa, void* scratch, uint8_t* keep,
                              hipStream_t stream);
hipError_t launch_lobe_range(int64_t n, int32_t k, const float* s, const float* lam, const float* amp, float* D,
                             hipStream_t stream);
hipError_t launch_prox_apply(int64_t count, const float* x, const float* lam, const uint8_t* keep, float* xt,
                             hipStream_t stream);
hipError_t launch_dual(int64_t count, float* lam, const float* x, const float* xt, hipStream_t stream);
hipError_t launch_penalty(int64_t count, float delta, const float* x, const float* xt, const float* lam, float* grad,
                          hipStream_t stream);

}  // namespace megs
