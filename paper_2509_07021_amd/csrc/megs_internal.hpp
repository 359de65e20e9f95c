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
// sqrt(log2(e) / 2): the blend's exponent in log2 units is -(w1^2 + w2^2) with w = kQ2 L' d (Shape)
constexpr float kQ2 = 0.84932180028801904f;

constexpr int kWave = 64;

// The hardware deals consecutive workgroups round-robin to the 8 XCDs (each with its own L2).
// xcd_item(b, n) maps workgroup b of an n-workgroup grid to an item so that XCD x runs one
// contiguous range of the n items: XCD x owns [x per + min(x, rem), ...) of length
// per + (x < rem), and receives exactly that many workgroups. Items processed close together in
// index order then share an L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_item(int64_t b, int64_t n_items) {
    const int64_t per = n_items / kXcds, rem = n_items % kXcds;
    const int64_t x = b % kXcds, k = b / kXcds;
    return x * per + (x < rem ? x : rem) + k;
}

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

// The most pairs a key table holds: positions are 32-bit and the counted total is reported in an int32.
constexpr uint32_t kMaxPairs = 0x7fffffffu;

// Words of the per-forward device status block (int32[8]).
constexpr int kStatusPairs = 0;     // pairs counted
constexpr int kStatusOverflow = 1;  // pair table overflowed its capacity
constexpr int kStatusBadLobes = 2;  // some compressed-row lobe offsets were malformed
constexpr int kStatusCulled = 3;    // records the projection culled (not rendered in their view)
// Work counters of a persistent launch: [0] for the per-tile kernels, one per slice of the items
// for the sub-tile kernels, each in its own 256 bytes (kQueueStride words apart: counters that share
// a cache line serialise each other's atomics); zeroed before each launch.
constexpr int kQueueStride = 64;
constexpr int kQueueWords = 8 * kQueueStride;

struct SceneDev {
    int64_t n;
    int32_t k;  // lobes per Gaussian (dense) or the most any Gaussian has (compressed rows)
    int32_t dt_geom, dt_color, dt_amp;
    const void *pos, *logscale, *quat, *op_logit, *pmask_logit;
    const void *base, *axis, *sharp, *amp, *lmask_logit;
    const int32_t* lobe_off;  // NULL: dense lobe planes; else compressed-row offsets [n + 1]
    int64_t n_lobes;
    int32_t* status;          // device status block, or NULL
    const void* sh;           // NULL: SG colour; else SH coefficients [(sh_degree + 1)^2][3][n]
    int32_t sh_degree;
};

struct GradDev {
    float *pos, *logscale, *quat, *op_logit, *pmask_logit;
    float *base, *axis, *sharp, *amp, *lmask_logit;
    float* sh;
};

// The 2D shape of a record. The conic Q = [[a, b], [b, c]] (q = d' Q d for a pixel offset d from the
// mean) is kept as the factors of Q = L L', L = [[l11, 0], [l11 r, l22]]:
//   q = (l11 (dx + r dy))^2 + (l22 dy)^2,
// with l11 = sqrt(C / det), r = -B / C, l22 = 1 / sqrt(C) for the dilated covariance [[A, B], [B, C]] and
// det = A C - B^2. Both terms are squares, so q never cancels; along a thin footprint the first factor
// does, and the ratio r is kept in FP64 so that the footprint's direction survives to hundreds of pixels.
// a = l11^2, b = l11^2 r, c = (l11 r)^2 + l22^2 and a c - b^2 = (l11 l22)^2 follow in FP64.
struct Shape {
    double a, b, c, det;
};
__device__ __forceinline__ Shape shape_of(float l11, double r, float l22) {
    Shape s;
    const double p = (double)l11, q = (double)l22;
    s.a = p * p;
    s.b = s.a * r;
    const double pr = p * r;
    s.c = pr * pr + q * q;
    const double pq = p * q;
    s.det = pq * pq;
    return s;
}

// One record in 48 bytes: what the blend and the projection backward read of it, gathered in
// depth and tile order (three 16-byte loads per gathered record instead of one per plane). The
// key emission forms the footprint radius from it (footprint_rho); its tile count is the step of
// the offsets' scan.
struct __align__(16) PackedRec {
    double2 mean;     // pixel-space mean
    double r;         // the conic's factor ratio (Shape)
    float l11, l22;   // the conic's diagonal factors (Shape); l22 = 0 when culled
    float o;          // effective opacity
    float rgb[3];     // colour
};
static_assert(sizeof(PackedRec) == 48, "three 16-byte vectors per record");

// Record planes written by the projection (record r = view * n + i).
struct Records {
    PackedRec* packed;  // the records, 48 bytes each
    // per-field planes (null unless MEGS_FLAG_RECORD_PLANES): mean .. radius, cutoff, chol
    double2* mean;      // pixel-space mean
    float4* conic_o;    // conic a, b, c (FP32 roundings of the factors' products) and effective opacity
    float4* rgbd;       // colour and camera depth
    int32_t* radius;    // -1 when culled
    uint32_t* ntiles_plane;  // copy of ntiles for the caller
    // the forward's own planes, in its sorting work space
    uint32_t* ntiles;   // tiles of the rectangle the footprint ellipse reaches
    uint32_t* dkey;     // depth sort key: float bits of depth, 0xffffffff when no tiles
    // initial values of the depth sort when non-null: record id r in the low order_idb bits and
    // min(ntiles, cap) above them, cap = 2^(32 - order_idb) - 1 marking a count that did not fit
    uint32_t* order0;
    int32_t order_idb;
    float* cutoff;      // k of the footprint ellipse q(d) = d' conic d <= k (with margin)
    double4* chol;      // the conic's factors as the blend uses them: l11, r, l22, 0
};

// Ellipse level that bounds every pixel with alpha >= 1/255: q <= 2 ln(255 o), widened by 0.2% (and
// 1e-4 absolute) so that FP32 rounding in the blend never reaches past a culled tile.
__device__ __forceinline__ float cutoff_of(float o_eff) {
    return 2.004f * __logf(255.0f * o_eff) + 1e-4f;
}

// Footprint radius before rounding up: every pixel with alpha >= 1/255 lies within
// rho = sqrt(2 ln(255 o) lmax) of the mean, lmax the larger eigenvalue of the 2D covariance. The
// covariance is taken from the stored factors of its inverse (Shape): S_xx = (r / l22)^2 + 1 / l11^2,
// S_yy = 1 / l22^2, det S = 1 / (l11 l22)^2, so the projection (which stores ceil(rho)) and the key
// emission (which needs it for the tile rectangle) form the same radius from the same record, and
// the emission need not gather a radius plane. Non-finite for a degenerate shape.
__device__ __forceinline__ float footprint_rho(float l11, double r, float l22, float o_eff) {
    const float il11 = 1.0f / l11, il22 = 1.0f / l22;
    const float rq = (float)r * il22, d = il11 * il22;
    const float sxx = __fmaf_rn(rq, rq, il11 * il11), syy = il22 * il22, det = d * d;
    const float mid = 0.5f * (sxx + syy);
    const float lmax = mid + sqrtf(fmaxf(__fmaf_rn(mid, mid, -det), 0.0f));
    return sqrtf(2.0f * __logf(255.0f * o_eff) * lmax);
}

// N parameter elements of one storage type (element j: plane p[j], index idx[j]; 0 where live[j] is
// false, and then not read), under one branch on the uniform storage type. FP32 elements are loaded
// straight into out. FP16 and BF16 ones are all loaded as 16-bit words before any is converted:
// converting each inside its load's branch (as load_elem does) makes the compiler wait for every
// 16-bit load before it issues the next.
template <int N>
__device__ __forceinline__ void load_n(int dt, const void* const (&p)[N], const int64_t (&idx)[N],
                                       const bool (&live)[N], float (&out)[N]) {
    if (dt == MEGS_F32) {
#pragma unroll
        for (int j = 0; j < N; ++j) out[j] = live[j] ? static_cast<const float*>(p[j])[idx[j]] : 0.0f;
        return;
    }
    uint32_t h[N];
#pragma unroll
    for (int j = 0; j < N; ++j) h[j] = live[j] ? static_cast<const uint16_t*>(p[j])[idx[j]] : 0u;
    if (dt == MEGS_F16) {
#pragma unroll
        for (int j = 0; j < N; ++j) out[j] = __half2float(__ushort_as_half((unsigned short)h[j]));
    } else {
#pragma unroll
        for (int j = 0; j < N; ++j) out[j] = __uint_as_float(h[j] << 16);
    }
}

__device__ __forceinline__ float load_elem(const void* p, int dt, int64_t idx) {
    if (dt == MEGS_F32) return static_cast<const float*>(p)[idx];
    if (dt == MEGS_F16) return __half2float(static_cast<const __half*>(p)[idx]);
    uint32_t bits = static_cast<uint32_t>(static_cast<const uint16_t*>(p)[idx]) << 16;
    return __uint_as_float(bits);
}

// FP32 to the storage dtype, round to nearest even (BF16: the upper half of the FP32 pattern after
// adding 0x7fff plus the lowest kept bit; NaNs stay NaN).
__device__ __forceinline__ void store_elem(void* p, int dt, int64_t idx, float v) {
    if (dt == MEGS_F32) { static_cast<float*>(p)[idx] = v; return; }
    if (dt == MEGS_F16) { static_cast<__half*>(p)[idx] = __float2half_rn(v); return; }
    const uint32_t b = __float_as_uint(v);
    const uint32_t r = isnan(v) ? ((b >> 16) | 0x40u) : ((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
    static_cast<uint16_t*>(p)[idx] = (uint16_t)r;
}

// Copies one stored element bit for bit.
__device__ __forceinline__ void copy_elem(void* dst, int64_t di, const void* src, int64_t si, int dt) {
    if (dt == MEGS_F32)
        static_cast<uint32_t*>(dst)[di] = static_cast<const uint32_t*>(src)[si];
    else
        static_cast<uint16_t*>(dst)[di] = static_cast<const uint16_t*>(src)[si];
}

// Where the lobes of Gaussian i live. Dense scenes: K lobes, element l n + i of a one-row plane
// (sharpness, lobe mask) and (3 l + c) n + i of a three-row plane (axis, amplitude). Compressed-row
// scenes: lobes lobe_off[i] .. lobe_off[i + 1] - 1, elements off + l and c n_lobes + off + l.
template <bool RAGGED>
struct LobeRef {
    int64_t off, n;
    int cnt;
    __device__ __forceinline__ int64_t at1(int l) const { return RAGGED ? off + l : (int64_t)l * n + off; }
    __device__ __forceinline__ int64_t at3(int l, int c) const {
        return RAGGED ? (int64_t)c * n + off + l : ((int64_t)l * 3 + c) * n + off;
    }
};

// Reads the lobe slice of Gaussian i (at most kmax lobes); false, with a flag in the status block,
// when compressed-row offsets are malformed: decreasing, outside [0, n_lobes], or more than kmax.
template <bool RAGGED>
__device__ __forceinline__ bool lobe_ref(const SceneDev& sc, int64_t i, int kmax, LobeRef<RAGGED>& r) {
    if (!RAGGED) {
        r.off = i; r.n = sc.n; r.cnt = kmax;
        return true;
    }
    const int64_t a = sc.lobe_off[i], b = sc.lobe_off[i + 1];
    r.off = a; r.n = sc.n_lobes; r.cnt = (int)(b - a);
    if (a < 0 || b < a || b > sc.n_lobes || b - a > kmax) {
        r.off = 0; r.cnt = 0;
        if (sc.status) sc.status[kStatusBadLobes] = 1;
        return false;
    }
    return true;
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
    const int sh = __ffs(tile) - 1;  // tile is a power of two and the indices are >= 0
    x0 = ixl >> sh; x1 = ixh >> sh; y0 = iyl >> sh; y1 = iyh >> sh;
    return static_cast<uint32_t>((x1 - x0 + 1) * (y1 - y0 + 1));
}

// Tile selection inside a record's rectangle: a tile is listed when the ellipse
// E = {p : (p - m)' C (p - m) <= k} (C = [[a, b], [b, c]] the conic, k the record's level) meets the box
// spanned by the centres of the tile's pixels inside the image. Evaluated per tile row: with
// band = the row's pixel-centre rows [Y0, Y1], E ∩ band is convex, so a tile's box meets it exactly
// when their x-ranges overlap. With S = C^-1, the points of E with extreme x lie at
// dy = +-S_xy sqrt(k / S_xx); the x-extent over the band is reached there, clamped into the band
// (x_max(dy) is concave, x_min(dy) convex). FP64 throughout.
struct EllipseRows {
    double u, v, b, det, ia, ka, ry, dys;
    bool full;  // degenerate conic: list the whole rectangle
};

__device__ __forceinline__ void ellipse_rows(double u, double v, const Shape& q, double k, EllipseRows& e) {
    e.u = u; e.v = v; e.b = q.b;
    e.det = q.det;
    e.full = !(e.det > 0.0) || !(q.a > 0.0) || !(k > 0.0);
    const double sxx = q.c / e.det, syy = q.a / e.det, sxy = -q.b / e.det;
    e.ry = sqrt(k * syy);
    e.dys = sxy * sqrt(k / sxx);
    e.ia = 1.0 / q.a;
    e.ka = k * q.a;
}

// Columns [lo, hi] of tile row ty listed for the record (within the rectangle columns [x0, x1]);
// returns false when the row lists no tile. The last tile column's box ends at the image's last pixel
// centre, width - 1/2.
__device__ __forceinline__ bool row_span(const EllipseRows& e, int width, int height, int tile, int ty, int x0,
                                         int x1, int& lo, int& hi) {
    if (e.full) { lo = x0; hi = x1; return true; }
    const int ye = (ty + 1) * tile < height ? (ty + 1) * tile : height;
    double dl = (ty * tile + 0.5) - e.v, dh = (ye - 0.5) - e.v;
    if (dl < -e.ry) dl = -e.ry;
    if (dh > e.ry) dh = e.ry;
    if (dl > dh) return false;
    double d1 = e.dys;
    if (d1 < dl) d1 = dl;
    if (d1 > dh) d1 = dh;
    double d2 = -e.dys;
    if (d2 < dl) d2 = dl;
    if (d2 > dh) d2 = dh;
    const double r1 = e.ka - (e.det * d1) * d1;
    const double r2 = e.ka - (e.det * d2) * d2;
    const double s1 = sqrt(r1 > 0.0 ? r1 : 0.0);
    const double s2 = sqrt(r2 > 0.0 ? r2 : 0.0);
    const double xmax = e.u + (s1 - e.b * d1) * e.ia;
    const double xmin = e.u - (s2 + e.b * d2) * e.ia;
    if (xmin > width - 0.5) return false;
    // division by the power-of-two tile size as an exact exponent shift (the same value as x / tile)
    const int sh = __ffs(tile) - 1;
    double flo = ceil(ldexp(xmin + 0.5, -sh) - 1.0), fhi = floor(ldexp(xmax - 0.5, -sh));
    if (flo < x0) flo = x0;
    if (fhi > x1) fhi = x1;
    if (flo > fhi) return false;
    lo = (int)flo;
    hi = (int)fhi;
    return true;
}

// Element comp (0..8) of record r in the backward's per-record sums: nine consecutive floats per
// record, the six exponent sums then the colour gradient (the blend's nine-lane atomic adds to one
// contiguous run; the projection backward's two passes each read their part of it).
__device__ __forceinline__ int64_t grad2d_index(int64_t r, int comp) { return 9 * r + comp; }

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
// rec: the forward's records (the backward reads each record's conic factors from them)
hipError_t launch_project_bwd(const SceneDev& sc, const ViewInfo* views, int nv, const float* grad2d,
                              const PackedRec* rec, const GradDev& g, hipStream_t stream);

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t stream);
hipError_t launch_iota(uint32_t* p, int64_t count, hipStream_t stream);

// Exclusive scan of x[idx[i]] (idx may be null) for i < n (n given on host), writing out[i];
// total written to *total (device). scratch: scan_scratch_bytes(n). With idx, `gathered` (n
// entries, optional) receives the gathered values, which saves the second pass a gather.
size_t scan_scratch_bytes(int64_t n);
// The same scan over depth-sorted values that carry the tile count above the record id (see
// Records::order0): counts come from the values themselves (ntiles[id] only for the escape value),
// and the values are rewritten in place as bare record ids.
hipError_t launch_scan_packed(uint32_t* order, const uint32_t* ntiles, int64_t n, int idb, uint32_t* out,
                              uint32_t* total, void* scratch, hipStream_t stream);
hipError_t launch_scan(const uint32_t* x, const uint32_t* idx, int64_t n, uint32_t* out, uint32_t* total,
                       void* scratch, hipStream_t stream, uint32_t* gathered = nullptr);

// Stable LSD radix sort of (key, value) pairs on bits [begin_bit, end_bit). The element count is
// read on device from *d_count (capped at max_count). Sorted output ends in keys/vals when
// the return flag `in_alt` is false, else in keys_alt/vals_alt.
size_t radix_scratch_bytes(int64_t max_count);
int radix_passes(int begin_bit, int end_bit);
hipError_t launch_radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                                 const uint32_t* d_count, int64_t max_count, int begin_bit, int end_bit,
                                 void* scratch, hipStream_t stream, bool* in_alt);
hipError_t launch_radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                                 const uint32_t* d_count, int64_t max_count, int begin_bit, int end_bit,
                                 void* scratch, hipStream_t stream, bool* in_alt);

// Key emission: for every record (in `order`, or index order when order is null) write its
// tiles' keys at offsets[pos]; total: the scan's grand total (device). Two-stage: u32 global tile ids;
// one-stage: u64 tile|depth keys. sub = 8: the upper 16 bits of each 32-bit tile key flag the 8 x 8
// sub-tiles the record reaches (two-stage sort, tile ids below 2^16); sub = 0: plain tile ids.
hipError_t launch_emit(const Records& rec, const ViewInfo* views, int nv, int64_t n, int tile,
                       const uint32_t* order, const uint32_t* offsets, const uint32_t* total, int64_t n_records,
                       uint32_t* tile_keys, uint64_t* keys64, uint32_t* vals, int64_t capacity,
                       int32_t* status, hipStream_t stream, int sub);
hipError_t launch_ranges_u32(const uint32_t* tile_keys, const uint32_t* d_count, int64_t max_count,
                             uint2* ranges, hipStream_t stream, uint32_t tmask);
hipError_t launch_ranges_u64(const uint64_t* keys, const uint32_t* d_count, int64_t max_count,
                             uint2* ranges, hipStream_t stream);
hipError_t launch_clamp_count(const uint32_t* total, int64_t capacity, uint32_t* count, int32_t* status,
                              hipStream_t stream);

struct BlendArgs {
    const ViewInfo* views;
    int nv;
    int64_t n_tiles;
    const PackedRec* rec;  // the projection's records, 48 bytes each
    const uint32_t* tkeys; // sorted tile keys carrying sub-tile flags in bits 16-31 (null: none)
    const uint32_t* vals;
    const uint2* ranges;
    float* image;
    float* T_final;
    uint32_t* last;
    const float* dl;      // backward only
    float* grad2d;        // backward only, [NR][9] (grad2d_index): sums over the record's fragments
                          // of e w1, e w2, e w1^2, e w1 w2, e w2^2 and e (e = dL/do_eff of an unclamped
                          // fragment, whose exponent gradient is o_eff e; w1, w2 the exponent's
                          // factors kQ2 L' d of the pixel offset d, Shape), then dL/dRGB
    float* grad_pair;     // deterministic backward: per list position [P][9] (null: atomics into grad2d)
    uint32_t* queue;      // persistent mode work counters (kQueueWords)
    unsigned long long* stats;  // forward fragment counters [blended, evaluated] (null: not counted)
    float* importance;          // forward: per-Gaussian sum of blending weights (null: not computed)
    int64_t n;                  // Gaussians per view (record r of view v is Gaussian r - v n)
};
// subtile 8 (with 16 x 16 or 32 x 32 tiles): one independent wave per 8 x 8 sub-tile walking its
// tile's list (the deterministic backward keeps the per-tile kernels).
hipError_t launch_blend_fwd(const BlendArgs& a, int tile, int waves, int batch, bool persistent, hipStream_t stream,
                            int subtile);
hipError_t launch_blend_bwd(const BlendArgs& a, int tile, int waves, int batch, bool persistent, hipStream_t stream,
                            int subtile);

// deterministic backward support (sort.hip)
hipError_t launch_copy_u32(uint32_t* dst, const uint32_t* src, int64_t count, hipStream_t stream);
// perm[s] = emission position of sorted position s (s < *d_count): rec_sorted[s] = rec_emit[perm[s]],
// inv[perm[s]] = s.
hipError_t launch_perm_gather(const uint32_t* perm, const uint32_t* rec_emit, const uint32_t* d_count,
                              int64_t max_count, uint32_t* rec_sorted, uint32_t* inv, hipStream_t stream);
// grad2d[r] = sum over record r's pairs, in emission order, of grad_pair[inv[e]] (records walked in
// the emission order `order`, or index order when null; offsets[i] = first emission position).
hipError_t launch_pair_reduce(const uint32_t* order, const uint32_t* offsets, const uint32_t* ntiles,
                              int64_t n_records, const uint32_t* inv, const uint32_t* d_count,
                              const float* grad_pair, float* grad2d, hipStream_t stream);

// post-processing compaction (compact.hip)
struct CompactArgs {
    SceneDev in;
    double opacity_min, sharp_min;
    uint32_t* keep;      // [n] 1 when Gaussian i is kept
    uint32_t* count;     // [n] lobes Gaussian i keeps
    uint32_t* new_idx;   // [n] exclusive scan of keep
    uint32_t* lobe_pos;  // [n] exclusive scan of count
    int64_t n_out, l_out;
    void *pos, *logscale, *quat, *op_logit, *base, *axis, *sharp, *amp;  // compacted planes
    int32_t* lobe_off;   // [n_out + 1]
    int32_t* kept;       // [n_out] source Gaussian
    int32_t* lobe_src;   // [l_out] source lobe element
};
hipError_t launch_compact_mark(const CompactArgs& a, hipStream_t stream);
hipError_t launch_compact_write(const CompactArgs& a, hipStream_t stream);

// training-step pieces (loss.hip)
struct LossView {
    int32_t width, height;
    int64_t pix_off;   // first pixel of the view in the concatenated image layout
    int64_t part_off;  // first loss partial of the view
    int64_t n_part;    // partials of the view (3 channels x tiles)
};
struct LossViews {
    LossView v[MEGS_MAX_VIEWS];
};
struct Window11 {
    double w[11];
};
int64_t loss_partials(int width, int height);
hipError_t launch_loss(const LossViews& vs, int nv, const float* x, const float* y, double* maps, double* partial,
                       double* terms, double* loss, float* dl, const Window11& g, double lam, hipStream_t stream);
hipError_t launch_adam(int64_t count, void* param, int dt, const float* grad, float* m, float* v, float lr, float b1,
                       float b2, float eps, int step, hipStream_t stream);

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
