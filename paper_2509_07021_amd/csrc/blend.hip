// blend.hip -- front-to-back alpha blending (forward) and its back-to-front replay (backward),
// gfx950: per-tile workgroup kernels, and the sub-tile kernels further down (one wave64 per 8 x 8
// sub-tile walking its tile's list; the configuration the benchmark runs).
//
// Compositing follows Sec. 3.1: C = sum_i c_i alpha_i prod_{j<i}(1 - alpha_j), alpha_i = o_i times
// the 2D Gaussian at the pixel, with the 3DGS conventions (alpha clamped to 0.99, fragments below
// 1/255 skipped, stop before the transmittance would fall under 1e-4).
//
// Mapping to CDNA4: a workgroup of 1, 2 or 4 wave64s per (view, tile), TILE^2 / (64 waves) pixels
// per lane, each wave owning a compact block of the tile (the whole tile, a half or a quadrant);
// every LDS read of a staged Gaussian is reused by all of a lane's pixels, and a wave skips a
// Gaussian whose footprint box misses its block or that reaches none of its pixels. More waves
// per tile shorten the serial walk of long tile lists (the latency of the densest tiles bounds a
// launch); one wave needs no workgroup barrier at all. Gaussians of the tile's list are staged into LDS in batches
// (one record per lane per load, gathered through the sorted record indices); their means are
// made tile-relative in FP64 while staging, so the per-fragment arithmetic works on small FP32
// offsets. The wave stops as soon as all its pixels have terminated.
//
// The backward walks each tile's list from the largest per-pixel last index down to 0, recovers
// the transmittance in front of each fragment by division, carries the colour seen behind the
// fragment (as its dot product with the pixel's colour gradient, the only form the gradient
// uses), and accumulates nine per-record sums: e = dL/do_eff of each unclamped fragment,
// its moments e w1, e w2, e w1^2, e w1 w2, e w2^2 in the exponent's factors (Staged; the exponent's
// gradient is o_eff e, so the projection backward turns them into the mean and conic gradients once
// per record), and the colour gradient. They are summed over the wave's pixels with a transposed butterfly of
// permlane swaps and DPP adds and added to the record's slot with nine lanes of one hardware
// float atomic, only when some lane of the wave contributed.
#include "megs_internal.hpp"

namespace megs {
namespace {

// A record as the blends use it, its shape folded into the exponent's affine factors over the
// pixel centres of one frame (a tile or a sub-tile, origin (X0, Y0), pixel centre (px, py) relative
// to it): the exponent in log2 units is -(w1^2 + w2^2) with
//   w1 = ax px + ay py + c1,  w2 = by py + c2,
// ax = kQ2 l11, ay = kQ2 l11 r, by = kQ2 l22 (Shape), c1 = kQ2 l11 ((X0 - u) + r (Y0 - v)) and
// c2 = kQ2 l22 (Y0 - v). c1 and c2 are formed in FP64 from the FP64 mean and ratio, so the
// cancellation along a thin footprint happens there, once per staged record; per pixel the FP32
// terms stay within a frame's width of the footprint. The backward needs the conic itself only per
// record, in the projection backward.
struct Staged {
    float4 box; // frame-relative bounding box of the cutoff ellipse: x - rx, x + rx, y - ry, y + ry
    float4 p0;  // ax, ay, c1, o
    float4 p1;  // by, c2, r, g
    float b;    // blue
};

// An entry kept for an 8x8 sub-tile, as the sub-tile blends read it back from LDS: the staged
// record without its box (the box only decides whether the entry is kept), plus the entry's list
// position and a record index, so that one LDS address serves every read of the entry (48 bytes).
struct Kept {
    float4 p0, p1;   // as in Staged
    float b;         // as in Staged
    uint32_t pos1;   // one past the entry's list position (relative to the tile's range start)
    uint64_t slot;   // forward: the record id (importance output); backward: the record's first
                     // element in the per-record sums (grad2d_index)
};
static_assert(sizeof(Kept) == 48 && offsetof(Kept, slot) % 8 == 0, "kept entries are 48 bytes, slot 8-aligned");

// &lds[k] through a VGPR copy of its byte offset. The compiler cannot rebuild the result of an asm
// statement, so every read of the entry (and, with immediate offsets, of the entries after it)
// shares this one address register, where it would otherwise re-derive the address from the
// scalar index with a VALU move before each group of reads.
__device__ __forceinline__ const Kept* kept_at(const Kept* lds, int k) {
    uint32_t off;
    asm("v_mov_b32 %0, %1" : "=v"(off) : "s"(k * (int)sizeof(Kept)));
    return reinterpret_cast<const Kept*>(reinterpret_cast<const char*>(lds) + off);
}

// Pixel layout of a (TILE, WAVES) workgroup: wave w owns a WW x WH block of the tile (the whole
// tile, its upper/lower half, or one quadrant), its lanes cover LW x LH pixels per slot, and
// pixel slot j of a lane lies LH j rows below slot 0. Compact blocks let a wave skip every staged
// Gaussian whose footprint box misses its block, which is most of them for small footprints.
template <int TILE, int WAVES>
struct Layout {
    static constexpr int WW = WAVES == 4 ? TILE / 2 : TILE;
    static constexpr int WH = WAVES == 1 ? TILE : TILE / 2;
    static constexpr int LW = WW;
    static constexpr int LH = 64 / LW;
    static constexpr int PPT = WW * WH / 64;
    static_assert(LW * LH == 64 && PPT * 64 == WW * WH, "tile and wave count mismatch");
    __device__ static int wx0(int wave) { return WAVES == 4 ? (wave & 1) * WW : 0; }
    __device__ static int wy0(int wave) { return WAVES == 4 ? (wave >> 1) * WH : (WAVES == 2 ? wave * WH : 0); }
};

// Stages record g for the frame with origin (x0, y0) (pixel coordinates of its top-left corner). Only
// t = (X0 - u) + r (Y0 - v), which cancels along a thin footprint, needs FP64; it is rounded once, and
// c1 = ax t and c2 = by (Y0 - v) then err by about one FP32 rounding of their own size. With box set,
// also the frame-relative box of the cutoff ellipse {d' Q d <= k}: its half-extents are sqrt(k A) and
// sqrt(k C) for the covariance Q^-1 = [[A, B], [B, C]], which the factors give without cancellation as
// A = (r / l22)^2 + 1 / l11^2 and C = 1 / l22^2; widened by 1e-3 relative and 1e-2 px, far more than
// FP32 rounding moves them, so every pixel with alpha >= 1/255 lies inside.
__device__ __forceinline__ void stage(const BlendArgs& a, uint32_t g, double x0, double y0, Staged* dst,
                                      bool box = true) {
    const float4* q = reinterpret_cast<const float4*>(a.rec + g);  // the record's three vectors
    const float4 q0 = q[0], q1 = q[1], q2 = q[2];
    const double mx = __hiloint2double(__float_as_int(q0.y), __float_as_int(q0.x));
    const double my = __hiloint2double(__float_as_int(q0.w), __float_as_int(q0.z));
    const double r = __hiloint2double(__float_as_int(q1.y), __float_as_int(q1.x));
    const double dx0 = x0 - mx, dy0 = y0 - my;
    const float t = (float)fma(r, dy0, dx0), dxf = (float)dx0, dyf = (float)dy0;
    const float ax = kQ2 * q1.z, by = kQ2 * q1.w;
    Staged s;
    s.p0 = make_float4(ax, ax * (float)r, ax * t, q2.x);
    s.p1 = make_float4(by, by * dyf, q2.y, q2.z);
    s.b = q2.w;
    s.box = make_float4(0.f, -1.f, 0.f, -1.f);
    if (box) {
        const float cut = cutoff_of(q2.x);
        const float il22 = __builtin_amdgcn_rcpf(q1.w), ra = (float)r * il22, il11 = __builtin_amdgcn_rcpf(q1.z);
        const float rx = __builtin_amdgcn_sqrtf(cut * __fmaf_rn(ra, ra, il11 * il11)) * 1.001f + 0.01f;
        const float ry = __builtin_amdgcn_sqrtf(cut) * il22 * 1.001f + 0.01f;
        s.box = make_float4(-dxf - rx, -dxf + rx, -dyf - ry, -dyf + ry);
    }
    *dst = s;
}

// Does the pixel block [x0, x1] x [y0, y1] (tile-relative, centres at +0.5) meet the staged
// footprint's box? Wave-uniform when the block is.
__device__ __forceinline__ bool box_meets(const float4& b, int x0, int x1, int y0, int y1) {
    return (x0 + 0.5f <= b.y) && (x1 + 0.5f >= b.x) && (y0 + 0.5f <= b.w) && (y1 + 0.5f >= b.z);
}

// Alpha test of one fragment (no branches): pass = alpha >= 1/255 with alpha = min(o G, 0.99) and
// G = 2^(-(w1^2 + w2^2)) (Staged). The compositing rule also skips fragments with a positive
// exponent, which a sum of squares never is. The threshold is tested on the unclamped value (the
// same decision for any number, and a NaN fails it). The forward and the backward call this same
// function, so both take identical decisions; w1 and w2 are returned for the backward's moments.
template <class E>  // Staged or Kept
__device__ __forceinline__ bool frag(const E& s, float px, float py, float& w1, float& w2, float& G,
                                     float& alpha, bool& clamped) {
    w1 = __fmaf_rn(s.p0.x, px, __fmaf_rn(s.p0.y, py, s.p0.z));
    w2 = __fmaf_rn(s.p1.x, py, s.p1.y);
    const float q2 = __fmaf_rn(-w1, w1, -(w2 * w2));
    G = __builtin_amdgcn_exp2f(q2);
    const float raw = s.p0.w * G;
    clamped = raw > kAlphaMax;
    alpha = fminf(raw, kAlphaMax);
    // keeps the clamp next to the product: moved into the callers' blend branches, it would need a
    // separate NaN-quieting step there
    asm volatile("" : "+v"(alpha));
    return raw >= kAlphaMin;
}

struct TileCtx {
    int view;
    int64_t tile;
    int x0, y0, width, height;
    int64_t pix_off;
    float bg[3];
};

__device__ __forceinline__ TileCtx tile_ctx(const BlendArgs& a, int64_t t, int TILE) {
    TileCtx c;
    c.tile = t;
    c.view = view_of_tile(a.views, a.nv, t);
    const ViewInfo& vw = a.views[c.view];
    const int64_t lt = t - vw.tile_off;
    c.x0 = (int)(lt % vw.tiles_x) * TILE;
    c.y0 = (int)(lt / vw.tiles_x) * TILE;
    c.width = vw.width;
    c.height = vw.height;
    c.pix_off = vw.pix_off;
    c.bg[0] = vw.bg[0]; c.bg[1] = vw.bg[1]; c.bg[2] = vw.bg[2];
    return c;
}

// Next work item: blockIdx.x when not persistent, else pulled from the queue counter (thread 0
// takes the item, the workgroup reads it back through LDS).
__device__ __forceinline__ int64_t next_tile(const BlendArgs& a, int64_t prev, bool persistent, uint32_t* slot) {
    if (!persistent) return prev < 0 ? (int64_t)blockIdx.x : a.n_tiles;
    __syncthreads();
    if (threadIdx.x == 0) *slot = atomicAdd(a.queue, 1u);
    __syncthreads();
    return (int64_t)*slot;
}

// Workgroup of WAVES wave64s per tile, PPT = TILE^2 / (64 WAVES) pixels per lane, each wave owning
// one compact block of the tile (Layout).
template <int TILE, int WAVES, bool STATS, bool IMP>
__global__ __launch_bounds__(64 * WAVES) void k_blend_fwd(BlendArgs a, int batch, int persistent) {
    using Ly = Layout<TILE, WAVES>;
    constexpr int NT = 64 * WAVES, PPT = Ly::PPT, LH = Ly::LH;
    extern __shared__ Staged lds[];
    uint32_t* lds_id = reinterpret_cast<uint32_t*>(lds + batch);  // record ids (importance only)
    __shared__ uint32_t work_slot;
    const int tid = threadIdx.x, lane = __lane_id(), wv = tid / 64;
    const int bx0 = Ly::wx0(wv), by0 = Ly::wy0(wv);   // this wave's block
    const int lx = bx0 + lane % Ly::LW, ly = by0 + lane / Ly::LW;
    uint32_t n_blended = 0, n_evaluated = 0;
    for (int64_t t = next_tile(a, -1, persistent, &work_slot); t < a.n_tiles;
         t = next_tile(a, t, persistent, &work_slot)) {
        const TileCtx c = tile_ctx(a, t, TILE);
        const uint2 rg = a.ranges[t];
        // T < 0 marks a pixel that has terminated (|T| is its final transmittance) or lies outside
        // the image; this keeps the per-pixel state in float registers.
        float T[PPT], C[PPT][3];
        uint32_t last[PPT];
        bool mine = false;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            T[j] = (c.x0 + lx < c.width && c.y0 + ly + LH * j < c.height) ? 1.0f : -1.0f;
            C[j][0] = C[j][1] = C[j][2] = 0.0f;
            last[j] = 0;
            mine |= T[j] > 0.0f;
        }
        const float px = lx + 0.5f;
        for (uint32_t base = rg.x; base < rg.y; base += batch) {
            // the workgroup stops once every pixel of the tile has terminated
            if (WAVES > 1 ? !__syncthreads_or(mine) : !__any(mine)) break;
            const int cnt = (int)min((uint32_t)batch, rg.y - base);
            for (int q = tid; q < cnt; q += NT) {
                const uint32_t g = a.vals[base + q];
                stage(a, g, (double)c.x0, (double)c.y0, &lds[q]);
                if (IMP) lds_id[q] = g;
            }
            __syncthreads();
            for (int jj = 0; jj < cnt; ++jj) {
                // the wave stops once all its pixels have terminated; checked every 4 Gaussians
                // (a terminated pixel has T < 0 and takes no further fragment in between)
                if ((jj & 3) == 0 && !__any(mine)) break;
                const float4 box = lds[jj].box;
                // wave-uniform: skip a Gaussian whose footprint box misses this wave's block
                if (!box_meets(box, bx0, bx0 + Ly::WW - 1, by0, by0 + Ly::WH - 1)) continue;
                const Staged s = lds[jj];
                const uint32_t pos = base + jj - rg.x;
                float alpha[PPT];
                bool pass[PPT];
                bool any_pass = false;
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    pass[j] = false;
                    alpha[j] = 0.0f;
                    // this wave's pixel rows of slot j; skip the slot when the footprint misses them
                    if (PPT > 1 && !box_meets(box, bx0, bx0 + Ly::WW - 1, by0 + LH * j, by0 + LH * j + LH - 1))
                        continue;
                    float w1, w2, G;
                    bool clamped;
                    pass[j] = frag(s, px, ly + LH * j + 0.5f, w1, w2, G, alpha[j], clamped) & (T[j] > 0.0f);
                    any_pass |= pass[j];
                    if (STATS) n_evaluated += T[j] > 0.0f;
                }
                if (!__any(any_pass)) continue;  // wave-uniform: none of this wave's pixels is hit
                float wsum = 0.0f;
                mine = false;
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    const float Tn = T[j] * (1.0f - alpha[j]);
                    const bool term = pass[j] & (Tn < kTMin);
                    const bool incl = pass[j] & !term;
                    const float w = incl ? alpha[j] * T[j] : 0.0f;
                    if (IMP) wsum += w;
                    C[j][0] = __fmaf_rn(w, s.p1.z, C[j][0]);
                    C[j][1] = __fmaf_rn(w, s.p1.w, C[j][1]);
                    C[j][2] = __fmaf_rn(w, s.b, C[j][2]);
                    T[j] = incl ? Tn : (term ? -T[j] : T[j]);
                    last[j] = incl ? pos + 1 : last[j];
                    mine |= T[j] > 0.0f;
                    if (STATS) n_blended += incl;
                }
                if (IMP) {
                    // importance score: blending weights of this record summed over the wave's pixels
#pragma unroll
                    for (int d = 32; d >= 1; d >>= 1) wsum += __shfl_xor(wsum, d);
                    if (lane == 0 && wsum != 0.0f)
                        unsafeAtomicAdd(a.importance + (lds_id[jj] - (int64_t)c.view * a.n), wsum);
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int x = c.x0 + lx, y = c.y0 + ly + LH * j;
            if (x >= c.width || y >= c.height) continue;
            const int64_t p = (int64_t)y * c.width + x;
            const int64_t plane = (int64_t)c.width * c.height;
            float* img = a.image + 3 * c.pix_off;
            const float Tf = fabsf(T[j]);
            img[p] = __fmaf_rn(Tf, c.bg[0], C[j][0]);
            img[plane + p] = __fmaf_rn(Tf, c.bg[1], C[j][1]);
            img[2 * plane + p] = __fmaf_rn(Tf, c.bg[2], C[j][2]);
            a.T_final[c.pix_off + p] = Tf;
            a.last[c.pix_off + p] = last[j];
        }
    }
    if (STATS) {
        unsigned long long nb = n_blended, ne = n_evaluated;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            nb += __shfl_xor(nb, d);
            ne += __shfl_xor(ne, d);
        }
        if (lane == 0) {
            atomicAdd(a.stats, nb);
            atomicAdd(a.stats + 1, ne);
        }
    }
}

// Cross-lane helpers on gfx950 VALU data paths (no LDS traffic). swap32(a, b): lanes 32-63 of a
// trade places with lanes 0-31 of b; swap16 does the same between odd and even 16-lane rows of each
// half. mirror16 / mirror8: the value of lane 15 - i (i - 8 ... ) within each 16- / 8-lane group.
__device__ __forceinline__ void swap32(float& a, float& b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap16(float& a, float& b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {  // lanes whose source lane is invalid read 0
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}
constexpr int kQuadXor1 = 0xb1, kQuadXor2 = 0x4e, kRowMirror = 0x140, kRowHalfMirror = 0x141;
constexpr int kRowBcast15 = 0x142;  // lane 15 of the previous 16-lane row (rows 1-3)
constexpr int kLaneSum8 = 63;       // the lane that ends with the wave total of v[8] in wave_sum9

// Sum over one 8-lane group (every lane of the group ends with the total).
__device__ __forceinline__ float sum8(float y) {
    y += dpp<kQuadXor1>(y);
    y += dpp<kQuadXor2>(y);
    y += dpp<kRowHalfMirror>(y);
    return y;
}

// Sum of v[0..8] over the wave: a transposed butterfly. After the swaps, lane group (b5 b4 b3) of
// the lane index holds partial sums of v[4 b5 + 2 b4 + b3] only; the last three steps finish
// them within each 8-lane group, so every lane of group m (lanes 8m..8m+7) holds the total of v[m].
// v[8] is summed within each 16-lane row, then across rows with the two row broadcasts, the last of
// which writes only lanes 60-63: on return lanes 8m (m < 8) hold the total of v[m] and lane
// kLaneSum8 (63) the total of v[8].
__device__ __forceinline__ float wave_sum9(const float v[9]) {
    const int lane = __lane_id();
    float w4[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {  // lanes < 32 gather v[i] pairs, lanes >= 32 v[i + 4] pairs
        float a = v[i], b = v[i + 4];
        swap32(a, b);
        w4[i] = a + b;
    }
    float w2[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {  // even rows keep w4[i], odd rows w4[i + 2]
        float a = w4[i], b = w4[i + 2];
        swap16(a, b);
        w2[i] = a + b;
    }
    const bool b3 = lane & 8;      // lanes 0-7 of a row pair with lanes 15..8 through the mirror
    const float y = (b3 ? w2[1] : w2[0]) + dpp<kRowMirror>(b3 ? w2[0] : w2[1]);
    float out = sum8(y);
    // (all rows take part in the first broadcast so it folds into one DPP add; only row 3's result,
    // which reads a valid lane, is used)
    float z = sum8(v[8]);
    z += dpp<kRowMirror>(z);   // row sums R0..R3 in every lane of their row
    z += dpp<kRowBcast15>(z);  // row 1: R0 + R1, row 3: R2 + R3
    // Lanes 60-63 (row mask 8: row 3; bank mask 8: its lanes 12-15) take R2 + R3 + lane 31's
    // R0 + R1 in place of the total of v[7], which lane 56 also holds; every other lane keeps out.
    // This masked DPP add has no builtin form (a masked DPP move keeps the old value in the move,
    // not in the sum), so it is written out, after the two wait states a DPP read of a VGPR that
    // the previous VALU instruction wrote needs.
    asm volatile("s_nop 1\n\tv_add_f32_dpp %0, %1, %1 row_bcast:31 row_mask:0x8 bank_mask:0x8"
                 : "+v"(out)
                 : "v"(z));
    return out;
}

// DET: instead of float atomics into the record's gradient, the tile's 9 sums for each list
// position go to that position's own slot a.grad_pair[pos] (written by exactly one workgroup), and
// a separate pass adds each record's slots in a fixed order: bit-reproducible gradients.
template <int TILE, int WAVES, bool DET>
__global__ __launch_bounds__(64 * WAVES) void k_blend_bwd(BlendArgs a, int batch, int persistent) {
    using Ly = Layout<TILE, WAVES>;
    constexpr int NT = 64 * WAVES, PPT = Ly::PPT, LH = Ly::LH;
    extern __shared__ Staged lds[];
    uint32_t* lds_id = reinterpret_cast<uint32_t*>(lds + batch);
    float* lds_part = reinterpret_cast<float*>(lds_id + batch);  // [batch][WAVES][9] (WAVES > 1)
    __shared__ uint32_t work_slot;
    __shared__ uint32_t red_slot[WAVES];
    const int tid = threadIdx.x, lane = __lane_id(), wv = tid / 64;
    const int bx0 = Ly::wx0(wv), by0 = Ly::wy0(wv);   // this wave's block
    const int lx = bx0 + lane % Ly::LW, ly = by0 + lane / Ly::LW;
    const float px = lx + 0.5f;
    for (int64_t t = next_tile(a, -1, persistent, &work_slot); t < a.n_tiles;
         t = next_tile(a, t, persistent, &work_slot)) {
        const TileCtx c = tile_ctx(a, t, TILE);
        const uint2 rg = a.ranges[t];
        const int64_t plane = (int64_t)c.width * c.height;
        float T[PPT], P[PPT], dl[PPT][3];  // P = S . dL/dC, as in the sub-tile backward
        uint32_t lst[PPT];
        uint32_t maxlast = 0;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int x = c.x0 + lx, y = c.y0 + ly + LH * j;
            const bool inside = x < c.width && y < c.height;
            const int64_t p = (int64_t)y * c.width + x;
            T[j] = inside ? a.T_final[c.pix_off + p] : 1.0f;
            lst[j] = inside ? a.last[c.pix_off + p] : 0u;
            const float* dimg = a.dl + 3 * c.pix_off;
            dl[j][0] = inside ? dimg[p] : 0.f;
            dl[j][1] = inside ? dimg[plane + p] : 0.f;
            dl[j][2] = inside ? dimg[2 * plane + p] : 0.f;
            P[j] = __fmaf_rn(c.bg[0], dl[j][0], __fmaf_rn(c.bg[1], dl[j][1], c.bg[2] * dl[j][2]));
            maxlast = max(maxlast, lst[j]);
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) maxlast = max(maxlast, (uint32_t)__shfl_xor((int)maxlast, d));
        const uint32_t wave_last = maxlast;
        if (WAVES > 1) {
            if (lane == 0) red_slot[wv] = maxlast;
            __syncthreads();
            for (int w = 0; w < WAVES; ++w) maxlast = max(maxlast, red_slot[w]);
            __syncthreads();
        }
        for (uint32_t end = rg.x + maxlast; end > rg.x;) {
            const uint32_t beg = end - rg.x > (uint32_t)batch ? end - batch : rg.x;
            const int cnt = (int)(end - beg);
            for (int q = tid; q < cnt; q += NT) {
                const uint32_t g = a.vals[end - 1 - q];
                stage(a, g, (double)c.x0, (double)c.y0, &lds[q]);
                lds_id[q] = g;
            }
            __syncthreads();
            for (int jj = 0; jj < cnt; ++jj) {
                const uint32_t pos = end - 1 - jj - rg.x;
                bool any_incl = false;
                float acc[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) acc[i] = 0.f;
                // wave-uniform: positions past every pixel's last, and Gaussians whose footprint
                // box misses this wave's block, are skipped
                if (pos < wave_last && box_meets(lds[jj].box, bx0, bx0 + Ly::WW - 1, by0, by0 + Ly::WH - 1)) {
                    const Staged s = lds[jj];
                    float alpha[PPT], G[PPT], w1s[PPT], w2s[PPT];
                    bool incl[PPT], clamped[PPT];
#pragma unroll
                    for (int j = 0; j < PPT; ++j) {
                        incl[j] = false;
                        alpha[j] = 0.0f; G[j] = 0.0f; w1s[j] = 0.0f; w2s[j] = 0.0f; clamped[j] = false;
                        if (PPT > 1 &&
                            !box_meets(s.box, bx0, bx0 + Ly::WW - 1, by0 + LH * j, by0 + LH * j + LH - 1))
                            continue;
                        incl[j] = frag(s, px, ly + LH * j + 0.5f, w1s[j], w2s[j], G[j], alpha[j], clamped[j]) &
                                  (pos < lst[j]);
                        any_incl |= incl[j];
                    }
                    any_incl = __any(any_incl);
                    if (any_incl) {
#pragma unroll
                        for (int j = 0; j < PPT; ++j) {
                            const float al = incl[j] ? alpha[j] : 0.0f;
                            const float Ti = T[j] * __builtin_amdgcn_rcpf(1.0f - al);
                            const float w = al * Ti;
                            const float dcs =
                                __fmaf_rn(s.p1.z, dl[j][0], __fmaf_rn(s.p1.w, dl[j][1], s.b * dl[j][2])) - P[j];
                            acc[6] = __fmaf_rn(w, dl[j][0], acc[6]);
                            acc[7] = __fmaf_rn(w, dl[j][1], acc[7]);
                            acc[8] = __fmaf_rn(w, dl[j][2], acc[8]);
                            const float dal = Ti * dcs;
                            P[j] = __fmaf_rn(al, dcs, P[j]);
                            T[j] = incl[j] ? Ti : T[j];
                            const bool live = incl[j] & !clamped[j];
                            // dL/do_eff of the fragment; its exponent gradient is o_eff times this
                            const float e = live ? G[j] * dal : 0.0f;
                            const float w1 = w1s[j], w2 = w2s[j];
                            acc[5] += e;
                            const float m1 = e * w1, m2 = e * w2;
                            acc[0] += m1;
                            acc[1] += m2;
                            acc[2] = __fmaf_rn(m1, w1, acc[2]);
                            acc[3] = __fmaf_rn(m1, w2, acc[3]);
                            acc[4] = __fmaf_rn(m2, w2, acc[4]);
                        }
                    }
                }
                if (WAVES == 1) {
                    if (!any_incl) continue;
                    const float tot = wave_sum9(acc);
                    if (DET) {
                        float* slot = a.grad_pair + 9 * (int64_t)(end - 1 - jj);
                        if ((lane & 7) == 0) slot[lane >> 3] = tot;
                        if (lane == kLaneSum8) slot[8] = tot;
                        continue;
                    }
                    // one 9-lane atomic: lanes 0, 8, .., 56 add sums 0..7, lane 63 adds sum 8
                    if ((lane & 7) == 0 || lane == kLaneSum8)
                        unsafeAtomicAdd(a.grad2d + grad2d_index(lds_id[jj], lane == kLaneSum8 ? 8 : lane >> 3), tot);
                } else {
                    // per-wave partial sums to LDS; summed across waves after the batch
                    float tot = 0.f;
                    if (any_incl) tot = wave_sum9(acc);
                    float* part = lds_part + ((int64_t)jj * WAVES + wv) * 9;
                    if ((lane & 7) == 0) part[lane >> 3] = tot;
                    if (lane == kLaneSum8) part[8] = tot;
                }
            }
            __syncthreads();
            if (WAVES > 1) {
                for (int i = tid; i < cnt * 9; i += NT) {
                    const int jj = i / 9, comp = i - jj * 9;
                    float sum = 0.f;
#pragma unroll
                    for (int w = 0; w < WAVES; ++w) sum += lds_part[((int64_t)jj * WAVES + w) * 9 + comp];
                    if (DET)
                        a.grad_pair[9 * (int64_t)(end - 1 - jj) + comp] = sum;
                    else if (sum != 0.f)
                        unsafeAtomicAdd(a.grad2d + grad2d_index(lds_id[jj], comp), sum);
                }
                __syncthreads();
            }
            end = beg;
        }
    }
}

// ------------------------------------------------------------- sub-tile kernels ----
// One wave64 per 8 x 8 sub-tile of a 16 x 16 or 32 x 32 tile: the tile's sorted list (and so the
// key table and its sort) stays at the tile's size, while blending runs at sub-tile size. The wave
// walks the list in chunks of 64 entries; each lane stages one entry and keeps it only when the
// tile key flags the sub-tile (the emission tested the entry's ellipse against it), or, without
// flags, when the entry's footprint box meets the sub-tile; the kept entries are packed in list
// order into the wave's own LDS (ballot prefix) and blended. Entries are staged relative to the
// sub-tile's corner, so each pixel's exponent factors stay within eight pixels of it. Sub-tiles of a tile never wait for each other: there
// is no workgroup barrier anywhere.

// LDS written by some lanes of a wave and read by others: order the wave's accesses.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Without the work queue, the forward's workgroup b runs item xcd_item(b): each XCD takes one
// contiguous eighth of the sub-tiles (with 8 views, one view each), so the records an XCD gathers
// stay in its own L2. The backward keeps identity order, which measured faster for it.
//
// With the work queue (persistent launch) the items are split into kSlices contiguous slices, one per
// XCD (the same eighths as above), with one counter each (queue[s * kQueueStride], one per 256 bytes).
// A wave pulls one item at a time from the slice of the XCD it runs on (the XCC_ID hardware register),
// so a tile's sub-tiles and its list stay in one L2. Once its slice is drained it reads all the
// counters at once (one lane each) and moves to the first slice with items left, its own XCD's first. Every pull advances a counter, so every item is handed out exactly once, and a wave
// ends when every counter has passed its slice's end. The register only steers locality: any value in
// it gives the same result. Measured on the 8-view 1080p workload (forward / backward blend): with the
// eight counters in one cache line, pulls serialised on it and the blends took 3.7 / 4.3 ms instead of
// 0.99 / 2.24 ms for one workgroup per item; a line per counter brings them to 1.35 / 2.48 ms. More
// slices per XCD (32, 64) lost L2 locality, and several items per pull lost balance (both slower).
// What remains is not the queue: issuing each next pull ahead of its item (its round trip overlapping
// the item's work) changed nothing, and a static assignment without atomics took as long (1.32 ms).
constexpr int kSlices = kXcds;
static_assert(kSlices % kXcds == 0 && kSlices <= 64 && kSlices * kQueueStride <= kQueueWords, "slice counters");

struct Pull {
    int slice = -1;  // the slice the wave pulls from (-1 before its first pull)
};

__device__ __forceinline__ void slice_of(int64_t n_items, int s, int64_t& base, int64_t& cnt) {
    const int64_t per = n_items / kSlices, rem = n_items % kSlices;
    base = s * per + (s < rem ? s : rem);
    cnt = per + (s < rem ? 1 : 0);
}

__device__ __forceinline__ int64_t next_item(const BlendArgs& a, int64_t prev, bool persistent, int64_t n_items,
                                             Pull& q, bool by_xcd) {
    if (!persistent) {
        if (prev >= 0) return n_items;
        return by_xcd ? xcd_item((int64_t)blockIdx.x, n_items) : (int64_t)blockIdx.x;
    }
    const int lane = __lane_id();
    constexpr int kPer = kSlices / kXcds;
    const int xcc = (int)(__builtin_amdgcn_s_getreg((3 << 11) | 20) & (kXcds - 1));  // XCC_ID
    if (q.slice < 0) q.slice = xcc * kPer + (int)((blockIdx.x / kXcds) % kPer);
    for (;;) {
        int64_t base, cnt;
        slice_of(n_items, q.slice, base, cnt);
        uint32_t j = 0;
        if (lane == 0) j = atomicAdd(a.queue + q.slice * kQueueStride, 1u);
        j = (uint32_t)__builtin_amdgcn_readfirstlane((int)j);
        if ((int64_t)j < cnt) return base + j;
        // this slice is drained: the slices with items left, one lane each, this XCD's first
        bool left = false;
        if (lane < kSlices) {
            int64_t b2, c2;
            slice_of(n_items, lane, b2, c2);
            left = (int64_t)__hip_atomic_load(a.queue + lane * kQueueStride, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT) < c2;
        }
        uint64_t m = __ballot(left);
        if (!m) return n_items;
        const int r = xcc * kPer;  // rotate so that this XCD's slices come first
        m = (m >> r) | (r ? m << (kSlices - r) : 0ull);
        m &= (kSlices == 64 ? ~0ull : ((1ull << kSlices) - 1ull));
        q.slice = (__builtin_ctzll(m) + r) % kSlices;
    }
}

// Rank of this lane among the lanes set in mask (lanes below it).
__device__ __forceinline__ int lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

struct SubCtx {
    TileCtx c;
    int sx, sy;       // sub-tile origin inside the tile
    int sidx;         // sub-tile index r S + c (the bit of its flag in the tile keys)
    int64_t t;
};

__device__ __forceinline__ SubCtx sub_ctx(const BlendArgs& a, int64_t w, int tile) {
    constexpr int SUB = 8;
    const int per_row = tile / SUB, nsub = per_row * per_row;
    SubCtx q;
    q.t = w / nsub;
    const int s = (int)(w - q.t * nsub);
    q.sidx = s;
    q.sx = (s % per_row) * SUB;
    q.sy = (s / per_row) * SUB;
    q.c = tile_ctx(a, q.t, tile);
    return q;
}

// FLAGS: the tile keys carry sub-tile flags (a.tkeys non-null), which decide which entries a
// sub-tile keeps; without them each entry's footprint box is tested instead. A template argument, so
// the flagged form (the default) carries no box code and no runtime test of the key pointer.
template <bool STATS, bool IMP, bool FLAGS>
__global__ __launch_bounds__(64) void k_blend_fwd_sub(BlendArgs a, int tile, int persistent) {
    constexpr int SUB = 8;
    __shared__ Kept lds[64];
    const int lane = __lane_id();
    const int64_t n_items = a.n_tiles * (int64_t)(tile / SUB) * (tile / SUB);
    uint32_t n_blended = 0, n_evaluated = 0;
    Pull pull;
    for (int64_t w = next_item(a, -1, persistent, n_items, pull, true); w < n_items;
         w = next_item(a, w, persistent, n_items, pull, true)) {
        const SubCtx q = sub_ctx(a, w, tile);
        const TileCtx& c = q.c;
        const int lx = q.sx + (lane & 7), ly = q.sy + (lane >> 3);
        const bool inside = c.x0 + lx < c.width && c.y0 + ly < c.height;
        if (!__any(inside)) continue;  // a sub-tile past the image edge has no pixel
        float T = inside ? 1.0f : -1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
        uint32_t last = 0;
        const uint2 rg = a.ranges[q.t];
        // pixel centre relative to the sub-tile, the frame the entries are staged in
        const float px = (lane & 7) + 0.5f, py = (lane >> 3) + 0.5f;
        const double fx0 = (double)(c.x0 + q.sx), fy0 = (double)(c.y0 + q.sy);
        // each chunk's tile keys and record ids are loaded one chunk ahead, while the previous
        // chunk's entries are blended
        uint32_t key_n = 0, id_n = 0;
        if (rg.x + lane < rg.y) {
            id_n = a.vals[rg.x + lane];
            key_n = FLAGS ? a.tkeys[rg.x + lane] : 0u;
        }
        for (uint32_t base = rg.x; base < rg.y; base += 64) {
            if (!__any(T > 0.0f)) break;
            const uint32_t idx = base + lane;
            const uint32_t key = key_n, gid = id_n;
            bool hit = false;
            Staged st;
            uint32_t g = 0;
            if (idx < rg.y) {
                // the key's sub-tile flags, when present, decide before the record is gathered
                g = gid;
                const bool flagged = !FLAGS || ((key >> (16 + q.sidx)) & 1u);
                if (flagged) {
                    stage(a, g, fx0, fy0, &st, !FLAGS);
                    // the flags already test the ellipse against the sub-tile; without them, its box
                    hit = FLAGS ? true : box_meets(st.box, 0, SUB - 1, 0, SUB - 1);
                }
            }
            const uint64_t m = __ballot(hit);
            const int nhit = __popcll(m);
            if (hit) {
                const int slot = lane_rank(m);
                lds[slot] = Kept{st.p0, st.p1, st.b, idx - rg.x + 1u, g};
            }
            if (idx + 64u < rg.y) {
                id_n = a.vals[idx + 64u];
                key_n = FLAGS ? a.tkeys[idx + 64u] : 0u;
            }
            wave_sync();
            for (int k0 = 0; k0 < nhit; k0 += 4) {
                // the wave stops once all its pixels have terminated; checked every 4 entries (a
                // terminated pixel has T < 0 and takes no further fragment in between)
                if (!__any(T > 0.0f)) break;
                const Kept* kp = kept_at(lds, k0);
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = k0 + kk;
                    if (k < nhit) {  // wave-uniform
                        const Kept s = kp[kk];
                        float w1, w2, G, alpha;
                        bool clamped;
                        // a live pixel has T >= kTMin, a terminated one (or one outside the image)
                        // T < 0; this compare, not shared with the termination test above, lets the
                        // wave vote below branch on the lane mask directly
                        const bool pass = frag(s, px, py, w1, w2, G, alpha, clamped) & (T >= kTMin);
                        if (STATS) n_evaluated += T > 0.0f;
                        if (__any(pass)) {
                            const float Tn = T * (1.0f - alpha);
                            const bool term = pass & (Tn < kTMin);
                            const bool incl = pass & !term;
                            const float wgt = incl ? alpha * T : 0.0f;
                            C0 = __fmaf_rn(wgt, s.p1.z, C0);
                            C1 = __fmaf_rn(wgt, s.p1.w, C1);
                            C2 = __fmaf_rn(wgt, s.b, C2);
                            T = incl ? Tn : (term ? -T : T);
                            last = incl ? s.pos1 : last;
                            if (STATS) n_blended += incl;
                            if (IMP) {
                                float wsum = wgt;
#pragma unroll
                                for (int d = 32; d >= 1; d >>= 1) wsum += __shfl_xor(wsum, d);
                                if (lane == 0 && wsum != 0.0f)
                                    unsafeAtomicAdd(a.importance + ((int64_t)s.slot - (int64_t)c.view * a.n), wsum);
                            }
                        }
                    }
                }
            }
            wave_sync();
        }
        if (inside) {
            const int x = c.x0 + lx, y = c.y0 + ly;
            const int64_t p = (int64_t)y * c.width + x;
            const int64_t plane = (int64_t)c.width * c.height;
            float* img = a.image + 3 * c.pix_off;
            const float Tf = fabsf(T);
            img[p] = __fmaf_rn(Tf, c.bg[0], C0);
            img[plane + p] = __fmaf_rn(Tf, c.bg[1], C1);
            img[2 * plane + p] = __fmaf_rn(Tf, c.bg[2], C2);
            a.T_final[c.pix_off + p] = Tf;
            a.last[c.pix_off + p] = last;
        }
    }
    if (STATS) {
        unsigned long long nb = n_blended, ne = n_evaluated;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            nb += __shfl_xor(nb, d);
            ne += __shfl_xor(ne, d);
        }
        if (lane == 0) {
            atomicAdd(a.stats, nb);
            atomicAdd(a.stats + 1, ne);
        }
    }
}

template <bool FLAGS>  // as in k_blend_fwd_sub
__global__ __launch_bounds__(64) void k_blend_bwd_sub(BlendArgs a, int tile, int persistent) {
    constexpr int SUB = 8;
    __shared__ Kept lds[64];
    const int lane = __lane_id();
    // the 9 sums leave through one 9-lane atomic: lanes 0, 8, .., 56 hold sums 0..7, lane 63 sum 8
    const bool adds = (lane & 7) == 0 || lane == kLaneSum8;
    const int comp = lane == kLaneSum8 ? 8 : lane >> 3;
    const int64_t n_items = a.n_tiles * (int64_t)(tile / SUB) * (tile / SUB);
    Pull pull;
    for (int64_t w = next_item(a, -1, persistent, n_items, pull, false); w < n_items;
         w = next_item(a, w, persistent, n_items, pull, false)) {
        const SubCtx q = sub_ctx(a, w, tile);
        const TileCtx& c = q.c;
        const int lx = q.sx + (lane & 7), ly = q.sy + (lane >> 3);
        const int x = c.x0 + lx, y = c.y0 + ly;
        const bool inside = x < c.width && y < c.height;
        const int64_t plane = (int64_t)c.width * c.height;
        const int64_t p = (int64_t)y * c.width + x;
        float T = 1.0f, dl0 = 0.f, dl1 = 0.f, dl2 = 0.f;
        uint32_t lst = 0;
        if (inside) {
            const float* dimg = a.dl + 3 * c.pix_off;
            T = a.T_final[c.pix_off + p];
            lst = a.last[c.pix_off + p];
            dl0 = dimg[p];
            dl1 = dimg[plane + p];
            dl2 = dimg[2 * plane + p];
        }
        // the colour accumulated behind the current fragment (background included) enters the
        // gradient only through its dot product with the pixel's colour gradient, so the replay
        // carries that one scalar: P = S . dL/dC, updated as S is (S += alpha (c - S))
        float P = __fmaf_rn(c.bg[0], dl0, __fmaf_rn(c.bg[1], dl1, c.bg[2] * dl2));
        uint32_t wave_last = lst;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) wave_last = max(wave_last, (uint32_t)__shfl_xor((int)wave_last, d));
        if (wave_last == 0) continue;  // wave-uniform: no pixel of the sub-tile blended anything
        const uint2 rg = a.ranges[q.t];
        const float px = (lane & 7) + 0.5f, py = (lane >> 3) + 0.5f;  // relative to the sub-tile
        const double fx0 = (double)(c.x0 + q.sx), fy0 = (double)(c.y0 + q.sy);
        // tile keys and record ids loaded one chunk ahead, as in the forward
        uint32_t key_n = 0, id_n = 0;
        if ((uint32_t)lane < wave_last) {
            const uint32_t i0 = rg.x + wave_last - 1u - (uint32_t)lane;
            id_n = a.vals[i0];
            key_n = FLAGS ? a.tkeys[i0] : 0u;
        }
        for (uint32_t end = rg.x + wave_last; end > rg.x;) {
            const uint32_t beg = end - rg.x > 64u ? end - 64u : rg.x;
            const uint32_t cnt = end - beg;
            const uint32_t idx = end - 1u - (uint32_t)lane;  // descending list positions
            const uint32_t key = key_n, gid = id_n;
            bool hit = false;
            Staged st;
            uint32_t g = 0;
            if ((uint32_t)lane < cnt) {
                g = gid;
                const bool flagged = !FLAGS || ((key >> (16 + q.sidx)) & 1u);
                if (flagged) {
                    stage(a, g, fx0, fy0, &st, !FLAGS);
                    // the flags already test the ellipse against the sub-tile; without them, its box
                    hit = FLAGS ? true : box_meets(st.box, 0, SUB - 1, 0, SUB - 1);
                }
            }
            const uint64_t m = __ballot(hit);
            const int nhit = __popcll(m);
            if (hit) {
                const int slot = lane_rank(m);
                lds[slot] = Kept{st.p0, st.p1, st.b, idx - rg.x + 1u, (uint64_t)grad2d_index(g, 0)};
            }
            if ((uint32_t)lane < beg - rg.x) {  // the next chunk: positions beg - 1 - lane downwards
                id_n = a.vals[beg - 1u - (uint32_t)lane];
                key_n = FLAGS ? a.tkeys[beg - 1u - (uint32_t)lane] : 0u;
            }
            wave_sync();
            for (int k = 0; k < nhit; ++k) {
                const Kept s = *kept_at(lds, k);
                float alpha, G, w1, w2;
                bool clamped;
                const bool incl = frag(s, px, py, w1, w2, G, alpha, clamped) & (s.pos1 <= lst);
                if (!__any(incl)) continue;
                float acc[9];
                // a lane the entry does not include takes alpha = 0: its T is then multiplied by the
                // reciprocal of 1.0, which is exactly 1.0, and its P by nothing, so it needs no select
                const float al = incl ? alpha : 0.0f;
                const float Ti = T * __builtin_amdgcn_rcpf(1.0f - al);
                const float wgt = al * Ti;
                // (c - S) . dL/dC, from c . dL/dC and the carried P
                const float dcs = __fmaf_rn(s.p1.z, dl0, __fmaf_rn(s.p1.w, dl1, __fmaf_rn(s.b, dl2, -P)));
                acc[6] = wgt * dl0;
                acc[7] = wgt * dl1;
                acc[8] = wgt * dl2;
                const float dal = Ti * dcs;
                P = __fmaf_rn(al, dcs, P);
                T = Ti;
                const bool live = incl & !clamped;
                acc[5] = live ? G * dal : 0.0f;  // dL/do_eff; the exponent gradient is o_eff times this
                acc[0] = acc[5] * w1;
                acc[1] = acc[5] * w2;
                acc[2] = acc[0] * w1;
                acc[3] = acc[0] * w2;
                acc[4] = acc[1] * w2;
                // (the sums' last add is a volatile statement, so their DPP adds stay in front of the
                // branch: sunk into it, where only the adding lanes run, each would split into a DPP
                // move and a separate add)
                const float val = wave_sum9(acc);
                if (adds) unsafeAtomicAdd(a.grad2d + (s.slot + comp), val);
            }
            wave_sync();
            end = beg;
        }
    }
}

constexpr int64_t kPersistentGroups = 256 * 24;  // resident workgroups pulling tiles in persistent mode

template <int TILE, int WAVES>
hipError_t launch_fwd_t(const BlendArgs& a, int batch, bool persistent, hipStream_t stream) {
    const size_t lds = (size_t)batch * (sizeof(Staged) + (a.importance ? sizeof(uint32_t) : 0));
    const int64_t groups = persistent ? kPersistentGroups / WAVES : a.n_tiles;
    const unsigned grid = (unsigned)(groups < a.n_tiles ? groups : a.n_tiles);
    const dim3 block(64 * WAVES);
    if (a.importance)
        hipLaunchKernelGGL((k_blend_fwd<TILE, WAVES, false, true>), dim3(grid), block, lds, stream, a, batch,
                           (int)persistent);
    else if (a.stats)
        hipLaunchKernelGGL((k_blend_fwd<TILE, WAVES, true, false>), dim3(grid), block, lds, stream, a, batch,
                           (int)persistent);
    else
        hipLaunchKernelGGL((k_blend_fwd<TILE, WAVES, false, false>), dim3(grid), block, lds, stream, a, batch,
                           (int)persistent);
    return hipGetLastError();
}

template <int TILE, int WAVES>
hipError_t launch_bwd_t(const BlendArgs& a, int batch, bool persistent, hipStream_t stream) {
    size_t lds = (size_t)batch * (sizeof(Staged) + sizeof(uint32_t));
    if (WAVES > 1) lds += (size_t)batch * WAVES * 9 * sizeof(float);
    const int64_t groups = persistent ? kPersistentGroups / WAVES : a.n_tiles;
    const unsigned grid = (unsigned)(groups < a.n_tiles ? groups : a.n_tiles);
    if (a.grad_pair)
        hipLaunchKernelGGL((k_blend_bwd<TILE, WAVES, true>), dim3(grid), dim3(64 * WAVES), lds, stream, a, batch,
                           (int)persistent);
    else
        hipLaunchKernelGGL((k_blend_bwd<TILE, WAVES, false>), dim3(grid), dim3(64 * WAVES), lds, stream, a, batch,
                           (int)persistent);
    return hipGetLastError();
}

// The sub-tile flags' presence is a template argument, so the flagged form (the default) carries no
// footprint-box code.
template <bool STATS, bool IMP>
void launch_fwd_sub_t(const BlendArgs& a, unsigned grid, int tile, bool persistent, hipStream_t stream) {
    if (a.tkeys)
        hipLaunchKernelGGL((k_blend_fwd_sub<STATS, IMP, true>), dim3(grid), dim3(64), 0, stream, a, tile, (int)persistent);
    else
        hipLaunchKernelGGL((k_blend_fwd_sub<STATS, IMP, false>), dim3(grid), dim3(64), 0, stream, a, tile,
                           (int)persistent);
}

hipError_t launch_fwd_sub(const BlendArgs& a, int tile, bool persistent, hipStream_t stream) {
    const int64_t items = a.n_tiles * (int64_t)(tile / 8) * (tile / 8);
    const int64_t groups = persistent ? kPersistentGroups : items;
    const unsigned grid = (unsigned)(groups < items ? groups : items);
    if (a.importance)
        launch_fwd_sub_t<false, true>(a, grid, tile, persistent, stream);
    else if (a.stats)
        launch_fwd_sub_t<true, false>(a, grid, tile, persistent, stream);
    else
        launch_fwd_sub_t<false, false>(a, grid, tile, persistent, stream);
    return hipGetLastError();
}

hipError_t launch_bwd_sub(const BlendArgs& a, int tile, bool persistent, hipStream_t stream) {
    const int64_t items = a.n_tiles * (int64_t)(tile / 8) * (tile / 8);
    const int64_t groups = persistent ? kPersistentGroups : items;
    const unsigned grid = (unsigned)(groups < items ? groups : items);
    if (a.tkeys)
        hipLaunchKernelGGL((k_blend_bwd_sub<true>), dim3(grid), dim3(64), 0, stream, a, tile, (int)persistent);
    else
        hipLaunchKernelGGL((k_blend_bwd_sub<false>), dim3(grid), dim3(64), 0, stream, a, tile, (int)persistent);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_blend_fwd(const BlendArgs& a, int tile, int waves, int batch, bool persistent, hipStream_t stream,
                            int subtile) {
    if (a.n_tiles <= 0) return hipSuccess;
    if (subtile == 8 && tile > 8) return launch_fwd_sub(a, tile, persistent, stream);
    if (tile == 8 && waves == 1) return launch_fwd_t<8, 1>(a, batch, persistent, stream);
    if (tile == 16 && waves == 1) return launch_fwd_t<16, 1>(a, batch, persistent, stream);
    if (tile == 16 && waves == 2) return launch_fwd_t<16, 2>(a, batch, persistent, stream);
    if (tile == 16 && waves == 4) return launch_fwd_t<16, 4>(a, batch, persistent, stream);
    if (tile == 32 && waves == 1) return launch_fwd_t<32, 1>(a, batch, persistent, stream);
    if (tile == 32 && waves == 2) return launch_fwd_t<32, 2>(a, batch, persistent, stream);
    if (tile == 32 && waves == 4) return launch_fwd_t<32, 4>(a, batch, persistent, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_blend_bwd(const BlendArgs& a, int tile, int waves, int batch, bool persistent, hipStream_t stream,
                            int subtile) {
    if (a.n_tiles <= 0) return hipSuccess;
    if (subtile == 8 && tile > 8 && !a.grad_pair) return launch_bwd_sub(a, tile, persistent, stream);
    if (tile == 8 && waves == 1) return launch_bwd_t<8, 1>(a, batch, persistent, stream);
    if (tile == 16 && waves == 1) return launch_bwd_t<16, 1>(a, batch, persistent, stream);
    if (tile == 16 && waves == 2) return launch_bwd_t<16, 2>(a, batch, persistent, stream);
    if (tile == 16 && waves == 4) return launch_bwd_t<16, 4>(a, batch, persistent, stream);
    if (tile == 32 && waves == 1) return launch_bwd_t<32, 1>(a, batch, persistent, stream);
    if (tile == 32 && waves == 2) return launch_bwd_t<32, 2>(a, batch, persistent, stream);
    if (tile == 32 && waves == 4) return launch_bwd_t<32, 4>(a, batch, persistent, stream);
    return hipErrorInvalidValue;
}

}  // namespace megs
