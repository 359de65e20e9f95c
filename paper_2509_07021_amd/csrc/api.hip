// api.hip -- C ABI of libmegs: argument checks, working-memory layout, stream orchestration of
// the forward and backward passes, hipGraph capture of the batched form, and the autotuner.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "megs_internal.hpp"

using namespace megs;

// Working memory of megs_render_forward_noalloc: one array per device in the library's code object, so
// that a forward can run where the caller cannot allocate. In host code the name `scratch` denotes a
// host-side stand-in, not device memory: host code takes the array's device address once per device
// (hipGetSymbolAddress, below) and uses only that address.
static __device__ __align__(256) unsigned char scratch[MEGS_NOALLOC_SCRATCH_BYTES];

namespace {

struct ProfileRec {
    int stage;
    hipEvent_t start, end;
};
struct Profiler {
    bool on = false;
    std::vector<ProfileRec> recs;
};
thread_local Profiler g_prof;

}  // namespace

namespace megs {

// Every stage's enqueue is also a named ROCTX range ("megs:project", ...), so a trace taken with
// rocprofv3 --marker-trace attributes each kernel to its stage (a no-op without a profiler).
const char* const kStageRange[MEGS_STAGE_COUNT] = {"megs:project", "megs:depth_sort", "megs:scan", "megs:emit",
                                                   "megs:pair_sort", "megs:ranges", "megs:blend_fwd",
                                                   "megs:blend_bwd", "megs:project_bwd"};

StageTimer::StageTimer(int st, hipStream_t s) : stage(st), stream(s), start(nullptr) {
    roctxRangePushA(kStageRange[st]);
    if (!g_prof.on) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    if (hipEventRecord(e, s) != hipSuccess) { (void)hipEventDestroy(e); return; }
    start = e;
}

StageTimer::~StageTimer() {
    roctxRangePop();
    if (!start) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    if (hipEventRecord(e, stream) != hipSuccess) { (void)hipEventDestroy(e); return; }
    g_prof.recs.push_back({stage, static_cast<hipEvent_t>(start), e});
}

}  // namespace megs

namespace {

thread_local char g_err[512] = "";

megs_status fail(megs_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

#define HIP_TRY(call)                                                                                     \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess) return fail(MEGS_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

constexpr int kViewChunk = 8;
struct ViewChunk {
    ViewInfo v[kViewChunk];
    int count;
};

__global__ void k_set_views(ViewInfo* dst, ViewChunk c) {
    if ((int)threadIdx.x < c.count) dst[threadIdx.x] = c.v[threadIdx.x];
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// The allocation callback's memory must be 256-byte aligned (the carved buffers inherit the
// alignment, and the kernels read records and index arrays with 16-byte vector accesses): NULL or
// a misaligned pointer is an allocation error, reported before anything is launched.
bool bad_alloc(const void* p) { return !p || (reinterpret_cast<uintptr_t>(p) & 255u) != 0; }

int waves_of(const megs_config* cfg) { return cfg->waves ? cfg->waves : (cfg->tile == 8 ? 1 : 4); }

// Bump allocator over one caller-provided block.
struct Carver {
    char* base;
    size_t off;
    template <typename T>
    T* take(int64_t count) {
        T* p = reinterpret_cast<T*>(base + off);
        off += align256((size_t)(count > 0 ? count : 1) * sizeof(T));
        return p;
    }
};

struct Layout {
    int nv;
    int64_t n, nr, n_tiles, n_pixels;
    int tile, tile_bits;
    bool planes;  // MEGS_FLAG_RECORD_PLANES
    std::vector<ViewInfo> views;
};

bool valid_dtype(int32_t d) { return d == MEGS_F32 || d == MEGS_F16 || d == MEGS_BF16; }

// Sub-tile flags in the tile keys: sub-tile blending with the two-stage sort and tile ids that
// leave the upper 16 bits of the 32-bit key free.
bool sub_masks(const megs_config* cfg, const Layout& L) {
    return cfg->subtile == 8 && cfg->tile > 8 && !(cfg->flags & MEGS_FLAG_ONE_STAGE_SORT) && L.n_tiles <= 65536;
}

// True when the scene has lobe planes to read (dense with k > 0, or compressed rows with lobes).
bool has_lobes(const megs_scene* sc) { return sc->k > 0 && (sc->lobe_off ? sc->n_lobes > 0 : true); }

megs_status check_scene(const megs_scene* sc) {
    if (!sc) return fail(MEGS_ERR_ARG, "null scene");
    if (sc->n < 0) return fail(MEGS_ERR_ARG, "n = %lld < 0", (long long)sc->n);
    if (sc->n >= (1ll << 31)) return fail(MEGS_ERR_ARG, "n must be < 2^31");
    if (sc->k < 0 || sc->k > MEGS_MAX_LOBES) return fail(MEGS_ERR_ARG, "k = %d outside [0, %d]", sc->k, MEGS_MAX_LOBES);
    if (!valid_dtype(sc->dt_geom) || !valid_dtype(sc->dt_color) || !valid_dtype(sc->dt_amp))
        return fail(MEGS_ERR_ARG, "unknown storage dtype");
    if (sc->lobe_off) {
        if (sc->n_lobes < 0 || sc->n_lobes >= (1ll << 31))
            return fail(MEGS_ERR_ARG, "n_lobes = %lld outside [0, 2^31)", (long long)sc->n_lobes);
        if (sc->n_lobes > sc->n * (int64_t)sc->k)
            return fail(MEGS_ERR_ARG, "n_lobes = %lld exceeds n * k", (long long)sc->n_lobes);
    } else if (sc->n_lobes != 0) {
        return fail(MEGS_ERR_ARG, "n_lobes must be 0 for the dense lobe layout");
    }
    if (sc->sh) {
        if (sc->sh_degree < 0 || sc->sh_degree > 3) return fail(MEGS_ERR_ARG, "sh_degree = %d outside [0, 3]", sc->sh_degree);
        if (sc->k != 0 || sc->lobe_off) return fail(MEGS_ERR_ARG, "a spherical-harmonic scene has no SG lobes (k = 0)");
    }
    if (sc->n > 0) {
        if (!sc->pos || !sc->logscale || !sc->quat || !sc->op_logit || (!sc->base && !sc->sh))
            return fail(MEGS_ERR_ARG, "null geometry or base plane");
        if (has_lobes(sc) && (!sc->axis || !sc->sharp || !sc->amp)) return fail(MEGS_ERR_ARG, "null lobe plane");
    }
    return MEGS_OK;
}

megs_status check_args(const megs_scene* sc, const megs_camera* cams, int32_t nv, const megs_config* cfg) {
    if (!sc || !cams || !cfg) return fail(MEGS_ERR_ARG, "null scene, camera or config");
    megs_status st = check_scene(sc);
    if (st != MEGS_OK) return st;
    if (nv < 1 || nv > MEGS_MAX_VIEWS) return fail(MEGS_ERR_ARG, "n_views = %d outside [1, %d]", nv, MEGS_MAX_VIEWS);
    if (sc->n * (int64_t)nv >= (1ll << 31)) return fail(MEGS_ERR_ARG, "n * n_views must be < 2^31");
    if (cfg->tile != 8 && cfg->tile != 16 && cfg->tile != 32) return fail(MEGS_ERR_ARG, "tile = %d not in {8, 16, 32}", cfg->tile);
    if (cfg->batch != 32 && cfg->batch != 64 && cfg->batch != 128 && cfg->batch != 256)
        return fail(MEGS_ERR_ARG, "batch = %d not in {32, 64, 128, 256}", cfg->batch);
    if (cfg->pair_capacity < 0 || cfg->pair_capacity >= (1ll << 31)) return fail(MEGS_ERR_ARG, "pair_capacity out of range");
    if (cfg->waves != 0 && cfg->waves != 1 && cfg->waves != 2 && cfg->waves != 4)
        return fail(MEGS_ERR_ARG, "waves = %d not in {0, 1, 2, 4}", cfg->waves);
    if (cfg->tile == 8 && cfg->waves > 1) return fail(MEGS_ERR_ARG, "8x8 tiles take one wave");
    if (cfg->subtile != 0 && cfg->subtile != 8) return fail(MEGS_ERR_ARG, "subtile = %d not in {0, 8}", cfg->subtile);
    if (cfg->subtile == 8 && cfg->tile == 8) return fail(MEGS_ERR_ARG, "subtile 8 needs 16x16 or 32x32 tiles");
    if (cfg->flags & ~(uint32_t)(MEGS_FLAG_ONE_STAGE_SORT | MEGS_FLAG_PERSISTENT | MEGS_FLAG_STATS |
                                 MEGS_FLAG_DETERMINISTIC | MEGS_FLAG_RECORD_PLANES))
        return fail(MEGS_ERR_ARG, "unknown flags 0x%x", cfg->flags);
    for (int v = 0; v < nv; ++v) {
        const megs_camera& c = cams[v];
        if (c.width <= 0 || c.height <= 0 || c.width > 16384 || c.height > 16384)
            return fail(MEGS_ERR_ARG, "view %d: image size %dx%d out of range", v, c.width, c.height);
        if (!(c.fx > 0) || !(c.fy > 0) || !(c.znear > 0)) return fail(MEGS_ERR_ARG, "view %d: fx, fy, znear must be > 0", v);
    }
    return MEGS_OK;
}

Layout make_layout(const megs_scene* sc, const megs_camera* cams, int nv, const megs_config* cfg) {
    const int tile = cfg->tile;
    Layout L;
    L.planes = cfg->flags & MEGS_FLAG_RECORD_PLANES;
    L.nv = nv;
    L.n = sc->n;
    L.nr = sc->n * nv;
    L.tile = tile;
    L.views.resize(nv);
    int64_t toff = 0, poff = 0;
    for (int v = 0; v < nv; ++v) {
        const megs_camera& c = cams[v];
        ViewInfo& w = L.views[v];
        memcpy(w.R, c.R, sizeof(w.R));
        memcpy(w.t, c.t, sizeof(w.t));
        w.fx = c.fx; w.fy = c.fy; w.cx = c.cx; w.cy = c.cy; w.znear = c.znear;
        memcpy(w.bg, c.bg, sizeof(w.bg));
        for (int a = 0; a < 3; ++a)
            w.campos[a] = (float)-((double)c.R[a] * c.t[0] + (double)c.R[3 + a] * c.t[1] + (double)c.R[6 + a] * c.t[2]);
        w.limx = (float)(1.3 * (0.5 * c.width) / (double)c.fx);
        w.limy = (float)(1.3 * (0.5 * c.height) / (double)c.fy);
        w.width = c.width; w.height = c.height;
        w.tiles_x = (c.width + tile - 1) / tile;
        w.tiles_y = (c.height + tile - 1) / tile;
        w.tile_off = toff;
        w.pix_off = poff;
        toff += (int64_t)w.tiles_x * w.tiles_y;
        poff += (int64_t)c.width * c.height;
    }
    L.n_tiles = toff;
    L.n_pixels = poff;
    int b = 1;
    while ((1ll << b) < L.n_tiles) ++b;
    L.tile_bits = b;
    return L;
}

SceneDev scene_dev(const megs_scene* sc, int32_t* status) {
    SceneDev d;
    d.n = sc->n; d.k = sc->k;
    d.dt_geom = sc->dt_geom; d.dt_color = sc->dt_color; d.dt_amp = sc->dt_amp;
    d.pos = sc->pos; d.logscale = sc->logscale; d.quat = sc->quat; d.op_logit = sc->op_logit;
    d.pmask_logit = sc->pmask_logit; d.base = sc->base; d.axis = sc->axis; d.sharp = sc->sharp; d.amp = sc->amp;
    d.lmask_logit = sc->lmask_logit;
    // a compressed-row scene without lobes reads no lobe plane and takes the dense k = 0 path
    d.lobe_off = has_lobes(sc) ? sc->lobe_off : nullptr;
    if (!has_lobes(sc)) d.k = 0;
    d.n_lobes = sc->n_lobes;
    d.status = status;
    d.sh = sc->sh;
    d.sh_degree = sc->sh_degree;
    return d;
}

// Device pointers of one forward. Its memory is one block: the part that lives as long as the state
// (views, records, per-tile ranges, per-pixel state, counters) and then the work space, which holds
// the depth sort, the scan and the key emission's per-record planes, is free once the pairs are
// emitted, and is then taken, when large enough, by the pair sort's alternate buffers and afterwards
// by the backward's scratch.
struct Frame {
    ViewInfo* views;
    Records rec;
    uint32_t *dkey_alt, *order, *order_alt, *offs;
    void *scan_scratch, *rs_scratch;
    uint32_t* counters;  // [0] pairs counted, [1] pairs used, [2] record count
    int32_t* status;     // [0] pairs counted, [1] overflow, [4..7] two uint64 fragment counters
    uint2* ranges;
    float* T_final;
    uint32_t* last;
    uint32_t* queue;     // the forward's work counters (persistent launch): [0] per-tile, [0..7] sub-tile
    char* work;          // the work space and its size
    size_t work_bytes;
};

size_t nr1(const Layout& L) { return (size_t)(L.nr ? L.nr : 1); }

// The part of the frame that lives as long as the state.
size_t frame_main_bytes(const Layout& L) {
    size_t b = 0;
    b += align256(sizeof(ViewInfo) * L.nv);
    b += align256(sizeof(PackedRec) * nr1(L));
    if (L.planes) {
        b += align256(sizeof(double2) * nr1(L));
        b += 2 * align256(sizeof(float4) * nr1(L));
        b += 3 * align256(sizeof(uint32_t) * nr1(L));
        b += align256(sizeof(double4) * nr1(L));
    }
    b += align256(sizeof(uint32_t) * 8) + align256(sizeof(int32_t) * 8);
    b += align256(sizeof(uint2) * L.n_tiles);
    b += 2 * align256(sizeof(float) * L.n_pixels);
    b += align256(sizeof(uint32_t) * kQueueWords);
    return b;
}

// What the forward itself needs of the work space: tile count, depth keys and order (each
// double-buffered), offsets, scan and sort scratch.
size_t work_fwd_bytes(const Layout& L) {
    return 6 * align256(sizeof(uint32_t) * nr1(L)) + align256(scan_scratch_bytes(L.nr)) +
           align256(radix_scratch_bytes(L.nr));
}

// The backward's scratch: the per-record sums of the blend backward [NR][9] (grad2d_index), the
// persistent launch's work counters, and in deterministic mode the per-pair slots [P][9].
size_t backward_bytes(const Layout& L, const megs_config* cfg, int64_t cap) {
    size_t b = align256(sizeof(float) * 9 * nr1(L)) + align256(sizeof(uint32_t) * kQueueWords);
    if (cfg->flags & MEGS_FLAG_DETERMINISTIC) b += align256(sizeof(float) * 9 * (cap > 0 ? cap : 1));
    return b;
}

// The pair sort's alternate keys and values and its scratch.
size_t pairs_alt_bytes(int64_t cap, bool one_stage) {
    const int64_t c = cap > 0 ? cap : 1;
    return align256(sizeof(uint32_t) * c) + align256((one_stage ? sizeof(uint64_t) : sizeof(uint32_t)) * c) +
           align256(radix_scratch_bytes(c));
}

// The work space is free for other use after the key emission unless the deterministic mode keeps
// its order and offsets for the backward. The pair sort's alternate buffers may go there only when
// the sort takes an even number of passes, so that the sorted pairs end in the pair block.
bool work_reusable(const megs_config* cfg) { return !(cfg->flags & MEGS_FLAG_DETERMINISTIC); }

bool alt_in_work(const Layout& L, const megs_config* cfg, int64_t cap, size_t work_bytes) {
    if (!work_reusable(cfg)) return false;
    const bool one_stage = cfg->flags & MEGS_FLAG_ONE_STAGE_SORT;
    if (radix_passes(0, one_stage ? 32 + L.tile_bits : L.tile_bits) % 2) return false;
    return pairs_alt_bytes(cap, one_stage) <= work_bytes;
}

// Size of the work space: the forward's own needs, and, where the frame is reusable, room for the
// backward's scratch (when one may follow) and for the pair sort's alternate buffers (when the pair
// capacity is known here: cap > 0).
size_t work_bytes(const Layout& L, const megs_config* cfg, int64_t cap, bool backward) {
    size_t w = work_fwd_bytes(L);
    if (!work_reusable(cfg)) return w;
    if (backward) w = std::max(w, backward_bytes(L, cfg, cap));
    const bool one_stage = cfg->flags & MEGS_FLAG_ONE_STAGE_SORT;
    if (cap > 0 && alt_in_work(L, cfg, cap, (size_t)-1)) w = std::max(w, pairs_alt_bytes(cap, one_stage));
    return w;
}

size_t frame_bytes(const Layout& L, size_t work) { return frame_main_bytes(L) + align256(work) + 256; }

Frame carve_frame(void* mem, const Layout& L, size_t work) {
    Carver c{static_cast<char*>(mem), 0};
    Frame f;
    f.views = c.take<ViewInfo>(L.nv);
    f.rec.packed = c.take<PackedRec>(L.nr);
    if (L.planes) {
        f.rec.mean = c.take<double2>(L.nr);
        f.rec.conic_o = c.take<float4>(L.nr);
        f.rec.rgbd = c.take<float4>(L.nr);
        f.rec.radius = c.take<int32_t>(L.nr);
        f.rec.cutoff = c.take<float>(L.nr);
        f.rec.chol = c.take<double4>(L.nr);
        f.rec.ntiles_plane = c.take<uint32_t>(L.nr);
    } else {
        f.rec.mean = nullptr;
        f.rec.conic_o = f.rec.rgbd = nullptr;
        f.rec.radius = nullptr;
        f.rec.cutoff = nullptr;
        f.rec.chol = nullptr;
        f.rec.ntiles_plane = nullptr;
    }
    f.counters = c.take<uint32_t>(8);
    f.status = c.take<int32_t>(8);
    f.ranges = c.take<uint2>(L.n_tiles);
    f.T_final = c.take<float>(L.n_pixels);
    f.last = c.take<uint32_t>(L.n_pixels);
    f.queue = c.take<uint32_t>(kQueueWords);
    // the work space
    f.work = c.take<char>((int64_t)align256(work));
    f.work_bytes = align256(work);
    Carver w{f.work, 0};
    f.rec.ntiles = w.take<uint32_t>(L.nr);
    f.rec.dkey = w.take<uint32_t>(L.nr);
    f.rec.order0 = nullptr;
    f.rec.order_idb = 0;
    f.dkey_alt = w.take<uint32_t>(L.nr);
    f.order = w.take<uint32_t>(L.nr);
    f.order_alt = w.take<uint32_t>(L.nr);
    f.offs = w.take<uint32_t>(L.nr);
    f.scan_scratch = w.take<char>((int64_t)scan_scratch_bytes(L.nr));
    f.rs_scratch = w.take<char>((int64_t)radix_scratch_bytes(L.nr));
    return f;
}

struct Pairs {
    int64_t capacity;
    uint32_t *tkeys, *tkeys_alt, *vals, *vals_alt;
    uint64_t *k64, *k64_alt;
    uint32_t *rec_emit, *inv;  // deterministic mode: record per emission position, sorted position per emission
    void* rs_scratch;
    bool alt_in_work;  // the alternate buffers and scratch are in the frame's work space
};

// The pair block: keys and values, and, unless they go to the frame's work space, the sort's
// alternate buffers and scratch; deterministic mode adds two permutations.
size_t pairs_bytes(int64_t cap, bool one_stage, bool det, bool alt_elsewhere) {
    const int64_t c = cap > 0 ? cap : 1;
    size_t b = align256(sizeof(uint32_t) * c) + align256((one_stage ? sizeof(uint64_t) : sizeof(uint32_t)) * c);
    if (!alt_elsewhere) b += pairs_alt_bytes(cap, one_stage);
    if (det) b += 2 * align256(sizeof(uint32_t) * c);
    return b + 256;
}

// alt: the frame's work space when the alternate buffers go there, else null.
Pairs carve_pairs(void* mem, int64_t cap, bool one_stage, bool det, char* alt) {
    Carver c{static_cast<char*>(mem), 0};
    Carver a{alt, 0};
    Carver& ca = alt ? a : c;
    Pairs p;
    p.capacity = cap;
    p.alt_in_work = alt != nullptr;
    p.tkeys = p.tkeys_alt = nullptr;
    p.k64 = p.k64_alt = nullptr;
    p.rec_emit = p.inv = nullptr;
    p.vals = c.take<uint32_t>(cap);
    p.vals_alt = ca.take<uint32_t>(cap);
    if (one_stage) {
        p.k64 = c.take<uint64_t>(cap);
        p.k64_alt = ca.take<uint64_t>(cap);
    } else {
        p.tkeys = c.take<uint32_t>(cap);
        p.tkeys_alt = ca.take<uint32_t>(cap);
    }
    p.rs_scratch = ca.take<char>((int64_t)radix_scratch_bytes(cap > 0 ? cap : 1));
    if (det) {
        p.rec_emit = c.take<uint32_t>(cap);
        p.inv = c.take<uint32_t>(cap);
    }
    return p;
}

megs_status upload_views(const Layout& L, ViewInfo* dst, hipStream_t s) {
    for (int v0 = 0; v0 < L.nv; v0 += kViewChunk) {
        ViewChunk ch;
        memset(&ch, 0, sizeof(ch));
        ch.count = L.nv - v0 < kViewChunk ? L.nv - v0 : kViewChunk;
        for (int i = 0; i < ch.count; ++i) ch.v[i] = L.views[v0 + i];
        hipLaunchKernelGGL(k_set_views, dim3(1), dim3(kViewChunk), 0, s, dst + v0, ch);
        HIP_TRY(hipGetLastError());
    }
    return MEGS_OK;
}

// Projection, depth pre-sort and tile-count scan (the part before the pair count is known).
megs_status enqueue_front(const megs_scene* sc, const Layout& L, const megs_config* cfg, Frame& f, hipStream_t s) {
    const bool one_stage = cfg->flags & MEGS_FLAG_ONE_STAGE_SORT;
    megs_status st = upload_views(L, f.views, s);
    if (st != MEGS_OK) return st;
    HIP_TRY(launch_fill_u32(f.counters, 0u, 8, s));
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(f.status), 0u, 8, s));
    // Two-stage sort: the projection writes the depth sort's initial values with each record's tile
    // count above its id (when the id leaves at least 4 bits), so the scan after the sort reads the
    // counts in depth order without gathering them.
    int idb = 1;
    while (idb < 32 && (1ll << idb) < L.nr) ++idb;
    const bool packed = !one_stage && idb <= 28;
    f.rec.order0 = packed ? f.order : nullptr;
    f.rec.order_idb = packed ? idb : 0;
    {
        StageTimer t(MEGS_STAGE_PROJECT, s);
        HIP_TRY(launch_project(scene_dev(sc, f.status), f.views, L.nv, L.tile, f.rec, s));
    }
    f.rec.order0 = nullptr;
    if (one_stage) {
        StageTimer t(MEGS_STAGE_SCAN, s);
        HIP_TRY(launch_scan(f.rec.ntiles, nullptr, L.nr, f.offs, f.counters + 0, f.scan_scratch, s));
        return MEGS_OK;
    }
    {
        StageTimer t(MEGS_STAGE_DEPTH_SORT, s);
        if (!packed) HIP_TRY(launch_iota(f.order, L.nr, s));
        HIP_TRY(launch_fill_u32(f.counters + 2, (uint32_t)L.nr, 1, s));
        bool alt = false;
        HIP_TRY(launch_radix_sort_u32(f.rec.dkey, f.order, f.dkey_alt, f.order_alt, f.counters + 2, L.nr, 0, 32,
                                      f.rs_scratch, s, &alt));
        if (alt) return fail(MEGS_ERR_HIP, "depth sort ended in the alternate buffer");
    }
    {
        StageTimer t(MEGS_STAGE_SCAN, s);
        if (packed) {
            HIP_TRY(launch_scan_packed(f.order, f.rec.ntiles, L.nr, idb, f.offs, f.counters + 0, f.scan_scratch, s));
        } else {
            // the depth keys' ping-pong buffer is free after the sort: it takes the gathered counts
            HIP_TRY(launch_scan(f.rec.ntiles, f.order, L.nr, f.offs, f.counters + 0, f.scan_scratch, s,
                                f.dkey_alt));
        }
    }
    return MEGS_OK;
}

// Emission, pair sort, ranges and the forward blend; fills the pair fields of state.
megs_status enqueue_back(const megs_scene* sc, const Layout& L, const megs_config* cfg, Frame& f, Pairs& p,
                         float* images, megs_state* state, hipStream_t s, float* importance = nullptr) {
    const bool one_stage = cfg->flags & MEGS_FLAG_ONE_STAGE_SORT;
    const bool persistent = cfg->flags & MEGS_FLAG_PERSISTENT;
    {
        StageTimer t(MEGS_STAGE_EMIT, s);
        HIP_TRY(launch_clamp_count(f.counters + 0, p.capacity, f.counters + 1, f.status, s));
        HIP_TRY(launch_emit(f.rec, f.views, L.nv, L.n, L.tile, one_stage ? nullptr : f.order, f.offs, f.counters + 0,
                            L.nr, p.tkeys,
                            p.k64, p.vals, p.capacity, f.status, s, sub_masks(cfg, L) ? 8 : 0));
    }
    const bool det = cfg->flags & MEGS_FLAG_DETERMINISTIC;
    if (det) {  // sort emission positions; the record ids are gathered back after the sort
        HIP_TRY(launch_copy_u32(p.rec_emit, p.vals, p.capacity, s));
        HIP_TRY(launch_iota(p.vals, p.capacity, s));
    }
    bool alt = false;
    const uint32_t* sorted_t = nullptr;
    const uint64_t* sorted_k = nullptr;
    const uint32_t* sorted_v = nullptr;
    {
        StageTimer t(MEGS_STAGE_PAIR_SORT, s);
        if (one_stage) {
            HIP_TRY(launch_radix_sort_u64(p.k64, p.vals, p.k64_alt, p.vals_alt, f.counters + 1, p.capacity, 0,
                                          32 + L.tile_bits, p.rs_scratch, s, &alt));
            sorted_k = alt ? p.k64_alt : p.k64;
        } else {
            HIP_TRY(launch_radix_sort_u32(p.tkeys, p.vals, p.tkeys_alt, p.vals_alt, f.counters + 1, p.capacity, 0,
                                          L.tile_bits, p.rs_scratch, s, &alt));
            sorted_t = alt ? p.tkeys_alt : p.tkeys;
        }
    }
    // the work space is reused after the forward: the sorted pairs must not end there
    if (alt && p.alt_in_work) return fail(MEGS_ERR_HIP, "the pair sort ended in the work space");
    sorted_v = alt ? p.vals_alt : p.vals;
    if (det) {
        uint32_t* rec_sorted = alt ? p.vals : p.vals_alt;  // the ping-pong buffer the sort left free
        StageTimer t(MEGS_STAGE_PAIR_SORT, s);
        HIP_TRY(launch_perm_gather(sorted_v, p.rec_emit, f.counters + 1, p.capacity, rec_sorted, p.inv, s));
        sorted_v = rec_sorted;
    }
    {
        StageTimer t(MEGS_STAGE_RANGES, s);
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(f.ranges), 0u, 2 * L.n_tiles, s));
        if (one_stage)
            HIP_TRY(launch_ranges_u64(sorted_k, f.counters + 1, p.capacity, f.ranges, s));
        else
            HIP_TRY(launch_ranges_u32(sorted_t, f.counters + 1, p.capacity, f.ranges, s,
                                      sub_masks(cfg, L) ? 0xffffu : ~0u));
    }
    BlendArgs a;
    memset(&a, 0, sizeof(a));
    a.views = f.views; a.nv = L.nv; a.n_tiles = L.n_tiles;
    a.rec = f.rec.packed;
    a.tkeys = sub_masks(cfg, L) ? sorted_t : nullptr;
    a.vals = sorted_v; a.ranges = f.ranges;
    a.image = images; a.T_final = f.T_final; a.last = f.last;
    a.queue = f.queue;
    a.stats = (cfg->flags & MEGS_FLAG_STATS) ? reinterpret_cast<unsigned long long*>(f.status + 4) : nullptr;
    a.importance = importance;
    a.n = L.n;
    if (persistent) HIP_TRY(launch_fill_u32(f.queue, 0u, kQueueWords, s));
    {
        StageTimer t(MEGS_STAGE_BLEND_FWD, s);
        HIP_TRY(launch_blend_fwd(a, L.tile, waves_of(cfg), cfg->batch, persistent, s, cfg->subtile));
    }

    state->n_records = L.nr;
    state->pair_capacity = p.capacity;
    state->n_pixels = L.n_pixels;
    state->n_views = L.nv;
    state->tile = L.tile;
    state->n_tiles = (int32_t)L.n_tiles;
    state->k = sc->k;
    state->mean = f.rec.mean;
    state->conic_o = f.rec.conic_o;
    state->rgbd = f.rec.rgbd;
    state->radius = f.rec.radius;
    // the work space's tile counts are the forward's own (the pair sort may reuse their memory): the
    // caller sees the copy in the record planes, or, in deterministic mode, the counts themselves
    state->ntiles = L.planes ? f.rec.ntiles_plane : (work_reusable(cfg) ? nullptr : f.rec.ntiles);
    state->cutoff = f.rec.cutoff;
    state->packed = f.rec.packed;
    state->chol = f.rec.chol;
    state->tile_keys = sorted_t;
    state->keys64 = sorted_k;
    state->vals = sorted_v;
    state->ranges = f.ranges;
    state->T_final = f.T_final;
    state->last = f.last;
    state->device_status = f.status;
    state->internal = f.views;
    state->det_inv = det ? p.inv : nullptr;
    state->det_order = one_stage ? nullptr : f.order;
    state->det_offsets = f.offs;
    state->det_count = f.counters + 1;
    state->work = work_reusable(cfg) ? f.work : nullptr;
    state->work_bytes = work_reusable(cfg) ? (int64_t)f.work_bytes : 0;
    return MEGS_OK;
}

megs_status enqueue_backward(const megs_scene* sc, const Layout& L, const megs_config* cfg, const megs_state* st,
                             const float* dl, void* scratch, const megs_scene_grad* gr, hipStream_t s) {
    Carver c{static_cast<char*>(scratch), 0};
    float* grad2d = c.take<float>(9 * L.nr);
    uint32_t* queue = c.take<uint32_t>(kQueueWords);
    float* grad_pair = nullptr;
    if (cfg->flags & MEGS_FLAG_DETERMINISTIC) {
        if (!st->det_inv) return fail(MEGS_ERR_ARG, "deterministic backward needs a deterministic forward state");
        grad_pair = c.take<float>(9 * st->pair_capacity);
    }
    const bool persistent = cfg->flags & MEGS_FLAG_PERSISTENT;
    BlendArgs a;
    memset(&a, 0, sizeof(a));
    a.views = static_cast<const ViewInfo*>(st->internal);
    a.nv = L.nv; a.n_tiles = L.n_tiles;
    a.n = L.n;
    a.rec = static_cast<const PackedRec*>(st->packed);
    a.tkeys = sub_masks(cfg, L) ? static_cast<const uint32_t*>(st->tile_keys) : nullptr;
    a.vals = static_cast<const uint32_t*>(st->vals);
    a.ranges = static_cast<const uint2*>(st->ranges);
    a.T_final = const_cast<float*>(static_cast<const float*>(st->T_final));
    a.last = const_cast<uint32_t*>(static_cast<const uint32_t*>(st->last));
    a.dl = dl;
    a.grad2d = grad2d;
    a.queue = queue;
    a.grad_pair = grad_pair;
    if (grad_pair)
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(grad_pair), 0u, 9 * st->pair_capacity, s));
    else
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(grad2d), 0u, 9 * L.nr, s));
    if (persistent) HIP_TRY(launch_fill_u32(queue, 0u, kQueueWords, s));
    {
        StageTimer t(MEGS_STAGE_BLEND_BWD, s);
        HIP_TRY(launch_blend_bwd(a, L.tile, waves_of(cfg), cfg->batch, persistent, s, cfg->subtile));
        if (grad_pair)
            HIP_TRY(launch_pair_reduce(static_cast<const uint32_t*>(st->det_order),
                                       static_cast<const uint32_t*>(st->det_offsets),
                                       static_cast<const uint32_t*>(st->ntiles), L.nr,
                                       static_cast<const uint32_t*>(st->det_inv),
                                       static_cast<const uint32_t*>(st->det_count), grad_pair, grad2d, s));
    }
    GradDev g;
    g.pos = gr->pos; g.logscale = gr->logscale; g.quat = gr->quat; g.op_logit = gr->op_logit;
    g.pmask_logit = gr->pmask_logit; g.base = gr->base; g.axis = gr->axis; g.sharp = gr->sharp; g.amp = gr->amp;
    g.lmask_logit = gr->lmask_logit;
    g.sh = gr->sh;
    {
        StageTimer t(MEGS_STAGE_PROJECT_BWD, s);
        HIP_TRY(launch_project_bwd(scene_dev(sc, nullptr), a.views, L.nv, grad2d, a.rec, g, s));
    }
    return MEGS_OK;
}

megs_status check_grads(const megs_scene* sc, const megs_scene_grad* g) {
    if (!g) return fail(MEGS_ERR_ARG, "null gradient struct");
    if (sc->n == 0) return MEGS_OK;
    if (!g->pos || !g->logscale || !g->quat || !g->op_logit || (sc->sh ? !g->sh : !g->base))
        return fail(MEGS_ERR_ARG, "null gradient plane");
    if (has_lobes(sc) && (!g->axis || !g->sharp || !g->amp)) return fail(MEGS_ERR_ARG, "null lobe gradient plane");
    if ((sc->pmask_logit != nullptr) != (g->pmask_logit != nullptr))
        return fail(MEGS_ERR_ARG, "pmask_logit gradient must be given exactly when the scene has primitive masks");
    if ((sc->lmask_logit != nullptr) != (g->lmask_logit != nullptr))
        return fail(MEGS_ERR_ARG, "lmask_logit gradient must be given exactly when the scene has lobe masks");
    return MEGS_OK;
}

bool backward_reuses(const megs_config* cfg, const megs_state* st, size_t gbytes) {
    return work_reusable(cfg) && st->work && st->work_bytes >= (int64_t)gbytes;
}

// reserve_backward: size the frame's work space to take the backward's scratch as well (a backward
// may follow); the pair sort's alternate buffers then also go there when they fit.
megs_status forward_impl(const megs_scene* sc, const megs_camera* cams, int32_t nv, const megs_config* cfg,
                         megs_alloc_fn alloc, void* ctx, float* images, megs_state* state, hipStream_t s,
                         float* importance = nullptr, bool reserve_backward = true) {
    megs_status st = check_args(sc, cams, nv, cfg);
    if (st != MEGS_OK) return st;
    if (!alloc || !images || !state) return fail(MEGS_ERR_ARG, "null allocator, image or state");
    const Layout L = make_layout(sc, cams, nv, cfg);
    const bool one_stage = cfg->flags & MEGS_FLAG_ONE_STAGE_SORT;
    const bool det = cfg->flags & MEGS_FLAG_DETERMINISTIC;
    memset(state, 0, sizeof(*state));
    const size_t work = work_bytes(L, cfg, cfg->pair_capacity, reserve_backward);
    void* fm = alloc(ctx, frame_bytes(L, work));
    if (bad_alloc(fm))
        return fail(MEGS_ERR_ALLOC, "allocation of %zu bytes failed or not 256-byte aligned", frame_bytes(L, work));
    Frame f = carve_frame(fm, L, work);
    st = enqueue_front(sc, L, cfg, f, s);
    if (st != MEGS_OK) return st;
    int64_t cap = cfg->pair_capacity;
    int64_t counted = -1;
    if (cap == 0) {
        uint32_t total = 0;
        int32_t flags[4] = {0, 0, 0, 0};
        HIP_TRY(hipMemcpyAsync(&total, f.counters, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(flags, f.status, sizeof(flags), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (flags[kStatusBadLobes]) return fail(MEGS_ERR_ARG, "malformed lobe_off (compressed-row lobes)");
        if (total > kMaxPairs)
            return fail(MEGS_ERR_CAPACITY, "the records list %s%u tile pairs; a key table holds at most %u",
                        total == 0xffffffffu ? "at least " : "", total, kMaxPairs);
        counted = total;
        cap = total;
    }
    const bool alt = alt_in_work(L, cfg, cap, f.work_bytes);
    const size_t pbytes = pairs_bytes(cap, one_stage, det, alt);
    void* pm = alloc(ctx, pbytes);
    if (bad_alloc(pm)) return fail(MEGS_ERR_ALLOC, "allocation of %zu bytes failed or not 256-byte aligned", pbytes);
    Pairs p = carve_pairs(pm, cap, one_stage, det, alt ? f.work : nullptr);
    st = enqueue_back(sc, L, cfg, f, p, images, state, s, importance);
    state->n_pairs = counted >= 0 ? counted : cap;
    return st;
}

// Device address of `scratch` on the calling thread's current device, taken once per device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices];

megs_status scratch_of_current_device(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MEGS_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(MEGS_ERR_HIP, "hipGetSymbolAddress returned a null address for the static scratch");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return MEGS_OK;
}

// Bump allocation over the static scratch, in place of the caller's allocation callback.
struct ScratchBump {
    char* base;
    size_t off, cap;
    size_t needed;  // the total the first request that did not fit would have needed (0: none)
};

void* scratch_take(void* ctx, size_t bytes) {
    ScratchBump* b = static_cast<ScratchBump*>(ctx);
    const size_t a = align256(bytes);
    if (a > b->cap - b->off) {
        if (!b->needed) b->needed = b->off + a;
        return nullptr;
    }
    void* p = b->base + b->off;
    b->off += a;
    return p;
}

// Working memory of the autotuner's sweep. Every forward+backward asks for the same sequence of blocks
// (frame, pair table, and the backward scratch when the frame's work space cannot take it), so the k-th
// request of a run reuses the pool's k-th block. The sweep sizes the blocks for its largest candidate
// before it starts, so the pool holds one candidate's working memory, not the sum over the sweep; a
// larger request would still get a new block (the caller's allocator never frees: the smaller block
// stays with it). All runs go to one stream, so a block is reused only after the run before has
// finished with it.
struct SweepPool {
    megs_alloc_fn alloc;
    void* ctx;
    std::vector<std::pair<void*, size_t>> blocks;
    size_t next;
    bool failed;
};

void* sweep_take(void* ctx, size_t bytes) {
    SweepPool* p = static_cast<SweepPool*>(ctx);
    const size_t k = p->next++;
    if (k < p->blocks.size() && p->blocks[k].second >= bytes) return p->blocks[k].first;
    void* m = p->alloc(p->ctx, bytes);
    if (bad_alloc(m)) {
        p->failed = true;
        return nullptr;
    }
    if (k < p->blocks.size())
        p->blocks[k] = {m, bytes};
    else
        p->blocks.push_back({m, bytes});
    return m;
}

}  // namespace

struct megs_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
    megs_state state;
};

extern "C" {

const char* megs_last_error(void) { return g_err; }

const char* megs_version(void) { return "megs 0.1 (gfx950)"; }

megs_status megs_profile_begin(void) {
    g_err[0] = 0;
    for (auto& r : g_prof.recs) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.end);
    }
    g_prof.recs.clear();
    g_prof.on = true;
    return MEGS_OK;
}

megs_status megs_profile_end(megs_profile* out) {
    g_err[0] = 0;
    megs_status st = MEGS_OK;
    if (out) memset(out, 0, sizeof(*out));
    for (auto& r : g_prof.recs) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.end);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.end);
        if (e != hipSuccess && st == MEGS_OK) st = fail(MEGS_ERR_HIP, "profile event: %s", hipGetErrorString(e));
        if (out && r.stage >= 0 && r.stage < MEGS_STAGE_COUNT) {
            out->ms[r.stage] += ms;
            out->count[r.stage] += 1;
        }
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.end);
    }
    g_prof.recs.clear();
    g_prof.on = false;
    return st;
}

megs_status megs_render_forward(const megs_scene* scene, const megs_camera* cams, int32_t n_views,
                                const megs_config* cfg, megs_alloc_fn alloc, void* alloc_ctx, float* images,
                                megs_state* state, void* stream) {
    g_err[0] = 0;
    return forward_impl(scene, cams, n_views, cfg, alloc, alloc_ctx, images, state, static_cast<hipStream_t>(stream));
}

megs_status megs_render_forward_noalloc(const megs_scene* scene, const megs_camera* cams, int32_t n_views,
                                        const megs_config* cfg, float* images, megs_state* state, void* stream) {
    g_err[0] = 0;
    megs_status st = check_args(scene, cams, n_views, cfg);
    if (st != MEGS_OK) return st;
    if (!images || !state) return fail(MEGS_ERR_ARG, "null image or state");
    const Layout L = make_layout(scene, cams, n_views, cfg);
    const bool one_stage = cfg->flags & MEGS_FLAG_ONE_STAGE_SORT;
    const bool det = cfg->flags & MEGS_FLAG_DETERMINISTIC;
    const size_t cap = MEGS_NOALLOC_SCRATCH_BYTES;
    // what is known before any launch: the frame, and the pair table when its capacity is fixed
    const size_t work = work_bytes(L, cfg, cfg->pair_capacity, false);
    size_t need = align256(frame_bytes(L, work));
    if (cfg->pair_capacity > 0)
        need += align256(pairs_bytes(cfg->pair_capacity, one_stage, det,
                                     alt_in_work(L, cfg, cfg->pair_capacity, align256(work))));
    if (need > cap)
        return fail(MEGS_ERR_CAPACITY, "this forward needs %zu bytes of working memory; the static scratch holds %zu",
                    need, cap);
    void* base = nullptr;
    st = scratch_of_current_device(&base);
    if (st != MEGS_OK) return st;
    ScratchBump b{static_cast<char*>(base), 0, cap, 0};
    st = forward_impl(scene, cams, n_views, cfg, scratch_take, &b, images, state, static_cast<hipStream_t>(stream),
                      nullptr, false);
    if (st == MEGS_ERR_ALLOC && b.needed)
        return fail(MEGS_ERR_CAPACITY,
                    "the counted pairs need %zu bytes of working memory in all; the static scratch holds %zu",
                    b.needed, cap);
    return st;
}

megs_status megs_render_backward(const megs_scene* scene, const megs_camera* cams, int32_t n_views,
                                 const megs_config* cfg, const megs_state* state, const float* dl_dimages,
                                 megs_alloc_fn alloc, void* alloc_ctx, megs_scene_grad* grads, void* stream) {
    g_err[0] = 0;
    megs_status st = check_args(scene, cams, n_views, cfg);
    if (st != MEGS_OK) return st;
    if (!state || !dl_dimages || !alloc) return fail(MEGS_ERR_ARG, "null state, dL/dimage or allocator");
    st = check_grads(scene, grads);
    if (st != MEGS_OK) return st;
    const Layout L = make_layout(scene, cams, n_views, cfg);
    if (state->n_records != L.nr || state->n_views != n_views || state->tile != cfg->tile || !state->internal)
        return fail(MEGS_ERR_ARG, "state does not belong to this scene, view set and tile size");
    const size_t gbytes = backward_bytes(L, cfg, state->pair_capacity);
    // the forward's work space when it is free and large enough, else new memory
    void* gm = backward_reuses(cfg, state, gbytes) ? state->work : alloc(alloc_ctx, gbytes);
    if (bad_alloc(gm)) return fail(MEGS_ERR_ALLOC, "allocation of %zu bytes failed or not 256-byte aligned", gbytes);
    return enqueue_backward(scene, L, cfg, state, dl_dimages, gm, grads, static_cast<hipStream_t>(stream));
}

megs_status megs_render_importance(const megs_scene* scene, const megs_camera* cams, int32_t n_views,
                                   const megs_config* cfg, megs_alloc_fn alloc, void* alloc_ctx, float* images,
                                   float* importance, megs_state* state, void* stream) {
    g_err[0] = 0;
    if (!importance) return fail(MEGS_ERR_ARG, "null importance output");
    if (cfg && (cfg->flags & MEGS_FLAG_STATS)) return fail(MEGS_ERR_UNSUPPORTED, "importance with MEGS_FLAG_STATS");
    return forward_impl(scene, cams, n_views, cfg, alloc, alloc_ctx, images, state, static_cast<hipStream_t>(stream),
                        importance);
}

megs_status megs_lobe_range(int64_t n, int32_t k, const float* sharp, const float* lam, const float* amp, float* D,
                            void* stream) {
    g_err[0] = 0;
    if (n < 0 || k < 0 || k > MEGS_MAX_LOBES) return fail(MEGS_ERR_ARG, "bad n or k");
    if (n * k > 0 && (!sharp || !amp || !D)) return fail(MEGS_ERR_ARG, "null sharpness, amplitude or output");
    HIP_TRY(launch_lobe_range(n, k, sharp, lam, amp, D, static_cast<hipStream_t>(stream)));
    return MEGS_OK;
}

megs_status megs_select_topk(const float* score, int64_t n, int64_t kappa, megs_alloc_fn alloc, void* alloc_ctx,
                             uint8_t* keep, void* stream) {
    g_err[0] = 0;
    if (n < 0 || n >= (1ll << 31)) return fail(MEGS_ERR_ARG, "n out of range");
    if (n == 0) return MEGS_OK;
    if (!score || !keep || !alloc) return fail(MEGS_ERR_ARG, "null score, keep or allocator");
    void* scratch = nullptr;
    if (kappa > 0 && kappa < n) {
        scratch = alloc(alloc_ctx, select_scratch_bytes(n));
        if (bad_alloc(scratch)) return fail(MEGS_ERR_ALLOC, "allocation of %zu bytes failed or not 256-byte aligned", select_scratch_bytes(n));
    }
    HIP_TRY(launch_select_topk(score, n, kappa, scratch, keep, static_cast<hipStream_t>(stream)));
    return MEGS_OK;
}

megs_status megs_prox_apply(int64_t count, const float* x, const float* lam, const uint8_t* keep, float* x_tilde,
                            void* stream) {
    g_err[0] = 0;
    if (count < 0) return fail(MEGS_ERR_ARG, "count < 0");
    if (count > 0 && (!x || !lam || !keep || !x_tilde)) return fail(MEGS_ERR_ARG, "null argument");
    HIP_TRY(launch_prox_apply(count, x, lam, keep, x_tilde, static_cast<hipStream_t>(stream)));
    return MEGS_OK;
}

megs_status megs_dual_update(int64_t count, float* lam, const float* x, const float* x_tilde, void* stream) {
    g_err[0] = 0;
    if (count < 0) return fail(MEGS_ERR_ARG, "count < 0");
    if (count > 0 && (!x || !lam || !x_tilde)) return fail(MEGS_ERR_ARG, "null argument");
    HIP_TRY(launch_dual(count, lam, x, x_tilde, static_cast<hipStream_t>(stream)));
    return MEGS_OK;
}

megs_status megs_penalty_grad(int64_t count, float delta, const float* x, const float* x_tilde, const float* lam,
                              float* grad, void* stream) {
    g_err[0] = 0;
    if (count < 0) return fail(MEGS_ERR_ARG, "count < 0");
    if (count > 0 && (!x || !lam || !x_tilde || !grad)) return fail(MEGS_ERR_ARG, "null argument");
    HIP_TRY(launch_penalty(count, delta, x, x_tilde, lam, grad, static_cast<hipStream_t>(stream)));
    return MEGS_OK;
}

megs_status megs_compact(const megs_scene* scene, double opacity_min, double sharp_min, megs_alloc_fn alloc,
                         void* alloc_ctx, void* stream, megs_compacted* out) {
    g_err[0] = 0;
    megs_status st = check_scene(scene);
    if (st != MEGS_OK) return st;
    if (!alloc || !out) return fail(MEGS_ERR_ARG, "null allocator or output");
    if (isnan(opacity_min) || isnan(sharp_min)) return fail(MEGS_ERR_ARG, "NaN threshold");
    if (scene->sh) return fail(MEGS_ERR_UNSUPPORTED, "compaction of spherical-harmonic scenes");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = scene->n;
    CompactArgs a;
    memset(&a, 0, sizeof(a));
    a.in = scene_dev(scene, nullptr);
    a.in.k = scene->k;  // the compaction keeps k as given
    a.in.lobe_off = scene->lobe_off;
    a.opacity_min = opacity_min;
    a.sharp_min = sharp_min;
    // working block: keep, count, new_idx, lobe_pos [n], totals [2], status [8], scan scratch
    const size_t wbytes = 4 * align256(sizeof(uint32_t) * (n ? n : 1)) + 2 * align256(32) +
                          align256(scan_scratch_bytes(n)) + 256;
    void* wm = alloc(alloc_ctx, wbytes);
    if (bad_alloc(wm)) return fail(MEGS_ERR_ALLOC, "allocation of %zu bytes failed or not 256-byte aligned", wbytes);
    Carver w{static_cast<char*>(wm), 0};
    a.keep = w.take<uint32_t>(n);
    a.count = w.take<uint32_t>(n);
    a.new_idx = w.take<uint32_t>(n);
    a.lobe_pos = w.take<uint32_t>(n);
    uint32_t* totals = w.take<uint32_t>(8);
    int32_t* status = w.take<int32_t>(8);
    void* scan_scratch = w.take<char>((int64_t)scan_scratch_bytes(n));
    a.in.status = status;
    HIP_TRY(launch_fill_u32(totals, 0u, 8, s));
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(status), 0u, 8, s));
    HIP_TRY(launch_compact_mark(a, s));
    if (n > 0) {
        HIP_TRY(launch_scan(a.keep, nullptr, n, a.new_idx, totals + 0, scan_scratch, s));
        HIP_TRY(launch_scan(a.count, nullptr, n, a.lobe_pos, totals + 1, scan_scratch, s));
    }
    uint32_t ht[2] = {0, 0};
    int32_t hs[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(ht, totals, sizeof(ht), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hs, status, sizeof(hs), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hs[kStatusBadLobes]) return fail(MEGS_ERR_ARG, "malformed lobe_off (compressed-row lobes)");
    const int64_t no = ht[0], lo = ht[1];
    a.n_out = no;
    a.l_out = lo;
    const size_t eg = scene->dt_geom == MEGS_F32 ? 4 : 2, ec = scene->dt_color == MEGS_F32 ? 4 : 2,
                 ea = scene->dt_amp == MEGS_F32 ? 4 : 2;
    const size_t obytes = align256(eg * 3 * no) * 2 + align256(eg * 4 * no) + align256(eg * no) +
                          align256(ec * 3 * no) + align256(ec * 3 * lo) + align256(ec * lo) + align256(ea * 3 * lo) +
                          align256(sizeof(int32_t) * (no + 1)) + align256(sizeof(int32_t) * no) +
                          align256(sizeof(int32_t) * lo) + 256 * 12;
    void* om = alloc(alloc_ctx, obytes);
    if (bad_alloc(om)) return fail(MEGS_ERR_ALLOC, "allocation of %zu bytes failed or not 256-byte aligned", obytes);
    Carver o{static_cast<char*>(om), 0};
    a.pos = o.take<char>((int64_t)(eg * 3 * no));
    a.logscale = o.take<char>((int64_t)(eg * 3 * no));
    a.quat = o.take<char>((int64_t)(eg * 4 * no));
    a.op_logit = o.take<char>((int64_t)(eg * no));
    a.base = o.take<char>((int64_t)(ec * 3 * no));
    a.axis = o.take<char>((int64_t)(ec * 3 * lo));
    a.sharp = o.take<char>((int64_t)(ec * lo));
    a.amp = o.take<char>((int64_t)(ea * 3 * lo));
    a.lobe_off = o.take<int32_t>(no + 1);
    a.kept = o.take<int32_t>(no);
    a.lobe_src = o.take<int32_t>(lo);
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(a.lobe_off + no), (uint32_t)lo, 1, s));
    HIP_TRY(launch_compact_write(a, s));

    memset(out, 0, sizeof(*out));
    megs_scene& r = out->scene;
    r.n = no;
    r.k = scene->k;
    r.dt_geom = scene->dt_geom; r.dt_color = scene->dt_color; r.dt_amp = scene->dt_amp;
    r.pos = a.pos; r.logscale = a.logscale; r.quat = a.quat; r.op_logit = a.op_logit; r.pmask_logit = nullptr;
    r.base = a.base; r.axis = a.axis; r.sharp = a.sharp; r.amp = a.amp; r.lmask_logit = nullptr;
    r.lobe_off = a.lobe_off;
    r.n_lobes = lo;
    out->kept = a.kept;
    out->lobe_src = a.lobe_src;
    return MEGS_OK;
}

megs_status megs_photometric_loss(const float* images, const float* targets, int32_t n_views, const int32_t* sizes,
                                  double lambda_dssim, megs_alloc_fn alloc, void* alloc_ctx, double* loss,
                                  float* dl_dimages, void* stream) {
    g_err[0] = 0;
    if (n_views < 1 || n_views > MEGS_MAX_VIEWS) return fail(MEGS_ERR_ARG, "n_views = %d outside [1, %d]", n_views, MEGS_MAX_VIEWS);
    if (!images || !targets || !sizes || !loss || !alloc) return fail(MEGS_ERR_ARG, "null argument");
    if (!(lambda_dssim >= 0.0 && lambda_dssim <= 1.0)) return fail(MEGS_ERR_ARG, "lambda outside [0, 1]");
    LossViews vs;
    memset(&vs, 0, sizeof(vs));
    int64_t pix = 0, parts = 0;
    for (int i = 0; i < n_views; ++i) {
        const int w = sizes[2 * i], h = sizes[2 * i + 1];
        if (w <= 0 || h <= 0 || w > 16384 || h > 16384) return fail(MEGS_ERR_ARG, "view %d: image size %dx%d out of range", i, w, h);
        vs.v[i].width = w; vs.v[i].height = h;
        vs.v[i].pix_off = pix;
        vs.v[i].part_off = parts;
        vs.v[i].n_part = loss_partials(w, h);
        pix += (int64_t)w * h;
        parts += vs.v[i].n_part;
    }
    const size_t bytes = align256(sizeof(double) * 9 * pix) + align256(sizeof(double) * 2 * parts) +
                         align256(sizeof(double) * n_views) + 256;
    void* mem = alloc(alloc_ctx, bytes);
    if (bad_alloc(mem)) return fail(MEGS_ERR_ALLOC, "allocation of %zu bytes failed or not 256-byte aligned", bytes);
    Carver c{static_cast<char*>(mem), 0};
    double* maps = c.take<double>(9 * pix);
    double* partial = c.take<double>(2 * parts);
    double* terms = c.take<double>(n_views);
    Window11 g;
    double sum = 0.0;
    for (int k = 0; k < 11; ++k) {
        g.w[k] = exp(-(double)((k - 5) * (k - 5)) / (2.0 * 1.5 * 1.5));
        sum += g.w[k];
    }
    for (int k = 0; k < 11; ++k) g.w[k] /= sum;
    HIP_TRY(launch_loss(vs, n_views, images, targets, maps, partial, terms, loss, dl_dimages, g, lambda_dssim,
                        static_cast<hipStream_t>(stream)));
    return MEGS_OK;
}

megs_status megs_adam_step(int64_t count, void* param, int32_t dtype, const float* grad, float* m, float* v, float lr,
                           float beta1, float beta2, float eps, int32_t step, void* stream) {
    g_err[0] = 0;
    if (count < 0) return fail(MEGS_ERR_ARG, "count < 0");
    if (!valid_dtype(dtype)) return fail(MEGS_ERR_ARG, "unknown storage dtype");
    if (step < 1) return fail(MEGS_ERR_ARG, "step must be >= 1");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f))
        return fail(MEGS_ERR_ARG, "beta1, beta2 must lie in [0, 1) and eps >= 0");
    if (count > 0 && (!param || !grad || !m || !v)) return fail(MEGS_ERR_ARG, "null argument");
    HIP_TRY(launch_adam(count, param, dtype, grad, m, v, lr, beta1, beta2, eps, step, static_cast<hipStream_t>(stream)));
    return MEGS_OK;
}

megs_status megs_state_status(const megs_state* state, int64_t* pairs_needed, void* stream) {
    g_err[0] = 0;
    if (!state || !state->device_status) return fail(MEGS_ERR_ARG, "null state");
    int32_t h[4] = {0, 0, 0, 0};
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(h, state->device_status, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (pairs_needed) *pairs_needed = (int64_t)(uint32_t)h[0];
    if (h[kStatusBadLobes]) return fail(MEGS_ERR_ARG, "malformed lobe_off (compressed-row lobes)");
    if (h[1]) return fail(MEGS_ERR_CAPACITY, "pair table overflow: %u pairs counted, capacity %lld", (uint32_t)h[0],
                          (long long)state->pair_capacity);
    return MEGS_OK;
}

megs_status megs_state_bytes(const megs_scene* scene, const megs_camera* cams, int32_t n_views,
                             const megs_config* cfg, int64_t n_pairs, megs_memory* out) {
    g_err[0] = 0;
    megs_status st = check_args(scene, cams, n_views, cfg);
    if (st != MEGS_OK) return st;
    if (!out) return fail(MEGS_ERR_ARG, "null output");
    if (cfg->pair_capacity == 0 && (n_pairs < 0 || n_pairs > (int64_t)kMaxPairs))
        return fail(MEGS_ERR_ARG, "n_pairs = %lld outside [0, 2^31 - 1]", (long long)n_pairs);
    const Layout L = make_layout(scene, cams, n_views, cfg);
    const bool one_stage = cfg->flags & MEGS_FLAG_ONE_STAGE_SORT;
    const bool det = cfg->flags & MEGS_FLAG_DETERMINISTIC;
    const int64_t cap = cfg->pair_capacity > 0 ? cfg->pair_capacity : n_pairs;
    const size_t work = align256(work_bytes(L, cfg, cfg->pair_capacity, true));
    out->work = work;
    out->frame = frame_bytes(L, work);
    out->pairs = pairs_bytes(cap, one_stage, det, alt_in_work(L, cfg, cap, work));
    const size_t gbytes = backward_bytes(L, cfg, cap);
    out->backward = work_reusable(cfg) && work >= gbytes ? 0 : gbytes;
    return MEGS_OK;
}

megs_status megs_state_counts(const megs_state* state, megs_counts* out, void* stream) {
    g_err[0] = 0;
    if (!state || !state->device_status || !out) return fail(MEGS_ERR_ARG, "null state or output");
    int32_t h[4] = {0, 0, 0, 0};
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(h, state->device_status, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    out->pairs_needed = (int64_t)(uint32_t)h[0];
    out->culled = (int64_t)(uint32_t)h[kStatusCulled];
    out->overflow = h[kStatusOverflow] != 0;
    out->bad_lobes = h[kStatusBadLobes] != 0;
    return MEGS_OK;
}

megs_status megs_graph_create(const megs_scene* scene, const megs_camera* cams, int32_t n_views,
                              const megs_config* cfg, megs_alloc_fn alloc, void* alloc_ctx, float* images,
                              const float* dl_dimages, megs_scene_grad* grads, int32_t with_backward, void* stream,
                              megs_graph** out) {
    g_err[0] = 0;
    megs_status st = check_args(scene, cams, n_views, cfg);
    if (st != MEGS_OK) return st;
    if (!out || !alloc || !images) return fail(MEGS_ERR_ARG, "null output, allocator or images");
    if (cfg->pair_capacity <= 0) return fail(MEGS_ERR_ARG, "graph mode needs pair_capacity > 0");
    if (!stream) return fail(MEGS_ERR_ARG, "graph capture needs a non-null stream");
    if (with_backward) {
        if (!dl_dimages) return fail(MEGS_ERR_ARG, "null dL/dimage");
        st = check_grads(scene, grads);
        if (st != MEGS_OK) return st;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Layout L = make_layout(scene, cams, n_views, cfg);
    const bool one_stage = cfg->flags & MEGS_FLAG_ONE_STAGE_SORT;
    const bool det = cfg->flags & MEGS_FLAG_DETERMINISTIC;
    const int64_t cap = cfg->pair_capacity;
    const size_t work = work_bytes(L, cfg, cap, with_backward);
    const bool alt = alt_in_work(L, cfg, cap, align256(work));
    void* fm = alloc(alloc_ctx, frame_bytes(L, work));
    void* pm = alloc(alloc_ctx, pairs_bytes(cap, one_stage, det, alt));
    if (bad_alloc(fm) || bad_alloc(pm)) return fail(MEGS_ERR_ALLOC, "allocation failed or not 256-byte aligned");
    Frame f = carve_frame(fm, L, work);
    const size_t gbytes = backward_bytes(L, cfg, cap);
    void* gm = nullptr;
    if (with_backward) {
        gm = work_reusable(cfg) && f.work_bytes >= gbytes ? static_cast<void*>(f.work) : alloc(alloc_ctx, gbytes);
        if (bad_alloc(gm)) return fail(MEGS_ERR_ALLOC, "allocation failed or not 256-byte aligned");
    }
    megs_graph* G = new (std::nothrow) megs_graph();
    if (!G) return fail(MEGS_ERR_ALLOC, "host allocation failed");
    Pairs p = carve_pairs(pm, cap, one_stage, det, alt ? f.work : nullptr);
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { delete G; return fail(MEGS_ERR_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e)); }
    st = enqueue_front(scene, L, cfg, f, s);
    if (st == MEGS_OK) st = enqueue_back(scene, L, cfg, f, p, images, &G->state, s);
    if (st == MEGS_OK && with_backward) st = enqueue_backward(scene, L, cfg, &G->state, dl_dimages, gm, grads, s);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    if (st != MEGS_OK) { if (graph) (void)hipGraphDestroy(graph); delete G; return st; }
    if (e != hipSuccess) { delete G; return fail(MEGS_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e)); }
    G->graph = graph;
    e = hipGraphInstantiate(&G->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete G;
        return fail(MEGS_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    G->state.n_pairs = cfg->pair_capacity;
    *out = G;
    return MEGS_OK;
}

megs_status megs_graph_capture(const megs_scene* scene, const megs_camera* cams, int32_t n_views,
                               const megs_config* cfg, megs_alloc_fn alloc, void* alloc_ctx, float* images,
                               const float* dl_dimages, megs_scene_grad* grads, int32_t with_backward, void* stream,
                               megs_graph** out) {
    return megs_graph_create(scene, cams, n_views, cfg, alloc, alloc_ctx, images, dl_dimages, grads, with_backward,
                             stream, out);
}

megs_status megs_graph_launch(megs_graph* graph, void* stream) {
    g_err[0] = 0;
    if (!graph) return fail(MEGS_ERR_ARG, "null graph");
    HIP_TRY(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)));
    return MEGS_OK;
}

megs_status megs_graph_status(megs_graph* graph, int64_t* pairs_needed, void* stream) {
    if (!graph) return fail(MEGS_ERR_ARG, "null graph");
    return megs_state_status(&graph->state, pairs_needed, stream);
}

const megs_state* megs_graph_state(const megs_graph* graph) { return graph ? &graph->state : nullptr; }

void megs_graph_destroy(megs_graph* graph) {
    if (!graph) return;
    (void)hipGraphExecDestroy(graph->exec);
    (void)hipGraphDestroy(graph->graph);
    delete graph;
}

megs_status megs_autotune(const megs_scene* scene, const megs_camera* cams, int32_t n_views, const megs_config* base,
                          megs_alloc_fn alloc, void* alloc_ctx, float* images, const float* dl_dimages,
                          megs_scene_grad* grads, int32_t reps, void* stream, megs_config* best, float* ms_out) {
    g_err[0] = 0;
    if (!base || !best || !dl_dimages || !alloc) return fail(MEGS_ERR_ARG, "null base config, best, dL/dimage or allocator");
    if (reps < 1) reps = 1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int combos[9][3] = {{8, 1, 0},  {16, 1, 0}, {16, 2, 0}, {16, 4, 0}, {32, 1, 0},
                              {32, 2, 0}, {32, 4, 0}, {16, 1, 8}, {32, 1, 8}};
    const int batches[4] = {32, 64, 128, 256};
    SweepPool pool{alloc, alloc_ctx, {}, 0, false};
    {
        // Sizing pass: each candidate's blocks are known before the sweep (the frame from its layout, the
        // pair table from the pairs its front end counts), so the pool takes the largest of each at once
        // and every run of the sweep reuses them.
        size_t need[3] = {0, 0, 0};
        for (int ci = 0; ci < 9; ++ci) {
            megs_config c = *base;
            c.tile = combos[ci][0]; c.waves = combos[ci][1]; c.subtile = combos[ci][2]; c.batch = 64;
            megs_status st = check_args(scene, cams, n_views, &c);
            if (st != MEGS_OK) return st;
            const Layout L = make_layout(scene, cams, n_views, &c);
            need[0] = std::max(need[0], frame_bytes(L, work_bytes(L, &c, c.pair_capacity, true)));
        }
        void* fm = alloc(alloc_ctx, need[0]);
        if (bad_alloc(fm)) return fail(MEGS_ERR_ALLOC, "allocation of %zu bytes failed or not 256-byte aligned", need[0]);
        for (int ci = 0; ci < 9; ++ci) {
            megs_config c = *base;
            c.tile = combos[ci][0]; c.waves = combos[ci][1]; c.subtile = combos[ci][2]; c.batch = 64;
            const Layout L = make_layout(scene, cams, n_views, &c);
            const size_t work = work_bytes(L, &c, c.pair_capacity, true);
            Frame f = carve_frame(fm, L, work);
            megs_status st = enqueue_front(scene, L, &c, f, s);
            if (st != MEGS_OK) return st;
            int64_t cap = c.pair_capacity;
            if (cap == 0) {
                uint32_t total = 0;
                HIP_TRY(hipMemcpyAsync(&total, f.counters, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                if (total > kMaxPairs)
                    return fail(MEGS_ERR_CAPACITY, "a candidate lists more than %u tile pairs", kMaxPairs);
                cap = total;
            }
            const bool one_stage = c.flags & MEGS_FLAG_ONE_STAGE_SORT;
            const bool det = c.flags & MEGS_FLAG_DETERMINISTIC;
            need[1] = std::max(need[1], pairs_bytes(cap, one_stage, det, alt_in_work(L, &c, cap, f.work_bytes)));
            const size_t gbytes = backward_bytes(L, &c, cap);
            if (!(work_reusable(&c) && f.work_bytes >= gbytes)) need[2] = std::max(need[2], gbytes);
        }
        pool.blocks.push_back({fm, need[0]});
        for (int k = 1; k < 3 && need[k]; ++k) {
            void* m = alloc(alloc_ctx, need[k]);
            if (bad_alloc(m)) return fail(MEGS_ERR_ALLOC, "allocation of %zu bytes failed or not 256-byte aligned", need[k]);
            pool.blocks.push_back({m, need[k]});
        }
    }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best_ms = 1e30f;
    megs_status result = MEGS_OK;
    for (int ci = 0; ci < 9 && result == MEGS_OK; ++ci)
        for (int bi = 0; bi < 4 && result == MEGS_OK; ++bi) {
            megs_config c = *base;
            c.tile = combos[ci][0];
            c.waves = combos[ci][1];
            c.subtile = combos[ci][2];
            c.batch = batches[bi];
            // the sub-tile blends stage no batches: one timing serves all four batch sizes
            if (c.subtile && bi > 0) {
                if (ms_out) ms_out[ci * 4 + bi] = ms_out[ci * 4];
                continue;
            }
            if (c.subtile) c.batch = 64;
            float ms_total = 0.f;
            for (int r = 0; r <= reps && result == MEGS_OK; ++r) {
                megs_state st;
                pool.next = 0;  // every run reuses the pool's blocks from the start
                if (r > 0) (void)hipEventRecord(e0, s);
                result = megs_render_forward(scene, cams, n_views, &c, sweep_take, &pool, images, &st, stream);
                if (result == MEGS_OK)
                    result = megs_render_backward(scene, cams, n_views, &c, &st, dl_dimages, sweep_take, &pool, grads,
                                                  stream);
                if (r > 0 && result == MEGS_OK) {
                    (void)hipEventRecord(e1, s);
                    (void)hipEventSynchronize(e1);
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    ms_total += ms;
                }
            }
            if (pool.failed) result = fail(MEGS_ERR_ALLOC, "allocation failed or not 256-byte aligned during the sweep");
            const float ms = ms_total / reps;
            if (ms_out) ms_out[ci * 4 + bi] = ms;
            if (result == MEGS_OK && ms < best_ms) {
                best_ms = ms;
                *best = c;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return result;
}

}  // extern "C"
