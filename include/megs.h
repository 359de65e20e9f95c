/*
 * megs.h -- C ABI of libmegs.so, the MI355X (gfx950) differentiable SG-splatting renderer.
 *
 * What the library computes (MEGS^2, arXiv 2509.07021):
 *   - colour per Gaussian and view from arbitrarily oriented Spherical-Gaussian lobes,
 *     c(d) = c0 + sum_k m_k a_k exp(lambda_k (mu_k . d - 1)) (Sec. 3.2, the SG lobe and colour
 *     equations), each lobe gated by a soft mask m_k = sigmoid(lobe mask logit);
 *   - front-to-back alpha compositing C = sum_i c_i alpha_i prod_{j<i}(1 - alpha_j), alpha_i the
 *     opacity (gated by a soft primitive mask) times the projected 2D Gaussian (Sec. 3.1);
 *   - the tile/depth key table of the tile rasteriser the paper builds on (Sec. 1, and the
 *     Appendix's evaluation details, which count it in the dynamic rendering memory);
 *   - the exact gradient of the images with respect to every raw parameter.
 *
 * Conventions (the paper prints none of them; they follow the 3DGS rasteriser it builds on):
 *   OpenCV camera axes (x right, y down, z forward), x_cam = R x_world + t; pixel (i, j) has
 *   its centre at (i + 0.5, j + 0.5); EWA projection with a 0.3 px^2 dilation; alpha clamped
 *   to 0.99; fragments with alpha < 1/255 skipped; a pixel stops before its transmittance
 *   would drop below 1e-4 (that fragment is not blended); near plane from the camera; the
 *   Jacobian is evaluated at the direction clamped to 1.3x the half field of view; the
 *   footprint radius is ceil(sqrt(2 ln(255 o) lambda_max)) so that every pixel with
 *   alpha >= 1/255 lies inside the tile rectangle (lambda_max in FP32 from the record's stored
 *   conic factors, so a radius can differ by one pixel from an FP64 evaluation where the root lies
 *   within rounding of an integer), and of that rectangle exactly the tiles are
 *   listed whose pixel-centre box (the centres of the tile's pixels inside the image) the ellipse
 *   (p - m)' conic (p - m) <= k reaches, k = 2.004 ln(255 o) + 1e-4, slightly above the level
 *   2 ln(255 o) of alpha = 1/255 (see megs_state.cutoff); depth ties are ordered by record index.
 *   Quaternions are (w, x, y, z) and normalised in the forward pass, lobe axes likewise;
 *   scales are exp(log-scale), opacity and masks are sigmoid(logit), sharpness is used as
 *   stored. Colours are not clamped.
 *
 * Memory: every device buffer belongs to the caller. The library never calls hipMalloc:
 * it asks the caller's allocation callback for its working memory and never frees it
 * (megs_render_forward_noalloc takes its working memory from a static per-device array instead).
 * All work is enqueued on the caller's stream (a hipStream_t passed as void*).
 *
 * Errors: every entry point returns a megs_status and never throws. Arguments are checked
 * before the first launch; megs_last_error() describes the last failure on the calling
 * thread.
 */
#ifndef MEGS_H
#define MEGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MEGS_OK = 0,
    MEGS_ERR_ARG = -1,         /* invalid argument (null pointer, bad size, bad dtype, ...) */
    MEGS_ERR_HIP = -2,         /* a HIP runtime call failed */
    MEGS_ERR_CAPACITY = -3,    /* the pair table overflowed its fixed capacity (graph mode), or the
                                  working memory exceeds the static scratch (no-allocation forward) */
    MEGS_ERR_UNSUPPORTED = -4, /* a configuration the library does not implement */
    MEGS_ERR_ALLOC = -5        /* the allocation callback returned NULL or memory not 256-byte aligned */
} megs_status;

typedef enum { MEGS_F32 = 0, MEGS_F16 = 1, MEGS_BF16 = 2 } megs_dtype;

#define MEGS_MAX_LOBES 8
#define MEGS_MAX_VIEWS 64

/*
 * Scene parameters: structure-of-arrays planes in device memory, plane row r of Gaussian i
 * at element r * n + i. Storage dtype per group: dt_geom for pos, logscale, quat, op_logit,
 * pmask_logit; dt_color for base, axis, sharp, lmask_logit; dt_amp for amp. All arithmetic is
 * FP32 (the camera-space mean and pixel mean in FP64); reduced-precision planes are widened in
 * registers, never copied.
 *   pos[3][n], logscale[3][n], quat[4][n] (w, x, y, z), op_logit[n],
 *   pmask_logit[n]      (NULL: no primitive mask, m = 1),
 *   base[3][n], and the lobes in one of two layouts:
 *   dense (lobe_off NULL): every Gaussian has k lobes,
 *     axis[k][3][n], sharp[k][n], amp[k][3][n], lmask_logit[k][n] (NULL: no lobe masks, m_k = 1);
 *   compressed rows (lobe_off non-NULL; the post-processed form of Sec. 3.3, where Gaussians keep
 *     different numbers of lobes): Gaussian i owns lobes lobe_off[i] .. lobe_off[i + 1] - 1, at
 *     most k of them, lobe_off[0] = 0, lobe_off non-decreasing, lobe_off[n] = n_lobes,
 *     axis[3][n_lobes], sharp[n_lobes], amp[3][n_lobes], lmask_logit[n_lobes] (or NULL).
 *     A Gaussian whose offsets break these rules is culled and the forward reports MEGS_ERR_ARG.
 * 0 <= k <= MEGS_MAX_LOBES; 0 <= n; n * n_views < 2^31; 0 <= n_lobes < 2^31.
 */
typedef struct {
    int64_t n;
    int32_t k;
    int32_t dt_geom, dt_color, dt_amp;
    int32_t reserved;
    const void *pos, *logscale, *quat, *op_logit, *pmask_logit;
    const void *base, *axis, *sharp, *amp, *lmask_logit;
    const int32_t *lobe_off; /* [n + 1] device, or NULL for the dense layout */
    int64_t n_lobes;         /* compressed rows only: total lobes */
    /* Spherical-harmonic colour instead of SG (3DGS's colour model, which the paper replaces;
     * kept for the same-renderer comparison of bytes per Gaussian): when sh is non-NULL the colour
     * is max(0, sum_m Y_m(d) sh[m] + 1/2) per channel, Y_m the real spherical harmonics of degree
     * <= sh_degree (0..3) in the 3DGS sign convention, sh[(sh_degree + 1)^2][3][n] in dt_color.
     * k must then be 0 and lobe_off NULL; base is not read (may be NULL). */
    const void *sh;
    int32_t sh_degree;
    int32_t reserved2;
} megs_scene;

/* FP32 gradient planes with the shapes of megs_scene's planes (compressed-row scenes: lobe planes
 * of n_lobes elements per row, same offsets); overwritten by the backward.
 * pmask_logit / lmask_logit may be NULL (and must be when the scene has no masks); sh is required
 * exactly for spherical-harmonic scenes, base for SG scenes. */
typedef struct {
    float *pos, *logscale, *quat, *op_logit, *pmask_logit;
    float *base, *axis, *sharp, *amp, *lmask_logit;
    float *sh;
} megs_scene_grad;

/* One pinhole view (host memory). R row-major world->camera, x_cam = R x + t. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float znear;
    float bg[3];
} megs_camera;

#define MEGS_FLAG_ONE_STAGE_SORT 1u /* sort 64-bit tile|depth keys in one radix sort instead of
                                       a depth pre-sort followed by a tile-only pair sort */
#define MEGS_FLAG_PERSISTENT 2u     /* blend kernels pull (view, tile) work items from a queue */
#define MEGS_FLAG_STATS 4u          /* forward also counts blended and evaluated fragments into
                                       device_status (a separate kernel instance; measurement only) */
#define MEGS_FLAG_DETERMINISTIC 8u  /* bit-reproducible backward: each (tile, Gaussian) pair's 9 gradient
                                       sums go to the pair's own slot (36 B per pair of scratch), then
                                       every record adds its slots in a fixed order; no float atomics.
                                       Set it on the forward and the backward alike. */
#define MEGS_FLAG_RECORD_PLANES 16u /* also write the per-field record planes of megs_state (mean,
                                       conic_o, rgbd, radius, cutoff, chol, ntiles) for inspection;
                                       without it those pointers are NULL (the packed records hold
                                       the same records) */

typedef struct {
    int32_t tile;          /* tile edge in pixels: 8, 16 or 32 */
    int32_t batch;         /* records staged in LDS per batch: 32, 64, 128 or 256 */
    uint32_t flags;        /* MEGS_FLAG_* */
    int32_t waves;         /* wave64s per tile workgroup: 1, 2 or 4 (1 for 8x8 tiles); 0: default
                              (1 for 8x8 tiles, 4 otherwise) */
    int64_t pair_capacity; /* 0: size the pair table from the counted pairs (one host sync per
                              forward); > 0: fixed capacity, no host sync, overflow reported
                              as MEGS_ERR_CAPACITY by megs_state_status */
    int32_t subtile;       /* 0: blend per tile (waves as above); 8: blend per 8x8 sub-tile with one
                              independent wave each, walking its 16x16 or 32x32 tile's list, so the
                              key table keeps the tile's size (the deterministic backward keeps the
                              per-tile kernel) */
    int32_t reserved;
} megs_config;

/* Allocation callback: returns device memory of at least `bytes` bytes, 256-byte aligned,
 * owned by the caller and valid until the caller drops it (the library never frees). */
typedef void *(*megs_alloc_fn)(void *ctx, size_t bytes);

/*
 * Forward state: filled by megs_render_forward, read by megs_render_backward. Every pointer is
 * device memory obtained from the allocation callback. Layouts (NR = n * n_views records,
 * record r = view * n + gaussian; P = pairs; T = tiles over all views; NP = pixels over all views):
 *   mean      double[NR][2]  pixel-space mean (u, v)          (this and conic_o, rgbd, radius,
 *                                                            cutoff, chol: MEGS_FLAG_RECORD_PLANES only)
 *   conic_o   float[NR][4]   conic (a, b, c) of q = -(a dx^2 + c dy^2)/2 - b dx dy, and o_eff
 *   rgbd      float[NR][4]   SG colour (r, g, b) and camera depth z
 *   radius    int32[NR]      footprint radius in pixels, -1 when culled
 *   ntiles    uint32[NR]     tiles of the record's rectangle that its footprint ellipse reaches
 *                            (MEGS_FLAG_RECORD_PLANES, or the deterministic mode; NULL otherwise: the
 *                            forward's own counts live in the work space below, which its pair sort
 *                            and the backward reuse)
 *   cutoff    float[NR]      k of that ellipse, {d : d' conic d <= k}; k bounds 2 ln(255 o_eff)
 *   chol      double[NR][4]  (l11, r, l22, 0): the conic as the key emission and the blend use it,
 *                            conic = L L', L = [[l11, 0], [l11 r, l22]], so that
 *                            q = (l11 (dx + r dy))^2 + (l22 dy)^2 (a sum of squares, no cancellation);
 *                            l11 = sqrt(C / det), r = -B / C, l22 = 1 / sqrt(C) for the dilated 2D
 *                            covariance [[A, B], [B, C]], det = A C - B^2, all formed in FP64; l11 and
 *                            l22 are stored as FP32, r as FP64. conic_o's (a, b, c) are the FP32
 *                            roundings of l11^2, l11^2 r, (l11 r)^2 + l22^2.
 *   tile_keys uint32[P]      sorted global tile ids (two-stage sort) or NULL; with subtile = 8 and
 *                            at most 65536 tiles, bits 16-31 flag the 8x8 sub-tiles of the tile that
 *                            the record's cutoff ellipse reaches (bit r S + c, S = tile / 8)
 *   keys64    uint64[P]      sorted tile<<32|depth keys (one-stage sort) or NULL
 *   vals      uint32[P]      sorted record indices
 *   ranges    uint32[T][2]   [start, end) of each tile in vals; (0, 0) when empty
 *   T_final   float[NP]      final transmittance per pixel
 *   last      uint32[NP]     1 + position (within its tile's list) of the last blended fragment
 *   device_status int32[8]   [0] pairs counted (at most 2^31 - 1), [1] overflow flag, [2] malformed
 *                            lobe offsets (compressed-row scenes), [3] culled records,
 *                            [4..5] uint64 blended fragments, [6..7] uint64 evaluated fragments
 *                            (written only with MEGS_FLAG_STATS)
 */
typedef struct {
    int64_t n_records, n_pairs, pair_capacity, n_pixels;
    int32_t n_views, tile, n_tiles, k;
    const void *mean, *conic_o, *rgbd, *radius, *ntiles, *cutoff;
    const void *tile_keys, *keys64, *vals, *ranges, *T_final, *last, *device_status;
    void *internal; /* library bookkeeping inside the caller's memory */
    /* deterministic mode bookkeeping (device): sorted position of each emitted pair (NULL unless
     * MEGS_FLAG_DETERMINISTIC), records in emission order (NULL: index order), the records'
     * first emission positions, and the pair count */
    const void *det_inv, *det_order, *det_offsets, *det_count;
    /* the records again, 48 bytes each (read by the key emission, the blend and the projection
     * backward, which gather records in depth and tile order): double mean[2]; double r; float l11,
     * l22 (the conic's factors, as in chol; l22 = 0 when culled); float o_eff; float rgb[3] */
    const void *packed;
    const void *chol; /* see above (MEGS_FLAG_RECORD_PLANES only) */
    /* the forward's work space (device, work_bytes bytes; NULL in deterministic mode): it holds the
     * depth sort, the scan, the key emission's tile counts and, when they
     * fit, the pair sort's alternate buffers; megs_render_backward takes its scratch from it when it is
     * large enough, so two backward calls on one state must not overlap (they would share it) */
    void *work;
    int64_t work_bytes;
} megs_state;

/* Per-view image layout: images are concatenated, view v's float[3][H][W] planes starting at
 * float offset 3 * sum_{u<v} W_u H_u. */

/*
 * Forward render of n_views views (front-to-back compositing, Sec. 3.1; SG colour, Sec. 3.2).
 * images: device float[3 * NP], written. state: host struct, filled. Returns MEGS_OK or an
 * error status; with pair_capacity == 0 it synchronises the stream once to size the pair table,
 * and returns MEGS_ERR_CAPACITY when the records list more than 2^31 - 1 tile pairs.
 */
megs_status megs_render_forward(const megs_scene *scene, const megs_camera *cams, int32_t n_views,
                                const megs_config *cfg, megs_alloc_fn alloc, void *alloc_ctx,
                                float *images, megs_state *state, void *stream);

/*
 * For callers that cannot allocate device memory (code under hipGraph capture, tight serving loops,
 * harnesses that forbid hipMalloc): megs_render_forward with its working memory (the records, sort
 * buffers, per-pixel state and pair table that megs_render_forward obtains from the allocation
 * callback) carved from one static array of MEGS_NOALLOC_SCRATCH_BYTES bytes per device instead. The
 * array lives in the library's code object: each device the library runs on holds it until the
 * process ends. The call allocates nothing; images and state are as for megs_render_forward, and the
 * state's buffers lie in the array, valid until the next call of this function on the same device
 * (megs_render_backward accepts that state). The device current on the calling thread must be the
 * stream's device. All calls on one device share its array, so calls that overlap in time on one
 * device (other streams, other threads) race: the caller serialises them.
 * pair_capacity == 0 synchronises the stream once, as megs_render_forward does; pair_capacity > 0
 * does not (overflow is then reported by megs_state_status).
 * Errors: as megs_render_forward, and MEGS_ERR_CAPACITY, before anything is launched, when the frame
 * (plus a fixed pair table) needs more than MEGS_NOALLOC_SCRATCH_BYTES, or, after the one
 * synchronisation, when the counted pairs do not fit beside it.
 */
#define MEGS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
megs_status megs_render_forward_noalloc(const megs_scene *scene, const megs_camera *cams, int32_t n_views,
                                        const megs_config *cfg, float *images, megs_state *state, void *stream);

/*
 * Backward: gradients of L with respect to every raw parameter plane, given dL/dimage
 * (dl_dimages, device float[3 * NP] in the image layout), summed over views. The blend is
 * replayed back to front from the stored final transmittance and last index; no per-fragment
 * state is kept. grads planes are overwritten. Scratch comes from alloc.
 */
megs_status megs_render_backward(const megs_scene *scene, const megs_camera *cams, int32_t n_views,
                                 const megs_config *cfg, const megs_state *state,
                                 const float *dl_dimages, megs_alloc_fn alloc, void *alloc_ctx,
                                 megs_scene_grad *grads, void *stream);

/* Reads state->device_status (synchronises the stream). Returns MEGS_ERR_CAPACITY when the
 * pair table overflowed (its capacity, or 2^31 - 1 pairs, the most a key table holds: its positions
 * are 32-bit) and MEGS_ERR_ARG when compressed-row lobe offsets were malformed; *pairs_needed receives
 * the counted pairs (may be NULL). */
megs_status megs_state_status(const megs_state *state, int64_t *pairs_needed, void *stream);

/* Device memory of one forward and backward, as megs_render_forward, megs_render_backward and
 * megs_graph_create ask the allocation callback for it (host only: nothing is launched). With
 * cfg->pair_capacity = 0, n_pairs is the count the sizing forward will find (the pair block is sized
 * for it); with a fixed capacity n_pairs is ignored. */
typedef struct {
    size_t frame;    /* first block: views, records, per-tile ranges, per-pixel state, then the work space */
    size_t pairs;    /* second block: the sorted tile keys and record indices (and, when they do not fit in
                        the work space, the sort's alternate buffers) */
    size_t backward; /* the backward's block; 0 when it takes the forward's work space */
    size_t work;     /* the part of frame that is the work space */
} megs_memory;
megs_status megs_state_bytes(const megs_scene *scene, const megs_camera *cams, int32_t n_views,
                             const megs_config *cfg, int64_t n_pairs, megs_memory *out);

/* The forward's counts (synchronises the stream): pairs the records list (saturated at 2^31 - 1),
 * records the projection culled (behind the near plane, anything non-finite, a zero quaternion or lobe
 * axis, effective opacity below 1/255, a mean or radius beyond 1e7 pixels, malformed compressed-row
 * lobes: the record takes part in no view's image), and the overflow and malformed-lobes flags. Records
 * that are valid but reach no tile of their view are not culled. */
typedef struct {
    int64_t pairs_needed;
    int64_t culled;
    int32_t overflow;
    int32_t bad_lobes;
} megs_counts;
megs_status megs_state_counts(const megs_state *state, megs_counts *out, void *stream);

/*
 * Batched form: forward (and optionally backward) of all views captured once into a hipGraph
 * and replayed with one launch. cfg->pair_capacity must be > 0. The camera table is uploaded
 * at creation; scene, images, dl_dimages and grads are read/written in place at every launch.
 * with_backward: 0 = forward only, 1 = forward + backward (dl_dimages and grads required).
 * stream must not be the null stream. Overflow is reported by megs_graph_status.
 */
typedef struct megs_graph megs_graph;

megs_status megs_graph_create(const megs_scene *scene, const megs_camera *cams, int32_t n_views,
                              const megs_config *cfg, megs_alloc_fn alloc, void *alloc_ctx,
                              float *images, const float *dl_dimages, megs_scene_grad *grads,
                              int32_t with_backward, void *stream, megs_graph **out);
/* The same call under the name of the capture step (identical arguments and behaviour). */
megs_status megs_graph_capture(const megs_scene *scene, const megs_camera *cams, int32_t n_views,
                               const megs_config *cfg, megs_alloc_fn alloc, void *alloc_ctx,
                               float *images, const float *dl_dimages, megs_scene_grad *grads,
                               int32_t with_backward, void *stream, megs_graph **out);
megs_status megs_graph_launch(megs_graph *graph, void *stream);
megs_status megs_graph_status(megs_graph *graph, int64_t *pairs_needed, void *stream);
const megs_state *megs_graph_state(const megs_graph *graph);
void megs_graph_destroy(megs_graph *graph);

/*
 * Autotuner: times forward+backward for every (tile, waves, subtile) in {(8,1,0), (16,1,0),
 * (16,2,0), (16,4,0), (32,1,0), (32,2,0), (32,4,0), (16,1,8), (32,1,8)} x batch in
 * {32, 64, 128, 256} on the given views (1 warm-up and `reps` timed runs each, HIP events on
 * `stream`) and writes the fastest configuration to *best (flags and pair_capacity copied from
 * *base). The sub-tile blends (subtile 8) stage no batches: each of those two candidates is timed
 * once, with batch 64, and its timing reported for all four batch sizes. Images are independent of
 * the choice up to FP32 rounding (the footprint lies inside the listed tiles), so the choice changes
 * speed only. ms_out (nullable) receives MEGS_AUTOTUNE_CANDIDATES timings in that order, batch
 * fastest-varying. Working memory: a sizing pass runs each candidate's front end (projection,
 * depth sort, pair count) once; then the frame, pair-table and (when needed) backward blocks are
 * taken from alloc once, each at its largest size over the candidates, and every run of the sweep
 * reuses them, so the sweep holds about one forward+backward's memory. */
#define MEGS_AUTOTUNE_CANDIDATES 36
megs_status megs_autotune(const megs_scene *scene, const megs_camera *cams, int32_t n_views,
                          const megs_config *base, megs_alloc_fn alloc, void *alloc_ctx,
                          float *images, const float *dl_dimages, megs_scene_grad *grads,
                          int32_t reps, void *stream, megs_config *best, float *ms_out);

/*
 * Per-stage timing with HIP events (eager calls only; graph capture records no events).
 * megs_profile_begin starts recording on the calling thread: every following
 * megs_render_forward / megs_render_backward on this thread brackets each stage's launches with
 * events on its stream. megs_profile_end waits for the recorded events, writes the summed
 * milliseconds and launch counts per stage, and stops recording.
 */
typedef enum {
    MEGS_STAGE_PROJECT = 0,   /* EWA projection and SG colour */
    MEGS_STAGE_DEPTH_SORT,    /* depth pre-sort of records */
    MEGS_STAGE_SCAN,          /* tile-count scan */
    MEGS_STAGE_EMIT,          /* key emission */
    MEGS_STAGE_PAIR_SORT,     /* pair sort on tile bits (or full keys) */
    MEGS_STAGE_RANGES,        /* per-tile ranges */
    MEGS_STAGE_BLEND_FWD,     /* front-to-back blend */
    MEGS_STAGE_BLEND_BWD,     /* back-to-front replay */
    MEGS_STAGE_PROJECT_BWD,   /* chain rule to raw parameters */
    MEGS_STAGE_COUNT
} megs_stage;

typedef struct {
    double ms[MEGS_STAGE_COUNT];
    int64_t count[MEGS_STAGE_COUNT];
} megs_profile;

megs_status megs_profile_begin(void);
megs_status megs_profile_end(megs_profile *out);

/*
 * ---- Memory-constrained optimisation steps (Sec. 3.3, Alg. 1; Appendix, proximal operators) ----
 * All pointers are device memory; all calls enqueue on `stream` and return without syncing.
 */

/* Forward render (as megs_render_forward) that also adds, for every Gaussian i, its blending
 * weights alpha * T summed over all pixels of all views into importance[i] (device float[n], not
 * cleared): the importance score of the Appendix's importance-based opacity selection. */
megs_status megs_render_importance(const megs_scene *scene, const megs_camera *cams, int32_t n_views,
                                   const megs_config *cfg, megs_alloc_fn alloc, void *alloc_ctx,
                                   float *images, float *importance, megs_state *state, void *stream);

/* Lobe dynamic range D = |a| (1 - exp(-2 z)) with z = sharp + lam (lam nullable) and |a| the
 * Euclidean norm of the RGB amplitude (Sec. 3.3.2, Eq. for D_i). sharp, lam, D: float[k][n];
 * amp: float[k][3][n]. */
megs_status megs_lobe_range(int64_t n, int32_t k, const float *sharp, const float *lam, const float *amp,
                            float *D, void *stream);

/* keep[i] = 1 for the kappa largest score[i] (equal scores taken in ascending index order), else
 * 0; kappa <= 0 keeps none, kappa >= n keeps all. score: float[n], keep: uint8[n]. Scratch of
 * O(n) bytes comes from alloc. The selection of both factorised proximal operators. */
megs_status megs_select_topk(const float *score, int64_t n, int64_t kappa, megs_alloc_fn alloc, void *alloc_ctx,
                             uint8_t *keep, void *stream);

/* Proximal step of Alg. 1 given the selection: x_tilde = keep ? x + lam : 0 (float[count]). */
megs_status megs_prox_apply(int64_t count, const float *x, const float *lam, const uint8_t *keep, float *x_tilde,
                            void *stream);

/* Dual update of Alg. 1: lam += x - x_tilde (float[count], lam updated in place). */
megs_status megs_dual_update(int64_t count, float *lam, const float *x, const float *x_tilde, void *stream);

/* Penalty term of the gradient step of Alg. 1: grad += delta (x - x_tilde + lam), with
 * delta = delta_o or delta_s (float[count], grad updated in place). */
megs_status megs_penalty_grad(int64_t count, float delta, const float *x, const float *x_tilde, const float *lam,
                              float *grad, void *stream);

/*
 * ---- Post-processing (Sec. 3.3, post-processing procedure; the compensation equation and its
 * derivation in the Appendix) ----
 * Keeps the Gaussians whose opacity o = sigmoid(op_logit) * sigmoid(pmask_logit) (the mask factor
 * is 1 without primitive masks) is >= opacity_min, and of those the lobes whose sharpness is
 * >= sharp_min. Every dropped lobe of a kept Gaussian adds its average over all directions,
 * m a (1 - e^{-2s}) / (2s) (a at s = 0; m its lobe mask, 1 without masks), to the base colour.
 * The masks are folded into the output, which has none: op_logit' = logit(o), amp' = m a.
 * Decisions and the compensation sum are FP64 on the stored values; each computed value is rounded
 * to FP32 and then to the plane's storage dtype; position, scale, rotation, axis and sharpness are
 * copied bit for bit. Kept Gaussians keep their order, kept lobes their order within a Gaussian.
 *
 * out->scene is the compacted scene in the compressed-row layout (same storage dtypes and k, no
 * mask planes); its planes, lobe_off, and the index maps below live in one block from alloc:
 *   kept      int32[scene.n]        source index of each kept Gaussian (ascending)
 *   lobe_src  int32[scene.n_lobes]  source element of each kept lobe in the input's sharp plane
 *                                   (dense input: l * n + i; compressed rows: the lobe index)
 * The call synchronises the stream once (to learn the output sizes). Thresholds must not be NaN.
 * Errors: MEGS_ERR_ARG for a bad scene or malformed lobe offsets, MEGS_ERR_ALLOC, MEGS_ERR_HIP.
 */
typedef struct {
    megs_scene scene;
    int32_t *kept;
    int32_t *lobe_src;
} megs_compacted;

megs_status megs_compact(const megs_scene *scene, double opacity_min, double sharp_min, megs_alloc_fn alloc,
                         void *alloc_ctx, void *stream, megs_compacted *out);

/*
 * ---- Training step around the renderer (the 3DGS loss and optimiser the paper trains with;
 * Appendix, experimental details) ----
 *
 * Photometric loss L = sum over views of (1 - lambda) mean|x - y| + lambda (1 - mean SSIM(x, y)),
 * each mean over the view's 3 channels and pixels; SSIM with an 11x11 Gaussian window of sigma 1.5,
 * zero padding, C1 = 0.01^2, C2 = 0.03^2 (3DGS uses lambda = 0.2). images and targets: device float
 * in the image layout of megs_render_forward; sizes: host int32[n_views][2] = (width, height).
 * loss: device double[1], written. dl_dimages: device float in the image layout, written with
 * dL/dimages (|.| has gradient 0 where x = y), or NULL for the loss alone. SSIM arithmetic is FP64.
 * Scratch (72 bytes per pixel) comes from alloc; the loss is deterministic.
 */
megs_status megs_photometric_loss(const float *images, const float *targets, int32_t n_views, const int32_t *sizes,
                                  double lambda_dssim, megs_alloc_fn alloc, void *alloc_ctx, double *loss,
                                  float *dl_dimages, void *stream);

/*
 * Adam step (Kingma and Ba, bias-corrected, eps added to the corrected root) on one parameter plane
 * of count elements stored as dtype (MEGS_F32, MEGS_F16 or MEGS_BF16): m = b1 m + (1 - b1) g,
 * v = b2 v + (1 - b2) g^2, p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps), in FP32,
 * the parameter rounded back to its storage dtype (nearest even). grad, m, v: device float[count];
 * m and v updated in place; step >= 1 is the 1-based step number.
 */
megs_status megs_adam_step(int64_t count, void *param, int32_t dtype, const float *grad, float *m, float *v, float lr,
                           float beta1, float beta2, float eps, int32_t step, void *stream);

/* Description of the last error on the calling thread ("" when none). */
const char *megs_last_error(void);

/* Library version string. */
const char *megs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MEGS_H */
