/*
 * qgs.h -- C ABI of libqgs, a differentiable tile rasterizer for quadric
 * (paraboloid) Gaussian primitives on AMD Instinct MI355X (gfx950).
 *
 * Method: Quadratic Gaussian Splatting (arXiv 2411.16392).  A primitive is a
 * Gaussian defined on a paraboloid patch: centre c, orientation R (a unit
 * quaternion), two tangent-plane standard deviations sigma_1, sigma_2, two
 * curvature coefficients lambda_1, lambda_2 of the explicit height
 * z = lambda_1 x^2 + lambda_2 y^2 in the local frame (Sec. 3.2, the explicit
 * form of the paraboloid and the curvature paragraph, lambda_i =
 * sign(s_i) s_3 / s_i^2), an opacity and an RGB colour.  A pixel's ray meets the
 * patch where the ray equals the paraboloid (supplement, ray-splat
 * intersection); the density at the hit is exp(-l^2 / (2 sigma(theta)^2)) with l
 * the arc length of the normal section through the vertex (Sec. 3.2, geodesic
 * and sigma(theta) equations); colour, depth and normal are alpha-composited
 * front to back (Eq. 1 and the normal/curvature render equation).
 *
 * Conventions for every entry point
 *  - All array pointers are DEVICE pointers unless stated otherwise, row-major,
 *    FP32 unless stated otherwise.  The caller owns every buffer; the library
 *    never frees caller memory and allocates nothing on these calls.
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream) unless stated otherwise, and returns a qgs_status (0 = OK,
 *    negative = error).  Arguments are validated on the host before anything is
 *    launched; on an argument error nothing is enqueued.
 *  - Invalid primitives (non-finite parameters, sigma <= 0, zero quaternion,
 *    centre at or behind the near plane) are culled, not errors.
 *  - Calls on one stream are ordered; concurrent calls on different streams may
 *    run together if they do not share output buffers.
 */
#ifndef QGS_H
#define QGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qgs_status;
#define QGS_OK               0
#define QGS_ERR_INVALID_ARG (-1) /* null pointer, n < 0, tile != 16, bad size */
#define QGS_ERR_WORKSPACE   (-2) /* workspace smaller than qgs_workspace_query says */
#define QGS_ERR_CAPACITY    (-3) /* more tile|primitive pairs than the list capacity */
#define QGS_ERR_BUDGET      (-4) /* serving: request can never fit the memory budget */
#define QGS_ERR_HIP         (-5) /* a HIP runtime call failed; see qgs_last_hip_error */
#define QGS_ERR_NOT_FOUND   (-6) /* serving: unknown request id */
#define QGS_ERR_STATE       (-7) /* serving: server stopped or request already finished */

typedef void *qgs_stream_t; /* hipStream_t */

/* Bytes of one preprocessed primitive record (see qgs_prim_buf). */
#define QGS_RECORD_BYTES 128

/* Primitive parameters (Sec. 3.2), structure of arrays, n primitives. */
typedef struct qgs_scene {
    const float *center;  /* [n][3] world-space centre c */
    const float *quat;    /* [n][4] orientation (w, x, y, z), any norm > 0; normalised internally */
    const float *scale;   /* [n][2] sigma_1, sigma_2 > 0: standard deviations along local x, y */
    const float *curv;    /* [n][2] lambda_1, lambda_2: local height z = lambda_1 x^2 + lambda_2 y^2 */
    const float *opacity; /* [n]    opacity in [0, 1] */
    const float *rgb;     /* [n][3] colour (unused, may be NULL, when sh is set) */
    int64_t n;
    /* optional view-dependent colour (the 3DGS colour model, kept by the paper,
       Sec. 3): [n][(sh_degree + 1)^2][3] real spherical-harmonics coefficients,
       sh_degree 0..3; colour = max(0, sum_k sh[k] Y_k(d) + 1/2) for the unit
       direction d from the camera centre to the primitive centre.  NULL: rgb. */
    const float *sh;
    int32_t sh_degree;
    int32_t pad;
} qgs_scene;

/* Pinhole camera (host memory).  R, t map world to camera: x_cam = R x + t,
   OpenCV axes (x right, y down, z forward).  Pixel (u, v) looks along the ray
   through ((u + 0.5 - cx) / fx, (v + 0.5 - cy) / fy, 1). */
typedef struct qgs_camera {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
} qgs_camera;

/* Rendering options (host memory).  Defaults: qgs_default_opts(). */
typedef struct qgs_render_opts {
    float near_plane; /* 0.2: centres and hits must have camera depth above it */
    float k_sigma;    /* 3: a hit is kept when l <= k_sigma * sigma(theta) (Sec. 3.2.1) */
    float alpha_min;  /* 1/255: hits with smaller alpha are skipped */
    float alpha_max;  /* 0.99: alpha = min(alpha_max, opacity * G) */
    float T_eps;      /* 1e-4: a pixel stops before blending a hit that would take T below it */
    float A_eps;      /* 1e-6: |A| below it (unit ray): nearly flat case (supplement), only the root
                         that tends to the tangent-plane intersection -C/B as A -> 0 is a candidate */
    float bg[3];      /* background colour, added with the final transmittance */
    int32_t tile;     /* must be 16 (16 x 16 tiles) */
    uint32_t flags;   /* QGS_* flags below; default QGS_TIGHT_BOUND */
    /* NULL, NULL (default), or two hipEvent_t handles created by the caller:
       qgs_render_fwd and qgs_render_bwd then record [0] on their stream just
       before their rasterizer kernel and [1] just after it (before the
       backward's deterministic reduction and preprocess adjoint), so that
       hipEventElapsedTime gives that kernel's duration alone.  The
       events stay the caller's; preprocess, bin_sort and the serving queue
       ignore them. */
    void *kernel_events[2];
} qgs_render_opts;

#define QGS_DETERMINISTIC_BWD 1u /* backward: two-pass, bit-reproducible reduction */
#define QGS_ACCUMULATE_GRADS  2u /* backward: add into qgs_scene_grads instead of overwriting */
#define QGS_COUNT_EVALS       4u /* forward: work counters into counters[2..7] */
/* The paper's full-model ordering (supplement, per-tile sorting and per-pixel
   resorting), both optional:
   QGS_TILE_DEPTH  qgs_bin_sort keys each (tile, primitive) pair by the depth at
                   which the ray through the tile's pixel nearest the projected
                   vertex meets the paraboloid (needs prims->frame).
   QGS_RESORT      the rasterizers pass accepted hits through a per-pixel buffer
                   of 8 and blend the nearest whenever it is full; the backward
                   then walks the lists front to back. */
#define QGS_TILE_DEPTH        8u
#define QGS_RESORT            16u
/* QGS_TIGHT_BOUND  qgs_preprocess bounds the support with the arc-length >=
                    chord inequality (below) instead of Q <= k^2 alone, and
                    with the cut-off where o G can still reach alpha_min for
                    faint primitives: a smaller, still conservative local box,
                    so fewer tiles and pixel tests for strongly curved or
                    faint primitives and the same image.  A provably conservative alternative to the paper's
                    tangent-plane box (supplement, bounding box calculation),
                    which can miss part of the support. */
#define QGS_TIGHT_BOUND       32u

/*
 * Per-primitive preprocess output (device memory, caller-allocated, n entries).
 *  records     n * QGS_RECORD_BYTES, 128-byte aligned.  Layout of record p as
 *              32 x 32-bit words: [0..3] pixel rectangle x0, x1, y0, y1 (int32,
 *              inclusive; x0 > x1 when empty), [4..7] projected centre split as
 *              U, 0.5 - frac(u_c), V, 0.5 - frac(v_c) (U, V integral floats),
 *              [8..11] Zc, lambda_1, lambda_2, opacity, [12..13] 1/sigma_1^2,
 *              1/sigma_2^2, [14..15] and [28..30] the screen conic a, b, c, d, e
 *              of the enclosing ellipsoid (below) in pixels relative to the
 *              projected centre, f = a dx^2 + b dx dy + c dy^2 + d dx + e dy - 1,
 *              [16..24] camera-from-local rotation row-major, [25..27] rgb,
 *              [31] zl: the centre's camera depth is Zc + zl, Zc its FP32
 *              rounding; u_c, v_c are projected at depth Zc.
 *  conic       [n][8] FP64: the image of an ellipsoid enclosing the support
 *              (c00, c01, c11, c02, c12, c22 in normalised camera coordinates),
 *              [6] 1 when it bounds the support on screen (ellipsoid in front of
 *              the near plane), [7] for a rectangle of at most 64 tiles the
 *              bits of a 64-bit integer, bit k set when the k-th tile
 *              (row-major) is kept, else 0: the tile decisions of
 *              qgs_preprocess, which qgs_bin_sort emits from instead of
 *              repeating the test.  Tiles of the rectangle that miss the conic
 *              are not emitted.
 *  depth_key   [n] FP32 bit pattern of the centre's camera-space depth (0 if culled)
 *  rect        [n][4] tile rectangle tx0, ty0, tx1, ty1 inclusive; (0, 0, -1, -1) if empty
 *  tiles       [n] number of tiles emitted (0 if culled or off screen)
 *  pair_offset [n] written by qgs_bin_sort: index of the primitive's first pair
 *              in emission order (pairs of one primitive are contiguous there)
 */
typedef struct qgs_prim_buf {
    void *records;
    uint32_t *depth_key;
    int32_t *rect;
    uint32_t *tiles;
    uint32_t *pair_offset;
    double *conic;
    int64_t n;
    /* optional (NULL: not written): [n][16] FP64 camera frame for the per-tile
       sort depth: c_cam[3], camera-from-local rotation [9] row-major, projected
       vertex u, v, lambda_1, lambda_2 */
    double *frame;
} qgs_prim_buf;

/*
 * Sorted tile lists (device memory, caller-allocated).
 *  pair_tile, pair_prim  [capacity] tile id and primitive index of each pair,
 *                        sorted by (tile, depth key, primitive index)
 *  emit_to_sorted        optional (NULL: not built): [capacity] position in
 *                        the sorted list of each pair, indexed by emission
 *                        order (primitive p's pairs are pair_offset[p] ...
 *                        pair_offset[p] + tiles[p] - 1).  The deterministic
 *                        backward needs it, and it must then have been set for
 *                        the qgs_bin_sort that built the lists; building it
 *                        costs a random gather and scatter over all pairs.
 *  ranges                [tiles_x * tiles_y][2] start, end of each tile's run
 *  tile_order            [tiles_x * tiles_y] tiles by decreasing forward work
 *                        (exact below 2048, then classes 16 wide up to 34800):
 *                        the order in which the rasterizer's workgroups take
 *                        tiles, so the costliest start first.  The work of a
 *                        tile is the largest, over its four 8 x 8 blocks, count
 *                        of its entries whose pixel rectangle and screen conic
 *                        (the forward's per-block filter) meet the block;
 *                        with QGS_TILE_DEPTH, and for the serving queue, the
 *                        list length
 *  counters              [8] uint32: [0] number of pairs, [1] overflow flag
 *                        (1 when [0] > capacity: lists and ranges are then empty
 *                        and the caller must grow and call again); with
 *                        QGS_COUNT_EVALS the forward adds [2] list entries
 *                        processed per pixel up to and including a stop, summed
 *                        over pixels, [3] (pixel, primitive) pairs whose
 *                        intersection was evaluated, [4] pairs blended, [5]
 *                        (wave, entry) steps whose rectangle meets the wave's
 *                        8 x 8 pixel block, [6] steps in which at least one lane
 *                        evaluated an intersection, [7] steps in which at least
 *                        one lane blended.
 *                        qgs_bin_sort resets [2..7] to zero.
 */
typedef struct qgs_tile_lists {
    uint32_t *pair_tile;
    uint32_t *pair_prim;
    uint32_t *emit_to_sorted;
    uint32_t *ranges;
    uint32_t *tile_order;
    uint32_t *counters;
    uint64_t capacity;
} qgs_tile_lists;

/*
 * Forward outputs, planar, [c][height][width].  w = alpha T is an entry's
 * blending weight and t its hit depth along the unit ray.
 * color is required.  depth and normal are optional together (both NULL:
 * colour-only rendering, which skips the normal computation); T_final and
 * last may be NULL (not written), but the backward needs both.  The four
 * geometry maps are optional: either all four pointers are NULL (not computed,
 * no cost) or all four are set, and then depth and normal must be set too.
 */
typedef struct qgs_images {
    float *color;    /* [3][H][W] sum w rgb + T_final bg */
    float *depth;    /* [H][W] sum w t */
    float *normal;   /* [3][H][W] sum w n, camera-space unit normals facing the camera */
    float *T_final;  /* [H][W] final transmittance */
    uint32_t *last;  /* [H][W] 1 + position in the tile list of the last blended entry (0: none) */
    /* curvature map (normal and curvature render equation, Sec. 3.2.1): sum w K,
       K = 4 l1 l2 / (1 + 4 l1^2 x^2 + 4 l2^2 y^2)^2 the Gaussian curvature at the hit */
    float *curvature;       /* [H][W] */
    /* median depth (output depth of the experiments, Sec. 4.1): the largest t
       among blended entries whose incoming transmittance exceeds 0.5 (0: none) */
    float *median_depth;    /* [H][W] */
    /* depth distortion (Sec. 3.3): sum_i sum_{j<i} w_i w_j (t_i - t_j)^2,
       accumulated in the running-mean form L += w (L/W + W (t - mean)^2) */
    float *distortion;      /* [H][W] */
    uint32_t *median_pos;   /* [H][W] 1 + tile-list position of the median entry (0: none) */
    /* optional replay bitmap for the backward (both or neither).  For 8 x 8
       pixel block b (0..3, row-major) of tile t, whose list is
       [start_t, start_t + len_t): bit j of word w is set when at least one of
       the block's pixels blended list entry 64 w + j (with QGS_RESORT: took it
       into its resort buffer).  The block's words start at
       steps[4 (floor(start_t / 64) + t) + b ceil(len_t / 64)];
       step_count[4 t + b] is the number of words written.  `steps` holds
       4 (ceil(capacity / 64) + tiles + 1) words.  The backward then visits only
       the marked entries (the others change nothing) and gives the same
       gradients.  The backward must get the bitmap of the same forward. */
    uint64_t *steps;
    uint32_t *step_count;   /* [4 * tiles] */
} qgs_images;

/* Upstream gradients, same layouts; a NULL plane means zero.  Any non-NULL
   geometry plane needs the geometry maps of the matching forward. */
typedef struct qgs_image_grads {
    const float *dcolor;
    const float *ddepth;
    const float *dnormal;
    const float *dcurvature;
    const float *dmedian_depth;
    const float *ddistortion;
} qgs_image_grads;

/* Parameter gradients, same shapes as qgs_scene. */
typedef struct qgs_scene_grads {
    float *center;
    float *quat;
    float *scale;
    float *curv;
    float *opacity;
    float *rgb;          /* the colour's gradient (after the SH evaluation when sh is set) */
    float *sh;           /* [n][K][3]; required when the scene has sh */
    /* optional densification statistics (both or neither), ADDED to, never
       overwritten: screen_grad[p] += |(W/2 z/fx g_x, H/2 z/fy g_y)| with g the
       centre gradient in camera axes and z the centre depth, i.e. the gradient
       with respect to the centre's image position in normalised device units
       (the 3D centre gradient projected to the screen, Sec. 4 implementation
       details); visible[p] += 1 when p covers a tile */
    float *screen_grad;
    float *visible;
} qgs_scene_grads;

/* Human-readable text for a status code (static storage). */
const char *qgs_status_string(qgs_status status);

/* Last HIP error code seen by this thread (0 if none). */
int32_t qgs_last_hip_error(void);

/* Build stamp: a hash of the sources and flags the library was compiled from
   (static storage; "unstamped" when built without one).  Bindings compare it
   with the sources they ship beside, so that a stale binary is refused. */
const char *qgs_build_id(void);

/* Fill *opts with the defaults listed in qgs_render_opts. Host only. */
void qgs_default_opts(qgs_render_opts *opts);

/*
 * Host-only size query.  For n primitives, a camera and a pair capacity:
 *  sort_ws_bytes  workspace of qgs_bin_sort
 *  bwd_ws_bytes   workspace of qgs_render_bwd for `flags`: the record
 *                 gradients (64 bytes per primitive) and the backward's order
 *                 of its 8 x 8 blocks with their costs (32 bytes per tile of
 *                 the camera); QGS_DETERMINISTIC_BWD
 *                 adds capacity * 256 bytes: one partial per pair and 8 x 8 block
 * Any output pointer may be NULL.
 */
qgs_status qgs_workspace_query(int64_t n, const qgs_camera *cam, uint64_t pair_capacity, uint32_t flags,
                               size_t *sort_ws_bytes, size_t *bwd_ws_bytes);

/*
 * Projection, culling and conservative screen bounds, one thread per primitive
 * (Sec. 3.2 congruent transform; supplement, bounding boxes).  Writes records,
 * depth_key, rect, tiles and conic of `out`.  The bounds hold every pixel whose
 * ray can meet the primitive inside k_sigma.  Since the arc-length factor is
 * >= 1, an accepted hit has |x| <= k sigma_1, |y| <= k sigma_2 and a height
 * between the extremes of lambda_1 x^2 + lambda_2 y^2 over that ellipse, capped
 * at k max(sigma).  With QGS_TIGHT_BOUND the arc is also at least its chord, so
 * Q + z^2 / max(sigma)^2 <= k^2, whose extremes in x, y and z give a smaller
 * box.  The rectangle is the projection of the part of this (slightly
 * inflated) local box in front of the near plane -- its corners there and the
 * points where its edges cross the plane -- and is empty when no corner is in
 * front; tiles of it are kept only if they meet the projection of an ellipsoid
 * enclosing the box's elliptic cylinder (when that ellipsoid lies in front of
 * the near plane).  Errors: QGS_ERR_INVALID_ARG.
 */
qgs_status qgs_preprocess(const qgs_scene *scene, const qgs_camera *cam, const qgs_render_opts *opts,
                          qgs_prim_buf *out, qgs_stream_t stream);

/*
 * Tile|depth key lists (supplement, per-tile sorting: one global sort keyed by
 * tile and depth).  Produces, for every tile, the primitives whose rectangle
 * covers it, ordered by depth key and then primitive index, bit-identical to a
 * stable sort of the 64-bit keys (tile << 32 | depth_key) emitted primitive by
 * primitive, tiles row-major within each rectangle.  Integer-only: a radix sort
 * of the depth keys, emission in that order, then a stable radix sort by tile.
 * Also writes prims->pair_offset and lists->counters.
 * host_num_pairs: if non-NULL the call synchronises `stream` once and stores the
 * pair count there, and returns QGS_ERR_CAPACITY if it exceeds the capacity; if
 * NULL the call never synchronises and the overflow is reported on the device
 * (counters[1]).  Errors: QGS_ERR_INVALID_ARG, QGS_ERR_WORKSPACE, QGS_ERR_CAPACITY.
 */
qgs_status qgs_bin_sort(qgs_prim_buf *prims, const qgs_camera *cam, const qgs_render_opts *opts,
                        qgs_tile_lists *lists, void *ws, size_t ws_bytes, uint64_t *host_num_pairs,
                        qgs_stream_t stream);

/*
 * Forward rasterizer: one 256-thread workgroup per 16 x 16 tile, each wave64
 * an 8 x 8 pixel block that walks the tile's list on its own; per-pixel
 * ray-paraboloid intersection with near/far root selection and the k_sigma
 * geodesic cut-off, geodesic Gaussian density, front-to-back compositing with
 * stop once T would fall below T_eps.  Writes all planes of `out`; depth and
 * normal only if set (both or neither), T_final, last and the replay list only
 * if set, the geometry maps only if they are set (all four or none).  With
 * QGS_RESORT, accepted hits pass through the per-pixel buffer (depth and
 * normal planes required) and `last` is 1 + the list position of the last hit
 * the pixel took in.  Errors: QGS_ERR_INVALID_ARG.
 */
qgs_status qgs_render_fwd(const qgs_prim_buf *prims, const qgs_tile_lists *lists, const qgs_camera *cam,
                          const qgs_render_opts *opts, qgs_images *out, qgs_stream_t stream);

/*
 * Backward: adjoint of qgs_render_fwd and qgs_preprocess.  Each tile's list is
 * walked back to front from each pixel's `last` entry (only the replay bitmap's
 * entries when `fwd` carries one; the tiles then run in decreasing order of
 * the entries their blocks' bitmaps hold), recomputing transmittance by division
 * (supplement, back-to-front adjoint), with per-primitive gradients reduced
 * across each 8 x 8 block's pixels in registers before one global atomic per
 * field per (block, primitive); QGS_DETERMINISTIC_BWD instead stores one
 * partial per (pair, block) and sums each primitive's partials in a fixed
 * order.  Then the chain rule to the scene parameters, one thread per
 * primitive.  With QGS_RESORT the lists are walked front to back instead,
 * replaying each pixel's resort buffer up to its `last` (supplement,
 * front-to-back form of the adjoint), and `fwd` must also hold the forward's
 * colour, depth and normal (and curvature with geometry gradients).
 * `fwd` must hold T_final and last from the matching forward, and
 * with any geometry gradient also its depth, distortion and median_pos (the
 * distortion adjoint needs the pixel's sum of weights, 1 - T_final, its mean
 * depth and its distortion; the median's gradient goes to the median entry).
 * ws: at least bwd_ws_bytes from qgs_workspace_query.
 * Errors: QGS_ERR_INVALID_ARG, QGS_ERR_WORKSPACE.
 */
qgs_status qgs_render_bwd(const qgs_scene *scene, const qgs_prim_buf *prims, const qgs_tile_lists *lists,
                          const qgs_camera *cam, const qgs_render_opts *opts, const qgs_images *fwd,
                          const qgs_image_grads *dL, qgs_scene_grads *out, void *ws, size_t ws_bytes,
                          qgs_stream_t stream);

/*
 * Backward without a caller workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving or training loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * qgs_render_bwd; the workspace is instead a static device array of
 * QGS_BWD_STATIC_BYTES that the library holds on each device it runs on until
 * the process ends.  Allocates nothing.
 * Limit: bwd_ws_bytes of qgs_workspace_query for (n, camera, capacity, flags)
 * must not exceed QGS_BWD_STATIC_BYTES (64 MiB: about 1M primitives at 1080p
 * without QGS_DETERMINISTIC_BWD, whose pair partials add 256 bytes per pair of
 * capacity); larger calls return QGS_ERR_WORKSPACE and launch nothing.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (the backward clears what it accumulates into): calls that
 * overlap on one device, on different streams or from different threads, race
 * and must be serialised by the caller.
 * Errors: QGS_ERR_INVALID_ARG, QGS_ERR_WORKSPACE, QGS_ERR_HIP.
 */
#define QGS_BWD_STATIC_BYTES ((size_t)64 << 20)
qgs_status qgs_render_bwd_static(const qgs_scene *scene, const qgs_prim_buf *prims, const qgs_tile_lists *lists,
                                 const qgs_camera *cam, const qgs_render_opts *opts, const qgs_images *fwd,
                                 const qgs_image_grads *dL, qgs_scene_grads *out, qgs_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of novel-view render requests               */
/* ------------------------------------------------------------------------ */

/*
 * A server keeps a scene resident in HBM and renders colour images of
 * requested views as they arrive.  Each request runs a count pass (preprocess,
 * depth sort, pair offsets) and is then admitted for rendering once the exact
 * memory its tile lists need is free in a pool of `budget_bytes`; requests are
 * admitted in arrival order as slots and memory free up, while earlier ones are
 * still on the device, and the requests in flight are spread over `n_streams`
 * HIP streams so their kernels overlap.  One scheduler thread owns all device
 * work.  qgs_serve_create and qgs_serve_destroy allocate and free the server's
 * pools; submit, poll and cancel only touch host queues and may be called from
 * any one client thread.
 */
typedef struct qgs_server qgs_server;

typedef struct qgs_serve_config {
    int64_t budget_bytes;            /* device bytes for per-request tile lists and sort temporaries */
    int32_t max_slots;               /* requests in flight (count pass or rendering) */
    int32_t max_width, max_height;   /* largest view accepted */
    int32_t n_streams;               /* HIP streams used by the scheduler (default priority) */
    int32_t device;                  /* HIP device ordinal */
    qgs_render_opts opts;
    uint32_t flags;                  /* QGS_SERVE_* below */
    uint32_t pad;
} qgs_serve_config;

/* Launch each request's work directly instead of through the slot's
   persistent graphs (for comparison). */
#define QGS_SERVE_NO_GRAPHS 1u

#define QGS_REQ_DONE      0
#define QGS_REQ_CANCELLED 1
#define QGS_REQ_FAILED    2

typedef struct qgs_completion {
    uint64_t req_id;
    int32_t state;     /* QGS_REQ_* */
    int32_t status;    /* qgs_status of a failed request (QGS_ERR_BUDGET: can never fit) */
    double t_submit;   /* seconds on the server clock (qgs_serve_clock) */
    double t_admit;    /* rendering admitted (memory reserved) */
    double t_done;     /* result complete in the caller's buffer */
    uint64_t num_pairs;
} qgs_completion;

typedef struct qgs_serve_stats {
    uint64_t submitted, completed, cancelled, failed;
    uint64_t peak_pool_bytes;   /* high-water mark of reserved list memory */
    int32_t peak_in_flight;     /* most requests on the device at once */
    int32_t pad;
    uint64_t graph_launches;    /* count and render passes launched as graphs */
    uint64_t graph_builds;      /* graphs instantiated (the rest were updated in place) */
} qgs_serve_stats;

/* scene: device arrays that must outlive the server.  Errors:
   QGS_ERR_INVALID_ARG, QGS_ERR_HIP (allocation failed). */
qgs_status qgs_serve_create(const qgs_scene *scene, const qgs_serve_config *cfg, qgs_server **out);

/* Queue a request; the colour image [3][height][width] FP32 is written to
   out_rgb (device, caller-owned, must stay valid until its completion is
   polled).  Errors: QGS_ERR_INVALID_ARG (bad camera or larger than max view),
   QGS_ERR_STATE (server stopping). */
qgs_status qgs_serve_submit(qgs_server *srv, const qgs_camera *cam, float *out_rgb, uint64_t *req_id);

/* Up to `max` completions in completion order; waits up to timeout_us for the
   first one (0: no wait). */
qgs_status qgs_serve_poll(qgs_server *srv, qgs_completion *out, int32_t max, int32_t *n, int32_t timeout_us);

/* Cancel a request that has not been admitted for rendering; its completion
   reports QGS_REQ_CANCELLED.  QGS_ERR_NOT_FOUND if unknown or already done,
   QGS_ERR_STATE if already rendering. */
qgs_status qgs_serve_cancel(qgs_server *srv, uint64_t req_id);

qgs_status qgs_serve_stats_get(qgs_server *srv, qgs_serve_stats *out);

/* Seconds on the server's steady clock. */
double qgs_serve_clock(qgs_server *srv);

/* Finishes the work in flight, stops the scheduler, frees the pools. */
qgs_status qgs_serve_destroy(qgs_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* QGS_H */
