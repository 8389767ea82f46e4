// C ABI of libqgs: argument checks, workspace layout and kernel launches.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <mutex>

#include "qgs.h"
#include "qgs_internal.hpp"

using namespace qgs;

namespace {

thread_local int32_t g_last_hip = 0;

qgs_status hip_status(hipError_t e)
{
    if (e == hipSuccess) return QGS_OK;
    g_last_hip = (int32_t)e;
    return QGS_ERR_HIP;
}

bool cam_ok(const qgs_camera *c)
{
    if (!c || c->width <= 0 || c->height <= 0) return false;
    if ((int64_t)c->width * c->height > (int64_t)1 << 31) return false;
    if (!(isfinite(c->fx) && isfinite(c->fy) && isfinite(c->cx) && isfinite(c->cy))) return false;
    if (!(c->fx > 0.0f) || !(c->fy > 0.0f)) return false;
    for (int i = 0; i < 9; ++i)
        if (!isfinite(c->R[i])) return false;
    for (int i = 0; i < 3; ++i)
        if (!isfinite(c->t[i])) return false;
    return true;
}

bool opts_ok(const qgs_render_opts *o)
{
    return o && o->tile == 16 && o->near_plane > 0.0f && o->k_sigma > 0.0f && o->alpha_max > 0.0f &&
           o->alpha_max < 1.0f && o->alpha_min >= 0.0f && o->T_eps >= 0.0f && o->A_eps >= 0.0f &&
           isfinite(o->bg[0]) && isfinite(o->bg[1]) && isfinite(o->bg[2]);
}

bool scene_ok(const qgs_scene *s)
{
    if (!s || s->n < 0 || s->n > 0x7FFFFFFFll) return false;
    if (s->n == 0) return true;
    if (s->sh && (s->sh_degree < 0 || s->sh_degree > 3)) return false;
    return s->center && s->quat && s->scale && s->curv && s->opacity && (s->rgb || s->sh);
}

bool prims_ok(const qgs_prim_buf *p, int64_t n)
{
    if (!p || p->n != n) return false;
    if (n == 0) return true;
    return p->records && ((uintptr_t)p->records % 16 == 0) && p->depth_key && p->rect && p->tiles && p->pair_offset &&
           p->conic;
}

bool lists_ok(const qgs_tile_lists *l)
{
    if (!l || !l->ranges || !l->counters) return false;
    if (l->capacity > 0xFFFFFFFFull) return false;
    if (l->capacity > 0 && (!l->pair_tile || !l->pair_prim)) return false;
    return true;
}

RasterParams raster_params(const qgs_camera *c, const qgs_render_opts *o)
{
    RasterParams p;
    p.fx = c->fx;
    p.fy = c->fy;
    p.cx = c->cx;
    p.cy = c->cy;
    p.ifx = 1.0f / c->fx;
    p.ify = 1.0f / c->fy;
    p.width = c->width;
    p.height = c->height;
    p.tiles_x = (c->width + 15) / 16;
    p.tiles_y = (c->height + 15) / 16;
    p.near_plane = o->near_plane;
    p.k2 = o->k_sigma * o->k_sigma;
    p.alpha_min = o->alpha_min;
    p.alpha_max = o->alpha_max;
    p.T_eps = o->T_eps;
    p.A_eps = o->A_eps;
    p.bg[0] = o->bg[0];
    p.bg[1] = o->bg[1];
    p.bg[2] = o->bg[2];
    p.flags = o->flags;
    return p;
}

RasterArgs raster_args(const qgs_prim_buf *prims, const qgs_tile_lists *lists, const qgs_camera *c)
{
    RasterArgs a{};
    a.records = reinterpret_cast<const float *>(prims->records);
    a.pair_prim = lists->pair_prim;
    a.pair_tile = lists->pair_tile;
    a.ranges = lists->ranges;
    a.tile_order = lists->tile_order;
    a.counters = lists->counters;
    a.pair_offset = prims->pair_offset;
    a.tiles = prims->tiles;
    a.emit_to_sorted = lists->emit_to_sorted;
    a.tiles_x = (c->width + 15) / 16;
    a.tiles_y = (c->height + 15) / 16;
    return a;
}

// backward workspace: record gradients [n][16] f32; the backward's tile cost
// and order [2][tiles] u32; deterministic mode: one 16-float partial per
// (pair, wave of the tile)
size_t bwd_grad_bytes(int64_t n) { return ((size_t)(n > 0 ? n : 1) * 64 + 255) & ~(size_t)255; }
size_t bwd_order_bytes(uint64_t ntiles) { return ((size_t)(ntiles > 0 ? ntiles : 1) * 32 + 255) & ~(size_t)255; }

size_t bwd_bytes(int64_t n, uint64_t capacity, uint32_t flags, uint64_t ntiles)
{
    size_t b = bwd_grad_bytes(n) + bwd_order_bytes(ntiles);
    if (flags & QGS_DETERMINISTIC_BWD) b += (size_t)(capacity > 0 ? capacity : 1) * 256;
    return b;
}

}  // namespace

extern "C" {

const char *qgs_status_string(qgs_status s)
{
    switch (s) {
    case QGS_OK: return "ok";
    case QGS_ERR_INVALID_ARG: return "invalid argument";
    case QGS_ERR_WORKSPACE: return "workspace too small";
    case QGS_ERR_CAPACITY: return "tile list capacity exceeded";
    case QGS_ERR_BUDGET: return "request exceeds the memory budget";
    case QGS_ERR_HIP: return "HIP runtime error";
    case QGS_ERR_NOT_FOUND: return "unknown request";
    case QGS_ERR_STATE: return "invalid state";
    default: return "unknown status";
    }
}

int32_t qgs_last_hip_error(void) { return g_last_hip; }

#ifndef QGS_BUILD_ID
#define QGS_BUILD_ID "unstamped"
#endif

const char *qgs_build_id(void) { return QGS_BUILD_ID; }

void qgs_default_opts(qgs_render_opts *o)
{
    if (!o) return;
    o->near_plane = 0.2f;
    o->k_sigma = 3.0f;
    o->alpha_min = 1.0f / 255.0f;
    o->alpha_max = 0.99f;
    o->T_eps = 1e-4f;
    o->A_eps = 1e-6f;
    o->bg[0] = o->bg[1] = o->bg[2] = 0.0f;
    o->tile = 16;
    o->flags = QGS_TIGHT_BOUND;
    o->kernel_events[0] = o->kernel_events[1] = nullptr;
}

qgs_status qgs_workspace_query(int64_t n, const qgs_camera *cam, uint64_t capacity, uint32_t flags,
                               size_t *sort_ws_bytes, size_t *bwd_ws_bytes)
{
    if (n < 0 || n > 0x7FFFFFFFll || !cam_ok(cam) || capacity > 0xFFFFFFFFull) return QGS_ERR_INVALID_ARG;
    const uint64_t ntiles = (uint64_t)((cam->width + 15) / 16) * (uint64_t)((cam->height + 15) / 16);
    if (sort_ws_bytes) *sort_ws_bytes = sort_workspace_layout(nullptr, n, capacity, ntiles).bytes;
    if (bwd_ws_bytes) *bwd_ws_bytes = bwd_bytes(n, capacity, flags, ntiles);
    return QGS_OK;
}

qgs_status qgs_preprocess(const qgs_scene *scene, const qgs_camera *cam, const qgs_render_opts *opts,
                          qgs_prim_buf *out, qgs_stream_t stream)
{
    if (!scene_ok(scene) || !cam_ok(cam) || !opts_ok(opts) || !prims_ok(out, scene->n)) return QGS_ERR_INVALID_ARG;
    PreprocessArgs a;
    a.center = scene->center;
    a.quat = scene->quat;
    a.scale = scene->scale;
    a.curv = scene->curv;
    a.opacity = scene->opacity;
    a.rgb = scene->rgb;
    a.n = scene->n;
    a.cam = *cam;
    a.near_plane = opts->near_plane;
    a.k_sigma = opts->k_sigma;
    a.alpha_min = opts->alpha_min;
    a.records = out->records;
    a.depth_key = out->depth_key;
    a.rect = out->rect;
    a.tiles = out->tiles;
    a.conic = out->conic;
    a.frame = out->frame;
    a.sh = scene->sh;
    a.sh_degree = scene->sh ? scene->sh_degree : -1;
    a.tight = (opts->flags & QGS_TIGHT_BOUND) ? 1 : 0;
    return hip_status(launch_preprocess(a, (hipStream_t)stream));
}

qgs_status qgs_bin_sort(qgs_prim_buf *prims, const qgs_camera *cam, const qgs_render_opts *opts,
                        qgs_tile_lists *lists, void *ws, size_t ws_bytes, uint64_t *host_num_pairs,
                        qgs_stream_t stream)
{
    if (!prims || !cam_ok(cam) || !opts_ok(opts) || !prims_ok(prims, prims->n) || !lists_ok(lists))
        return QGS_ERR_INVALID_ARG;
    const uint64_t ntiles = (uint64_t)((cam->width + 15) / 16) * (uint64_t)((cam->height + 15) / 16);
    const SortWorkspace need = sort_workspace_layout(nullptr, prims->n, lists->capacity, ntiles);
    if (!ws || ws_bytes < need.bytes) return QGS_ERR_WORKSPACE;
    const SortWorkspace w = sort_workspace_layout(ws, prims->n, lists->capacity, ntiles);
    BinSortArgs a;
    a.n = prims->n;
    a.depth_key = prims->depth_key;
    a.tiles = prims->tiles;
    a.rect = prims->rect;
    a.conic = prims->conic;
    a.cam = *cam;
    a.pair_offset = prims->pair_offset;
    a.tiles_x = (cam->width + 15) / 16;
    a.tiles_y = (cam->height + 15) / 16;
    a.pair_tile = lists->pair_tile;
    a.pair_prim = lists->pair_prim;
    a.emit_to_sorted = lists->emit_to_sorted;
    a.ranges = lists->ranges;
    a.tile_order = lists->tile_order;
    a.counters = lists->counters;
    a.capacity = lists->capacity;
    a.frame = (opts->flags & QGS_TILE_DEPTH) ? prims->frame : nullptr;
    a.near_plane = opts->near_plane;
    a.records = reinterpret_cast<const float *>(prims->records);
    if ((opts->flags & QGS_TILE_DEPTH) && !prims->frame) return QGS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    qgs_status st = hip_status(bin_sort_phase1(a, w, s));
    if (st != QGS_OK) return st;
    uint64_t bound = lists->capacity;
    bool overflow = false;
    if (host_num_pairs) {
        uint32_t c[2] = {0, 0};
        st = hip_status(hipMemcpyAsync(c, lists->counters, sizeof c, hipMemcpyDeviceToHost, s));
        if (st != QGS_OK) return st;
        st = hip_status(hipStreamSynchronize(s));
        if (st != QGS_OK) return st;
        *host_num_pairs = c[0];
        overflow = c[1] != 0;
        bound = overflow ? 0 : c[0];
    }
    st = hip_status(bin_sort_phase2(a, w, bound, s));
    if (st != QGS_OK) return st;
    return overflow ? QGS_ERR_CAPACITY : QGS_OK;
}

qgs_status qgs_render_fwd(const qgs_prim_buf *prims, const qgs_tile_lists *lists, const qgs_camera *cam,
                          const qgs_render_opts *opts, qgs_images *out, qgs_stream_t stream)
{
    if (!prims || !prims_ok(prims, prims->n) || !lists_ok(lists) || !cam_ok(cam) || !opts_ok(opts) || !out)
        return QGS_ERR_INVALID_ARG;
    // depth and normal: both or neither (colour-only rendering)
    if (!out->color || (out->depth == nullptr) != (out->normal == nullptr)) return QGS_ERR_INVALID_ARG;
    const int n_geo = (out->curvature != nullptr) + (out->median_depth != nullptr) + (out->distortion != nullptr) +
                      (out->median_pos != nullptr);
    if (n_geo != 0 && n_geo != 4) return QGS_ERR_INVALID_ARG;
    if (n_geo == 4 && !out->depth) return QGS_ERR_INVALID_ARG;
    if ((opts->flags & QGS_RESORT) && !out->depth) return QGS_ERR_INVALID_ARG;
    if ((out->steps == nullptr) != (out->step_count == nullptr)) return QGS_ERR_INVALID_ARG;
    FwdOut o;
    o.flags = opts->flags;
    o.color = out->color;
    o.depth = out->depth;
    o.normal = out->normal;
    o.T_final = out->T_final;
    o.last = out->last;
    o.counters = (opts->flags & QGS_COUNT_EVALS) ? lists->counters : nullptr;
    o.curvature = out->curvature;
    o.median_depth = out->median_depth;
    o.distortion = out->distortion;
    o.median_pos = out->median_pos;
    o.steps = out->steps;
    o.step_count = out->step_count;
    o.ev_begin = (hipEvent_t)opts->kernel_events[0];
    o.ev_end = (hipEvent_t)opts->kernel_events[1];
    return hip_status(launch_render_fwd(raster_args(prims, lists, cam), raster_params(cam, opts), o,
                                        (hipStream_t)stream));
}

}  // extern "C"

namespace {

qgs_status render_bwd_impl(const qgs_scene *scene, const qgs_prim_buf *prims, const qgs_tile_lists *lists,
                           const qgs_camera *cam, const qgs_render_opts *opts, const qgs_images *fwd,
                           const qgs_image_grads *dL, qgs_scene_grads *out, void *ws, size_t ws_bytes,
                           qgs_stream_t stream)
{
    if (!scene_ok(scene) || !prims || !prims_ok(prims, scene->n) || !lists_ok(lists) || !cam_ok(cam) ||
        !opts_ok(opts) || !fwd || !fwd->T_final || !fwd->last || !dL || !out)
        return QGS_ERR_INVALID_ARG;
    if (scene->n > 0 && (!out->center || !out->quat || !out->scale || !out->curv || !out->opacity || !out->rgb))
        return QGS_ERR_INVALID_ARG;
    if (scene->n > 0 && scene->sh && !out->sh) return QGS_ERR_INVALID_ARG;
    if ((out->screen_grad == nullptr) != (out->visible == nullptr)) return QGS_ERR_INVALID_ARG;
    const bool geo = dL->dcurvature || dL->dmedian_depth || dL->ddistortion;
    if (geo && (!fwd->depth || !fwd->distortion || !fwd->median_pos)) return QGS_ERR_INVALID_ARG;
    const bool det = (opts->flags & QGS_DETERMINISTIC_BWD) != 0;
    if (det && lists->capacity > 0 && !lists->emit_to_sorted) return QGS_ERR_INVALID_ARG;
    // the front-to-back adjoint of the resort mode needs every composited output
    if ((opts->flags & QGS_RESORT) && (!fwd->color || !fwd->depth || !fwd->normal)) return QGS_ERR_INVALID_ARG;
    if ((opts->flags & QGS_RESORT) && geo && !fwd->curvature) return QGS_ERR_INVALID_ARG;
    if ((fwd->steps == nullptr) != (fwd->step_count == nullptr)) return QGS_ERR_INVALID_ARG;
    const uint64_t ntiles = (uint64_t)((cam->width + 15) / 16) * (uint64_t)((cam->height + 15) / 16);
    if (!ws || ws_bytes < bwd_bytes(scene->n, lists->capacity, opts->flags, ntiles)) return QGS_ERR_WORKSPACE;
    float *grad_rec = reinterpret_cast<float *>(ws);
    const size_t off = bwd_grad_bytes(scene->n);
    uint32_t *order_ws = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(ws) + off);
    const size_t off2 = off + bwd_order_bytes(ntiles);
    float *pair_partials = det ? reinterpret_cast<float *>(reinterpret_cast<char *>(ws) + off2) : nullptr;
    hipStream_t s = (hipStream_t)stream;
    BwdIn in;
    in.T_final = fwd->T_final;
    in.last = fwd->last;
    in.dcolor = dL->dcolor;
    in.ddepth = dL->ddepth;
    in.dnormal = dL->dnormal;
    in.dcurvature = dL->dcurvature;
    in.dmedian = dL->dmedian_depth;
    in.ddistortion = dL->ddistortion;
    in.depth = fwd->depth;
    in.distortion = fwd->distortion;
    in.median_pos = fwd->median_pos;
    in.color = fwd->color;
    in.normal = fwd->normal;
    in.curvature = fwd->curvature;
    in.steps = fwd->steps;
    in.step_count = fwd->step_count;
    in.flags = opts->flags;
    in.ev_begin = (hipEvent_t)opts->kernel_events[0];
    in.ev_end = (hipEvent_t)opts->kernel_events[1];
    qgs_status st = hip_status(launch_render_bwd(raster_args(prims, lists, cam), raster_params(cam, opts), in,
                                                 grad_rec, pair_partials, order_ws, scene->n, lists->capacity, s));
    if (st != QGS_OK) return st;
    PreprocessBwdArgs b;
    b.center = scene->center;
    b.quat = scene->quat;
    b.scale = scene->scale;
    b.sh = scene->sh;
    b.sh_degree = scene->sh ? scene->sh_degree : -1;
    b.n = scene->n;
    b.cam = *cam;
    b.grad_rec = grad_rec;
    b.tiles = prims->tiles;
    b.out = *out;
    b.accumulate = (opts->flags & QGS_ACCUMULATE_GRADS) ? 1 : 0;
    return hip_status(launch_preprocess_bwd(b, s));
}

// Backward workspace of qgs_render_bwd_static: one copy per device, held until
// the process ends.  Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[QGS_BWD_STATIC_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

qgs_status static_scratch(void **out)
{
    int dev = -1;
    qgs_status st = hip_status(hipGetDevice(&dev));
    if (st != QGS_OK) return st;
    if (dev < 0 || dev >= kMaxDevices) return QGS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        st = hip_status(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (st != QGS_OK) return st;
        if (!p) return QGS_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return QGS_OK;
}

}  // namespace

extern "C" {

qgs_status qgs_render_bwd(const qgs_scene *scene, const qgs_prim_buf *prims, const qgs_tile_lists *lists,
                          const qgs_camera *cam, const qgs_render_opts *opts, const qgs_images *fwd,
                          const qgs_image_grads *dL, qgs_scene_grads *out, void *ws, size_t ws_bytes,
                          qgs_stream_t stream)
{
    return render_bwd_impl(scene, prims, lists, cam, opts, fwd, dL, out, ws, ws_bytes, stream);
}

qgs_status qgs_render_bwd_static(const qgs_scene *scene, const qgs_prim_buf *prims, const qgs_tile_lists *lists,
                                 const qgs_camera *cam, const qgs_render_opts *opts, const qgs_images *fwd,
                                 const qgs_image_grads *dL, qgs_scene_grads *out, qgs_stream_t stream)
{
    if (!scene_ok(scene) || !lists_ok(lists) || !cam_ok(cam) || !opts_ok(opts)) return QGS_ERR_INVALID_ARG;
    const uint64_t ntiles = (uint64_t)((cam->width + 15) / 16) * (uint64_t)((cam->height + 15) / 16);
    if (bwd_bytes(scene->n, lists->capacity, opts->flags, ntiles) > QGS_BWD_STATIC_BYTES) return QGS_ERR_WORKSPACE;
    void *ws = nullptr;
    const qgs_status st = static_scratch(&ws);
    if (st != QGS_OK) return st;
    return render_bwd_impl(scene, prims, lists, cam, opts, fwd, dL, out, ws, QGS_BWD_STATIC_BYTES, stream);
}

}  // extern "C"
