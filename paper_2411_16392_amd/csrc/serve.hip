// Serving: a resident scene, render requests of mixed resolutions admitted as
// slots and tile-list memory free up, their work spread over several HIP
// streams so that requests in flight overlap on the device.
//
// Request life cycle (one scheduler thread issues all device work):
//   queued     submitted, waiting for a slot (FIFO)
//   counting   count pass on the slot's stream: preprocess, depth sort, pair
//              offsets; the pair count is copied to pinned host memory
//   waiting    count known; waits, oldest first, until the exact bytes its
//              tile lists and sort temporaries need are free in the pool
//   rendering  emission, tile sort, ranges and the forward rasterizer write
//              the colour image into the caller's buffer
// Completion is observed with hipEventQuery; memory and slot are released
// and the completion is queued for qgs_serve_poll.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "qgs.h"
#include "qgs_internal.hpp"
#include "serve_pool.hpp"

namespace qgs {
namespace {

size_t a256(size_t x) { return pool_align(x); }
uint64_t cdiv64(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// bytes one request's lists and tile-sort temporaries take in the pool
size_t list_bytes(uint64_t pairs)
{
    const uint64_t c = pairs > 0 ? pairs : 1;
    const uint64_t nb = cdiv64(c, TILE_SORT_CHUNK) + 1;
    // pair_tile, pair_prim and their two sort buffers (no emission map: the
    // server runs no deterministic backward)
    return 4 * a256(4 * c) + a256(4 * 256 * nb) + a256(8 * (cdiv64(256 * nb, SCAN_CHUNK) + 64));
}

enum Phase { IDLE = 0, COUNTING = 1, WAITING = 2, RENDERING = 3 };

struct Req {
    uint64_t id = 0;
    qgs_camera cam{};
    float *out = nullptr;
    double t_submit = 0, t_admit = 0;
    uint64_t pairs = 0;
    bool cancelled = false;
    bool admitting = false;  // taken by the scheduler for admission: no longer cancellable
    size_t mem_off = 0, mem_bytes = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    void *records = nullptr;
    uint32_t *depth_key = nullptr, *tiles = nullptr, *pair_offset = nullptr;
    int32_t *rect = nullptr;
    double *conic = nullptr;
    uint32_t *dkA = nullptr, *dvA = nullptr, *dkB = nullptr, *dvB = nullptr, *hist = nullptr;
    uint64_t *off = nullptr, *part = nullptr;
    uint32_t *ranges = nullptr, *tile_order = nullptr, *counters = nullptr, *counters_host = nullptr;
    std::shared_ptr<Req> req;
    Phase phase = IDLE;
    // persistent graphs of the count pass and of the render pass
    hipGraphExec_t count_exec = nullptr, render_exec = nullptr;
};

}  // namespace
}  // namespace qgs

struct qgs_server {
    qgs_scene scene{};
    qgs_serve_config cfg{};
    std::vector<qgs::Slot> slots;
    std::vector<hipStream_t> streams;
    void *pool_base = nullptr;
    qgs::Pool pool;
    std::vector<void *> allocations;

    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<std::shared_ptr<qgs::Req>> queued;
    std::map<uint64_t, std::shared_ptr<qgs::Req>> live;  // submitted, not yet completed
    std::deque<qgs_completion> done;
    bool stopping = false;
    uint64_t next_id = 1;
    qgs_serve_stats stats{};
    std::thread thread;
    std::chrono::steady_clock::time_point t0;
    int32_t in_flight = 0;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace qgs {
namespace {

hipError_t dev_alloc(qgs_server *s, void **p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes > 0 ? bytes : 256);
    if (e == hipSuccess) s->allocations.push_back(*p);
    return e;
}

RasterParams params_for(const qgs_camera &c, const qgs_render_opts &o)
{
    RasterParams p;
    p.fx = c.fx; p.fy = c.fy; p.cx = c.cx; p.cy = c.cy;
    p.ifx = 1.0f / c.fx; p.ify = 1.0f / c.fy;
    p.width = c.width; p.height = c.height;
    p.tiles_x = (c.width + 15) / 16; p.tiles_y = (c.height + 15) / 16;
    p.near_plane = o.near_plane; p.k2 = o.k_sigma * o.k_sigma;
    p.alpha_min = o.alpha_min; p.alpha_max = o.alpha_max; p.T_eps = o.T_eps; p.A_eps = o.A_eps;
    p.bg[0] = o.bg[0]; p.bg[1] = o.bg[1]; p.bg[2] = o.bg[2];
    p.flags = 0;
    return p;
}

BinSortArgs sort_args(qgs_server *s, Slot &sl, const qgs_camera &cam)
{
    BinSortArgs a{};
    a.n = s->scene.n;
    a.depth_key = sl.depth_key;
    a.tiles = sl.tiles;
    a.rect = sl.rect;
    a.conic = sl.conic;
    a.cam = cam;
    a.pair_offset = sl.pair_offset;
    a.tiles_x = (cam.width + 15) / 16;
    a.tiles_y = (cam.height + 15) / 16;
    a.ranges = sl.ranges;
    a.tile_order = sl.tile_order;
    a.counters = sl.counters;
    return a;
}

SortWorkspace fixed_ws(Slot &sl)
{
    SortWorkspace w{};
    w.dkA = sl.dkA; w.dvA = sl.dvA; w.dkB = sl.dkB; w.dvB = sl.dvB;
    w.off = sl.off; w.part = sl.part; w.hist = sl.hist;
    return w;
}

// Runs issue(stream) on the slot's stream, normally through a graph: the
// launches are captured, the slot's executable graph for this pass is updated
// in place with the new arguments (same topology: same kernels and grids
// shape, different camera, sizes and pool addresses) or instantiated when the
// topology differs, and launched as one unit.  Every fill in these passes is
// a kernel, so the graphs hold no memset nodes.
hipError_t enqueue_count(qgs_server *s, Slot &sl, hipStream_t stream);

template <class F>
hipError_t run_pass(qgs_server *s, Slot &sl, hipGraphExec_t &exec, F &&issue)
{
    if (s->cfg.flags & QGS_SERVE_NO_GRAPHS) return issue(sl.stream);
    hipError_t e = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t ei = issue(sl.stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(sl.stream, &g);
    if (ei != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return ei != hipSuccess ? ei : e;
    }
    bool updated = false;
    if (exec) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        updated = hipGraphExecUpdate(exec, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
        if (!updated) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(exec);
            exec = nullptr;
        }
    }
    if (!updated) {
        e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            exec = nullptr;
            (void)hipGraphDestroy(g);
            return e;
        }
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.graph_builds++;
    }
    (void)hipGraphDestroy(g);
    e = hipGraphLaunch(exec, sl.stream);
    if (e == hipSuccess) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.graph_launches++;
    }
    return e;
}

hipError_t issue_count(qgs_server *s, Slot &sl)
{
    hipError_t e = run_pass(s, sl, sl.count_exec, [&](hipStream_t st) { return enqueue_count(s, sl, st); });
    if (e != hipSuccess) return e;
    return hipEventRecord(sl.ev, sl.stream);
}

hipError_t enqueue_count(qgs_server *s, Slot &sl, hipStream_t stream)
{
    const Req &r = *sl.req;
    PreprocessArgs pa{};
    pa.center = s->scene.center; pa.quat = s->scene.quat; pa.scale = s->scene.scale;
    pa.curv = s->scene.curv; pa.opacity = s->scene.opacity; pa.rgb = s->scene.rgb;
    pa.sh = s->scene.sh; pa.sh_degree = s->scene.sh ? s->scene.sh_degree : -1;
    pa.n = s->scene.n;
    pa.cam = r.cam;
    pa.near_plane = s->cfg.opts.near_plane;
    pa.k_sigma = s->cfg.opts.k_sigma;
    pa.alpha_min = s->cfg.opts.alpha_min;
    pa.tight = (s->cfg.opts.flags & QGS_TIGHT_BOUND) ? 1 : 0;
    pa.records = sl.records; pa.depth_key = sl.depth_key; pa.rect = sl.rect; pa.tiles = sl.tiles;
    pa.conic = sl.conic;
    hipError_t e = launch_preprocess(pa, stream);
    if (e != hipSuccess) return e;
    BinSortArgs a = sort_args(s, sl, r.cam);
    a.capacity = 0xFFFFFFFFull;  // the count pass never overflows
    e = bin_sort_phase1(a, fixed_ws(sl), stream);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(sl.counters_host, sl.counters, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, stream);
}

hipError_t enqueue_render(qgs_server *s, Slot &sl, hipStream_t stream);

hipError_t issue_render(qgs_server *s, Slot &sl)
{
    hipError_t e = run_pass(s, sl, sl.render_exec, [&](hipStream_t st) { return enqueue_render(s, sl, st); });
    if (e != hipSuccess) return e;
    return hipEventRecord(sl.ev, sl.stream);
}

hipError_t enqueue_render(qgs_server *s, Slot &sl, hipStream_t stream)
{
    Req &r = *sl.req;
    const uint64_t c = r.pairs > 0 ? r.pairs : 1;
    const uint64_t nb = cdiv64(c, TILE_SORT_CHUNK) + 1;
    char *base = (char *)s->pool_base + r.mem_off;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        void *p = base + o;
        o += a256(bytes);
        return p;
    };
    uint32_t *pair_tile = (uint32_t *)take(4 * c);
    uint32_t *pair_prim = (uint32_t *)take(4 * c);
    SortWorkspace w = fixed_ws(sl);
    w.tileT = (uint32_t *)take(4 * c);
    w.primT = (uint32_t *)take(4 * c);
    w.emit_prim = nullptr;
    w.hist = (uint32_t *)take(4 * 256 * nb);
    w.part = (uint64_t *)take(8 * (cdiv64(256 * nb, SCAN_CHUNK) + 64));
    BinSortArgs a = sort_args(s, sl, r.cam);
    a.pair_tile = pair_tile;
    a.pair_prim = pair_prim;
    a.emit_to_sorted = nullptr;
    a.capacity = c;
    hipError_t e = bin_sort_phase2(a, w, r.pairs, stream);
    if (e != hipSuccess) return e;
    RasterArgs ra{};
    ra.records = (const float *)sl.records;
    ra.pair_prim = pair_prim; ra.pair_tile = pair_tile;
    ra.ranges = sl.ranges; ra.tile_order = sl.tile_order; ra.counters = sl.counters;
    ra.pair_offset = sl.pair_offset; ra.tiles = sl.tiles; ra.emit_to_sorted = nullptr;
    ra.tiles_x = a.tiles_x; ra.tiles_y = a.tiles_y;
    FwdOut fo{};
    // colour only: no depth, normal, transmittance or last-entry planes
    fo.color = r.out; fo.depth = nullptr; fo.normal = nullptr; fo.T_final = nullptr; fo.last = nullptr;
    fo.counters = nullptr;
    return launch_render_fwd(ra, params_for(r.cam, s->cfg.opts), fo, stream);
}

void complete(qgs_server *s, const Req &r, int32_t state, int32_t status)
{
    qgs_completion c{};
    c.req_id = r.id;
    c.state = state;
    c.status = status;
    c.t_submit = r.t_submit;
    c.t_admit = r.t_admit;
    c.t_done = s->now();
    c.num_pairs = r.pairs;
    std::lock_guard<std::mutex> g(s->mu);
    s->live.erase(r.id);
    s->done.push_back(c);
    if (state == QGS_REQ_DONE) s->stats.completed++;
    else if (state == QGS_REQ_CANCELLED) s->stats.cancelled++;
    else s->stats.failed++;
    s->cv_done.notify_all();
}

void scheduler(qgs_server *s)
{
    (void)hipSetDevice(s->cfg.device);
    const size_t budget = (size_t)s->cfg.budget_bytes;
    for (;;) {
        bool progressed = false;
        // 1. observe finished device work
        for (auto &sl : s->slots) {
            if (sl.phase != COUNTING && sl.phase != RENDERING) continue;
            const hipError_t q = hipEventQuery(sl.ev);
            if (q == hipErrorNotReady) continue;
            progressed = true;
            Req &r = *sl.req;
            if (q != hipSuccess) {
                // the slot's device work failed: the request fails with the
                // HIP error, its memory and slot are released
                if (sl.phase == RENDERING) s->pool.release(r.mem_off, r.mem_bytes);
                complete(s, r, QGS_REQ_FAILED, QGS_ERR_HIP);
            } else if (sl.phase == COUNTING) {
                r.pairs = sl.counters_host[0];
                bool cancelled;
                {
                    std::lock_guard<std::mutex> g(s->mu);
                    cancelled = r.cancelled;
                }
                if (cancelled) {
                    complete(s, r, QGS_REQ_CANCELLED, QGS_OK);
                } else if (list_bytes(r.pairs) > budget) {
                    complete(s, r, QGS_REQ_FAILED, QGS_ERR_BUDGET);
                } else {
                    sl.phase = WAITING;
                    continue;
                }
            } else {
                s->pool.release(r.mem_off, r.mem_bytes);
                complete(s, r, QGS_REQ_DONE, QGS_OK);
            }
            sl.req.reset();
            sl.phase = IDLE;
            s->in_flight--;
        }
        // 2. admit waiting requests for rendering in arrival order: only the
        // oldest request not yet admitted may go, so a younger request whose
        // count pass finished first waits behind an older one still counting
        for (;;) {
            Slot *oldest = nullptr;
            for (auto &sl : s->slots)
                if ((sl.phase == WAITING || sl.phase == COUNTING) && (!oldest || sl.req->id < oldest->req->id))
                    oldest = &sl;
            if (!oldest || oldest->phase != WAITING) break;
            Req &r = *oldest->req;
            bool cancelled;
            {
                // the cancel check and the mark that ends cancellability in
                // one critical section: a cancel after it returns QGS_ERR_STATE
                std::lock_guard<std::mutex> g(s->mu);
                cancelled = r.cancelled;
                if (!cancelled) r.admitting = true;
            }
            if (cancelled) {
                complete(s, r, QGS_REQ_CANCELLED, QGS_OK);
                oldest->req.reset();
                oldest->phase = IDLE;
                s->in_flight--;
                progressed = true;
                continue;
            }
            r.mem_bytes = list_bytes(r.pairs);
            if (!s->pool.alloc(r.mem_bytes, r.mem_off)) {
                // not admitted yet (keep arrival order): cancellable again
                std::lock_guard<std::mutex> g(s->mu);
                r.admitting = false;
                break;
            }
            {
                std::lock_guard<std::mutex> g(s->mu);
                r.t_admit = s->now();
                if (s->pool.peak > s->stats.peak_pool_bytes) s->stats.peak_pool_bytes = s->pool.peak;
            }
            if (issue_render(s, *oldest) != hipSuccess) {
                s->pool.release(r.mem_off, r.mem_bytes);
                complete(s, r, QGS_REQ_FAILED, QGS_ERR_HIP);
                oldest->req.reset();
                oldest->phase = IDLE;
                s->in_flight--;
            } else {
                oldest->phase = RENDERING;
            }
            progressed = true;
        }
        // 3. start count passes for queued requests on free slots
        for (auto &sl : s->slots) {
            if (sl.phase != IDLE) continue;
            std::shared_ptr<Req> r;
            {
                std::lock_guard<std::mutex> g(s->mu);
                while (!s->queued.empty() && !r) {
                    r = s->queued.front();
                    s->queued.pop_front();
                }
            }
            if (!r) break;
            sl.req = r;
            sl.phase = COUNTING;
            s->in_flight++;
            {
                std::lock_guard<std::mutex> g(s->mu);
                if (s->in_flight > s->stats.peak_in_flight) s->stats.peak_in_flight = s->in_flight;
            }
            if (issue_count(s, sl) != hipSuccess) {
                complete(s, *r, QGS_REQ_FAILED, QGS_ERR_HIP);
                sl.req.reset();
                sl.phase = IDLE;
                s->in_flight--;
            }
            progressed = true;
        }
        // 4. sleep or stop
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stopping && s->queued.empty() && s->in_flight == 0) break;
        if (s->in_flight == 0 && s->queued.empty()) {
            s->cv_sched.wait(lk, [&] { return s->stopping || !s->queued.empty(); });
        } else if (!progressed) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
}

}  // namespace
}  // namespace qgs

using namespace qgs;

extern "C" {

qgs_status qgs_serve_create(const qgs_scene *scene, const qgs_serve_config *cfg, qgs_server **out)
{
    if (!scene || !cfg || !out || scene->n < 0 || scene->n > 0x7FFFFFFFll) return QGS_ERR_INVALID_ARG;
    if (scene->n > 0 && (!scene->center || !scene->quat || !scene->scale || !scene->curv || !scene->opacity ||
                         !scene->rgb))
        return QGS_ERR_INVALID_ARG;
    if (cfg->max_slots <= 0 || cfg->max_slots > 64 || cfg->n_streams <= 0 || cfg->n_streams > 16 ||
        cfg->max_width <= 0 || cfg->max_height <= 0 || cfg->budget_bytes <= 0 || cfg->opts.tile != 16)
        return QGS_ERR_INVALID_ARG;
    *out = nullptr;
    qgs_server *s = new qgs_server();
    s->scene = *scene;
    s->cfg = *cfg;
    s->t0 = std::chrono::steady_clock::now();
    hipError_t e = hipSetDevice(cfg->device);
    const uint64_t n = (uint64_t)(scene->n > 0 ? scene->n : 1);
    const uint64_t ntiles = (uint64_t)((cfg->max_width + 15) / 16) * ((cfg->max_height + 15) / 16);
    // count table of the per-slot depth sort
    const uint64_t nb_n = cdiv64(n, DEPTH_SORT_CHUNK) + 1;
    for (int i = 0; i < cfg->n_streams && e == hipSuccess; ++i) {
        hipStream_t st;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) s->streams.push_back(st);
    }
    s->slots.resize(cfg->max_slots);
    for (int i = 0; i < cfg->max_slots && e == hipSuccess; ++i) {
        Slot &sl = s->slots[i];
        sl.stream = s->streams[i % s->streams.size()];
        e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
        if (e != hipSuccess) break;
        void *p;
        if ((e = dev_alloc(s, &p, 128 * n)) != hipSuccess) break;
        sl.records = p;
        if ((e = dev_alloc(s, &p, 4 * n)) != hipSuccess) break;
        sl.depth_key = (uint32_t *)p;
        if ((e = dev_alloc(s, &p, 16 * n)) != hipSuccess) break;
        sl.rect = (int32_t *)p;
        if ((e = dev_alloc(s, &p, 64 * n)) != hipSuccess) break;
        sl.conic = (double *)p;
        if ((e = dev_alloc(s, &p, 4 * n)) != hipSuccess) break;
        sl.tiles = (uint32_t *)p;
        if ((e = dev_alloc(s, &p, 4 * n)) != hipSuccess) break;
        sl.pair_offset = (uint32_t *)p;
        if ((e = dev_alloc(s, &p, 16 * n)) != hipSuccess) break;
        sl.dkA = (uint32_t *)p;
        sl.dvA = sl.dkA + n;
        sl.dkB = sl.dkA + 2 * n;
        sl.dvB = sl.dkA + 3 * n;
        if ((e = dev_alloc(s, &p, 8 * (n + 1))) != hipSuccess) break;
        sl.off = (uint64_t *)p;
        if ((e = dev_alloc(s, &p, 8 * (cdiv64(n + 1, SCAN_CHUNK) + cdiv64(256 * nb_n, SCAN_CHUNK) + 64))) !=
            hipSuccess)
            break;
        sl.part = (uint64_t *)p;
        if ((e = dev_alloc(s, &p, 4 * 256 * nb_n)) != hipSuccess) break;
        sl.hist = (uint32_t *)p;
        if ((e = dev_alloc(s, &p, 8 * ntiles)) != hipSuccess) break;
        sl.ranges = (uint32_t *)p;
        if ((e = dev_alloc(s, &p, 4 * ntiles)) != hipSuccess) break;
        sl.tile_order = (uint32_t *)p;
        if ((e = dev_alloc(s, &p, 32)) != hipSuccess) break;
        sl.counters = (uint32_t *)p;

        if ((e = hipHostMalloc((void **)&sl.counters_host, 32, hipHostMallocDefault)) != hipSuccess) break;
    }
    if (e == hipSuccess) e = dev_alloc(s, &s->pool_base, (size_t)cfg->budget_bytes);
    if (e != hipSuccess) {
        qgs_serve_destroy(s);
        return QGS_ERR_HIP;
    }
    s->pool.init((size_t)cfg->budget_bytes);
    s->thread = std::thread(scheduler, s);
    *out = s;
    return QGS_OK;
}

qgs_status qgs_serve_submit(qgs_server *s, const qgs_camera *cam, float *out_rgb, uint64_t *req_id)
{
    if (!s || !cam || !out_rgb) return QGS_ERR_INVALID_ARG;
    if (cam->width <= 0 || cam->height <= 0 || cam->width > s->cfg.max_width || cam->height > s->cfg.max_height ||
        !(cam->fx > 0.0f) || !(cam->fy > 0.0f))
        return QGS_ERR_INVALID_ARG;
    auto r = std::make_shared<Req>();
    r->cam = *cam;
    r->out = out_rgb;
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stopping) return QGS_ERR_STATE;
        r->id = s->next_id++;
        r->t_submit = s->now();
        s->queued.push_back(r);
        s->live[r->id] = r;
        s->stats.submitted++;
    }
    if (req_id) *req_id = r->id;
    s->cv_sched.notify_one();
    return QGS_OK;
}

qgs_status qgs_serve_poll(qgs_server *s, qgs_completion *out, int32_t max, int32_t *n, int32_t timeout_us)
{
    if (!s || !n || max < 0 || (max > 0 && !out)) return QGS_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && timeout_us > 0)
        s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return !s->done.empty(); });
    int32_t k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n = k;
    return QGS_OK;
}

qgs_status qgs_serve_cancel(qgs_server *s, uint64_t id)
{
    if (!s) return QGS_ERR_INVALID_ARG;
    std::shared_ptr<Req> hit;
    {
        std::lock_guard<std::mutex> g(s->mu);
        auto lv = s->live.find(id);
        if (lv == s->live.end()) return QGS_ERR_NOT_FOUND;
        for (auto it = s->queued.begin(); it != s->queued.end(); ++it) {
            if ((*it)->id == id) {
                hit = *it;
                s->queued.erase(it);
                break;
            }
        }
        if (!hit) {
            // in a slot: cancellable until admitted for rendering; the scheduler
            // completes it when it next looks at the slot
            if (lv->second->admitting || lv->second->t_admit > 0) return QGS_ERR_STATE;
            lv->second->cancelled = true;
            return QGS_OK;
        }
    }
    complete(s, *hit, QGS_REQ_CANCELLED, QGS_OK);
    return QGS_OK;
}

qgs_status qgs_serve_stats_get(qgs_server *s, qgs_serve_stats *out)
{
    if (!s || !out) return QGS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    return QGS_OK;
}

double qgs_serve_clock(qgs_server *s) { return s ? s->now() : 0.0; }

qgs_status qgs_serve_destroy(qgs_server *s)
{
    if (!s) return QGS_ERR_INVALID_ARG;
    std::vector<std::shared_ptr<Req>> dropped;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stopping = true;
        for (auto &r : s->queued) dropped.push_back(r);
        s->queued.clear();
    }
    for (auto &r : dropped) complete(s, *r, QGS_REQ_CANCELLED, QGS_OK);
    s->cv_sched.notify_all();
    if (s->thread.joinable()) s->thread.join();
    (void)hipSetDevice(s->cfg.device);
    for (auto &st : s->streams) (void)hipStreamSynchronize(st);
    for (auto &sl : s->slots) {
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.count_exec) (void)hipGraphExecDestroy(sl.count_exec);
        if (sl.render_exec) (void)hipGraphExecDestroy(sl.render_exec);
        if (sl.counters_host) (void)hipHostFree(sl.counters_host);
    }
    for (void *p : s->allocations) (void)hipFree(p);
    for (auto &st : s->streams) (void)hipStreamDestroy(st);
    delete s;
    return QGS_OK;
}

}  // extern "C"
