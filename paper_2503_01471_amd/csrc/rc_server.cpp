// rc_server.cpp -- request loop over a renderer context's resident scene.
//
// One worker thread owns all device work of the server.  Requests wait in a
// FIFO; each admission round takes, in arrival order (with backfill of later
// requests that still fit), the requests whose in-flight bytes fit the
// server budget and launches them on a free stream: in batched mode all of
// them in ONE persistent render launch whose work list concatenates their
// tiles and whose per-sensor-instance output table points into each
// request's own buffers; in plain mode one request at a time, one launch per
// environment.  Completion is detected through one event per stream; while
// a batch runs, newly arrived requests are admitted on the other streams, so
// their work overlaps on the device.  The admission round itself and the
// arena that holds library-allocated outputs are the host-only code of
// rc_sched.hpp.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rc_runtime.hpp"
#include "rc_sched.hpp"

using namespace rc;

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
    uint64_t ticket = 0;
    std::vector<int32_t> envs;
    int32_t model = 0;
    std::vector<float> poses;  // 12 per environment
    float *depth = nullptr;    // outputs: caller buffers, or carved from the arena at admission
    int32_t *seg = nullptr;
    int32_t *tri = nullptr;
    float *hit = nullptr;
    int32_t lib_outputs = 0;   // RC_OUT_* kinds the library allocates (0: caller buffers)
    int64_t rays_per_env = 0;
    int64_t tiles = 0;  // work items
    sched::Pending pending;  // bytes charged while in flight; arena block of library outputs
    double t_submit = 0.0, t_done = 0.0;
    int state = 0;  // 0 queued, 1 running, 2 done
};

// Bytes per ray of each output kind, in the order the arena block holds them.
constexpr int kOutKinds = 4;
constexpr int kOutBit[kOutKinds] = {RC_OUT_DEPTH, RC_OUT_SEG, RC_OUT_TRI, RC_OUT_HIT};
constexpr int64_t kOutBytes[kOutKinds] = {4, 4, 4, 12};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<Req *> reqs;
    size_t charged = 0;
    DBuf items, si_env, si_model, ray_off, pose, dtab, stab, ttab, htab, head;
    int64_t cap_items = 0, cap_si = 0;
    void *host = nullptr;
    size_t host_cap = 0;
    // tables replaced by larger ones: kept until the server is destroyed, so
    // growing one never waits for the device
    std::vector<std::unique_ptr<DBuf>> retired;
};

constexpr int64_t kMaxBatchRays = int64_t(48) << 20;  // bound on one admission round
constexpr int kLookahead = 256;                       // backfill window of the FIFO

}  // namespace

struct rc_server {
    rc_context *ctx = nullptr;
    int mode = RC_SERVE_BATCHED;
    size_t budget = 0, in_use = 0;
    sched::Arena arena;  // library-allocated outputs: offsets into `slab`
    DBuf slab;           // allocated by the first request that asks for library outputs
    std::vector<SensorModel> models;  // host copies, current tile shape
    std::vector<float> env_pose;      // first attached pose per environment
    std::vector<uint8_t> env_has_pose;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    uint64_t next_ticket = 1;
    std::vector<std::unique_ptr<Slot>> slots;
    std::thread worker;
    bool stop = false;
    rc_status error = RC_OK;
    std::string error_msg;
};

namespace {

// Grow a device table of a slot (no budget check beyond the context pool).
rc_status ensure(rc_context *c, Slot &sl, DBuf &b, size_t bytes)
{
    if (b.n >= bytes)
        return RC_OK;
    if (b.p) {
        auto old = std::make_unique<DBuf>();
        std::swap(old->p, b.p);
        std::swap(old->n, b.n);
        std::swap(old->pool, b.pool);
        sl.retired.push_back(std::move(old));
    }
    return c->pool.alloc(b, bytes + bytes / 2);
}

// Byte offsets of the pinned staging block:
// items | si_env | si_model | pose | dtab | stab | ttab | htab.
struct Staging {
    size_t o_items, o_env, o_model, o_pose, o_dtab, o_stab, o_ttab, o_htab, total;
    Staging(int64_t n_items, int64_t S)
    {
        o_items = 0;
        o_env = o_items + 8 * n_items;
        o_model = o_env + 4 * S;
        o_pose = o_model + 4 * S;
        o_dtab = o_pose + 48 * S;
        o_stab = o_dtab + 8 * S;
        o_ttab = o_stab + 8 * S;
        o_htab = o_ttab + 8 * S;
        total = o_htab + 8 * S;
    }
};

// Make the slot's tables hold a batch of S sensor instances and n_items tiles.
rc_status reserve(rc_context *c, Slot &sl, int64_t S, int64_t n_items)
{
    if (S > sl.cap_si) {
        RC_TRY(ensure(c, sl, sl.si_env, 4 * S));
        RC_TRY(ensure(c, sl, sl.si_model, 4 * S));
        RC_TRY(ensure(c, sl, sl.ray_off, 8 * (S + 1)));
        RC_TRY(ensure(c, sl, sl.pose, 48 * S));
        RC_TRY(ensure(c, sl, sl.dtab, 8 * S));
        RC_TRY(ensure(c, sl, sl.stab, 8 * S));
        RC_TRY(ensure(c, sl, sl.ttab, 8 * S));
        RC_TRY(ensure(c, sl, sl.htab, 8 * S));
        RC_HIP(hipMemsetAsync(sl.ray_off.p, 0, sl.ray_off.n, sl.stream));
        sl.cap_si = (int64_t)(sl.si_env.n / 4);
    }
    if (n_items > sl.cap_items) {
        RC_TRY(ensure(c, sl, sl.items, 8 * n_items));
        sl.cap_items = (int64_t)(sl.items.n / 8);
    }
    if (!sl.head.p)
        RC_TRY(c->pool.alloc(sl.head, sizeof(unsigned int) * kQueues * kQueueStride));
    const Staging g(n_items, S);
    if (g.total > sl.host_cap) {
        // the slot is idle here: its previous batch has completed
        if (sl.host)
            RC_HIP(hipHostFree(sl.host));
        sl.host = nullptr;
        sl.host_cap = 0;
        RC_HIP(hipHostMalloc(&sl.host, g.total + g.total / 2, hipHostMallocDefault));
        sl.host_cap = g.total + g.total / 2;
    }
    return RC_OK;
}

// Launch one admitted batch on slot `sl` (worker thread, no lock held).
rc_status launch(rc_server *sv, Slot &sl)
{
    rc_context *c = sv->ctx;
    const Scene &sc = *c->scene;
    const Sensors &se = *c->sensors;
    int64_t S = 0, n_items = 0;
    for (Req *r : sl.reqs) {
        S += (int64_t)r->envs.size();
        n_items += r->tiles;
    }
    RC_TRY(reserve(c, sl, S, n_items));
    const Staging g(n_items, S);
    const size_t o_items = g.o_items, o_env = g.o_env, o_model = g.o_model, o_pose = g.o_pose, o_dtab = g.o_dtab,
                 o_stab = g.o_stab, o_ttab = g.o_ttab, o_htab = g.o_htab;
    char *h = (char *)sl.host;
    int2 *items = (int2 *)(h + o_items);
    int32_t *si_env = (int32_t *)(h + o_env);
    int32_t *si_model = (int32_t *)(h + o_model);
    float *pose = (float *)(h + o_pose);
    float **dtab = (float **)(h + o_dtab);
    int32_t **stab = (int32_t **)(h + o_stab);
    int32_t **ttab = (int32_t **)(h + o_ttab);
    float **htab = (float **)(h + o_htab);
    int64_t k = 0;
    std::vector<int64_t> item_begin;  // per sensor instance, request order (plain mode)
    std::vector<int64_t> order, tiles;  // batched mode: queue order of the sensor instances
    for (Req *r : sl.reqs) {
        const SensorModel &m = sv->models[r->model];
        for (size_t i = 0; i < r->envs.size(); ++i, ++k) {
            si_env[k] = r->envs[i];
            si_model[k] = r->model;
            memcpy(pose + 12 * k, r->poses.data() + 12 * i, 48);
            const int64_t at = (int64_t)i * r->rays_per_env;
            dtab[k] = r->depth ? r->depth + at : nullptr;
            stab[k] = r->seg ? r->seg + at : nullptr;
            ttab[k] = r->tri ? r->tri + at : nullptr;
            htab[k] = r->hit ? r->hit + 3 * at : nullptr;
            order.push_back(k);
            tiles.push_back(m.tiles);
        }
    }
    int64_t qoff[kQueues + 1];
    if (sv->mode == RC_SERVE_BATCHED) {
        std::vector<int2> dealt;
        deal_queues(order, tiles, dealt, qoff);
        memcpy(items, dealt.data(), sizeof(int2) * dealt.size());
    } else {
        int64_t it = 0;
        for (int64_t s = 0; s < k; ++s) {
            item_begin.push_back(it);
            for (int64_t t = 0; t < tiles[s]; ++t)
                items[it++] = make_int2((int)s, (int)t);
        }
        item_begin.push_back(it);
    }
    hipStream_t st = sl.stream;
    RC_HIP(hipMemcpyAsync(sl.items.p, h + o_items, 8 * n_items, hipMemcpyHostToDevice, st));
    RC_HIP(hipMemcpyAsync(sl.si_env.p, h + o_env, 4 * S, hipMemcpyHostToDevice, st));
    RC_HIP(hipMemcpyAsync(sl.si_model.p, h + o_model, 4 * S, hipMemcpyHostToDevice, st));
    RC_HIP(hipMemcpyAsync(sl.pose.p, h + o_pose, 48 * S, hipMemcpyHostToDevice, st));
    RC_HIP(hipMemcpyAsync(sl.dtab.p, h + o_dtab, 8 * S, hipMemcpyHostToDevice, st));
    RC_HIP(hipMemcpyAsync(sl.stab.p, h + o_stab, 8 * S, hipMemcpyHostToDevice, st));
    RC_HIP(hipMemcpyAsync(sl.ttab.p, h + o_ttab, 8 * S, hipMemcpyHostToDevice, st));
    RC_HIP(hipMemcpyAsync(sl.htab.p, h + o_htab, 8 * S, hipMemcpyHostToDevice, st));
    SensorView ev;
    ev.models = se.models.as<SensorModel>();
    ev.tables = se.tables.as<float>();
    ev.si_env = sl.si_env.as<int32_t>();
    ev.si_model = sl.si_model.as<int32_t>();
    ev.ray_off = sl.ray_off.as<int64_t>();
    ev.pose = sl.pose.as<float>();
    ev.items = sl.items.as<int2>();
    OutView ov;
    ov.depth_tab = sl.dtab.as<float *>();
    ov.seg_tab = sl.stab.as<int32_t *>();
    ov.tri_tab = sl.ttab.as<int32_t *>();
    ov.hit_tab = sl.htab.as<float *>();
    if (sv->mode == RC_SERVE_BATCHED && c->tuning.chunk == 0) {  // the tuned one-launch form, no queue
        RC_HIP(launch_render_flat(sc.sview(), ev, ov, 0, n_items, st));
    } else if (sv->mode == RC_SERVE_BATCHED) {
        QueueView qv;
        qv.items = ev.items;
        for (int i = 0; i <= kQueues; ++i)
            qv.off[i] = qoff[i];
        qv.head = sl.head.as<unsigned int>();
        qv.chunk = c->tuning.chunk;
        RC_HIP(launch_render_batched(sc.sview(), ev, ov, qv, c->batched_grid(), st));
    } else {
        for (int64_t s = 0; s < S; ++s)
            RC_HIP(launch_render_flat(sc.sview(), ev, ov, item_begin[s], item_begin[s + 1] - item_begin[s], st));
    }
    RC_HIP(hipEventRecord(sl.done, st));
    return RC_OK;
}

// Point a request's library-allocated outputs into its arena block (kinds in
// kOutBit order, each starting on an arena alignment boundary).
void carve_outputs(rc_server *sv, Req &r)
{
    char *p = (char *)sv->slab.p + r.pending.arena_off;
    const int64_t n = r.rays_per_env * (int64_t)r.envs.size();
    void *dst[kOutKinds] = {};
    for (int k = 0; k < kOutKinds; ++k)
        if (r.lib_outputs & kOutBit[k]) {
            dst[k] = p;
            p += sched::align_up((size_t)(kOutBytes[k] * n));
        }
    r.depth = (float *)dst[0];
    r.seg = (int32_t *)dst[1];
    r.tri = (int32_t *)dst[2];
    r.hit = (float *)dst[3];
}

// Arena bytes of a request's library-allocated outputs.
size_t lib_output_bytes(int32_t kinds, int64_t rays)
{
    size_t b = 0;
    for (int k = 0; k < kOutKinds; ++k)
        if (kinds & kOutBit[k])
            b += sched::align_up((size_t)(kOutBytes[k] * rays));
    return b;
}

void worker_main(rc_server *sv)
{
    (void)hipSetDevice(sv->ctx->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    while (true) {
        // completions
        bool any_busy = false;
        for (auto &slp : sv->slots) {
            Slot &sl = *slp;
            if (!sl.busy)
                continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) {
                const double t = now_s();
                for (Req *r : sl.reqs) {
                    r->state = 2;
                    r->t_done = t;
                }
                sl.reqs.clear();
                sv->in_use -= sl.charged;  // library outputs stay charged until released
                sl.charged = 0;
                sl.busy = false;
                sv->cv.notify_all();
            } else if (q != hipErrorNotReady) {
                sv->error = RC_E_HIP;
                sv->error_msg = hipGetErrorString(q);
                sv->stop = true;
                for (Req *r : sl.reqs)
                    r->state = 2;
                sl.reqs.clear();
                sl.busy = false;
                sv->cv.notify_all();
            } else {
                any_busy = true;
            }
        }
        if (sv->stop && (sv->queue.empty() || sv->error != RC_OK) && !any_busy)
            break;
        // admission
        bool launched = false;
        for (auto &slp : sv->slots) {
            Slot &sl = *slp;
            if (sl.busy || sv->queue.empty() || sv->error != RC_OK)
                continue;
            sched::RoundLimits lim;
            lim.budget = sv->budget;
            lim.max_rays = kMaxBatchRays;
            lim.lookahead = kLookahead;
            lim.fifo_only = sv->mode == RC_SERVE_PLAIN;
            std::vector<Req *> batch = sched::admit(sv->queue, sv->in_use, sv->arena, lim);
            if (batch.empty())
                continue;
            size_t charged = 0;
            for (Req *r : batch) {
                r->state = 1;
                charged += r->pending.bytes - r->pending.arena_bytes;
                if (r->lib_outputs)
                    carve_outputs(sv, *r);
            }
            sl.reqs = batch;
            sl.charged = charged;
            sl.busy = true;
            lk.unlock();
            const rc_status s = launch(sv, sl);
            lk.lock();
            if (s != RC_OK) {
                sv->error = s;
                sv->error_msg = last_error();
                sv->stop = true;
                for (Req *r : sl.reqs)
                    r->state = 2;
                sl.reqs.clear();
                sl.busy = false;
                sv->in_use -= sl.charged;
                sl.charged = 0;
                sv->cv.notify_all();
            }
            launched = true;
        }
        if (!launched) {
            // short wait: new requests notify; running batches are polled
            sv->cv.wait_for(lk, std::chrono::microseconds(any_busy ? 20 : 500));
        }
    }
    // after a failure, release whatever is still queued so that no client waits forever
    for (Req *r : sv->queue)
        r->state = 2;
    sv->queue.clear();
    sv->cv.notify_all();
}

}  // namespace

extern "C" {

rc_status rc_server_create(rc_context *c, int32_t mode, int32_t n_streams, size_t hbm_budget, rc_server **out)
{
    RC_CHECK(c && out, "NULL argument");
    *out = nullptr;
    RC_CHECK(mode == RC_SERVE_PLAIN || mode == RC_SERVE_BATCHED, "unknown server mode %d", mode);
    RC_CHECK(n_streams >= 1 && n_streams <= 16, "n_streams must be in [1, 16]");
    if (!c->scene || !c->scene->built || !c->sensors || !c->sensors->poses_set)
        return fail(RC_E_STATE, "server needs a built scene and attached, posed sensors");
    RC_TRY(set_device(c));
    size_t free_b = 0, total_b = 0;
    RC_HIP(hipMemGetInfo(&free_b, &total_b));
    // 0: half of the device memory free now; never more than is free
    const size_t budget = hbm_budget ? std::min(hbm_budget, free_b) : free_b / 2;
    RC_CHECK(budget > 0, "no device memory free for the server budget");
    auto sv = new rc_server;
    sv->ctx = c;
    sv->mode = mode;
    sv->budget = budget;
    const Sensors &se = *c->sensors;
    // host copies of the models (current tile shape) and of the attached poses
    sv->models.resize(c->models.size());
    if (!c->models.empty() &&
        hipMemcpy(sv->models.data(), se.models.p, sizeof(SensorModel) * c->models.size(), hipMemcpyDeviceToHost) !=
            hipSuccess) {
        delete sv;
        return fail(RC_E_HIP, "reading sensor models");
    }
    std::vector<float> pose(12 * (size_t)se.n_si);
    if (se.n_si && hipMemcpy(pose.data(), se.pose.p, 48 * se.n_si, hipMemcpyDeviceToHost) != hipSuccess) {
        delete sv;
        return fail(RC_E_HIP, "reading sensor poses");
    }
    const int32_t E = c->scene->n_envs;
    sv->env_pose.assign(12 * (size_t)E, 0.f);
    sv->env_has_pose.assign(E, 0);
    for (int32_t e = 0; e < E; ++e) {
        const int64_t s = se.sens_offsets[e];
        if (s < se.sens_offsets[e + 1]) {
            memcpy(&sv->env_pose[12 * (size_t)e], &pose[12 * (size_t)s], 48);
            sv->env_has_pose[e] = 1;
        }
    }
    const int n_slots = mode == RC_SERVE_PLAIN ? 1 : n_streams;
    for (int i = 0; i < n_slots; ++i)
        sv->slots.push_back(std::make_unique<Slot>());
    for (auto &slp : sv->slots) {
        Slot &sl = *slp;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            rc_server_destroy(sv);
            return fail(RC_E_HIP, "creating server streams");
        }
    }
    // size every slot's tables for the largest batch one admission round
    // forms (bounded by kMaxBatchRays, or one larger request alone), so the
    // worker rarely has to allocate
    {
        int64_t max_tiles = 0;
        for (const SensorModel &m : sv->models)
            max_tiles = std::max<int64_t>(max_tiles, (int64_t)m.tiles);
        const int64_t S0 = std::max<int64_t>(E, 1);
        const int64_t items0 = kMaxBatchRays / 64 + S0 * std::max<int64_t>(max_tiles / 16, 1);
        for (auto &slp : sv->slots) {
            rc_status st = reserve(c, *slp, S0, mode == RC_SERVE_PLAIN ? 1 : items0);
            if (st != RC_OK) {
                rc_server_destroy(sv);
                return st;
            }
        }
        for (auto &slp : sv->slots)
            if (hipStreamSynchronize(slp->stream) != hipSuccess) {
                rc_server_destroy(sv);
                return fail(RC_E_HIP, "server table setup");
            }
    }
    c->servers += 1;
    sv->worker = std::thread(worker_main, sv);
    *out = sv;
    return RC_OK;
}

rc_status rc_server_submit(rc_server *sv, const rc_request *q, uint64_t *ticket)
{
    RC_CHECK(sv && q && ticket, "NULL argument");
    rc_context *c = sv->ctx;
    RC_CHECK(q->n_envs >= 1 && q->env_ids, "request needs n_envs >= 1 and env_ids");
    RC_CHECK(q->sensor_id >= 0 && q->sensor_id < (int32_t)sv->models.size(), "sensor_id %d invalid", q->sensor_id);
    auto r = std::make_unique<Req>();
    r->envs.assign(q->env_ids, q->env_ids + q->n_envs);
    for (int32_t e : r->envs) {
        RC_CHECK(e >= 0 && e < c->scene->n_envs, "environment id %d out of range", e);
        RC_CHECK(q->sensor_T || sv->env_has_pose[e], "environment %d has no attached sensor pose", e);
    }
    r->model = q->sensor_id;
    r->poses.resize(12 * (size_t)q->n_envs);
    for (int32_t i = 0; i < q->n_envs; ++i)
        memcpy(&r->poses[12 * (size_t)i], q->sensor_T ? q->sensor_T + 12 * (size_t)i : &sv->env_pose[12 * (size_t)r->envs[i]],
               48);
    const rc_outputs &o = q->out;
    RC_CHECK(!o.normal && !o.bary && !o.point && !o.vert && !o.shadow,
             "served requests write depth, seg, tri and hit_xyz only");
    RC_CHECK((q->lib_outputs & ~(RC_OUT_DEPTH | RC_OUT_SEG | RC_OUT_TRI | RC_OUT_HIT)) == 0,
             "lib_outputs has unknown bits 0x%x", q->lib_outputs);
    RC_CHECK(!q->lib_outputs || (!o.depth && !o.seg && !o.tri && !o.hit_xyz),
             "lib_outputs needs every output pointer NULL");
    r->depth = o.depth;
    r->seg = o.seg;
    r->tri = o.tri;
    r->hit = o.hit_xyz;
    r->lib_outputs = q->lib_outputs;
    const SensorModel &m = sv->models[r->model];
    r->rays_per_env = (int64_t)m.W * m.H;
    r->tiles = (int64_t)m.tiles * q->n_envs;
    const int64_t rays = r->rays_per_env * q->n_envs;
    // in flight: the outputs (the arena block, or for caller buffers the bytes
    // they stand for, at least depth and seg) and the work lists
    int64_t caller_b = 0;
    const void *given[kOutKinds] = {o.depth, o.seg, o.tri, o.hit_xyz};
    for (int k = 0; k < kOutKinds; ++k)
        caller_b += given[k] ? kOutBytes[k] : 0;
    r->pending.rays = rays;
    r->pending.arena_bytes = lib_output_bytes(r->lib_outputs, rays);
    const size_t out_b = r->lib_outputs ? r->pending.arena_bytes : (size_t)(std::max<int64_t>(caller_b, 8) * rays);
    r->pending.bytes = out_b + (size_t)(8 * r->tiles + 80 * q->n_envs);
    sched::RoundLimits alone;
    alone.budget = sv->budget;
    if (!sched::fits_alone(r->pending, alone))
        return fail(RC_E_OOM, "request needs %zu bytes in flight, server budget is %zu", r->pending.bytes,
                    sv->budget);
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->error != RC_OK)
        return fail(sv->error, "server failed: %s", sv->error_msg.c_str());
    if (sv->stop)
        return fail(RC_E_STATE, "server is stopping");
    if (r->lib_outputs && !sv->slab.p) {  // first request with library outputs: the arena slab
        RC_TRY(set_device(c));
        RC_TRY(c->pool.alloc(sv->slab, sv->budget));
        sv->arena.reset(sv->budget);
    }
    r->ticket = sv->next_ticket++;
    r->t_submit = now_s();
    *ticket = r->ticket;
    sv->queue.push_back(r.get());
    sv->reqs.emplace(r->ticket, std::move(r));
    sv->cv.notify_all();
    return RC_OK;
}

// Completion of a ticket: a request with caller buffers is released by the
// call that reports it; one with library outputs stays until rc_server_release.
static rc_status finish(rc_server *sv, uint64_t ticket, bool block, int32_t *done, double *latency)
{
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end())
        return fail(RC_E_INVALID, "unknown or already released ticket %llu", (unsigned long long)ticket);
    Req *r = it->second.get();
    if (block)
        sv->cv.wait(lk, [&] { return r->state == 2; });
    if (r->state != 2) {
        if (done)
            *done = 0;
        return RC_OK;
    }
    if (done)
        *done = 1;
    if (latency)
        *latency = r->t_done - r->t_submit;
    if (!r->lib_outputs)
        sv->reqs.erase(it);
    if (sv->error != RC_OK)
        return fail(sv->error, "server failed: %s", sv->error_msg.c_str());
    return RC_OK;
}

rc_status rc_server_poll(rc_server *sv, uint64_t ticket, int32_t *done, double *latency_s)
{
    RC_CHECK(sv && done, "NULL argument");
    return finish(sv, ticket, false, done, latency_s);
}

rc_status rc_server_wait(rc_server *sv, uint64_t ticket, double *latency_s)
{
    RC_CHECK(sv, "NULL server");
    return finish(sv, ticket, true, nullptr, latency_s);
}

rc_status rc_server_outputs(rc_server *sv, uint64_t ticket, rc_outputs *out)
{
    RC_CHECK(sv && out, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end())
        return fail(RC_E_INVALID, "unknown or already released ticket %llu", (unsigned long long)ticket);
    const Req &r = *it->second;
    if (!r.lib_outputs)
        return fail(RC_E_INVALID, "ticket %llu writes caller buffers", (unsigned long long)ticket);
    if (r.state != 2)
        return fail(RC_E_STATE, "ticket %llu has not completed", (unsigned long long)ticket);
    *out = rc_outputs{};
    out->depth = r.depth;
    out->seg = r.seg;
    out->tri = r.tri;
    out->hit_xyz = r.hit;
    return RC_OK;
}

rc_status rc_server_release(rc_server *sv, uint64_t ticket)
{
    RC_CHECK(sv, "NULL server");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end())
        return fail(RC_E_INVALID, "unknown or already released ticket %llu", (unsigned long long)ticket);
    Req &r = *it->second;
    if (!r.lib_outputs)
        return fail(RC_E_INVALID, "ticket %llu writes caller buffers (released by poll or wait)",
                    (unsigned long long)ticket);
    if (r.state != 2)
        return fail(RC_E_STATE, "ticket %llu has not completed", (unsigned long long)ticket);
    if (r.depth || r.seg || r.tri || r.hit) {  // admitted: its block and charge are held
        sv->arena.release(r.pending.arena_off, r.pending.arena_bytes);
        sv->in_use -= r.pending.arena_bytes;
    }
    sv->reqs.erase(it);
    sv->cv.notify_all();
    return RC_OK;
}

rc_status rc_server_destroy(rc_server *sv)
{
    if (!sv)
        return RC_OK;
    if (sv->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stop = true;
        }
        sv->cv.notify_all();
        sv->worker.join();
        sv->ctx->servers -= 1;
    }
    (void)hipSetDevice(sv->ctx->device);
    for (auto &slp : sv->slots) {
        Slot &sl = *slp;
        if (sl.stream)
            (void)hipStreamSynchronize(sl.stream);
        if (sl.done)
            (void)hipEventDestroy(sl.done);
        if (sl.stream)
            (void)hipStreamDestroy(sl.stream);
        if (sl.host)
            (void)hipHostFree(sl.host);
    }
    delete sv;
    return RC_OK;
}

}  // extern "C"
