// rc_api.cpp -- host runtime behind the C ABI in include/rc.h.
//
// Owns the device copies of meshes, scenes, BVHs and sensors of one context,
// enforces the memory budget, validates arguments before queueing work, and
// dispatches the kernels of rc_build.hip / rc_render.hip on HIP streams.
#include "rc.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "rc_runtime.hpp"

using namespace rc;

namespace rc {

namespace {
thread_local std::string g_err;
}

rc_status fail(rc_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

rc_status hip_fail(hipError_t e, const char *what) { return fail(RC_E_HIP, "%s: %s", what, hipGetErrorString(e)); }

const char *last_error() { return g_err.c_str(); }

void DBuf::reset()
{
    if (p) {
        if (pool)
            pool->release(p, n);
        else
            (void)hipFree(p);
    }
    p = nullptr;
    n = 0;
}

void Pool::release(void *p, size_t bytes)
{
    if (hook.alloc) {
        // the caller's allocator may hand the block out at once: let every
        // queued use of it finish first (hipFree does the same implicitly)
        (void)hipDeviceSynchronize();
        hook.free(hook.user, p, bytes, (void *)stream);
    } else {
        (void)hipFree(p);
    }
    used -= bytes;
}

rc_status Pool::alloc(DBuf &b, size_t bytes)
{
    b.reset();
    if (bytes == 0)
        bytes = 16;
    if (budget && used + bytes > budget)
        return fail(RC_E_OOM, "memory budget exceeded: %zu used + %zu requested > %zu", (size_t)used, bytes, budget);
    void *p = nullptr;
    if (hook.alloc) {
        p = hook.alloc(hook.user, bytes, (void *)stream);
        if (!p)
            return fail(RC_E_OOM, "allocator hook returned NULL for %zu bytes", bytes);
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(RC_E_OOM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        }
    }
    b.p = p;
    b.n = bytes;
    b.pool = this;
    used += bytes;
    return RC_OK;
}

BuildView Scene::view() const
{
    BuildView v;
    v.n_envs = n_envs;
    v.n_tris = n_tris;
    v.env_tri_off = d_env_tri_off.as<int64_t>();
    v.tri_env = tri_env.as<int32_t>();
    v.tri_src = tri_src.as<int2>();
    v.proto_xyz = proto_xyz.as<float>();
    v.proto_tri = proto_tri.as<int32_t>();
    v.inst_T = inst_T.as<float>();
    v.world = world.as<float>();
    v.box_lo = box_lo.as<float4>();
    v.box_hi = box_hi.as<float4>();
    v.prim = prim.as<int32_t>();
    v.tmp = tmp.as<int32_t>();
    v.nodes = nodes.as<Node>();
    v.recs = recs.as<TriRec>();
    v.pos_of = pos_of.as<int32_t>();
    v.leaf_src = leaf_src.as<int4>();
    v.inst_dyn = inst_dyn.as<uint8_t>();
    v.env_root = env_root.as<int32_t>();
    v.env_nodes = env_nodes.as<int32_t>();
    v.env_micro = env_micro.as<int32_t>();
    v.micro = micro.as<int4>();
    v.micro_off = micro_off.as<int64_t>();
    v.env_local = env_local.as<int32_t>();
    v.local_off = local_off.as<int64_t>();
    v.level_nodes = level_nodes.as<int32_t>();
    v.level_off = level_off.as<int32_t>();
    v.env_mask = nullptr;
    v.wide = wide_on ? wide.as<WideRec>() : nullptr;
    return v;
}

// Words of the per-environment stale flags (one byte per environment).
static int64_t stale_words(int64_t n_envs) { return (n_envs + 3) / 4 + 1; }

SceneView Scene::sview() const
{
    SceneView s;
    s.env_tri_off = d_env_tri_off.as<int64_t>();
    s.env_root = env_root.as<int32_t>();
    s.nodes = nodes.as<Node>();
    s.recs = recs.as<TriRec>();
    s.tri_seg = tri_seg.as<int32_t>();
    s.world = world.as<float>();
    s.tri_src = tri_src.as<int2>();
    s.proto_tri = proto_tri.as<int32_t>();
    s.n_envs = n_envs;
    s.wide = wide_on ? wide.as<WideRec>() : nullptr;
    if (two_level) {
        InstView &v = s.inst;
        v.tnodes = top->nodes.as<Node>();
        v.trecs = top->recs.as<TriRec>();
        v.troot = top->env_root.as<int32_t>();
        v.inst_off = top->d_env_tri_off.as<int64_t>();
        v.bnodes = bottom->nodes.as<Node>();
        v.brecs = bottom->recs.as<TriRec>();
        v.broot = bottom->env_root.as<int32_t>();
        v.mesh_tri_off = bottom->d_env_tri_off.as<int64_t>();
        v.inst_info = inst_info.as<int4>();
        v.inst_seg = top->tri_seg.as<int32_t>();  // one primitive per instance, in instance order
        v.inv = inst_inv.as<double>();
        v.n_inst = n_inst;
        v.bnode_count = node_base(bottom->n_tris, bottom->n_envs) + 16;
        v.brec_count = bottom->n_tris;
    }
    return s;
}

QueueView Sensors::queue(int chunk) const
{
    QueueView q;
    q.items = lpt_items.as<int2>();
    for (int i = 0; i <= kQueues; ++i)
        q.off[i] = qoff[i];
    q.head = head.as<unsigned int>();
    q.chunk = chunk;
    return q;
}

void deal_queues(const std::vector<int64_t> &order, const std::vector<int64_t> &tiles, std::vector<int2> &items,
                 int64_t off[kQueues + 1])
{
    std::vector<std::vector<int2>> per(kQueues);
    for (size_t i = 0; i < order.size(); ++i) {
        const int64_t s = order[i];
        std::vector<int2> &dst = per[i % kQueues];
        for (int64_t t = 0; t < tiles[s]; ++t)
            dst.push_back(make_int2((int)s, (int)t));
    }
    items.clear();
    off[0] = 0;
    for (int q = 0; q < kQueues; ++q) {
        items.insert(items.end(), per[q].begin(), per[q].end());
        off[q + 1] = (int64_t)items.size();
    }
}

SensorView Sensors::view() const
{
    SensorView v;
    v.models = models.as<SensorModel>();
    v.tables = tables.as<float>();
    v.si_env = si_env_d.as<int32_t>();
    v.si_model = si_model_d.as<int32_t>();
    v.ray_off = d_ray_off.as<int64_t>();
    v.pose = pose.as<float>();
    v.items = items.as<int2>();
    return v;
}

rc_status set_device(const rc_context *c)
{
    RC_HIP(hipSetDevice(c->device));
    return RC_OK;
}

}  // namespace rc

namespace {

hipStream_t pick(const rc_context *c, void *stream) { return stream ? (hipStream_t)stream : c->stream; }

template <class T>
rc_status upload(rc_context *c, DBuf &b, const T *src, size_t count, hipStream_t st)
{
    RC_TRY(c->pool.alloc(b, count * sizeof(T)));
    if (count)
        RC_HIP(hipMemcpyAsync(b.p, src, count * sizeof(T), hipMemcpyHostToDevice, st));
    return RC_OK;
}

rc_status busy_check(const rc_context *c)
{
    if (c->servers.load() > 0)
        return fail(RC_E_BUSY, "a request server is using this context");
    return RC_OK;
}

// Models with the current tile shape, concatenated direction tables.
void models_for(const rc_context *c, std::vector<SensorModel> &models, std::vector<float> &tables)
{
    models.clear();
    tables.clear();
    for (const ModelHost &h : c->models) {
        SensorModel m = h.m;
        m.tw_shift = c->tuning.tw_shift;
        const int tw = 1 << m.tw_shift, th = 64 >> m.tw_shift;
        m.tiles_x = (m.W + tw - 1) / tw;
        m.tiles = m.tiles_x * ((m.H + th - 1) / th);
        m.table_off = (int64_t)tables.size() / 3;
        tables.insert(tables.end(), h.table.begin(), h.table.end());
        models.push_back(m);
    }
}

}  // namespace

namespace rc {

// Traversal on four-wide records (tuning node width 4): the records are
// allocated on first use and filled from the binary tree whenever it is
// current (the next single-level build or refit fills them otherwise).
rc_status set_node_width(rc_context *c, int width)
{
    if (!c->scene)
        return RC_OK;
    Scene &sc = *c->scene;
    if (width != 4 || sc.two_only) {  // (two-level scenes never traverse the four-wide records)
        sc.wide_on = false;
        return RC_OK;
    }
    if (!sc.wide.p)
        RC_TRY(c->pool.alloc(sc.wide, sizeof(WideRec) * (size_t)(node_base(sc.n_tris, sc.n_envs) + 16)));
    sc.wide_on = true;
    if (sc.built && !sc.two_level)
        RC_HIP(launch_wide_fill(sc.view(), c->stream));
    return RC_OK;
}

rc_status rebuild_items(rc_context *c, Sensors &se)
{
    const Scene &sc = *c->scene;
    hipStream_t st = c->stream;
    std::vector<SensorModel> models;
    std::vector<float> tables;
    models_for(c, models, tables);
    const int64_t S = se.n_si;
    se.item_off.assign(S + 1, 0);
    for (int64_t s = 0; s < S; ++s)
        se.item_off[s + 1] = se.item_off[s] + models[se.si_model[s]].tiles;
    se.n_items = se.item_off[S];
    RC_CHECK(se.n_items < kPairFlag, "too many tiles");  // tile indices leave kPairFlag free
    std::vector<int2> items(se.n_items);
    for (int64_t s = 0; s < S; ++s)
        for (int64_t k = se.item_off[s]; k < se.item_off[s + 1]; ++k)
            items[k] = make_int2((int)s, (int)(k - se.item_off[s]));
    // queue order of the persistent form: sensor instances by estimated cost
    // (rays x log2 of the environment's triangle count), largest first; the
    // tiles of one instance stay together
    std::vector<int64_t> order(S);
    std::iota(order.begin(), order.end(), 0);
    if (c->tuning.lpt) {
        std::vector<double> cost(S);
        for (int64_t s = 0; s < S; ++s) {
            const int e = se.si_env[s];
            const double ntri = (double)(sc.env_tri_off[e + 1] - sc.env_tri_off[e]);
            cost[s] = (double)(se.ray_off[s + 1] - se.ray_off[s]) * log2(ntri + 2.0);
        }
        std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return cost[a] > cost[b]; });
    }
    std::vector<int64_t> tiles(S);
    for (int64_t s = 0; s < S; ++s)
        tiles[s] = se.item_off[s + 1] - se.item_off[s];
    std::vector<int2> lpt;
    deal_queues(order, tiles, lpt, se.qoff);
    // output pairs (kPairFlag): a 16-column tile and its right-hand
    // neighbour at an even offset from the queue's start, so that a pop of
    // an even number of tiles always holds both
    if ((1 << c->tuning.tw_shift) == kPairCols && c->tuning.chunk > 0 && c->tuning.chunk % 2 == 0)
        for (int q = 0; q < kQueues; ++q)
            for (int64_t j = se.qoff[q]; j + 1 < se.qoff[q + 1]; j += 2) {
                const int2 a = lpt[j], b = lpt[j + 1];
                const int tiles_x = models[se.si_model[a.x]].tiles_x, tx = a.y % tiles_x;
                if (b.x == a.x && b.y == a.y + 1 && tx % 2 == 0 && tx + 1 < tiles_x)
                    lpt[j].y |= kPairFlag;
            }
    RC_HIP(hipStreamSynchronize(st));  // previous users of the old lists are done
    RC_TRY(upload(c, se.models, models.data(), models.size(), st));
    RC_TRY(upload(c, se.tables, tables.data(), tables.size(), st));
    RC_TRY(upload(c, se.items, items.data(), items.size(), st));
    RC_TRY(upload(c, se.lpt_items, lpt.data(), lpt.size(), st));
    RC_HIP(hipStreamSynchronize(st));
    return RC_OK;
}

}  // namespace rc

extern "C" {

const char *rc_status_string(rc_status s)
{
    switch (s) {
    case RC_OK: return "ok";
    case RC_E_INVALID: return "invalid argument";
    case RC_E_OOM: return "out of memory";
    case RC_E_HIP: return "HIP error";
    case RC_E_STATE: return "invalid state";
    case RC_E_BUSY: return "busy";
    case RC_E_DEVICE: return "device error";
    default: return "unknown status";
    }
}

const char *rc_last_error(void) { return rc::last_error(); }

// Queue heads of rc_render_noalloc: a fixed device array (2 KiB), one copy
// per GPU, resident until the process ends and shared by every context on
// that GPU.  Host code never passes `scratch` itself to a kernel (on the
// host the name is a stand-in, not a device address): rc_create looks up
// each device's address once, with that device current, and keeps it in
// g_scratch.
static __device__ __align__(256) unsigned int scratch[kQueues * kQueueStride];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned int *g_scratch[kScratchDevices] = {};
}  // namespace

// The current device is `device`.
static rc_status scratch_setup(int device)
{
    RC_CHECK(device < kScratchDevices, "device %d: above the %d devices with static queue heads", device,
             kScratchDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device])
        return RC_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(RC_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    }
    g_scratch[device] = (unsigned int *)p;
    return RC_OK;
}

rc_status rc_create(int32_t device, void *stream, const rc_allocator *alloc, size_t hbm_budget, rc_context **out)
{
    RC_CHECK(out, "out is NULL");
    *out = nullptr;
    RC_CHECK(!alloc || (alloc->alloc && alloc->free), "allocator needs both alloc and free");
    int n = 0;
    RC_HIP(hipGetDeviceCount(&n));
    RC_CHECK(device >= 0 && device < n, "device %d out of range (%d devices)", device, n);
    RC_HIP(hipSetDevice(device));
    RC_TRY(scratch_setup(device));
    auto *c = new rc_context;
    c->device = device;
    c->stream = (hipStream_t)stream;
    c->pool.budget = hbm_budget;
    c->pool.stream = (hipStream_t)stream;
    if (alloc)
        c->pool.hook = *alloc;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return fail(RC_E_HIP, "hipGetDeviceProperties failed");
    }
    c->n_cu = prop.multiProcessorCount;
    c->blocks_per_cu = batched_blocks_per_cu(false);
    c->blocks_per_cu_two = batched_blocks_per_cu(true);
    *out = c;
    return RC_OK;
}

rc_status rc_destroy(rc_context *c)
{
    if (!c)
        return RC_OK;
    RC_TRY(busy_check(c));
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    c->sensors.reset();
    c->scene.reset();
    delete c;
    return RC_OK;
}

rc_status rc_memory_used(const rc_context *c, size_t *bytes)
{
    RC_CHECK(c && bytes, "NULL argument");
    *bytes = c->pool.used;
    return RC_OK;
}

rc_status rc_mesh_add(rc_context *c, const float *xyz, int32_t n_verts, const int32_t *tri3, int32_t n_tris,
                      int32_t *mesh_id)
{
    RC_CHECK(c && mesh_id, "NULL argument");
    RC_CHECK(n_verts >= 0 && n_tris >= 0, "negative sizes");
    RC_CHECK((n_verts == 0 || xyz) && (n_tris == 0 || tri3), "NULL mesh arrays");
    for (int64_t i = 0; i < 3 * (int64_t)n_verts; ++i)
        RC_CHECK(isfinite(xyz[i]), "vertex coordinate %lld is not finite", (long long)i);
    for (int64_t i = 0; i < 3 * (int64_t)n_tris; ++i)
        RC_CHECK(tri3[i] >= 0 && tri3[i] < n_verts, "triangle index %lld out of range", (long long)i);
    Mesh m{(int64_t)c->mesh_xyz.size() / 3, n_verts, (int64_t)c->mesh_tri.size() / 3, n_tris};
    c->mesh_xyz.insert(c->mesh_xyz.end(), xyz, xyz + 3 * (int64_t)n_verts);
    for (int64_t i = 0; i < 3 * (int64_t)n_tris; ++i)
        c->mesh_tri.push_back((int32_t)(tri3[i] + m.vert_off));
    *mesh_id = (int32_t)c->meshes.size();
    c->meshes.push_back(m);
    return RC_OK;
}

// Device tables of a scene over `n_envs` environments with the given CSR
// instance lists (validated by the caller).  Every instance contributes its
// mesh's triangles, or one primitive each with one_prim (a two-level scene's
// top level: one box per instance, built like triangles).  `prim_limit`
// bounds the primitives per environment.
// per_tri = false (RC_SCENE_TWO_LEVEL_ONLY): no per-triangle array is
// allocated, only the meshes and the per-instance and per-environment tables.
static rc_status make_scene(rc_context *c, int32_t n_envs, const int64_t *inst_offsets, const int32_t *inst_mesh,
                            const int32_t *inst_seg, const uint8_t *inst_dynamic, bool one_prim, int64_t prim_limit,
                            std::unique_ptr<Scene> &out, bool per_tri = true)
{
    hipStream_t st = c->stream;
    const int64_t n_inst = inst_offsets[n_envs];
    auto sc = std::make_unique<Scene>();
    sc->n_envs = n_envs;
    sc->n_inst = n_inst;
    sc->inst_offsets.assign(inst_offsets, inst_offsets + n_envs + 1);
    sc->env_tri_off.assign(n_envs + 1, 0);
    for (int32_t e = 0; e < n_envs; ++e) {
        int64_t t = 0;
        for (int64_t i = inst_offsets[e]; i < inst_offsets[e + 1]; ++i)
            t += one_prim ? 1 : c->meshes[inst_mesh[i]].n_tris;
        RC_CHECK(t <= prim_limit, "environment %d has %lld %s (limit %lld)", e, (long long)t,
                 one_prim ? "instances" : "triangles", (long long)prim_limit);
        sc->env_tri_off[e + 1] = sc->env_tri_off[e] + t;
    }
    const int64_t N = sc->env_tri_off[n_envs];
    RC_CHECK(N < INT32_MAX, "too many triangles");
    sc->n_tris = N;
    sc->two_only = !per_tri;
    std::vector<int32_t> tri_env, tri_seg, dyn;
    std::vector<int2> tri_src;
    if (per_tri) {
        tri_env.resize(N);
        tri_seg.resize(N);
        tri_src.resize(N);
    }
    std::vector<uint8_t> dynf(n_inst, 0);
    std::vector<int32_t> inst_env(n_inst, 0);
    int64_t g = 0, n_dyn = 0;
    for (int32_t e = 0; e < n_envs; ++e) {
        for (int64_t i = inst_offsets[e]; i < inst_offsets[e + 1]; ++i) {
            const Mesh &m = c->meshes[inst_mesh[i]];
            const bool d = inst_dynamic && inst_dynamic[i];
            dynf[i] = d;
            inst_env[i] = e;
            const int64_t n = one_prim ? 1 : m.n_tris;
            if (d)
                n_dyn += n;
            if (!per_tri) {
                g += n;
                continue;
            }
            for (int64_t k = 0; k < n; ++k, ++g) {
                tri_env[g] = e;
                tri_seg[g] = inst_seg[i];
                tri_src[g] = make_int2((int)i, (int)(m.tri_off + k));
                if (d)
                    dyn.push_back((int32_t)g);
            }
        }
    }
    sc->n_dyn = n_dyn;
    RC_TRY(upload(c, sc->proto_xyz, c->mesh_xyz.data(), c->mesh_xyz.size(), st));
    RC_TRY(upload(c, sc->proto_tri, c->mesh_tri.data(), c->mesh_tri.size(), st));
    RC_TRY(upload(c, sc->d_env_tri_off, sc->env_tri_off.data(), sc->env_tri_off.size(), st));
    RC_TRY(upload(c, sc->inst_dyn, dynf.data(), n_inst, st));
    RC_TRY(upload(c, sc->inst_env, inst_env.data(), n_inst, st));
    RC_TRY(c->pool.alloc(sc->inst_T, 48 * n_inst));
    RC_TRY(c->pool.alloc(sc->inst_T0, 48 * n_inst));
    RC_TRY(c->pool.alloc(sc->inst_Tw, 48 * n_inst));
    RC_TRY(c->pool.alloc(sc->stale_env, 4 * stale_words(n_envs)));
    RC_HIP(launch_fill_u32(sc->stale_env.as<unsigned int>(), stale_words(n_envs), 0u, st));
    RC_TRY(c->pool.alloc(sc->env_root, 4 * (size_t)n_envs));
    RC_TRY(c->pool.alloc(sc->env_nodes, 4 * (size_t)n_envs));
    RC_TRY(c->pool.alloc(sc->env_micro, 4 * (size_t)n_envs));
    RC_TRY(c->pool.alloc(sc->level_off, 4 * (size_t)n_envs * (kLevels + 1)));
    RC_TRY(c->pool.alloc(sc->micro_off, 8 * ((size_t)n_envs + 1)));
    RC_TRY(c->pool.alloc(sc->env_local, 4 * (size_t)n_envs));
    RC_TRY(c->pool.alloc(sc->local_off, 8 * ((size_t)n_envs + 1)));
    RC_TRY(c->pool.alloc(sc->sah_mask, (size_t)n_envs + 16));
    if (per_tri) {
        RC_TRY(upload(c, sc->tri_env, tri_env.data(), N, st));
        RC_TRY(upload(c, sc->tri_seg, tri_seg.data(), N, st));
        RC_TRY(upload(c, sc->tri_src, tri_src.data(), N, st));
        RC_TRY(upload(c, sc->dyn_tris, dyn.data(), dyn.size(), st));
        RC_TRY(c->pool.alloc(sc->world, 36 * N));
        RC_TRY(c->pool.alloc(sc->box_lo, 16 * N));
        RC_TRY(c->pool.alloc(sc->box_hi, 16 * N));
        RC_TRY(c->pool.alloc(sc->prim, 4 * N));
        RC_TRY(c->pool.alloc(sc->tmp, 4 * N));
        RC_TRY(c->pool.alloc(sc->nodes, sizeof(Node) * (size_t)(node_base(N, n_envs) + 16)));
        RC_TRY(c->pool.alloc(sc->recs, sizeof(TriRec) * N));
        RC_TRY(c->pool.alloc(sc->pos_of, 4 * N));
        RC_TRY(c->pool.alloc(sc->micro, 16 * N));
        RC_TRY(c->pool.alloc(sc->level_nodes, 4 * (size_t)(node_base(N, n_envs) + 16)));
        RC_TRY(c->pool.alloc(sc->leaf_src, 16 * N));
    }
    out = std::move(sc);
    return RC_OK;
}

rc_status rc_scene_options(rc_context *c, int32_t flags)
{
    RC_CHECK(c, "NULL context");
    RC_CHECK((flags & ~RC_SCENE_TWO_LEVEL_ONLY) == 0, "unknown scene option bits 0x%x", (unsigned)flags);
    c->scene_flags = flags;
    return RC_OK;
}

rc_status rc_scene_load(rc_context *c, int32_t n_envs, const int64_t *inst_offsets, const int32_t *inst_mesh,
                        const int32_t *inst_seg, const uint8_t *inst_dynamic)
{
    RC_CHECK(c, "NULL context");
    RC_TRY(busy_check(c));
    RC_CHECK(n_envs >= 0, "n_envs < 0");
    RC_CHECK(inst_offsets, "inst_offsets is NULL");
    RC_CHECK(inst_offsets[0] == 0, "inst_offsets[0] != 0");
    for (int32_t e = 0; e < n_envs; ++e)
        RC_CHECK(inst_offsets[e + 1] >= inst_offsets[e], "inst_offsets not non-decreasing at %d", e);
    const int64_t n_inst = inst_offsets[n_envs];
    RC_CHECK(n_inst == 0 || (inst_mesh && inst_seg), "NULL instance arrays");
    const int64_t n_meshes = (int64_t)c->meshes.size();
    for (int64_t i = 0; i < n_inst; ++i)
        RC_CHECK(inst_mesh[i] >= 0 && inst_mesh[i] < n_meshes, "inst_mesh[%lld] = %d is not a mesh id",
                 (long long)i, inst_mesh[i]);
    RC_TRY(set_device(c));
    std::unique_ptr<Scene> sc;
    const bool two_only = (c->scene_flags & RC_SCENE_TWO_LEVEL_ONLY) != 0;
    RC_TRY(make_scene(c, n_envs, inst_offsets, inst_mesh, inst_seg, inst_dynamic, false,
                      two_only ? INT32_MAX : kMaxEnvTris, sc, !two_only));
    sc->inst_mesh.assign(inst_mesh, inst_mesh + n_inst);
    sc->inst_seg_h.assign(inst_seg, inst_seg + n_inst);
    RC_HIP(hipStreamSynchronize(c->stream));
    c->sensors.reset();
    c->scene = std::move(sc);
    ++c->generation;
    return RC_OK;
}

rc_status rc_sensor_add(rc_context *c, const rc_sensor_desc *d, int32_t *sensor_id)
{
    RC_CHECK(c && d && sensor_id, "NULL argument");
    RC_CHECK(d->kind == RC_PINHOLE || d->kind == RC_LIDAR || d->kind == RC_TABLE, "unknown sensor kind %d", d->kind);
    RC_CHECK(d->width > 0 && d->height > 0, "sensor size must be positive");
    RC_CHECK((int64_t)d->width * d->height < (1ll << 31), "sensor too large");
    RC_CHECK(isfinite(d->near_) && isfinite(d->far_) && d->near_ >= 0.f && d->near_ <= d->far_,
             "need 0 <= near <= far (finite)");
    for (int k = 0; k < 3; ++k)
        RC_CHECK(isfinite(d->stereo[k]), "stereo baseline not finite");
    ModelHost h{};
    SensorModel &m = h.m;
    m.kind = d->kind;
    m.stereo = d->stereo[0] != 0.f || d->stereo[1] != 0.f || d->stereo[2] != 0.f;
    for (int k = 0; k < 3; ++k)
        m.sb[k] = d->stereo[k];
    m.W = d->width;
    m.H = d->height;
    m.tw_shift = 3;
    m.tiles_x = 0;  // set per tile shape when work lists are built
    m.tiles = 0;
    m.hw = (float)d->width * 0.5f;
    m.hh = (float)d->height * 0.5f;
    m.tn = d->near_;
    m.tf = d->far_;
    m.s = 0.f;
    m.table_off = 0;
    if (d->kind == RC_PINHOLE) {
        RC_CHECK(d->hfov > 0.f && d->hfov < 3.14159f, "pinhole hfov must be in (0, pi)");
        m.s = (float)(tan((double)d->hfov * 0.5) / ((double)d->width * 0.5));
    } else if (d->kind == RC_LIDAR) {
        RC_CHECK(isfinite(d->vmin) && isfinite(d->vmax) && isfinite(d->hmin) && isfinite(d->hmax),
                 "lidar angles must be finite");
        const int W = d->width, H = d->height;
        h.table.resize(3 * (size_t)W * H);
        for (int ch = 0; ch < H; ++ch) {
            const double el = H > 1 ? (double)d->vmax - (double)ch * ((double)d->vmax - (double)d->vmin) / (double)(H - 1)
                                    : (double)d->vmax;
            const double ce = cos(el), se = sin(el);
            for (int a = 0; a < W; ++a) {
                const double az = (double)d->hmin + (double)a * ((double)d->hmax - (double)d->hmin) / (double)W;
                float *t = &h.table[3 * ((size_t)ch * W + a)];
                t[0] = (float)(ce * cos(az));
                t[1] = (float)(ce * sin(az));
                t[2] = (float)se;
            }
        }
    } else {
        RC_CHECK(d->dir_table, "table sensor needs dir_table");
        const size_t n = 3 * (size_t)d->width * d->height;
        for (size_t i = 0; i < n; ++i)
            RC_CHECK(isfinite(d->dir_table[i]), "dir_table entry %zu not finite", i);
        h.table.assign(d->dir_table, d->dir_table + n);
    }
    *sensor_id = (int32_t)c->models.size();
    c->models.push_back(std::move(h));
    return RC_OK;
}

rc_status rc_sensors_attach(rc_context *c, const int64_t *sens_offsets, const int32_t *sensor_ids)
{
    RC_CHECK(c && sens_offsets, "NULL argument");
    RC_TRY(busy_check(c));
    if (!c->scene)
        return fail(RC_E_STATE, "rc_sensors_attach before rc_scene_load");
    const Scene &sc = *c->scene;
    const int32_t E = sc.n_envs;
    RC_CHECK(sens_offsets[0] == 0, "sens_offsets[0] != 0");
    for (int32_t e = 0; e < E; ++e)
        RC_CHECK(sens_offsets[e + 1] >= sens_offsets[e], "sens_offsets not non-decreasing at %d", e);
    const int64_t S = sens_offsets[E];
    RC_CHECK(S == 0 || sensor_ids, "sensor_ids is NULL");
    for (int64_t s = 0; s < S; ++s)
        RC_CHECK(sensor_ids[s] >= 0 && sensor_ids[s] < (int32_t)c->models.size(), "sensor_ids[%lld] invalid",
                 (long long)s);
    RC_TRY(set_device(c));
    hipStream_t st = c->stream;
    auto se = std::make_unique<Sensors>();
    se->n_si = S;
    se->sens_offsets.assign(sens_offsets, sens_offsets + E + 1);
    se->si_env.assign(S, 0);
    se->si_model.assign(S, 0);
    se->ray_off.assign(S + 1, 0);
    for (int32_t e = 0; e < E; ++e)
        for (int64_t s = sens_offsets[e]; s < sens_offsets[e + 1]; ++s)
            se->si_env[s] = e;
    for (int64_t s = 0; s < S; ++s) {
        se->si_model[s] = sensor_ids[s];
        const SensorModel &m = c->models[sensor_ids[s]].m;
        se->ray_off[s + 1] = se->ray_off[s] + (int64_t)m.W * m.H;
    }
    se->total_rays = se->ray_off[S];
    RC_TRY(upload(c, se->si_env_d, se->si_env.data(), S, st));
    RC_TRY(upload(c, se->si_model_d, se->si_model.data(), S, st));
    RC_TRY(upload(c, se->d_ray_off, se->ray_off.data(), S + 1, st));
    RC_TRY(c->pool.alloc(se->pose, 48 * (size_t)S));
    RC_TRY(c->pool.alloc(se->head, sizeof(unsigned int) * kQueues * kQueueStride));
    RC_TRY(c->pool.alloc(se->counters, 256));
    RC_TRY(rebuild_items(c, *se));
    c->sensors = std::move(se);
    ++c->generation;
    return RC_OK;
}

rc_status rc_ray_layout(const rc_context *c, int64_t *ray_offsets, int64_t *total_rays)
{
    RC_CHECK(c, "NULL context");
    if (!c->sensors)
        return fail(RC_E_STATE, "no sensors attached");
    if (ray_offsets)
        memcpy(ray_offsets, c->sensors->ray_off.data(), sizeof(int64_t) * c->sensors->ray_off.size());
    if (total_rays)
        *total_rays = c->sensors->total_rays;
    return RC_OK;
}

rc_status rc_env_tri_offsets(const rc_context *c, int64_t *off)
{
    RC_CHECK(c && off, "NULL argument");
    if (!c->scene)
        return fail(RC_E_STATE, "no scene loaded");
    memcpy(off, c->scene->env_tri_off.data(), sizeof(int64_t) * c->scene->env_tri_off.size());
    return RC_OK;
}

rc_status rc_set_instance_poses(rc_context *c, const float *d_inst_T, void *stream)
{
    RC_CHECK(c, "NULL context");
    RC_TRY(busy_check(c));
    if (!c->scene)
        return fail(RC_E_STATE, "no scene loaded");
    Scene &sc = *c->scene;
    RC_CHECK(sc.n_inst == 0 || d_inst_T, "d_inst_T is NULL");
    RC_TRY(set_device(c));
    hipStream_t st = pick(c, stream);
    if (sc.n_inst) {
        RC_HIP(hipMemcpyAsync(sc.inst_T.p, d_inst_T, 48 * sc.n_inst, hipMemcpyDeviceToDevice, st));
        RC_HIP(hipMemcpyAsync(sc.inst_T0.p, d_inst_T, 48 * sc.n_inst, hipMemcpyDeviceToDevice, st));
    }
    sc.poses_set = true;
    return RC_OK;
}

rc_status rc_set_sensor_poses(rc_context *c, const float *d_sensor_T, void *stream)
{
    RC_CHECK(c, "NULL context");
    if (!c->sensors)
        return fail(RC_E_STATE, "no sensors attached");
    Sensors &se = *c->sensors;
    RC_CHECK(se.n_si == 0 || d_sensor_T, "d_sensor_T is NULL");
    RC_TRY(set_device(c));
    if (se.n_si)
        RC_HIP(hipMemcpyAsync(se.pose.p, d_sensor_T, 48 * se.n_si, hipMemcpyDeviceToDevice, pick(c, stream)));
    se.poses_set = true;
    return RC_OK;
}

rc_status rc_move_instances(rc_context *c, const float *d_vel, int32_t step, float dt, void *stream)
{
    RC_CHECK(c, "NULL context");
    RC_TRY(busy_check(c));
    if (!c->scene || !c->scene->poses_set)
        return fail(RC_E_STATE, "instance poses not set");
    Scene &sc = *c->scene;
    RC_CHECK(sc.n_inst == 0 || d_vel, "d_vel is NULL");
    RC_CHECK(isfinite(dt), "dt not finite");
    RC_TRY(set_device(c));
    RC_HIP(launch_move(sc.n_inst, sc.inst_T0.as<float>(), d_vel, sc.inst_dyn.as<uint8_t>(), step, nullptr, dt,
                       sc.inst_T.as<float>(), pick(c, stream)));
    return RC_OK;
}

// The world copy of every environment matches its records again.
static rc_status world_fresh(Scene &sc, hipStream_t st)
{
    if (sc.world_stale)
        RC_HIP(launch_fill_u32(sc.stale_env.as<unsigned int>(), stale_words(sc.n_envs), 0u, st));
    sc.world_stale = sc.stale_all = false;
    return RC_OK;
}


// Per-instance inverse poses and top-level boxes of a two-level scene (with
// recs: also the top level's leaf records, for its refit).
static rc_status inst_prep(Scene &sc, const uint8_t *d_env_mask, bool recs, hipStream_t st)
{
    InstPrep p;
    p.n_inst = sc.n_inst;
    p.inst_T = sc.inst_T.as<float>();
    p.inst_env = sc.inst_env.as<int32_t>();
    p.env_mask = d_env_mask;
    p.inst_info = sc.inst_info.as<int4>();
    p.mesh_box = sc.mesh_box.as<float>();
    p.env_off = sc.top->d_env_tri_off.as<int64_t>();
    p.inv = sc.inst_inv.as<double>();
    p.world = sc.top->world.as<float>();
    p.recs = recs ? sc.top->recs.as<TriRec>() : nullptr;
    p.pos_of = sc.top->pos_of.as<int32_t>();
    RC_HIP(launch_inst_prep(p, st));
    return RC_OK;
}

// The bottom level (one BVH per mesh in the mesh's own frame, shared by all
// its instances) and the per-instance tables of a two-level scene; rebuilt
// only when meshes were added since.
static rc_status two_level_tables(rc_context *c, Scene &sc, hipStream_t st)
{
    const int64_t M = (int64_t)c->meshes.size();
    const int64_t bottom_limit = (int64_t)kLeafMax << (kBottomDepth + 1);
    for (int64_t m = 0; m < M; ++m)
        RC_CHECK(c->meshes[m].n_tris <= bottom_limit,
                 "mesh %lld has %lld triangles: a two-level build admits %lld per mesh", (long long)m,
                 (long long)c->meshes[m].n_tris, (long long)bottom_limit);
    if (!sc.bottom || sc.bottom_meshes != M) {
        std::vector<int64_t> off(M + 1);
        std::vector<int32_t> mesh(M), seg(M, 0);
        for (int64_t m = 0; m <= M; ++m)
            off[m] = m;
        for (int64_t m = 0; m < M; ++m)
            mesh[m] = (int32_t)m;
        std::unique_ptr<Scene> bot;
        RC_TRY(make_scene(c, (int32_t)M, off.data(), mesh.data(), seg.data(), nullptr, false, bottom_limit, bot));
        std::vector<float> eye(12 * M, 0.f);
        for (int64_t m = 0; m < M; ++m)
            eye[12 * m + 0] = eye[12 * m + 5] = eye[12 * m + 10] = 1.f;
        RC_HIP(hipMemcpyAsync(bot->inst_T.p, eye.data(), 48 * M, hipMemcpyHostToDevice, st));
        BuildView bv = bot->view();
        bv.max_depth = kBottomDepth;
        RC_HIP(launch_transform(bv, nullptr, bot->n_tris, false, st));
        RC_HIP(launch_build_sah(bv, st));
        // each mesh's vertex bounds (of the vertices its triangles use)
        std::vector<float> box(6 * M);
        for (int64_t m = 0; m < M; ++m) {
            const Mesh &h = c->meshes[m];
            float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
            for (int64_t k = 0; k < 3 * h.n_tris; ++k) {
                const float *v = &c->mesh_xyz[3 * (size_t)c->mesh_tri[3 * h.tri_off + k]];
                for (int a = 0; a < 3; ++a) {
                    lo[a] = fminf(lo[a], v[a]);
                    hi[a] = fmaxf(hi[a], v[a]);
                }
            }
            for (int a = 0; a < 3; ++a) {
                box[6 * m + a] = lo[a];
                box[6 * m + 3 + a] = hi[a];
            }
        }
        RC_TRY(upload(c, sc.mesh_box, box.data(), box.size(), st));
        RC_HIP(hipStreamSynchronize(st));  // the host tables above go out of scope
        sc.bottom = std::move(bot);
        sc.bottom_meshes = M;
    }
    if (!sc.top) {
        std::vector<int32_t> one(sc.n_inst, 0);
        std::unique_ptr<Scene> top;
        RC_TRY(make_scene(c, sc.n_envs, sc.inst_offsets.data(), one.data(), sc.inst_seg_h.data(), nullptr, true,
                          (int64_t)kLeafMax << (kTopDepth + 1), top));
        std::vector<int4> info(sc.n_inst);
        for (int32_t e = 0; e < sc.n_envs; ++e) {
            int64_t t = 0;
            for (int64_t i = sc.inst_offsets[e]; i < sc.inst_offsets[e + 1]; ++i) {
                info[i] = make_int4(sc.inst_mesh[i], (int)t, 0, 0);
                t += c->meshes[sc.inst_mesh[i]].n_tris;
            }
        }
        RC_TRY(upload(c, sc.inst_info, info.data(), info.size(), st));
        RC_TRY(c->pool.alloc(sc.inst_inv, 96 * (size_t)sc.n_inst));
        RC_HIP(hipStreamSynchronize(st));
        sc.top = std::move(top);
    }
    return RC_OK;
}

rc_status rc_build(rc_context *c, const uint8_t *d_env_mask, int32_t builder, void *stream)
{
    RC_CHECK(c, "NULL context");
    RC_TRY(busy_check(c));
    RC_CHECK(builder == RC_BUILD_SAH || builder == RC_BUILD_LBVH || builder == RC_BUILD_TWO_LEVEL,
             "unknown builder %d", builder);
    if (!c->scene || !c->scene->poses_set)
        return fail(RC_E_STATE, "rc_build needs a scene and instance poses");
    Scene &sc = *c->scene;
    const bool two = builder == RC_BUILD_TWO_LEVEL;
    if (d_env_mask && !sc.built)
        return fail(RC_E_STATE, "a masked rc_build needs a full build first");
    if (d_env_mask && two != sc.two_level)
        return fail(RC_E_STATE, "a masked rc_build must use the form (two-level or not) of the last full build");
    if (sc.two_only && !two)
        return fail(RC_E_STATE, "a scene loaded with RC_SCENE_TWO_LEVEL_ONLY builds with RC_BUILD_TWO_LEVEL only");
    RC_TRY(set_device(c));
    hipStream_t st = pick(c, stream);
    if (two)  // before any work is queued: this may fail on the mesh size limit
        RC_TRY(two_level_tables(c, sc, st));
    BuildView v = sc.view();
    v.env_mask = d_env_mask;
    if (!sc.two_only)  // the world copy
        RC_HIP(launch_transform(v, nullptr, sc.n_tris, false, st));
    // the rebuilt environments' world triangles and records use these poses
    RC_HIP(launch_pose_snapshot(sc.n_inst, sc.inst_env.as<int32_t>(), sc.inst_dyn.as<uint8_t>(), d_env_mask, false,
                                sc.inst_T.as<float>(), sc.inst_Tw.as<float>(), nullptr, st));
    if (!d_env_mask)
        RC_TRY(world_fresh(sc, st));
    if (two) {
        // the single-level BVH is not built
        RC_TRY(inst_prep(sc, d_env_mask, false, st));
        BuildView tv = sc.top->view();
        tv.env_mask = d_env_mask;
        tv.max_depth = kTopDepth;
        RC_HIP(launch_build_sah(tv, st));
    } else {
        if (builder == RC_BUILD_LBVH)
            RC_HIP(launch_build_lbvh(v, sc.sah_mask.as<uint8_t>(), st));
        else
            RC_HIP(launch_build_sah(v, st));
    }
    if (!d_env_mask && two != sc.two_level)
        ++c->generation;  // captured step graphs hold the other form's kernels
    if (!d_env_mask)
        sc.two_level = two;
    sc.built = true;
    return RC_OK;
}

rc_status rc_refit(rc_context *c, const uint8_t *d_env_mask, void *stream)
{
    RC_CHECK(c, "NULL context");
    RC_TRY(busy_check(c));
    if (!c->scene || !c->scene->built)
        return fail(RC_E_STATE, "rc_refit before rc_build");
    Scene &sc = *c->scene;
    RC_TRY(set_device(c));
    hipStream_t st = pick(c, stream);
    if (sc.two_level) {
        // new inverse poses and top-level boxes, then the top level's refit;
        // the mesh-frame bottom level never changes
        RC_TRY(inst_prep(sc, d_env_mask, true, st));
        BuildView tv = sc.top->view();
        tv.env_mask = d_env_mask;
        RC_HIP(launch_refit(tv, st));
        if (sc.n_dyn > 0) {
            RC_HIP(launch_pose_snapshot(sc.n_inst, sc.inst_env.as<int32_t>(), sc.inst_dyn.as<uint8_t>(), d_env_mask,
                                        true, sc.inst_T.as<float>(), sc.inst_Tw.as<float>(),
                                        d_env_mask ? sc.stale_env.as<uint8_t>() : nullptr, st));
            sc.world_stale = true;
            if (!d_env_mask)
                sc.stale_all = true;
        }
        return RC_OK;
    }
    BuildView v = sc.view();
    v.env_mask = d_env_mask;
    if (sc.n_dyn > 0) {
        RC_HIP(launch_transform_leaf(v, st));
        // the poses of the moved records; a masked refit marks its environments
        RC_HIP(launch_pose_snapshot(sc.n_inst, sc.inst_env.as<int32_t>(), sc.inst_dyn.as<uint8_t>(), d_env_mask,
                                    true, sc.inst_T.as<float>(), sc.inst_Tw.as<float>(),
                                    d_env_mask ? sc.stale_env.as<uint8_t>() : nullptr, st));
        sc.world_stale = true;
        if (!d_env_mask)
            sc.stale_all = true;
    }
    RC_HIP(launch_refit(v, st));
    return RC_OK;
}

// Brings the original-order world copy up to date (on stream st) if a
// per-step transform left it stale: the stale environments (all of them
// after an unmasked refit or a step graph) are transformed with the poses
// their records were made with.
static rc_status fresh_world(rc_context *c, hipStream_t st)
{
    Scene &sc = *c->scene;
    if (sc.world_stale) {
        BuildView v = sc.view();
        v.inst_T = sc.inst_Tw.as<float>();
        v.env_mask = sc.stale_all ? nullptr : sc.stale_env.as<uint8_t>();
        RC_HIP(launch_transform(v, nullptr, sc.n_tris, false, st));
        RC_TRY(world_fresh(sc, st));
    }
    return RC_OK;
}

static rc_status render_ready(const rc_context *c)
{
    if (!c->scene || !c->scene->built)
        return fail(RC_E_STATE, "render before rc_build");
    if (!c->sensors)
        return fail(RC_E_STATE, "render before rc_sensors_attach");
    if (!c->sensors->poses_set)
        return fail(RC_E_STATE, "render before rc_set_sensor_poses");
    return RC_OK;
}

// One render on stream st; the batched form's queue heads are `heads`
// (kQueues * kQueueStride words, cleared here by a fill kernel).
static rc_status render_on(rc_context *c, const rc_outputs *out, int32_t mode, hipStream_t st, unsigned int *heads)
{
    const Scene &sc = *c->scene;
    Sensors &se = *c->sensors;
    const SceneView sv = sc.sview();
    const SensorView ev = se.view();
    const OutView ov = out_view(*out);
    const bool extras = out->normal || out->bary || out->point || out->vert;
    RC_CHECK(!(extras || out->shadow) || out->tri, "normal, bary, point, vert and shadow need the tri output");
    if (out->shadow && sc.two_level)
        return fail(RC_E_STATE, "stereo shadows need the single-level BVH (rc_build with RC_BUILD_SAH or LBVH)");
    if (sc.two_only && (mode == RC_RENDER_BRUTE || extras))
        return fail(RC_E_STATE, "the brute-force render and the further outputs read the world copy, which a scene "
                                "loaded with RC_SCENE_TWO_LEVEL_ONLY does not keep");
    if (mode == RC_RENDER_BRUTE || extras || out->shadow)
        RC_TRY(fresh_world(c, st));
    switch (mode) {
    case RC_RENDER_PLAIN:
        for (int64_t s = 0; s < se.n_si; ++s)
            RC_HIP(launch_render_flat(sv, ev, ov, se.item_off[s], se.item_off[s + 1] - se.item_off[s], st));
        break;
    case RC_RENDER_FLAT:
        RC_HIP(launch_render_flat(sv, ev, ov, 0, se.n_items, st));
        break;
    case RC_RENDER_BATCHED: {
        if (c->tuning.chunk == 0) {  // the tuned choice: one launch over every tile, no queue
            RC_HIP(launch_render_flat(sv, ev, ov, 0, se.n_items, st));
            break;
        }
        QueueView q = se.queue(c->tuning.chunk);
        q.head = heads;
        RC_HIP(launch_render_batched(sv, ev, ov, q, c->batched_grid(), st));
        break;
    }
    case RC_RENDER_BRUTE:
        RC_HIP(launch_render_brute(sv, ev, ov, se.n_items, st));
        break;
    }
    if (extras)
        RC_HIP(launch_hit_extras(sv, ev, ov, se.n_items, st));
    if (out->shadow)
        RC_HIP(launch_stereo_shadow(sv, ev, ov, se.n_items, st));
    return RC_OK;
}

rc_status rc_render(rc_context *c, const rc_outputs *out, int32_t mode, void *stream)
{
    RC_CHECK(c && out, "NULL argument");
    RC_TRY(render_ready(c));
    RC_CHECK(mode >= RC_RENDER_PLAIN && mode <= RC_RENDER_BRUTE, "unknown render mode %d", mode);
    RC_TRY(set_device(c));
    return render_on(c, out, mode, pick(c, stream), c->sensors->head.as<unsigned int>());
}

rc_status rc_render_noalloc(rc_context *c, const rc_outputs *out, void *stream)
{
    RC_CHECK(c && out, "NULL argument");
    RC_TRY(render_ready(c));
    RC_TRY(set_device(c));
    RC_CHECK(c->device < kScratchDevices && g_scratch[c->device], "no static queue heads for device %d", c->device);
    const Sensors &se = *c->sensors;
    // each queue's head counts popped tiles in 32 bits and may pass the end by one pop
    for (int i = 0; i < kQueues; ++i)
        RC_CHECK(se.qoff[i + 1] - se.qoff[i] <= (int64_t)(0xffffffffu - (unsigned)c->tuning.chunk),
                 "queue %d holds %lld tiles: above the 32-bit queue head's limit of %u", i,
                 (long long)(se.qoff[i + 1] - se.qoff[i]), 0xffffffffu - (unsigned)c->tuning.chunk);
    return render_on(c, out, RC_RENDER_BATCHED, pick(c, stream), g_scratch[c->device]);
}

rc_status rc_render_stats(rc_context *c, void *stream, int64_t *counters)
{
    RC_CHECK(c && counters, "NULL argument");
    RC_TRY(render_ready(c));
    RC_TRY(set_device(c));
    hipStream_t st = pick(c, stream);
    Sensors &se = *c->sensors;
    const OutView ov{};
    RC_HIP(launch_fill_u32(se.counters.as<unsigned int>(), 8, 0u, st));
    RC_HIP(launch_render_stats(c->scene->sview(), se.view(), ov, se.n_items, se.counters.as<unsigned long long>(),
                               st));
    unsigned long long h[3];
    RC_HIP(hipMemcpyAsync(h, se.counters.p, sizeof h, hipMemcpyDeviceToHost, st));
    RC_HIP(hipStreamSynchronize(st));
    counters[0] = (int64_t)h[0];
    counters[1] = (int64_t)h[1];
    counters[2] = (int64_t)h[2];
    counters[3] = se.total_rays;
    return RC_OK;
}

rc_status rc_debug_world(rc_context *c, float *tris9)
{
    RC_CHECK(c && tris9, "NULL argument");
    if (!c->scene || !c->scene->built)
        return fail(RC_E_STATE, "no built scene");
    if (c->scene->two_only)
        return fail(RC_E_STATE, "a scene loaded with RC_SCENE_TWO_LEVEL_ONLY keeps no world copy");
    RC_TRY(set_device(c));
    RC_TRY(fresh_world(c, c->stream));
    RC_HIP(hipStreamSynchronize(c->stream));
    RC_HIP(hipMemcpy(tris9, c->scene->world.p, 36 * c->scene->n_tris, hipMemcpyDeviceToHost));
    return RC_OK;
}

rc_status rc_debug_rays(rc_context *c, int32_t s, int64_t n, const int64_t *ray_idx, float *o, float *d)
{
    RC_CHECK(c && (n == 0 || (ray_idx && o && d)), "NULL argument");
    if (!c->sensors || !c->sensors->poses_set)
        return fail(RC_E_STATE, "sensors or sensor poses missing");
    Sensors &se = *c->sensors;
    RC_CHECK(s >= 0 && s < se.n_si, "sensor instance %d out of range", s);
    const int64_t nr = se.ray_off[s + 1] - se.ray_off[s];
    for (int64_t i = 0; i < n; ++i)
        RC_CHECK(ray_idx[i] >= 0 && ray_idx[i] < nr, "ray index %lld out of range", (long long)ray_idx[i]);
    RC_TRY(set_device(c));
    hipStream_t st = c->stream;
    DBuf di, dout;
    RC_TRY(c->pool.alloc(di, 8 * n));
    RC_TRY(c->pool.alloc(dout, 24 * n));
    RC_HIP(hipMemcpyAsync(di.p, ray_idx, 8 * n, hipMemcpyHostToDevice, st));
    float *od = dout.as<float>();
    RC_HIP(launch_debug_rays(se.view(), s, n, di.as<int64_t>(), od, od + 3 * n, st));
    RC_HIP(hipMemcpyAsync(o, od, 12 * n, hipMemcpyDeviceToHost, st));
    RC_HIP(hipMemcpyAsync(d, od + 3 * n, 12 * n, hipMemcpyDeviceToHost, st));
    RC_HIP(hipStreamSynchronize(st));
    return RC_OK;
}

rc_status rc_debug_bvh(rc_context *c, int32_t e, int32_t *n_nodes, float *boxes, int32_t *children, int32_t *parent,
                       int32_t *leaf_ids, int32_t *root)
{
    RC_CHECK(c && n_nodes && boxes && children && parent && leaf_ids && root, "NULL argument");
    if (!c->scene || !c->scene->built)
        return fail(RC_E_STATE, "no built scene");
    const Scene &sc = *c->scene;
    if (sc.two_level)
        return fail(RC_E_STATE, "the scene's last build was two-level");
    RC_CHECK(e >= 0 && e < sc.n_envs, "environment %d out of range", e);
    RC_TRY(set_device(c));
    RC_HIP(hipStreamSynchronize(c->stream));
    const int64_t base = sc.env_tri_off[e], n = sc.env_tri_off[e + 1] - base;
    int32_t nn = 0;
    RC_HIP(hipMemcpy(&nn, sc.env_nodes.as<int32_t>() + e, 4, hipMemcpyDeviceToHost));
    RC_HIP(hipMemcpy(root, sc.env_root.as<int32_t>() + e, 4, hipMemcpyDeviceToHost));
    std::vector<Node> nodes(nn);
    std::vector<TriRec> recs(n);
    if (nn)
        RC_HIP(hipMemcpy(nodes.data(), sc.nodes.as<Node>() + node_base(base, e), sizeof(Node) * nn,
                         hipMemcpyDeviceToHost));
    if (n)
        RC_HIP(hipMemcpy(recs.data(), sc.recs.as<TriRec>() + base, sizeof(TriRec) * n, hipMemcpyDeviceToHost));
    *n_nodes = nn;
    for (int32_t i = 0; i < nn; ++i) {
        const Node &d = nodes[i];
        const float b[12] = {d.xy0.x, d.xy0.z, d.z01.x, d.xy0.y, d.xy0.w, d.z01.y,
                             d.xy1.x, d.xy1.z, d.z01.z, d.xy1.y, d.xy1.w, d.z01.w};
        memcpy(boxes + 12 * (int64_t)i, b, sizeof b);
        children[2 * i] = d.ch.x;
        children[2 * i + 1] = d.ch.y;
        parent[i] = d.ch.z;
    }
    for (int64_t i = 0; i < n; ++i) {
        int32_t id;
        memcpy(&id, &recs[i].c.y, 4);
        leaf_ids[i] = id;
    }
    return RC_OK;
}

}  // extern "C"
