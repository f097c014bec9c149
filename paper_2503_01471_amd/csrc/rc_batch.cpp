// rc_batch.cpp -- the batched form: autotuned launch choices and the
// per-step HIP graph (motion -> transform -> refit -> queue reset -> render).
#include <stdio.h>
#include <string.h>

#include <cmath>

#include <string>
#include <vector>

#include "rc_runtime.hpp"

using namespace rc;

struct rc_graph {
    rc_context *ctx = nullptr;
    uint64_t generation = 0;
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    DBuf step;
    bool world_kept = false;  // the graph refreshes the original-order world copy itself
};

namespace {

rc_status ready(const rc_context *c)
{
    if (!c->scene || !c->scene->built)
        return fail(RC_E_STATE, "needs a built scene");
    if (!c->sensors || !c->sensors->poses_set)
        return fail(RC_E_STATE, "needs attached sensors with poses");
    return RC_OK;
}

std::string workload_key(const rc_context *c)
{
    hipDeviceProp_t p;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&p, c->device) == hipSuccess)
        arch = p.gcnArchName;
    for (char &ch : arch)
        if (ch == ' ' || ch == ':')
            ch = '_';
    char buf[256];
    snprintf(buf, sizeof buf, "%s/cu%d/envs%d/tris%lld/rays%lld/si%lld", arch.c_str(), c->n_cu, c->scene->n_envs,
             (long long)c->scene->n_tris, (long long)c->sensors->total_rays, (long long)c->sensors->n_si);
    std::string key = buf;
    if (c->scene->two_level)
        key += "/two";
    for (const ModelHost &h : c->models) {
        snprintf(buf, sizeof buf, "/m%d.%dx%d", h.m.kind, h.m.W, h.m.H);
        key += buf;
    }
    return key;
}

}  // namespace

extern "C" {

rc_status rc_autotune(rc_context *c, const char *cache_path, int32_t *choice)
{
    RC_CHECK(c, "NULL context");
    if (c->servers.load() > 0)
        return fail(RC_E_BUSY, "a request server is using this context");
    RC_TRY(ready(c));
    RC_TRY(set_device(c));
    Sensors &se = *c->sensors;
    const Scene &sc = *c->scene;
    const std::string key = workload_key(c);
    Tuning best = c->tuning;
    bool found = false;
    if (cache_path) {
        if (FILE *f = fopen(cache_path, "r")) {
            char line[1200], k[1024];
            int tw, ch, lpt, width;
            while (fgets(line, sizeof line, f)) {
                if (sscanf(line, "%1023s %d %d %d %d", k, &tw, &ch, &lpt, &width) != 5)
                    continue;  // a line of another format
                if (key == k && (tw == 4 || tw == 8 || tw == 16 || tw == 32) && ch >= 0 && ch <= 64 &&
                    (width == 2 || width == 4)) {
                    best.tw_shift = __builtin_ctz(tw);
                    best.chunk = ch;
                    best.lpt = lpt != 0;
                    best.width = width;
                    found = true;
                }
            }
            fclose(f);
        }
    }
    if (!found) {
        hipStream_t st = c->stream;
        DBuf depth, seg;
        RC_TRY(c->pool.alloc(depth, 4 * (size_t)se.total_rays));
        RC_TRY(c->pool.alloc(seg, 4 * (size_t)se.total_rays));
        OutView ov;
        ov.depth = depth.as<float>();
        ov.seg = seg.as<int32_t>();
        hipEvent_t e0, e1;
        RC_HIP(hipEventCreate(&e0));
        RC_HIP(hipEventCreate(&e1));
        float best_ms = 1e30f;
        const int chunks[4] = {0, 2, 4, 16};  // 0: one launch over every tile, no queue
        // node width 4 (four-wide records) for single-level scenes only
        for (int width = 2; width <= (sc.two_level ? 2 : 4); width += 2)
        for (int tws = 2; tws <= 5; ++tws)
            for (int ci = 0; ci < 4; ++ci)
                for (int lpt = 1; lpt >= (chunks[ci] == 0 ? 1 : 0); --lpt) {  // without a queue, no order
                    c->tuning = Tuning{tws, chunks[ci], lpt != 0, width};
                    rc_status s = set_node_width(c, width);
                    if (s == RC_OK)
                        s = rebuild_items(c, se);
                    if (s != RC_OK) {
                        (void)hipEventDestroy(e0);
                        (void)hipEventDestroy(e1);
                        return s;
                    }
                    const SensorView ev = se.view();
                    float ms = 0.f;
                    for (int rep = 0; rep < 4; ++rep) {
                        if (rep == 1)
                            RC_HIP(hipEventRecord(e0, st));
                        if (c->tuning.chunk == 0)
                            RC_HIP(launch_render_flat(sc.sview(), ev, ov, 0, se.n_items, st));
                        else
                            RC_HIP(launch_render_batched(sc.sview(), ev, ov, se.queue(c->tuning.chunk),
                                                         c->batched_grid(), st));
                    }
                    RC_HIP(hipEventRecord(e1, st));
                    RC_HIP(hipEventSynchronize(e1));
                    RC_HIP(hipEventElapsedTime(&ms, e0, e1));
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = c->tuning;
                    }
                }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (cache_path) {
            if (FILE *f = fopen(cache_path, "a")) {
                fprintf(f, "%s %d %d %d %d\n", key.c_str(), 1 << best.tw_shift, best.chunk, best.lpt ? 1 : 0,
                        best.width);
                fclose(f);
            }
        }
    }
    c->tuning = best;
    RC_TRY(set_node_width(c, best.width));
    RC_TRY(rebuild_items(c, se));
    ++c->generation;
    if (choice) {
        choice[0] = 1 << best.tw_shift;
        choice[1] = best.chunk;
        choice[2] = best.lpt ? 1 : 0;
        choice[3] = best.width;
    }
    return RC_OK;
}

rc_status rc_tuning_set(rc_context *c, const int32_t *choice)
{
    RC_CHECK(c && choice, "NULL argument");
    if (c->servers.load() > 0)
        return fail(RC_E_BUSY, "a request server is using this context");
    const int tw = choice[0];
    RC_CHECK(tw == 4 || tw == 8 || tw == 16 || tw == 32, "tile columns must be 4, 8, 16 or 32");
    RC_CHECK(choice[1] >= 0 && choice[1] <= 64, "tiles per pop must be in [0, 64] (0: no queue)");
    RC_CHECK(choice[2] == 0 || choice[2] == 1, "cost order must be 0 or 1");
    RC_CHECK(choice[3] == 2 || choice[3] == 4, "node width must be 2 or 4");
    c->tuning = Tuning{__builtin_ctz(tw), choice[1], choice[2] != 0, choice[3]};
    RC_TRY(set_device(c));
    RC_TRY(set_node_width(c, c->tuning.width));
    if (c->sensors)
        RC_TRY(rebuild_items(c, *c->sensors));
    ++c->generation;
    return RC_OK;
}

rc_status rc_step_graph_create(rc_context *c, const rc_outputs *out, const float *d_vel, float dt, rc_graph **graph)
{
    RC_CHECK(c && out && graph, "NULL argument");
    *graph = nullptr;
    RC_TRY(ready(c));
    Scene &sc = *c->scene;
    Sensors &se = *c->sensors;
    RC_CHECK(sc.n_inst == 0 || d_vel, "d_vel is NULL");
    RC_CHECK(std::isfinite(dt), "dt not finite");
    const bool extras = out->normal || out->bary || out->point || out->vert;
    RC_CHECK(!(extras || out->shadow) || out->tri, "normal, bary, point, vert and shadow need the tri output");
    if (out->shadow && sc.two_level)
        return fail(RC_E_STATE, "stereo shadows need the single-level BVH (rc_build with RC_BUILD_SAH or LBVH)");
    if (extras && sc.two_only)
        return fail(RC_E_STATE, "the further outputs read the world copy, which a scene loaded with "
                                "RC_SCENE_TWO_LEVEL_ONLY does not keep");
    RC_TRY(set_device(c));
    auto g = new rc_graph;
    g->ctx = c;
    g->generation = c->generation;
    rc_status s = c->pool.alloc(g->step, 256);
    if (s != RC_OK) {
        delete g;
        return s;
    }
    hipError_t e = launch_fill_u32(g->step.as<unsigned int>(), 1, 0u, c->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&g->capture, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete g;
        return hip_fail(e, "step graph setup");
    }
    const BuildView v = sc.view();
    const OutView ov = out_view(*out);
    hipStream_t cs = g->capture;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t k = launch_move(sc.n_inst, sc.inst_T0.as<float>(), d_vel, sc.inst_dyn.as<uint8_t>(), 0,
                                   g->step.as<int32_t>(), dt, sc.inst_T.as<float>(), cs);
        // With the further outputs or shadows in the graph (they read the
        // original-order world copy) both copies are transformed; otherwise
        // the leaf-ordered records only.
        g->world_kept = extras || out->shadow;
        if (sc.two_level) {
            // two-level: the moved triangles go to the world copy only (when
            // the further outputs read it); each instance's inverse pose and
            // box, then the refit of the instance BVH
            if (k == hipSuccess && sc.n_dyn > 0 && g->world_kept)
                k = launch_transform(v, sc.dyn_tris.as<int32_t>(), sc.n_dyn, false, cs);
            if (k == hipSuccess) {
                InstPrep p;
                p.n_inst = sc.n_inst;
                p.inst_T = sc.inst_T.as<float>();
                p.inst_env = sc.inst_env.as<int32_t>();
                p.env_mask = nullptr;
                p.inst_info = sc.inst_info.as<int4>();
                p.mesh_box = sc.mesh_box.as<float>();
                p.env_off = sc.top->d_env_tri_off.as<int64_t>();
                p.inv = sc.inst_inv.as<double>();
                p.world = sc.top->world.as<float>();
                p.recs = sc.top->recs.as<TriRec>();
                p.pos_of = sc.top->pos_of.as<int32_t>();
                k = launch_inst_prep(p, cs);
            }
        } else if (k == hipSuccess && sc.n_dyn > 0) {
            k = g->world_kept ? launch_transform(v, sc.dyn_tris.as<int32_t>(), sc.n_dyn, true, cs)
                              : launch_transform_leaf(v, cs);
        }
        if (k == hipSuccess && sc.n_dyn > 0)
            k = launch_pose_snapshot(sc.n_inst, sc.inst_env.as<int32_t>(), sc.inst_dyn.as<uint8_t>(), nullptr, true,
                                     sc.inst_T.as<float>(), sc.inst_Tw.as<float>(), nullptr, cs);
        if (k == hipSuccess)
            k = launch_refit(sc.two_level ? sc.top->view() : v, cs);
        if (k == hipSuccess)
            k = c->tuning.chunk == 0 ? launch_render_flat(sc.sview(), se.view(), ov, 0, se.n_items, cs)
                                     : launch_render_batched(sc.sview(), se.view(), ov, se.queue(c->tuning.chunk),
                                                             c->batched_grid(), cs);
        if (k == hipSuccess && extras)
            k = launch_hit_extras(sc.sview(), se.view(), ov, se.n_items, cs);
        if (k == hipSuccess && out->shadow)
            k = launch_stereo_shadow(sc.sview(), se.view(), ov, se.n_items, cs);
        if (k == hipSuccess)
            k = launch_bump(g->step.as<int32_t>(), cs);
        e = hipStreamEndCapture(cs, &g->graph);
        if (k != hipSuccess)
            e = k;
    }
    if (e == hipSuccess)
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        rc_graph_destroy(g);
        return hip_fail(e, "step graph capture");
    }
    *graph = g;
    return RC_OK;
}

rc_status rc_graph_set_step(rc_graph *g, int32_t step, void *stream)
{
    RC_CHECK(g, "NULL graph");
    RC_TRY(set_device(g->ctx));
    RC_HIP(launch_fill_u32(g->step.as<unsigned int>(), 1, (unsigned int)step,
                           stream ? (hipStream_t)stream : g->ctx->stream));
    return RC_OK;
}

rc_status rc_graph_launch(rc_graph *g, void *stream)
{
    RC_CHECK(g, "NULL graph");
    if (g->generation != g->ctx->generation)
        return fail(RC_E_STATE, "the scene, sensors or tuning changed after the graph was captured");
    RC_TRY(set_device(g->ctx));
    RC_HIP(hipGraphLaunch(g->exec, stream ? (hipStream_t)stream : g->ctx->stream));
    if (!g->world_kept && g->ctx->scene->n_dyn > 0)
        g->ctx->scene->world_stale = g->ctx->scene->stale_all = true;
    return RC_OK;
}

rc_status rc_graph_destroy(rc_graph *g)
{
    if (!g)
        return RC_OK;
    (void)hipSetDevice(g->ctx->device);
    if (g->capture)
        (void)hipStreamSynchronize(g->capture);
    if (g->exec)
        (void)hipGraphExecDestroy(g->exec);
    if (g->graph)
        (void)hipGraphDestroy(g->graph);
    if (g->capture)
        (void)hipStreamDestroy(g->capture);
    (void)hipDeviceSynchronize();
    delete g;
    return RC_OK;
}

}  // extern "C"
