// rc_runtime.hpp -- host-side state of a renderer context (internal).
//
// Shared by the ABI implementation (rc_api.cpp) and the request server
// (rc_server.cpp).  All device memory of a context goes through its Pool,
// which enforces the context's memory budget.
#pragma once

#include <stdint.h>

#include <atomic>
#include <memory>
#include <string>
#include <vector>

#include "rc.h"
#include "rc_common.hpp"

namespace rc {

rc_status fail(rc_status s, const char *fmt, ...);
rc_status hip_fail(hipError_t e, const char *what);

#define RC_HIP(call)                        \
    do {                                    \
        hipError_t e_ = (call);             \
        if (e_ != hipSuccess)               \
            return ::rc::hip_fail(e_, #call); \
    } while (0)
#define RC_CHECK(cond, ...)                                   \
    do {                                                      \
        if (!(cond))                                          \
            return ::rc::fail(RC_E_INVALID, __VA_ARGS__);     \
    } while (0)
#define RC_TRY(expr)                 \
    do {                             \
        rc_status s_ = (expr);       \
        if (s_ != RC_OK)             \
            return s_;               \
    } while (0)

struct Pool;

// Device buffer owned by a context (freed on destruction, budget released).
struct DBuf {
    void *p = nullptr;
    size_t n = 0;
    Pool *pool = nullptr;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { reset(); }
    void reset();
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

struct Pool {
    size_t budget = 0;
    std::atomic<size_t> used{0};
    rc_allocator hook{};      // caller allocator (hook.alloc == nullptr: hipMalloc)
    hipStream_t stream = nullptr;
    rc_status alloc(DBuf &b, size_t bytes);
    void release(void *p, size_t bytes);
};

struct Mesh {
    int64_t vert_off, n_verts, tri_off, n_tris;
};

struct Scene {
    int32_t n_envs = 0;
    int64_t n_inst = 0, n_tris = 0, n_dyn = 0;
    std::vector<int64_t> env_tri_off;  // host copy
    std::vector<int64_t> inst_offsets;
    DBuf proto_xyz, proto_tri, d_env_tri_off, tri_env, tri_src, tri_seg, inst_T, inst_T0, inst_dyn, dyn_tris;
    DBuf world, box_lo, box_hi, prim, tmp, nodes, recs, pos_of, env_root, env_nodes, env_micro, micro;
    DBuf level_nodes, level_off, micro_off, env_local, local_off;
    DBuf sah_mask;  // LBVH builds: environments left to the SAH kernels
    DBuf leaf_src;  // leaf order: instance, prototype triangle, env-local id, 0 (written by the build)
    bool poses_set = false;
    bool built = false;
    // RC_SCENE_TWO_LEVEL_ONLY: the per-triangle arrays of the single-level
    // form (world copy, records, nodes, build lists) were not allocated
    bool two_only = false;
    // The per-step transform writes the leaf-ordered records only; the
    // original-order world copy (read by the brute-force render, the further
    // outputs, the stereo shadows and the debug readback) is then stale until
    // refreshed by fresh_world().  The refresh transforms with inst_Tw, the
    // poses each instance's records were last made with (a caller may set new
    // poses in between), and only the environments marked in stale_env unless
    // stale_all is set; an environment outside a masked refit keeps its world
    // triangles.
    DBuf inst_Tw;    // [I][12] poses of the last build / refit per instance
    DBuf inst_env;   // [I] owning environment
    DBuf stale_env;  // [E] (padded to whole words) environments whose world copy is stale
    bool world_stale = false;  // some environment may be stale
    bool stale_all = false;    // every environment may be stale
    std::vector<int32_t> inst_mesh, inst_seg_h;  // host copies of the instance lists
    // Two-level form (rc_build with RC_BUILD_TWO_LEVEL): `top` holds one box
    // primitive per instance, `bottom` one environment per mesh (identity
    // pose), each built with the depth bound of its level.
    std::unique_ptr<Scene> top, bottom;
    DBuf inst_info;  // [I] int4: mesh, environment-local id of the instance's first triangle
    DBuf inst_inv;   // [I][12] double (InstView::inv)
    DBuf mesh_box;   // [M][6] float: each mesh's vertex bounds
    int64_t bottom_meshes = 0;  // meshes the bottom level covers
    bool two_level = false;     // the last full build was two-level
    DBuf wide;                  // four-wide records (WideRec), same index as nodes
    bool wide_on = false;       // traverse the four-wide records
    BuildView view() const;
    SceneView sview() const;
};

struct ModelHost {
    SensorModel m;
    std::vector<float> table;  // lidar / table directions (FP32)
};

struct Sensors {
    int64_t n_si = 0, n_items = 0, total_rays = 0;
    std::vector<int64_t> ray_off, item_off, sens_offsets;
    std::vector<int32_t> si_env, si_model;
    DBuf models, tables, si_env_d, si_model_d, d_ray_off, pose, items, lpt_items, head, counters;
    int64_t qoff[kQueues + 1] = {};  // queue ranges of lpt_items
    bool poses_set = false;
    SensorView view() const;
    QueueView queue(int chunk) const;
};

// Kernel view of caller output buffers.
inline OutView out_view(const rc_outputs &o)
{
    OutView v;
    v.depth = o.depth;
    v.seg = o.seg;
    v.tri = o.tri;
    v.hit = o.hit_xyz;
    v.normal = o.normal;
    v.bary = o.bary;
    v.point = o.point;
    v.vert = o.vert;
    v.shadow = o.shadow;
    return v;
}

// Launch choices of the batched form (set by rc_autotune).
struct Tuning {
    int tw_shift = 3;     // ray tile 8 x 8
    int chunk = 4;        // tiles per queue pop
    bool lpt = true;      // queue in decreasing estimated cost
    int width = 2;        // node width of the single-level traversal (2 or 4)
};

}  // namespace rc

struct rc_context {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    rc::Pool pool;
    std::vector<float> mesh_xyz;
    std::vector<int32_t> mesh_tri;  // global vertex indices
    std::vector<rc::Mesh> meshes;
    std::vector<rc::ModelHost> models;
    std::unique_ptr<rc::Scene> scene;
    std::unique_ptr<rc::Sensors> sensors;
    rc::Tuning tuning;
    int n_cu = 0, blocks_per_cu = 1, blocks_per_cu_two = 1;
    uint64_t generation = 0;   // bumped whenever scene or sensors are replaced
    int32_t scene_flags = 0;   // rc_scene_options, read by the next rc_scene_load
    std::atomic<int> servers{0};  // live request servers (scene is read-only meanwhile)
    int batched_grid() const { return n_cu * (scene && scene->two_level ? blocks_per_cu_two : blocks_per_cu); }
};

namespace rc {
// Deal sensor instances (in priority order) round-robin to the kQueues
// queues; each queue keeps the order and the tiles of one instance together.
// tiles[s] = number of tiles of sensor instance s.
void deal_queues(const std::vector<int64_t> &order, const std::vector<int64_t> &tiles, std::vector<int2> &items,
                 int64_t off[kQueues + 1]);
rc_status set_device(const rc_context *c);
const char *last_error();
// (Re)build the tile work lists of sensors `se` for the current tuning.
rc_status rebuild_items(rc_context *c, Sensors &se);
// Traverse the scene's four-wide records (width 4) or its binary nodes.
rc_status set_node_width(rc_context *c, int width);
}  // namespace rc
