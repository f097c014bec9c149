// rc_common.hpp -- data layouts shared by the renderer's host runtime and its
// gfx950 kernels (internal to the library; the public ABI is include/rc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rc {

// ---------------------------------------------------------------------------
// BVH layout.  Binary BVH with both child boxes stored in the parent (one
// 64-byte node fetch tests two children).  Child refs: >= 0 internal node
// index (environment-local, node array of environment e starts at
// env_tri_off[e]); < 0 leaf ~(first << 3 | (count - 1)) over the
// environment's leaf-ordered triangle records.
// ---------------------------------------------------------------------------
// The depth bound sizes the per-lane traversal stack in LDS, and that stack
// is what limits how many render waves a CU holds: 18 keeps seven waves per
// SIMD resident (20 KB of stack and 2 KB of output-pair slots per 256-thread
// block, seven blocks in a CU's 160 KB) and still admits 2^21 triangles per
// environment.
#ifndef RC_MAX_NODE_DEPTH
#define RC_MAX_NODE_DEPTH 18
#endif
constexpr int kLeafMax = 4;                        // triangles per leaf (<= 8 by the encoding)
constexpr int kMaxNodeDepth = RC_MAX_NODE_DEPTH;   // internal-node depth bound enforced by the builder
constexpr int kStack = RC_MAX_NODE_DEPTH + 2;      // traversal stack entries (> kMaxNodeDepth)
// Largest environment the bound admits: a balanced tree over this many
// triangles has its deepest internal node at depth kMaxNodeDepth.
constexpr int64_t kMaxEnvTris = (int64_t)kLeafMax << (kMaxNodeDepth + 1);
constexpr int kLevels = kMaxNodeDepth + 1;  // internal-node depths 0 .. kMaxNodeDepth
static_assert(kMaxEnvTris <= (int64_t(1) << 28), "leaf references hold 28-bit record offsets");
#ifndef RC_BINS
#define RC_BINS 32
#endif
constexpr int kBins = RC_BINS;     // SAH bins per axis
constexpr int kEmptyRoot = INT32_MIN;

struct alignas(16) Node {
    float4 xy0;  // child 0: lo.x hi.x lo.y hi.y
    float4 xy1;  // child 1: lo.x hi.x lo.y hi.y
    float4 z01;  // lo0.z hi0.z lo1.z hi1.z
    int4 ch;     // child0, child1, parent (-1 at the root), depth (root 0)
};
static_assert(sizeof(Node) == 64, "node is one 64-byte fetch");

// Four-wide view of the same tree: for internal node m, the boxes one level
// further down, stored beside the node array (same index).  Slots 0 and 1
// come from child 0 of m, slots 2 and 3 from child 1: an internal child
// contributes its two children (refs and boxes as stored in the child), a
// leaf child occupies its first slot with its own box (as stored in m) and
// leaves the second one empty (ref kDoneRef, the box [+inf, +inf] on every
// axis, which no slab test accepts).  pair.x / pair.y
// are m's two children themselves.  Box components are stored slot-major
// (lox = the low x of slots 0..3), so that one 16-byte load gives one plane
// of all four boxes.  Rebuilt by k_wide_fill after every build and refit.
constexpr int kDoneRef = INT32_MIN;  // "nothing": an empty slot, the end of a traversal
struct alignas(16) WideRec {
    float4 lox, hix, loy, hiy, loz, hiz;
    int4 ref;
    int4 pair;  // child 0, child 1 of m, 0, 0
};
static_assert(sizeof(WideRec) == 128, "wide record is two 64-byte lines");

// Leaf-ordered triangle record: 3 vertices + environment-local triangle id.
struct alignas(16) TriRec {
    float4 a;  // v0.x v0.y v0.z v1.x
    float4 b;  // v1.y v1.z v2.x v2.y
    float4 c;  // v2.z, id (bits), 0, 0
};
static_assert(sizeof(TriRec) == 48, "record is three 16-byte fetches");

__host__ __device__ inline int leaf_ref(int first, int count) { return ~((first << 3) | (count - 1)); }

// First node slot of environment e (tri_off = env_tri_off[e]).  Each
// environment gets n + n/4 + 2 slots for n triangles; its internal nodes and
// the unused ids the builder reserves for small ranges together stay below n.
__host__ __device__ inline int64_t node_base(int64_t tri_off, int e) { return tri_off + (tri_off >> 2) + 2 * (int64_t)e; }

// ---------------------------------------------------------------------------
// Sensors.
// ---------------------------------------------------------------------------
struct SensorModel {
    int32_t kind;     // 0 pinhole, 1 lidar, 2 table
    int32_t W, H;     // pinhole W x H; lidar azimuths x channels
    int32_t tw_shift; // ray tile = (1 << tw_shift) columns x (64 >> tw_shift) rows (one wavefront)
    int32_t tiles_x;  // ray tiles per row of tiles
    int32_t tiles;    // tiles per sensor instance
    float s;          // pinhole: tan(hfov/2)/(W/2)
    float hw, hh;     // W/2, H/2
    float tn, tf;     // near, far
    int64_t table_off;  // float3 entries into the direction table (lidar/table)
    float sb[3];      // stereo pair's second centre in the sensor frame
    int32_t stereo;   // nonzero when sb is set
};

// ---------------------------------------------------------------------------
// Kernel argument views.
// ---------------------------------------------------------------------------
// Two-level scenes: a top-level BVH per environment over its instances'
// world boxes and one bottom-level BVH per mesh in the mesh's own frame,
// shared by every instance of the mesh; rays enter each visited instance's
// frame.  The top level is a BVH over one box primitive per instance, stored
// with the layout of the triangle BVH: environment e's nodes start at
// node_base(inst_off[e], e), and each leaf record holds the box (lo, hi, lo)
// as a triangle and the environment-local instance index as its id.
constexpr int kTopDepth = 10;     // top-level internal-node depth bound (<= 4 << 11 instances per env)
constexpr int kBottomDepth = 11;  // bottom-level bound (<= 4 << 12 triangles per mesh)
// The two-level kernels run at four waves per SIMD (their registers, not LDS,
// bound them) and have a deeper stack of their own.
constexpr int kStackTwo = 24;
static_assert((kTopDepth + 1) + (kBottomDepth + 1) <= kStackTwo, "both levels share the traversal stack");
static_assert(kTopDepth <= kMaxNodeDepth && kBottomDepth <= kMaxNodeDepth, "levels within the builder's bound");
struct InstView {
    const Node *tnodes = nullptr;        // top level; tnodes == nullptr: a flat scene
    const TriRec *trecs = nullptr;       // top-level leaf records, env e from inst_off[e]
    const int32_t *troot = nullptr;      // [E]
    const int64_t *inst_off = nullptr;   // [E+1]
    const Node *bnodes = nullptr;        // bottom levels, mesh m at node_base(mesh_tri_off[m], m)
    const TriRec *brecs = nullptr;       // mesh triangles in their own frame, mesh m from mesh_tri_off[m]
    const int32_t *broot = nullptr;      // [M]
    const int64_t *mesh_tri_off = nullptr;  // [M+1]
    const int4 *inst_info = nullptr;     // [I] mesh, environment-local id of the instance's first triangle
    const int32_t *inst_seg = nullptr;   // [I] segment label of each instance
    const double *inv = nullptr;         // [I][12] FP64 rows (M_r0 M_r1 M_r2 p_r) with M the inverse of
                                         // the pose's linear part and p its translation
    int64_t n_inst = 0, bnode_count = 0, brec_count = 0;  // sizes of the arrays above (range-checked loads)
};

struct SceneView {
    const int64_t *env_tri_off;  // [E+1]
    const int32_t *env_root;     // [E]
    const Node *nodes;           // env e starts at node_base(env_tri_off[e], e)
    const TriRec *recs;          // [N] leaf order
    const int32_t *tri_seg;      // [N] global original order
    const float *world;          // [N][9] original order (reference path)
    const int2 *tri_src;         // [N] (instance, global prototype triangle)
    const int32_t *proto_tri;    // prototype triangles (global vertex ids)
    int32_t n_envs;
    InstView inst;               // set for a two-level scene
    const WideRec *wide = nullptr;  // set: four-wide traversal (same index as nodes)
};

struct SensorView {
    const SensorModel *models;
    const float *tables;     // float3 directions
    const int32_t *si_env;   // [S]
    const int32_t *si_model; // [S]
    const int64_t *ray_off;  // [S+1]
    const float *pose;       // [S][12]
    const int2 *items;       // (sensor instance, tile)
};

// Outputs: either one buffer per kind in the ray layout (ray_off), or, when
// the tables are set, one buffer per sensor instance (requests of a served
// batch write into their own buffers).
struct OutView {
    float *depth = nullptr;
    int32_t *seg = nullptr;
    int32_t *tri = nullptr;
    float *hit = nullptr;
    float *normal = nullptr;  // [ray][3]
    float *bary = nullptr;    // [ray][2]
    float *point = nullptr;   // [ray][3] sensor frame
    int32_t *vert = nullptr;  // [ray][3]
    uint8_t *shadow = nullptr;  // [ray] hidden from the second camera
    float *const *depth_tab = nullptr;  // per sensor instance (served batches)
    int32_t *const *seg_tab = nullptr;
    int32_t *const *tri_tab = nullptr;
    float *const *hit_tab = nullptr;    // [ray][3] per sensor instance
};

struct BuildView {
    int32_t n_envs;
    int64_t n_tris;
    const int64_t *env_tri_off;  // [E+1]
    const int32_t *tri_env;      // [N]
    const int2 *tri_src;         // [N] (instance, global prototype triangle)
    const float *proto_xyz;      // prototype vertices
    const int32_t *proto_tri;    // prototype triangles (global vertex indices)
    const float *inst_T;         // [I][12]
    float *world;                // [N][9] original order
    float4 *box_lo, *box_hi;     // [N] build scratch
    int32_t *prim, *tmp;         // [N] build scratch
    Node *nodes;                 // env e starts at node_base(env_tri_off[e], e)
    TriRec *recs;                // [N]
    int32_t *pos_of;             // [N] leaf position of env-local id
    int4 *leaf_src;              // [N] leaf order: instance, prototype triangle, env-local id, 0
    const uint8_t *inst_dyn;     // [I] dynamic flag per instance
    int32_t *env_root;           // [E]
    int32_t *env_nodes;          // [E] node slots per environment
    int32_t *env_micro;          // [E] deferred small ranges per environment
    int4 *micro;                 // [N] deferred ranges (node, begin, end, depth)
    int64_t *micro_off;          // [E+1] start of env e's ranges in the list of all ranges
    int32_t *env_local;          // [E] subtrees of at most kSmall primitives deferred per environment
    int64_t *local_off;          // [E+1] start of env e's subtrees in the list of all subtrees
    int32_t *level_nodes;        // node slots of env e grouped by depth (same base as nodes)
    int32_t *level_off;          // [E][kLevels + 1] depth d of env e = level_nodes[off[d] .. off[d+1])
    const uint8_t *env_mask;     // [E] environments to process (nullptr: all)
    int32_t max_depth = kMaxNodeDepth;  // internal-node depth bound of the trees built (<= kMaxNodeDepth)
    WideRec *wide = nullptr;            // four-wide records, refreshed by launch_wide_fill
};

// True when environment e is excluded by the build/refit mask.
__host__ __device__ inline bool masked_out(const BuildView &v, int e) { return v.env_mask && !v.env_mask[e]; }

// ---------------------------------------------------------------------------
// Launch wrappers (rc_build.hip / rc_render.hip).
// ---------------------------------------------------------------------------
hipError_t launch_transform(const BuildView &v, const int32_t *tri_list, int64_t n, bool to_recs,
                            hipStream_t st);
// The dynamic instances' triangles straight into their leaf-ordered records
// (the original-order world copy is not written).
hipError_t launch_transform_leaf(const BuildView &v, hipStream_t st);
// Copies the pose rows of the instances of the environments in env_mask (all
// when null; dynamic instances only with dyn_only) from src to dst, marking
// each such environment in stale_env when it is set.
hipError_t launch_pose_snapshot(int64_t n_inst, const int32_t *inst_env, const uint8_t *dyn, const uint8_t *env_mask,
                                bool dyn_only, const float *src, float *dst, uint8_t *stale_env, hipStream_t st);
// Two-level scenes, per instance: the FP64 inverse of the pose (InstView::inv)
// and the world box of its mesh's box under the pose, as the box primitive
// (lo, hi, lo) of the top level in original order (world, 9 floats per
// instance) and, with recs set, in the top level's leaf-ordered records
// (recs[env_off[e] + pos_of[i]]).  A pose with a singular linear part gets a
// zero-volume box at its translation and an all-NaN inverse (its instance
// is never hit).  Only environments in env_mask (all when null).
struct InstPrep {
    int64_t n_inst;
    const float *inst_T;        // [I][12]
    const int32_t *inst_env;    // [I]
    const uint8_t *env_mask;
    const int4 *inst_info;      // [I] mesh, ...
    const float *mesh_box;      // [M][6] lo.xyz hi.xyz of the mesh's vertices
    const int64_t *env_off;     // [E+1] instances per environment (top-level primitive ranges)
    double *inv;                // [I][12]
    float *world;               // [I][9]
    TriRec *recs;               // nullptr: records not written
    const int32_t *pos_of;      // [I] leaf position of an environment's instance
};
hipError_t launch_inst_prep(const InstPrep &p, hipStream_t st);
hipError_t launch_move(int64_t n_inst, const float *T0, const float *vel, const uint8_t *dyn, int32_t step,
                       const int32_t *d_step, float dt, float *T, hipStream_t st);
hipError_t launch_bump(int32_t *d_step, hipStream_t st);
hipError_t launch_build_sah(const BuildView &v, hipStream_t st);
hipError_t launch_build_lbvh(const BuildView &v, uint8_t *sah_mask, hipStream_t st);
hipError_t launch_refit(const BuildView &v, hipStream_t st);
// The four-wide records of every internal node of the environments the view
// admits (v.wide must be set).
hipError_t launch_wide_fill(const BuildView &v, hipStream_t st);

hipError_t launch_render_flat(const SceneView &sc, const SensorView &se, const OutView &o, int64_t item_begin,
                              int64_t n_items, hipStream_t st);
// Persistent-form work queues: one per XCD (blocks are dealt round-robin to
// the 8 XCDs, so block b serves queue b % 8 first), counters kQueueStride
// words apart; a wavefront pops `chunk` tiles at a time and moves on to the
// next queue when its own is empty.
constexpr int kQueues = 8;
constexpr int kQueueStride = 64;
// Output pairs: with 16-column tiles and an even pop size, the queue marks a
// tile whose right-hand neighbour (same sensor instance, same tile row)
// follows it at an even offset from the queue's start, so that both are
// always popped together: kPairFlag set in the first tile's index.  The
// render then writes the two tiles' depth and segmentation rows together,
// as whole 128-byte lines.
constexpr int kPairCols = 16;
constexpr int kPairFlag = 1 << 30;
struct QueueView {
    const int2 *items;          // kQueues consecutive ranges of (sensor instance, tile [| kPairFlag])
    int64_t off[kQueues + 1];   // range q = [off[q], off[q+1])
    unsigned int *head;         // kQueues * kQueueStride counters
    int chunk;                  // tiles per pop
};
hipError_t launch_render_batched(const SceneView &sc, const SensorView &se, const OutView &o, const QueueView &q,
                                 int grid, hipStream_t st);
int batched_blocks_per_cu(bool two_level);  // resident blocks per CU of the persistent kernel
// Normals, barycentrics, sensor-frame points and vertex ids of rendered rays
// (needs o.tri from a preceding render of the same rays).
hipError_t launch_hit_extras(const SceneView &sc, const SensorView &se, const OutView &o, int64_t n_items,
                             hipStream_t st);
// Stereo shadows of rendered rays (needs o.tri from a preceding render).
hipError_t launch_stereo_shadow(const SceneView &sc, const SensorView &se, const OutView &o, int64_t n_items,
                                hipStream_t st);
hipError_t launch_render_brute(const SceneView &sc, const SensorView &se, const OutView &o, int64_t n_items,
                               hipStream_t st);
hipError_t launch_render_stats(const SceneView &sc, const SensorView &se, const OutView &o, int64_t n_items,
                               unsigned long long *counters, hipStream_t st);
hipError_t launch_debug_rays(const SensorView &se, int32_t s, int64_t n, const int64_t *ray_idx, float *o,
                             float *d, hipStream_t st);
hipError_t launch_fill_u32(unsigned int *p, int64_t n, unsigned int value, hipStream_t st);

}  // namespace rc
