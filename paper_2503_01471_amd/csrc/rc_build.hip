// rc_build.hip -- transform, BVH build and refit kernels (gfx950).
//
// Paper, Sec. III-D: every sub-mesh of environment i is moved by its own
// transform and a BVH is computed over the transformed mesh; the paper
// rebuilds it when static environments are randomised.  Here the build is a
// surface-area-heuristic builder over all environments at once: one wavefront
// per environment takes the binned splits of the large nodes, then one
// wavefront per subtree of at most kSmall primitives takes exact sweeps over
// sorted centroids, and one 16-lane group per subtree of 5..16 primitives
// finishes it; plus a bottom-up refit on the fixed topology for moving
// instances.
#include "rc_common.hpp"

namespace rc {

namespace {

// Order-preserving float <-> int mapping for LDS atomic min/max.
__device__ __forceinline__ int f2o(float f)
{
    const int i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7fffffff;
}
__device__ __forceinline__ float o2f(int i) { return __int_as_float(i >= 0 ? i : i ^ 0x7fffffff); }

// Outward expansion of a bound by one float step (never onto a subnormal or
// zero), so that a ray origin equal to a stored bound lies strictly outside the
// true box: together with IEEE infinities for zero direction components this
// keeps the slab test conservative.
__device__ __forceinline__ float expand_lo(float x)
{
    if (fabsf(x) < 0x1p-100f)
        return -0x1p-100f;
    const int i = __float_as_int(x);
    return __int_as_float(x > 0.f ? i - 1 : i + 1);
}
__device__ __forceinline__ float expand_hi(float x)
{
    if (fabsf(x) < 0x1p-100f)
        return 0x1p-100f;
    const int i = __float_as_int(x);
    return __int_as_float(x > 0.f ? i + 1 : i - 1);
}

// DPP lane moves (gfx9 encodings): row_shr:n = 0x110 + n and row_shl:n =
// 0x100 + n within rows of 16 lanes, wave_shr:1 = 0x138 and wave_shl:1 = 0x130
// across the wavefront.  Lane i reads lane i - n (shr) or i + n (shl); a lane
// whose source lies outside its row (or the wavefront) keeps `old`.  The
// wavefront helpers below (scans, reductions, readlane) are called from
// uniform control flow with all 64 lanes active; the row helpers (row_scan,
// row_xor and the 16-lane group operations built on them) read only their own
// row and need its 16 lanes active.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float old, float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float readlane_f(float x, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
template <bool MIN>
__device__ __forceinline__ float mm(float a, float b) { return MIN ? fminf(a, b) : fmaxf(a, b); }

// Inclusive in-row scan (Hillis-Steele over shifts 1, 2, 4, 8): lanes
// 16 r .. i of the row (UP) or i .. 16 r + 15.
template <bool MIN, bool UP>
__device__ __forceinline__ float row_scan(float x)
{
    constexpr float id = MIN ? INFINITY : -INFINITY;
    x = mm<MIN>(x, dpp_mov<UP ? 0x111 : 0x101>(id, x));
    x = mm<MIN>(x, dpp_mov<UP ? 0x112 : 0x102>(id, x));
    x = mm<MIN>(x, dpp_mov<UP ? 0x114 : 0x104>(id, x));
    x = mm<MIN>(x, dpp_mov<UP ? 0x118 : 0x108>(id, x));
    return x;
}
// Inclusive scan over the wavefront: lanes 0 .. i (UP) or i .. 63; the row
// totals are combined through readlane.
template <bool MIN, bool UP>
__device__ __forceinline__ float lane_scan(float x, int row)
{
    constexpr float id = MIN ? INFINITY : -INFINITY;
    x = row_scan<MIN, UP>(x);
    if (UP) {
        const float r0 = readlane_f(x, 15);
        const float r1 = mm<MIN>(r0, readlane_f(x, 31));
        const float r2 = mm<MIN>(r1, readlane_f(x, 47));
        return mm<MIN>(x, row == 0 ? id : (row == 1 ? r0 : (row == 2 ? r1 : r2)));
    }
    const float r3 = readlane_f(x, 48);
    const float r2 = mm<MIN>(r3, readlane_f(x, 32));
    const float r1 = mm<MIN>(r2, readlane_f(x, 16));
    return mm<MIN>(x, row == 3 ? id : (row == 2 ? r3 : (row == 1 ? r2 : r1)));
}
// Value of lane l ^ M within the lane's row of 16 (gl = l mod 16): quad_perm
// [1,0,3,2] (M = 1) and [2,3,0,1] (M = 2), row_ror:8 (M = 8), and for M = 4
// row_shl:4 or row_shr:4 by the lane's bit 2.
template <int M>
__device__ __forceinline__ int row_xor(int x, int gl)
{
    static_assert(M == 1 || M == 2 || M == 4 || M == 8, "partner within the row");
    if (M == 1)
        return __builtin_amdgcn_update_dpp(x, x, 0xb1, 0xf, 0xf, false);
    if (M == 2)
        return __builtin_amdgcn_update_dpp(x, x, 0x4e, 0xf, 0xf, false);
    if (M == 8)
        return __builtin_amdgcn_update_dpp(x, x, 0x128, 0xf, 0xf, false);
    const int up = __builtin_amdgcn_update_dpp(x, x, 0x104, 0xf, 0xf, false);
    const int dn = __builtin_amdgcn_update_dpp(x, x, 0x114, 0xf, 0xf, false);
    return (gl & 4) ? dn : up;
}
template <int M>
__device__ __forceinline__ float row_xor_f(float x, int gl) { return __int_as_float(row_xor<M>(__float_as_int(x), gl)); }

// Lexicographic minimum of (c, w) over the wavefront, left in every lane:
// partners 1..8 through DPP, 16 and 32 through ds_bpermute.
__device__ __forceinline__ void take_min(float &c, int &w, float oc, int ow)
{
    if (oc < c || (oc == c && ow < w)) {
        c = oc;
        w = ow;
    }
}
__device__ __forceinline__ void wave_argmin(float &c, int &w, int lane)
{
    const int gl = lane & 15;
    take_min(c, w, row_xor_f<1>(c, gl), row_xor<1>(w, gl));
    take_min(c, w, row_xor_f<2>(c, gl), row_xor<2>(w, gl));
    take_min(c, w, row_xor_f<4>(c, gl), row_xor<4>(w, gl));
    take_min(c, w, row_xor_f<8>(c, gl), row_xor<8>(w, gl));
    take_min(c, w, __shfl_xor(c, 16, 64), __shfl_xor(w, 16, 64));
    take_min(c, w, __shfl_xor(c, 32, 64), __shfl_xor(w, 32, 64));
}

template <bool MIN>
__device__ __forceinline__ float lane_reduce(float x)
{
    x = row_scan<MIN, true>(x);
    return mm<MIN>(mm<MIN>(readlane_f(x, 15), readlane_f(x, 31)), mm<MIN>(readlane_f(x, 47), readlane_f(x, 63)));
}
__device__ __forceinline__ float wave_min(float v) { return lane_reduce<true>(v); }
__device__ __forceinline__ float wave_max(float v) { return lane_reduce<false>(v); }

// ---------------------------------------------------------------------------
// K1: sub-mesh transform, one thread per world triangle.  Coordinate r of a
// world vertex is fma(A_r0, x, fma(A_r1, y, fma(A_r2, z, A_r3))).  With
// to_recs the leaf-ordered record of the triangle is refreshed as well.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_transform(BuildView v, const int32_t *__restrict__ tri_list, int64_t n,
                                                   int to_recs)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n)
        return;
    const int64_t g = tri_list ? tri_list[k] : k;
    if (masked_out(v, v.tri_env[g]))
        return;
    const int2 src = v.tri_src[g];
    const float *A = v.inst_T + 12 * (int64_t)src.x;
    float w[9];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int vi = v.proto_tri[3 * (int64_t)src.y + c];
        const float x = v.proto_xyz[3 * (int64_t)vi + 0];
        const float y = v.proto_xyz[3 * (int64_t)vi + 1];
        const float z = v.proto_xyz[3 * (int64_t)vi + 2];
#pragma unroll
        for (int r = 0; r < 3; ++r)
            w[3 * c + r] = fmaf(A[4 * r + 0], x, fmaf(A[4 * r + 1], y, fmaf(A[4 * r + 2], z, A[4 * r + 3])));
    }
#pragma unroll
    for (int j = 0; j < 9; ++j)
        v.world[9 * g + j] = w[j];
    if (to_recs) {
        const int e = v.tri_env[g];
        const int64_t base = v.env_tri_off[e];
        const int id = (int)(g - base);
        TriRec rec;
        rec.a = make_float4(w[0], w[1], w[2], w[3]);
        rec.b = make_float4(w[4], w[5], w[6], w[7]);
        rec.c = make_float4(w[8], __int_as_float(id), 0.f, 0.f);
        v.recs[base + v.pos_of[g]] = rec;
    }
}

// K1b: the per-step form of K1 for a built scene: one thread per leaf-ordered
// record, so reads and writes are coalesced; a record of a static instance is
// left as it is.  Same arithmetic as K1, so the record is bit-identical to
// the one K1 writes.  The original-order world copy is not updated (the
// library refreshes it before a path that reads it).
__global__ __launch_bounds__(256) void k_transform_leaf(BuildView v)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // a record stays inside its environment's range, so tri_env[p] is its environment
    if (p >= v.n_tris || masked_out(v, v.tri_env[p]))
        return;
    const int4 src = v.leaf_src[p];
    if (!v.inst_dyn[src.x])
        return;
    const float *A = v.inst_T + 12 * (int64_t)src.x;
    float w[9];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int vi = v.proto_tri[3 * (int64_t)src.y + c];
        const float x = v.proto_xyz[3 * (int64_t)vi + 0];
        const float y = v.proto_xyz[3 * (int64_t)vi + 1];
        const float z = v.proto_xyz[3 * (int64_t)vi + 2];
#pragma unroll
        for (int r = 0; r < 3; ++r)
            w[3 * c + r] = fmaf(A[4 * r + 0], x, fmaf(A[4 * r + 1], y, fmaf(A[4 * r + 2], z, A[4 * r + 3])));
    }
    TriRec rec;
    rec.a = make_float4(w[0], w[1], w[2], w[3]);
    rec.b = make_float4(w[4], w[5], w[6], w[7]);
    rec.c = make_float4(w[8], __int_as_float(src.z), 0.f, 0.f);
    v.recs[p] = rec;
}

// Pose record of the original-order world copy: copies the pose rows of the
// instances whose triangles a build or refit just transformed (environments
// in env_mask, dynamic instances only with dyn_only), so that a later refresh
// of the world copy uses the poses its records were made with.  With
// stale_env set, every environment touched is marked there.
__global__ __launch_bounds__(256) void k_pose_snapshot(int64_t n, const int32_t *__restrict__ inst_env,
                                                       const uint8_t *__restrict__ dyn,
                                                       const uint8_t *__restrict__ env_mask, int dyn_only,
                                                       const float *__restrict__ src, float *__restrict__ dst,
                                                       uint8_t *__restrict__ stale_env)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int e = inst_env[i];
    if ((env_mask && !env_mask[e]) || (dyn_only && !dyn[i]))
        return;
#pragma unroll
    for (int k = 0; k < 12; ++k)
        dst[12 * i + k] = src[12 * i + k];
    if (stale_env)
        stale_env[e] = 1;  // every writer stores the same value
}

// K1c: two-level scenes, one thread per instance.  The inverse of the pose's
// linear part A comes from its adjugate in FP64 (the pose's FP32 entries are
// exact in FP64, so M = adj(A) / det(A) is A^-1 to FP64 rounding); the world
// box of the mesh box [lo, hi] under x -> A x + p is p_r + sum_j min / max
// (A_rj lo_j, A_rj hi_j) per row, the exact interval image (the products are
// exact in FP64), rounded outward to FP32.
__global__ __launch_bounds__(256) void k_inst_prep(InstPrep q)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= q.n_inst)
        return;
    const int e = q.inst_env[i];
    if (q.env_mask && !q.env_mask[e])
        return;
    const float *T = q.inst_T + 12 * i;
    double a[3][3], p[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            a[r][c] = (double)T[4 * r + c];
        p[r] = (double)T[4 * r + 3];
    }
    // adjugate (transpose of the cofactor matrix)
    double m[3][3];
    m[0][0] = a[1][1] * a[2][2] - a[1][2] * a[2][1];
    m[0][1] = a[0][2] * a[2][1] - a[0][1] * a[2][2];
    m[0][2] = a[0][1] * a[1][2] - a[0][2] * a[1][1];
    m[1][0] = a[1][2] * a[2][0] - a[1][0] * a[2][2];
    m[1][1] = a[0][0] * a[2][2] - a[0][2] * a[2][0];
    m[1][2] = a[0][2] * a[1][0] - a[0][0] * a[1][2];
    m[2][0] = a[1][0] * a[2][1] - a[1][1] * a[2][0];
    m[2][1] = a[0][1] * a[2][0] - a[0][0] * a[2][1];
    m[2][2] = a[0][0] * a[1][1] - a[0][1] * a[1][0];
    const double det = a[0][0] * m[0][0] + a[0][1] * m[1][0] + a[0][2] * m[2][0];
    const bool ok = det != 0.0 && isfinite(det);
    double *inv = q.inv + 12 * i;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            inv[4 * r + c] = ok ? m[r][c] / det : __builtin_nan("");
        inv[4 * r + 3] = p[r];
    }
    const float *mb = q.mesh_box + 6 * (int64_t)q.inst_info[i].x;
    float lo[3], hi[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double l = p[r], h = p[r];
        if (ok) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double u0 = a[r][c] * (double)mb[c], u1 = a[r][c] * (double)mb[3 + c];
                l += fmin(u0, u1);
                h += fmax(u0, u1);
            }
        }
        lo[r] = __double2float_rd(l);
        hi[r] = __double2float_ru(h);
    }
    float *w = q.world + 9 * i;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        w[r] = lo[r];
        w[3 + r] = hi[r];
        w[6 + r] = lo[r];
    }
    if (q.recs) {
        const int64_t base = q.env_off[e];
        TriRec rec;
        rec.a = make_float4(lo[0], lo[1], lo[2], hi[0]);
        rec.b = make_float4(hi[1], hi[2], lo[0], lo[1]);
        rec.c = make_float4(lo[2], __int_as_float((int)(i - base)), 0.f, 0.f);
        q.recs[base + q.pos_of[i]] = rec;
    }
}

// K8: constant-velocity motion of dynamic instances.
// The step comes from d_step when it is set (a captured step graph advances
// it on the device), else from the argument.
__global__ __launch_bounds__(256) void k_move(int64_t n, const float *__restrict__ T0, const float *__restrict__ vel,
                                              const uint8_t *__restrict__ dyn, int32_t step,
                                              const int32_t *__restrict__ d_step, float dt, float *__restrict__ T)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float sdt = (float)(d_step ? *d_step : step) * dt;
    float a[12];
#pragma unroll
    for (int k = 0; k < 12; ++k)
        a[k] = T0[12 * i + k];
    if (dyn[i]) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
            a[4 * r + 3] = fmaf(vel[3 * i + r], sdt, a[4 * r + 3]);
    }
#pragma unroll
    for (int k = 0; k < 12; ++k)
        T[12 * i + k] = a[k];
}

// K2: per-triangle bounds (build scratch).
__global__ __launch_bounds__(256) void k_bounds(BuildView v)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= v.n_tris || masked_out(v, v.tri_env[g]))
        return;
    const float *w = v.world + 9 * g;
    const float lx = fminf(fminf(w[0], w[3]), w[6]), hx = fmaxf(fmaxf(w[0], w[3]), w[6]);
    const float ly = fminf(fminf(w[1], w[4]), w[7]), hy = fmaxf(fmaxf(w[1], w[4]), w[7]);
    const float lz = fminf(fminf(w[2], w[5]), w[8]), hz = fmaxf(fmaxf(w[2], w[5]), w[8]);
    v.box_lo[g] = make_float4(lx, ly, lz, 0.f);
    v.box_hi[g] = make_float4(hx, hy, hz, 0.f);
}

// ---------------------------------------------------------------------------
// K5: SAH build, one wavefront (64 lanes) per environment.
// Tasks are processed depth first (left child next) and node ids are assigned
// when a task is popped.  Nodes above kSmall primitives take the cheapest of
// 3 x (kBins - 1) binned planes and the cuts in triangle-id order, split by a
// stable partition; a task of at most kSmall primitives is deferred whole to
// k_build_local, which builds it from LDS with the exact sweep below.  Every
// step is deterministic.  A node whose subtree could exceed kMaxNodeDepth is
// split at the index median (balanced), which bounds the traversal stack.
// Within a deferred subtree, depth-first order guarantees that every task
// popped after its root, until the stack is empty again, is one of its
// descendants.
// ---------------------------------------------------------------------------
constexpr int kTaskCap = kMaxNodeDepth + 4;
#ifndef RC_SMALL
#define RC_SMALL 128
#endif
constexpr int kSmall = RC_SMALL;  // subtrees up to this size are built from LDS
constexpr int kMicro = 16;    // ranges of 5..16 go to the per-thread builder
constexpr int kU = 4;         // chunks of 64 primitives loaded together by the passes over large ranges

struct WaveBox {
    float lx, ly, lz, hx, hy, hz;
};

__device__ __forceinline__ int levels_needed(int n)
{
    const int leaves = (n + kLeafMax - 1) / kLeafMax;
    return leaves <= 1 ? 0 : 32 - __clz(leaves - 1);
}

__device__ __forceinline__ float half_area(float lx, float ly, float lz, float hx, float hy, float hz)
{
    const float dx = hx - lx, dy = hy - ly, dz = hz - lz;
    return dx * dy + dy * dz + dz * dx;
}

__device__ __forceinline__ int bin_of(float c, float cmin, float scale)
{
    const int b = (int)((c - cmin) * scale);
    return b < 0 ? 0 : (b >= kBins ? kBins - 1 : b);
}

struct BuildShared {
    int cnt[3 * kBins];
    int lo[3 * kBins * 3];
    int hi[3 * kBins * 3];
    int tp[kTaskCap], ts[kTaskCap], tb[kTaskCap], te[kTaskCap], td[kTaskCap];
    float box[6][kSmall];  // local mode: primitive bounds by slot
    int id[kSmall];        // local mode: environment-local id by slot
    int perm[kSmall];      // local mode: slot at each position
    int ord[4][kSmall];    // local mode: slots of each task in each sweep order
    int side[kSmall];      // local mode: side of each slot in the current split
};

__device__ __forceinline__ void write_boxes(Node &nd, const WaveBox &L, const WaveBox &R)
{
    nd.xy0 = make_float4(expand_lo(L.lx), expand_hi(L.hx), expand_lo(L.ly), expand_hi(L.hy));
    nd.xy1 = make_float4(expand_lo(R.lx), expand_hi(R.hx), expand_lo(R.ly), expand_hi(R.hy));
    nd.z01 = make_float4(expand_lo(L.lz), expand_hi(L.hz), expand_lo(R.lz), expand_hi(R.hz));
}

// ---------------------------------------------------------------------------
// Exact SAH sweep for a task of at most kSmall primitives held in LDS (local
// mode).  Slots number the subtree's primitives in the order they had when it
// entered LDS, which is ascending triangle id (every earlier split is a stable
// partition of the identity order).  On entry the wavefront sorts the slots
// once per centroid axis by (centroid, slot) with a bitonic network (kSweepE
// keys per lane, key h of lane l at index 64 h + l); the fourth order is the
// slot order itself (mesh order).  Every split then stable-partitions the four
// lists, so each task finds its primitives sorted in every order (a subset of
// a sorted list is sorted).  Per order the sweep scans the boxes from both
// ends, costs every split position, and the cheapest wins (lowest order, then
// fewest left primitives, on ties).
// ---------------------------------------------------------------------------
constexpr int kSweepE = kSmall / 64;
static_assert(kSmall % 64 == 0 && (kSweepE & (kSweepE - 1)) == 0, "kSmall must be 64 times a power of two");
constexpr WaveBox kEmptyBox{INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
constexpr uint64_t kNoKey = ~0ull;

__device__ __forceinline__ WaveBox box_union(const WaveBox &a, const WaveBox &b)
{
    return WaveBox{fminf(a.lx, b.lx), fminf(a.ly, b.ly), fminf(a.lz, b.lz),
                   fmaxf(a.hx, b.hx), fmaxf(a.hy, b.hy), fmaxf(a.hz, b.hz)};
}

// Inclusive union over lanes 0 .. i (UP) or i .. 63 (row = lane / 16).
template <bool UP>
__device__ __forceinline__ WaveBox box_scan(const WaveBox &b, int row)
{
    return WaveBox{lane_scan<true, UP>(b.lx, row),  lane_scan<true, UP>(b.ly, row),  lane_scan<true, UP>(b.lz, row),
                   lane_scan<false, UP>(b.hx, row), lane_scan<false, UP>(b.hy, row), lane_scan<false, UP>(b.hz, row)};
}
// Box of lane i - 1 (UP) or i + 1; the empty box at the end of the wavefront.
template <bool UP>
__device__ __forceinline__ WaveBox box_shift(const WaveBox &b)
{
    constexpr int C = UP ? 0x138 : 0x130;
    return WaveBox{dpp_mov<C>(INFINITY, b.lx),  dpp_mov<C>(INFINITY, b.ly),  dpp_mov<C>(INFINITY, b.lz),
                   dpp_mov<C>(-INFINITY, b.hx), dpp_mov<C>(-INFINITY, b.hy), dpp_mov<C>(-INFINITY, b.hz)};
}
// Box of lane src (wave-uniform).
__device__ __forceinline__ WaveBox box_lane(const WaveBox &b, int src)
{
    return WaveBox{readlane_f(b.lx, src), readlane_f(b.ly, src), readlane_f(b.lz, src),
                   readlane_f(b.hx, src), readlane_f(b.hy, src), readlane_f(b.hz, src)};
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int m)
{
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, m, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Partner j < 16 through DPP (j is a compile-time constant after unrolling).
__device__ __forceinline__ uint64_t row_xor_u64(uint64_t x, int j, int lane)
{
    const int lo = (int)(uint32_t)x, hi = (int)(uint32_t)(x >> 32);
    const int gl = lane & 15;
    int olo, ohi;
    if (j == 1) {
        olo = row_xor<1>(lo, gl);
        ohi = row_xor<1>(hi, gl);
    } else if (j == 2) {
        olo = row_xor<2>(lo, gl);
        ohi = row_xor<2>(hi, gl);
    } else if (j == 4) {
        olo = row_xor<4>(lo, gl);
        ohi = row_xor<4>(hi, gl);
    } else {
        olo = row_xor<8>(lo, gl);
        ohi = row_xor<8>(hi, gl);
    }
    return ((uint64_t)(uint32_t)ohi << 32) | (uint32_t)olo;
}

template <int E>
__device__ __forceinline__ void wave_sort(uint64_t (&key)[E], int lane)
{
#pragma unroll
    for (int k = 2; k <= 64 * E; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 64) {  // partner in the same lane
#pragma unroll
                for (int h = 0; h < E; ++h) {
                    const int h2 = h ^ (j >> 6);
                    if (h2 < h)
                        continue;
                    const bool up = ((64 * h + lane) & k) == 0;
                    const uint64_t a = key[h], c = key[h2];
                    const bool swap = up ? c < a : a < c;
                    key[h] = swap ? c : a;
                    key[h2] = swap ? a : c;
                }
            } else {
#pragma unroll
                for (int h = 0; h < E; ++h) {
                    const uint64_t o = j < 16 ? row_xor_u64(key[h], j, lane) : shfl_xor_u64(key[h], j);
                    const int i = 64 * h + lane;
                    const bool keep_min = ((i & k) == 0) == ((i & j) == 0);
                    key[h] = keep_min == (o < key[h]) ? o : key[h];
                }
            }
        }
    }
}

// The three centroid orders of the cnt slots of a subtree entering LDS, and
// the slot order; 64 E >= cnt.
template <int E>
__device__ __forceinline__ void local_sort(BuildShared &S, int cnt, int lane)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        uint64_t key[E];
#pragma unroll
        for (int h = 0; h < E; ++h) {
            const int s = 64 * h + lane;
            const float c = s < cnt ? 0.5f * (S.box[a][s] + S.box[3 + a][s]) : 0.f;
            key[h] = s < cnt ? ((uint64_t)((uint32_t)f2o(c) ^ 0x80000000u) << 32) | (uint32_t)s : kNoKey;
        }
        wave_sort<E>(key, lane);
#pragma unroll
        for (int h = 0; h < E; ++h) {
            const int p = 64 * h + lane;
            if (p < cnt)
                S.ord[a][p] = (int)(uint32_t)key[h];
        }
    }
    for (int p = lane; p < cnt; p += 64)
        S.ord[3][p] = p;
}

// Split of the cnt primitives at positions pb .. pb + cnt - 1 of the sorted
// lists.  Lane l holds positions E l .. E l + E - 1 (64 E >= cnt).  Returns
// the left count (0 if no split has a finite cost) and, when it splits, the
// child boxes; S.perm then holds the chosen order over the range.
template <int E>
__device__ int sweep_split(BuildShared &S, int pb, int cnt, int lane, WaveBox &L, WaveBox &R)
{
    constexpr int W = kSmall + 1;  // candidate rank: order * W + left count
    const int row = lane >> 4;
    float best_c = INFINITY;
    int best_w = INT32_MAX;
    WaveBox bl = kEmptyBox, br = kEmptyBox;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        WaveBox lp[E], ls[E];  // unions of the lane's positions up to / from h
#pragma unroll
        for (int h = 0; h < E; ++h) {
            const int p = E * lane + h;
            const int s = p < cnt ? S.ord[a][pb + p] : -1;
            lp[h] = s >= 0 ? WaveBox{S.box[0][s], S.box[1][s], S.box[2][s], S.box[3][s], S.box[4][s], S.box[5][s]}
                           : kEmptyBox;
        }
        ls[E - 1] = lp[E - 1];
#pragma unroll
        for (int h = E - 2; h >= 0; --h)
            ls[h] = box_union(lp[h], ls[h + 1]);
#pragma unroll
        for (int h = 1; h < E; ++h)
            lp[h] = box_union(lp[h - 1], lp[h]);
        const WaveBox before = box_shift<true>(box_scan<true>(lp[E - 1], row));  // positions < E l
        const WaveBox after = box_shift<false>(box_scan<false>(ls[0], row));     // positions >= E l + E
#pragma unroll
        for (int h = 0; h < E; ++h) {
            const int k = E * lane + h + 1;  // left = positions 0 .. k - 1
            if (k < cnt) {
                const WaveBox P = box_union(before, lp[h]);
                const WaveBox Q = h + 1 < E ? box_union(ls[h + 1], after) : after;
                const float c = half_area(P.lx, P.ly, P.lz, P.hx, P.hy, P.hz) * (float)k +
                                half_area(Q.lx, Q.ly, Q.lz, Q.hx, Q.hy, Q.hz) * (float)(cnt - k);
                const int w = a * W + k;
                if (c < best_c || (c == best_c && w < best_w)) {
                    best_c = c;
                    best_w = w;
                    bl = P;
                    br = Q;
                }
            }
        }
    }
    float bc = best_c;
    int bw = best_w;
    wave_argmin(bc, bw, lane);
    if (!(bc < INFINITY))
        return 0;
    bw = __builtin_amdgcn_readfirstlane(bw);
    const int a = bw / W, k = bw % W;
    const int src = (k - 1) / E;  // the lane that costed this split (its own best)
    L = box_lane(bl, src);
    R = box_lane(br, src);
    for (int p = lane; p < cnt; p += 64)
        S.perm[pb + p] = S.ord[a][pb + p];
    return k;
}

// Local mode, after the task at positions pb .. pb + cnt - 1 has been split
// into the first nl positions of S.perm and the rest: stable partition of the
// four sorted lists by side.
__device__ __forceinline__ void local_partition(BuildShared &S, int pb, int cnt, int nl, int lane)
{
    for (int p = lane; p < cnt; p += 64)
        S.side[S.perm[pb + p]] = p < nl;
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        int s[kSweepE];
        bool left[kSweepE];
#pragma unroll
        for (int h = 0; h < kSweepE; ++h) {
            const int p = 64 * h + lane;
            s[h] = p < cnt ? S.ord[a][pb + p] : -1;
            left[h] = s[h] >= 0 && S.side[s[h]] != 0;
        }
        __syncthreads();  // the whole list is read before any of it is rewritten
        int lc = 0, rc = 0;
#pragma unroll
        for (int h = 0; h < kSweepE; ++h) {
            const uint64_t m = __ballot(left[h]);
            const int rank = __popcll(m & ((1ull << lane) - 1));  // left entries in lower lanes
            const int nvalid = min(64, max(0, cnt - 64 * h));
            if (s[h] >= 0)
                S.ord[a][pb + (left[h] ? lc + rank : nl + rc + (lane - rank))] = s[h];
            const int cl = __popcll(m);
            lc += cl;
            rc += nvalid - cl;
        }
    }
    __syncthreads();
}

// One SAH job for one wavefront.  JOB = false: environment e from its root;
// every task of at most kSmall primitives is deferred whole to k_build_local
// (its root id assigned and linked now, followed by cnt - 2 reserved ids, the
// task stored at the end of the environment's range list).  JOB = true: one
// such deferred subtree, built from LDS, its ranges of 5..kMicro primitives
// appended to the environment's range list with an atomic counter.
template <bool JOB>
__device__ __forceinline__ void sah_job(const BuildView &v, BuildShared &S, int e, int4 job)
{
    const int lane = threadIdx.x;
    const int64_t base = v.env_tri_off[e];
    const int n = (int)(v.env_tri_off[e + 1] - base);
    int32_t *prim = v.prim + base;
    int32_t *tmp = v.tmp + base;
    Node *nodes = v.nodes + node_base(base, e);
    const float4 *blo = v.box_lo + base;
    const float4 *bhi = v.box_hi + base;
    int n_nodes = 0;
    if (!JOB) {
        for (int i = lane; i < n; i += 64)
            prim[i] = i;
        if (n == 0) {
            if (lane == 0) {
                v.env_root[e] = kEmptyRoot;
                v.env_nodes[e] = 0;
                v.env_micro[e] = 0;
                v.env_local[e] = 0;
            }
            return;
        }
        __syncthreads();
    } else {
        n_nodes = job.x;  // the subtree's root id (linked, parent and depth written)
    }
    bool local = false;
    int b0 = 0, cnt0 = 0, h0 = 0;
    int nm = 0;   // deferred small ranges (environment job)
    int nlt = 0;  // deferred subtrees (environment job)
    // Ranges from the start of the list, subtrees from its end: a range holds at
    // least 5 primitives and a subtree (other than a root) at least kMicro + 1,
    // so n/5 + n/(kMicro + 1) + 1 <= n entries never meet.
    int4 *micro = v.micro + base;

    // bounds of the primitive at list position i of the LDS copy (local mode)
    auto local_box = [&](int i) {
        const int slot = S.perm[i - b0];
        return WaveBox{S.box[0][slot], S.box[1][slot], S.box[2][slot], S.box[3][slot], S.box[4][slot], S.box[5][slot]};
    };
    // Boxes of the global list at positions c + lane, c = g0 + 64 u (g0 - 64 u
    // when down), u < kU, and the primitives there (-1 and the empty box
    // outside [rb, re)): the loads of kU chunks are issued together, so a
    // pass over a large range waits for one round trip per kU chunks.
    auto load_boxes = [&](int g0, bool down, int rb, int re, WaveBox(&xs)[kU], int(&ps)[kU]) {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int i = (down ? g0 - 64 * u : g0 + 64 * u) + lane;
            ps[u] = (i >= rb && i < re) ? prim[i] : -1;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            xs[u] = kEmptyBox;
            if (ps[u] >= 0) {
                const float4 lo = blo[ps[u]], hi = bhi[ps[u]];
                xs[u] = WaveBox{lo.x, lo.y, lo.z, hi.x, hi.y, hi.z};
            }
        }
    };
    auto reduce_range = [&](int rb, int re) {
        WaveBox acc = kEmptyBox;
        if (local) {
            for (int i = rb + lane; i < re; i += 64)
                acc = box_union(acc, local_box(i));
        } else {
            for (int g0 = rb; g0 < re; g0 += 64 * kU) {
                WaveBox xs[kU];
                int ps[kU];
                load_boxes(g0, false, rb, re, xs, ps);
#pragma unroll
                for (int u = 0; u < kU; ++u)
                    acc = box_union(acc, xs[u]);
            }
        }
        return WaveBox{wave_min(acc.lx), wave_min(acc.ly), wave_min(acc.lz),
                       wave_max(acc.hx), wave_max(acc.hy), wave_max(acc.hz)};
    };

    if (!JOB && n <= kLeafMax) {
        if (lane == 0)
            v.env_root[e] = leaf_ref(0, n);
    } else {
        int sp = 0;
        S.tp[0] = JOB ? -2 : -1;  // -2: the subtree's root, already linked
        S.ts[0] = 0;
        S.tb[0] = JOB ? job.y : 0;
        S.te[0] = JOB ? job.z : n;
        S.td[0] = JOB ? job.w : 0;
        sp = 1;
        __syncthreads();
        while (sp > 0) {
            --sp;
            const int parent = S.tp[sp], side = S.ts[sp], b = S.tb[sp], en = S.te[sp], depth = S.td[sp];
            const int cnt = en - b;
            __syncthreads();
            if (!JOB && cnt <= kSmall) {
                const int cid = n_nodes;
                n_nodes += cnt - 1;  // the most internal nodes cnt primitives can need
                if (lane == 0) {
                    if (parent < 0)
                        v.env_root[e] = cid;
                    else if (side == 0)
                        nodes[parent].ch.x = cid;
                    else
                        nodes[parent].ch.y = cid;
                    nodes[cid].ch.z = parent;
                    nodes[cid].ch.w = depth;
                    micro[n - 1 - nlt] = make_int4(cid, b, en, depth);
                }
                ++nlt;
                continue;
            }
            if (JOB && !local) {
                // enter local mode: copy the task's primitives into LDS
                b0 = b;
                cnt0 = cnt;
                h0 = sp;
                for (int i = lane; i < cnt; i += 64) {
                    const int p = prim[b + i];
                    const float4 lo = blo[p], hi = bhi[p];
                    S.id[i] = p;
                    S.perm[i] = i;
                    S.box[0][i] = lo.x;
                    S.box[1][i] = lo.y;
                    S.box[2][i] = lo.z;
                    S.box[3][i] = hi.x;
                    S.box[4][i] = hi.y;
                    S.box[5][i] = hi.z;
                }
                local = true;
                __syncthreads();
                if (cnt <= 64)
                    local_sort<1>(S, cnt, lane);
                else
                    local_sort<kSweepE>(S, cnt, lane);
                __syncthreads();
            }
            const int id = n_nodes++;
            if (lane == 0 && parent != -2) {
                if (parent < 0)
                    v.env_root[e] = id;
                else if (side == 0)
                    nodes[parent].ch.x = id;
                else
                    nodes[parent].ch.y = id;
                nodes[id].ch.z = parent;
                nodes[id].ch.w = depth;
            }
            // Nodes above kSmall primitives, one pass: centroid bounds for the bins
            // (centroid = midpoint of the primitive's box) and the half-area of every
            // prefix of the range in its own order, for the cuts in that order (kept in
            // tmp, which the partition below reuses only afterwards).  The range is in
            // ascending triangle id order (every split above local mode is a stable
            // partition of the identity order) and mesh order is spatially coherent,
            // so those cuts separate whole objects and clusters of equal centroids
            // that no binned plane can split.
            float cmin[3] = {0.f, 0.f, 0.f}, scale[3] = {0.f, 0.f, 0.f};
            bool usable = false;
            float *parea = reinterpret_cast<float *>(tmp);
            if (!local) {
                float cl0 = INFINITY, cl1 = INFINITY, cl2 = INFINITY, ch0 = -INFINITY, ch1 = -INFINITY, ch2 = -INFINITY;
                WaveBox carry = kEmptyBox;
                for (int g0 = b; g0 < en; g0 += 64 * kU) {
                    WaveBox xs[kU];
                    int ps[kU];
                    load_boxes(g0, false, b, en, xs, ps);
#pragma unroll
                    for (int u = 0; u < kU; ++u) {
                        const int i = g0 + 64 * u + lane;
                        WaveBox x = xs[u];
                        if (i < en) {
                            const float cx = 0.5f * (x.lx + x.hx), cy = 0.5f * (x.ly + x.hy), cz = 0.5f * (x.lz + x.hz);
                            cl0 = fminf(cl0, cx);
                            cl1 = fminf(cl1, cy);
                            cl2 = fminf(cl2, cz);
                            ch0 = fmaxf(ch0, cx);
                            ch1 = fmaxf(ch1, cy);
                            ch2 = fmaxf(ch2, cz);
                        }
                        x = box_union(box_scan<true>(x, lane >> 4), carry);
                        if (i < en)
                            parea[i] = half_area(x.lx, x.ly, x.lz, x.hx, x.hy, x.hz);
                        carry = box_lane(x, 63);
                    }
                }
                const float mn[3] = {wave_min(cl0), wave_min(cl1), wave_min(cl2)};
                const float mx[3] = {wave_max(ch0), wave_max(ch1), wave_max(ch2)};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const float ext = mx[a] - mn[a];
                    cmin[a] = mn[a];
                    scale[a] = ext > 0.f ? (float)kBins / ext : 0.f;
                    usable |= ext > 0.f;
                }
            }
            const bool forced = depth + levels_needed(cnt) - 1 >= v.max_depth;

            int mid = -1, best_axis = -1, best_k = -1;
            WaveBox L{}, R{};
            if (local && !forced) {
                __syncthreads();
                const int k = cnt <= 64 ? sweep_split<1>(S, b - b0, cnt, lane, L, R)
                                        : sweep_split<kSweepE>(S, b - b0, cnt, lane, L, R);
                __syncthreads();
                if (k > 0)
                    mid = b + k;
            } else if (usable && !forced) {
                for (int j = lane; j < 3 * kBins; j += 64) {
                    S.cnt[j] = 0;
                    S.lo[3 * j] = S.lo[3 * j + 1] = S.lo[3 * j + 2] = f2o(INFINITY);
                    S.hi[3 * j] = S.hi[3 * j + 1] = S.hi[3 * j + 2] = f2o(-INFINITY);
                }
                __syncthreads();  // bins cleared, prefix areas visible to every lane
                // One pass, chunks from the end: binning (order-free) and, for the cuts in
                // the range's own order, suffix boxes and the cost of every cut.
                float ic = INFINITY;
                int ik = 0;
                {
                    WaveBox carry = kEmptyBox;  // union of the positions after the current chunk
                    for (int g0 = b + ((cnt - 1) & ~63); g0 >= b; g0 -= 64 * kU) {
                        WaveBox xs[kU];
                        int ps[kU];
                        float pa[kU];
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int i = g0 - 64 * u + lane;
                            pa[u] = (i >= b && i < en - 1) ? parea[i] : 0.f;
                        }
                        load_boxes(g0, true, b, en, xs, ps);
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int i = g0 - 64 * u + lane;
                            WaveBox x = xs[u];
                            if (i >= b && i < en) {
                                const float cc[3] = {0.5f * (x.lx + x.hx), 0.5f * (x.ly + x.hy), 0.5f * (x.lz + x.hz)};
#pragma unroll
                                for (int a = 0; a < 3; ++a) {
                                    if (scale[a] == 0.f)
                                        continue;
                                    const int j = a * kBins + bin_of(cc[a], cmin[a], scale[a]);
                                    atomicAdd(&S.cnt[j], 1);
                                    atomicMin(&S.lo[3 * j + 0], f2o(x.lx));
                                    atomicMin(&S.lo[3 * j + 1], f2o(x.ly));
                                    atomicMin(&S.lo[3 * j + 2], f2o(x.lz));
                                    atomicMax(&S.hi[3 * j + 0], f2o(x.hx));
                                    atomicMax(&S.hi[3 * j + 1], f2o(x.hy));
                                    atomicMax(&S.hi[3 * j + 2], f2o(x.hz));
                                }
                            }
                            x = box_scan<false>(x, lane >> 4);
                            const WaveBox suf = box_union(x, carry);                    // positions i .. en - 1
                            const WaveBox rn = box_union(box_shift<false>(x), carry);  // positions i + 1 .. en - 1
                            if (i >= b && i < en - 1) {
                                const int k = i - b + 1;
                                const float c = pa[u] * (float)k + half_area(rn.lx, rn.ly, rn.lz, rn.hx, rn.hy, rn.hz) * (float)(cnt - k);
                                if (c < ic || (c == ic && k < ik)) {
                                    ic = c;
                                    ik = k;
                                }
                            }
                            carry = box_lane(suf, 0);
                        }
                    }
                    wave_argmin(ic, ik, lane);
                }
                __syncthreads();
                // evaluate the 3 x (kBins-1) split planes, plane index pl = lane,
                // lane + 64, ...; each lane keeps its cheapest (lowest index on ties)
                float cost = INFINITY;
                int nl = 0, bw = lane;
                WaveBox bl{INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
                WaveBox br = bl;
                for (int pl = lane; pl < 3 * (kBins - 1); pl += 64) {
                    const int a = pl / (kBins - 1), k = pl % (kBins - 1);
                    if (scale[a] == 0.f)
                        continue;
                    WaveBox cl{INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
                    WaveBox cr = cl;
                    int ml = 0, mr = 0;
                    for (int j = 0; j < kBins; ++j) {
                        const int q = a * kBins + j;
                        const int c = S.cnt[q];
                        if (c == 0)
                            continue;
                        WaveBox &B = j <= k ? cl : cr;
                        B.lx = fminf(B.lx, o2f(S.lo[3 * q]));
                        B.ly = fminf(B.ly, o2f(S.lo[3 * q + 1]));
                        B.lz = fminf(B.lz, o2f(S.lo[3 * q + 2]));
                        B.hx = fmaxf(B.hx, o2f(S.hi[3 * q]));
                        B.hy = fmaxf(B.hy, o2f(S.hi[3 * q + 1]));
                        B.hz = fmaxf(B.hz, o2f(S.hi[3 * q + 2]));
                        if (j <= k)
                            ml += c;
                        else
                            mr += c;
                    }
                    if (ml > 0 && mr > 0) {
                        const float c = half_area(cl.lx, cl.ly, cl.lz, cl.hx, cl.hy, cl.hz) * (float)ml +
                                        half_area(cr.lx, cr.ly, cr.lz, cr.hx, cr.hy, cr.hz) * (float)mr;
                        if (c < cost) {
                            cost = c;
                            nl = ml;
                            bw = pl;
                            bl = cl;
                            br = cr;
                        }
                    }
                }
                // argmin over lanes, ties to the lower plane index
                float bc = cost;
                wave_argmin(bc, bw, lane);
                if (ic < bc) {  // cut in id order: both sides are already contiguous
                    mid = b + ik;
                    L = reduce_range(b, mid);
                    R = reduce_range(mid, en);
                } else if (bc < INFINITY) {
                    best_axis = bw / (kBins - 1);
                    best_k = bw % (kBins - 1);
                    const int src = __builtin_amdgcn_readfirstlane(bw) & 63;  // the lane that evaluated plane bw
                    const int nL = __builtin_amdgcn_readlane(nl, src);
                    L = box_lane(bl, src);
                    R = box_lane(br, src);
                    mid = b + nL;
                    // stable partition into tmp, then copy back (global list only:
                    // local mode always takes the sweep)
                    int lc = 0, rc = 0;
                    const float cm = cmin[best_axis], sc = scale[best_axis];
                    for (int g0 = b; g0 < en; g0 += 64 * kU) {
                        WaveBox xs[kU];
                        int ps[kU];
                        load_boxes(g0, false, b, en, xs, ps);
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int c0 = g0 + 64 * u;
                            if (c0 >= en)
                                break;
                            const int i = c0 + lane;
                            const bool valid = i < en;
                            const WaveBox &x = xs[u];
                            const float cc = best_axis == 0 ? 0.5f * (x.lx + x.hx)
                                                            : (best_axis == 1 ? 0.5f * (x.ly + x.hy) : 0.5f * (x.lz + x.hz));
                            const bool left = valid && bin_of(cc, cm, sc) <= best_k;
                            const uint64_t m = __ballot(left);
                            const uint64_t below = lane == 0 ? 0ull : (m & (~0ull >> (64 - lane)));
                            const int rank = __popcll(below);
                            const int nvalid = min(64, en - c0);
                            const int dst = left ? b + lc + rank : mid + rc + (lane - rank);
                            if (valid)
                                tmp[dst] = ps[u];
                            const int cl = __popcll(m);
                            lc += cl;
                            rc += nvalid - cl;
                        }
                    }
                    __syncthreads();
                    for (int g0 = b; g0 < en; g0 += 64 * kU) {
                        int t[kU];
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int i = g0 + 64 * u + lane;
                            t[u] = i < en ? tmp[i] : 0;
                        }
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int i = g0 + 64 * u + lane;
                            if (i < en)
                                prim[i] = t[u];
                        }
                    }
                    __syncthreads();
                }
            }
            if (mid < 0) {  // index-median split (forced depth bound or no usable plane)
                mid = b + cnt / 2;
                L = reduce_range(b, mid);
                R = reduce_range(mid, en);
            }
            if (local)
                local_partition(S, b - b0, cnt, mid - b, lane);
            // write the node's child boxes (expanded outward by one step)
            const int nl = mid - b, nr = en - mid;
            if (lane == 0) {
                Node &nd = nodes[id];
                write_boxes(nd, L, R);
                if (nl <= kLeafMax)
                    nd.ch.x = leaf_ref(b, nl);
                if (nr <= kLeafMax)
                    nd.ch.y = leaf_ref(mid, nr);
            }
            // Children of 5..kMicro primitives are deferred to k_build_micro
            // (their node id is assigned now, followed by c - 2 reserved ids
            // for the rest of their subtree); larger ones are pushed, right
            // first so that the left child is popped next.
            const int cb[2] = {b, mid}, ce[2] = {mid, en};
            for (int sd = 1; sd >= 0; --sd) {
                const int c = ce[sd] - cb[sd];
                if (c <= kLeafMax)
                    continue;
                if (c <= kMicro) {
                    const int cid = n_nodes;
                    n_nodes += c - 1;  // the most internal nodes c primitives can need
                    if (lane == 0) {
                        if (sd == 0)
                            nodes[id].ch.x = cid;
                        else
                            nodes[id].ch.y = cid;
                        nodes[cid].ch.z = id;
                        nodes[cid].ch.w = depth + 1;
                        micro[JOB ? atomicAdd(&v.env_micro[e], 1) : nm] = make_int4(cid, cb[sd], ce[sd], depth + 1);
                    }
                    ++nm;
                } else {
                    S.tp[sp] = id;
                    S.ts[sp] = sd;
                    S.tb[sp] = cb[sd];
                    S.te[sp] = ce[sd];
                    S.td[sp] = depth + 1;
                    ++sp;
                }
            }
            __syncthreads();
            if (local && sp == h0) {
                // subtree finished: write its primitive order back
                for (int i = lane; i < cnt0; i += 64)
                    prim[b0 + i] = S.id[S.perm[i]];
                local = false;
                __syncthreads();
            }
        }
    }
    if (lane == 0) {
        if (!JOB) {
            v.env_nodes[e] = n_nodes;
            v.env_micro[e] = nm;
            v.env_local[e] = nlt;
        } else {
            // unused reserved ids: never referenced; a depth of -1 keeps refit away
            for (int h = n_nodes; h < job.x + (job.z - job.y) - 1; ++h) {
                Node &u = nodes[h];
                u.xy0 = u.xy1 = u.z01 = make_float4(0.f, 0.f, 0.f, 0.f);
                u.ch = make_int4(0, 0, -1, -1);
            }
        }
    }
}

__global__ __launch_bounds__(64) void k_build_sah(BuildView v)
{
    const int e = blockIdx.x;
    if (masked_out(v, e))
        return;
    __shared__ BuildShared S;
    sah_job<false>(v, S, e, make_int4(0, 0, 0, 0));
}

// K5a: the subtrees deferred by k_build_sah, one wavefront each (a persistent
// grid over the list of all of them), so an environment's LDS-resident levels
// are built in parallel instead of one after another.
__global__ __launch_bounds__(64) void k_build_local(BuildView v)
{
    __shared__ BuildShared S;
    const int64_t total = v.local_off[v.n_envs];
    for (int64_t T = blockIdx.x; T < total; T += gridDim.x) {
        // environment of task T: local_off[e] <= T < local_off[e + 1]
        int lo = 0, hi = v.n_envs;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (v.local_off[mid] <= T)
                lo = mid;
            else
                hi = mid;
        }
        const int64_t base = v.env_tri_off[lo];
        const int n = (int)(v.env_tri_off[lo + 1] - base);
        const int4 job = v.micro[base + n - 1 - (T - v.local_off[lo])];
        __syncthreads();  // the previous job's LDS is no longer read
        sah_job<true>(v, S, lo, job);
    }
}

// ---------------------------------------------------------------------------
// K5b: ranges of 5..16 primitives deferred by k_build_sah and k_build_local.  One 16-lane group
// per range (four per wavefront), one primitive per lane, builds the whole
// subtree: every node takes the full-sweep SAH split over the three centroid
// axes (per axis the group sorts (centroid, triangle id) with a bitonic
// network across its lanes, scans the sorted boxes from both ends and takes
// the cheapest split: lowest axis, then fewest left primitives, on ties), and
// every side above kLeafMax primitives becomes a node of its own.  A side of
// 2..kLeafMax primitives becomes a leaf unless splitting it is cheaper under
// the SAH with a node visit costing one triangle test (n A > A + A_L n_L +
// A_R n_R, half areas).  The only limit on a split is the depth bound
// (micro_cap).  Centroids are compared through their ordered-integer
// image, a total order, so the network is a permutation for any input.
// ---------------------------------------------------------------------------
constexpr int kMicroBlock = 256;
constexpr int kGroup = 16;

// Compare-exchange of the bitonic network: partner lane gl ^ j, block size k.
template <int K, int J>
__device__ __forceinline__ void group_cx(int &key, int &id, int gl)
{
    const int ok = row_xor<J>(key, gl);
    const int oi = row_xor<J>(id, gl);
    const bool other_less = ok < key || (ok == key && oi < id);
    const bool take = (((gl & K) == 0) == ((gl & J) == 0)) ? other_less : !other_less;
    if (take) {
        key = ok;
        id = oi;
    }
}

// Ascending (key, id) across the 16 lanes of a group (ids distinct).
__device__ __forceinline__ void group_sort(int &key, int &id, int gl)
{
    group_cx<2, 1>(key, id, gl);
    group_cx<4, 2>(key, id, gl);
    group_cx<4, 1>(key, id, gl);
    group_cx<8, 4>(key, id, gl);
    group_cx<8, 2>(key, id, gl);
    group_cx<8, 1>(key, id, gl);
    group_cx<16, 8>(key, id, gl);
    group_cx<16, 4>(key, id, gl);
    group_cx<16, 2>(key, id, gl);
    group_cx<16, 1>(key, id, gl);
}

// Minimum or maximum over the group: quad_perm [1,0,3,2], [2,3,0,1], then
// row_half_mirror (lane j with 7 - j of its half) and row_mirror (j with 15 - j).
template <bool MIN>
__device__ __forceinline__ float group_reduce(float x)
{
    x = mm<MIN>(x, dpp_mov<0xb1>(x, x));
    x = mm<MIN>(x, dpp_mov<0x4e>(x, x));
    x = mm<MIN>(x, dpp_mov<0x141>(x, x));
    return mm<MIN>(x, dpp_mov<0x140>(x, x));
}

__device__ __forceinline__ WaveBox group_box_reduce(const WaveBox &b)
{
    return WaveBox{group_reduce<true>(b.lx),  group_reduce<true>(b.ly),  group_reduce<true>(b.lz),
                   group_reduce<false>(b.hx), group_reduce<false>(b.hy), group_reduce<false>(b.hz)};
}

// Inclusive union over lanes 0 .. gl (UP) or gl .. 15 of the group.
template <bool UP>
__device__ __forceinline__ WaveBox group_scan(const WaveBox &b)
{
    return WaveBox{row_scan<true, UP>(b.lx),  row_scan<true, UP>(b.ly),  row_scan<true, UP>(b.lz),
                   row_scan<false, UP>(b.hx), row_scan<false, UP>(b.hy), row_scan<false, UP>(b.hz)};
}

// Box of lane gl + 1 of the group (row_shl:1); the empty box at lane 15.
__device__ __forceinline__ WaveBox group_next(const WaveBox &b)
{
    return WaveBox{dpp_mov<0x101>(INFINITY, b.lx),  dpp_mov<0x101>(INFINITY, b.ly),  dpp_mov<0x101>(INFINITY, b.lz),
                   dpp_mov<0x101>(-INFINITY, b.hx), dpp_mov<0x101>(-INFINITY, b.hy), dpp_mov<0x101>(-INFINITY, b.hz)};
}

// One step of the group's argmin of (cost, k): partner lane gl ^ M.
template <int M>
__device__ __forceinline__ void group_min_step(float &bc, int &bk, int gl)
{
    const float oc = row_xor_f<M>(bc, gl);
    const int ok = row_xor<M>(bk, gl);
    if (oc < bc || (oc == bc && ok < bk)) {
        bc = oc;
        bk = ok;
    }
}

// Cross-lane read within the group.  Call it from every lane of the group
// (never inside a per-lane condition): a lane that skips it cannot be read.
__device__ __forceinline__ WaveBox box_shfl(const WaveBox &b, int src)
{
    return WaveBox{__shfl(b.lx, src, kGroup), __shfl(b.ly, src, kGroup), __shfl(b.lz, src, kGroup),
                   __shfl(b.hx, src, kGroup), __shfl(b.hy, src, kGroup), __shfl(b.hz, src, kGroup)};
}

// Split of the `cnt` primitives that lanes [first, first + cnt) hold (lane r
// holds box `bx`; positions outside are ignored), both sides at most `cap`.
// On return lane q holds in `order` the lane whose primitive comes q-th along
// the chosen axis (q < cnt), and the function returns the left count.
__device__ __forceinline__ int group_split(const WaveBox &bx, int pid, int gl, int first, int cnt, int cap, int &order,
                                           WaveBox &L, WaveBox &R)
{
    const bool mine = gl >= first && gl < first + cnt;
    const int kmin = cnt - cap > 1 ? cnt - cap : 1;
    const int kmax = cap < cnt - 1 ? cap : cnt - 1;
    float best_c = INFINITY;
    int best_k = cnt / 2, best_a = 0;  // no finite cost: middle split along the first axis
    int orders[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float c = a == 0 ? 0.5f * (bx.lx + bx.hx) : (a == 1 ? 0.5f * (bx.ly + bx.hy) : 0.5f * (bx.lz + bx.hz));
        int key = mine ? f2o(c) : INT32_MAX;
        int id = mine ? (pid << 4) | gl : 0x7ffffff0 | gl;  // ties: lower triangle id first
        group_sort(key, id, gl);
        orders[a] = id;
        // boxes in sorted order; identity beyond the range (every lane takes
        // part in the shuffle: its source may lie outside [0, cnt))
        const WaveBox got = box_shfl(bx, id & (kGroup - 1));
        const WaveBox s = gl < cnt ? got : kEmptyBox;
        const WaveBox pre = group_scan<true>(s);
        // lane r: split after k = r + 1 (left = sorted 0..r, right = r+1..cnt-1)
        const WaveBox rs = group_next(group_scan<false>(s));
        const int k = gl + 1;
        float cost = INFINITY;
        if (k >= kmin && k <= kmax && k < cnt)
            cost = half_area(pre.lx, pre.ly, pre.lz, pre.hx, pre.hy, pre.hz) * (float)k +
                   half_area(rs.lx, rs.ly, rs.lz, rs.hx, rs.hy, rs.hz) * (float)(cnt - k);
        // cheapest over the group, fewest left primitives on ties
        float bc = cost;
        int bk = k;
        group_min_step<1>(bc, bk, gl);
        group_min_step<2>(bc, bk, gl);
        group_min_step<4>(bc, bk, gl);
        group_min_step<8>(bc, bk, gl);
        if (bc < best_c) {
            best_c = bc;
            best_k = bk;
            best_a = a;
        }
    }
    order = best_a == 0 ? orders[0] : (best_a == 1 ? orders[1] : orders[2]);
    // child boxes of the chosen split
    const WaveBox got = box_shfl(bx, order & (kGroup - 1));
    const WaveBox s = gl < cnt ? got : kEmptyBox;
    L = group_box_reduce(gl < best_k ? s : kEmptyBox);
    R = group_box_reduce(gl >= best_k && gl < cnt ? s : kEmptyBox);
    return best_k;
}

// Largest side a micro split at depth dd may leave: a side of s > kLeafMax
// primitives becomes a node at depth dd + 1 whose subtree needs
// levels_needed(s) more levels, and internal nodes stay within the depth
// bound md.
__device__ __forceinline__ int micro_cap(int dd, int md)
{
    const int m = md - dd;
    return m >= 2 ? kGroup : (kLeafMax << (m < 0 ? 0 : m));
}

// SAH leaf test for the c <= kLeafMax primitives of lanes first .. first + c - 1
// at depth dd (call from every lane of the group): true if they stay a leaf.
// The split cost is the cheapest over every two-way partition of the c
// primitives (a superset of the sweep's candidates): lane j costs the
// partition whose left side is the bit set of j + 1 (primitive c - 1 always
// right, so each partition once).
// gbox: the group's boxes in LDS, lane r's at gbox[r] (lo.x lo.y lo.z hi.x,
// hi.y hi.z).
__device__ __forceinline__ bool micro_leaf(const float4 (*gbox)[2], int gl, int first, int c, int dd, int md)
{
    static_assert(kLeafMax <= 5, "2^(kLeafMax-1) - 1 partitions must fit in the 16-lane group");
    if (c <= 1 || dd >= md)  // a split would put a node below the depth bound
        return true;
    WaveBox B[kLeafMax];
    WaveBox U = kEmptyBox;
#pragma unroll
    for (int i = 0; i < kLeafMax; ++i) {
        B[i] = kEmptyBox;
        if (i < c) {  // group-uniform: every lane reads the same slot
            const float4 a = gbox[first + i][0], b = gbox[first + i][1];
            B[i] = WaveBox{a.x, a.y, a.z, a.w, b.x, b.y};
        }
        U = box_union(U, B[i]);
    }
    const int m = gl + 1;
    float cost = INFINITY;
    if (m < (1 << (c - 1))) {
        WaveBox l = kEmptyBox, r = kEmptyBox;
        int nl = 0;
#pragma unroll
        for (int i = 0; i < kLeafMax; ++i) {
            if (i < c) {
                if ((m >> i) & 1) {
                    l = box_union(l, B[i]);
                    ++nl;
                } else {
                    r = box_union(r, B[i]);
                }
            }
        }
        cost = half_area(l.lx, l.ly, l.lz, l.hx, l.hy, l.hz) * (float)nl +
               half_area(r.lx, r.ly, r.lz, r.hx, r.hy, r.hz) * (float)(c - nl);
    }
    cost = group_reduce<true>(cost);
    const float a = half_area(U.lx, U.ly, U.lz, U.hx, U.hy, U.hz);
    return !((float)c * a > a + cost);
}

__global__ __launch_bounds__(kMicroBlock) void k_build_micro(BuildView v)
{
    // each lane's current box, for the leaf tests' reads of the group's boxes
    __shared__ float4 sbox[kMicroBlock][2];
    const float4(*gbox)[2] = sbox + (threadIdx.x & ~(kGroup - 1));
    const int gl = threadIdx.x & (kGroup - 1);
    const int64_t n_groups = ((int64_t)gridDim.x * kMicroBlock) / kGroup;
    const int64_t total = v.micro_off[v.n_envs];
    for (int64_t T = ((int64_t)blockIdx.x * kMicroBlock + threadIdx.x) / kGroup; T < total; T += n_groups) {
        // environment of task T: micro_off[e] <= T < micro_off[e + 1]
        int lo = 0, hi = v.n_envs;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (v.micro_off[mid] <= T)
                lo = mid;
            else
                hi = mid;
        }
        const int e = lo;
        const int64_t base = v.env_tri_off[e];
        const int4 task = v.micro[base + (T - v.micro_off[e])];  // node, begin, end, depth
        int32_t *prim = v.prim + base;
        Node *nodes = v.nodes + node_base(base, e);
        const int cnt = task.z - task.y;
        // lane r holds primitive r of the range
        int pid = -1;
        WaveBox bx = kEmptyBox;
        if (gl < cnt) {
            pid = prim[task.y + gl];
            const float4 lo4 = v.box_lo[base + pid], hi4 = v.box_hi[base + pid];
            bx = WaveBox{lo4.x, lo4.y, lo4.z, hi4.x, hi4.y, hi4.z};
        }
        // Depth-first over the subtree's nodes.  Pending nodes form a stack
        // held across the group, entry s in lane s: (first | count << 8, node
        // id, depth); at most three ranges of five or more fit in sixteen.
        int s_range = 0, s_id = 0, s_depth = 0, sp = 0;
        int next = task.x + 1;  // next reserved node id
        int f = 0, c = cnt, id = task.x, dd = task.w;
        while (true) {
            int order;
            WaveBox L, R;
            const int k = group_split(bx, pid, gl, f, c, micro_cap(dd, v.max_depth), order, L, R);
            // lanes f .. f + c - 1 take the chosen axis order
            const int src = __shfl(order, (gl - f) & (kGroup - 1), kGroup) & (kGroup - 1);
            const WaveBox nb = box_shfl(bx, src);
            const int np = __shfl(pid, src, kGroup);
            if (gl >= f && gl < f + c) {
                bx = nb;
                pid = np;
            }
            sbox[threadIdx.x][0] = make_float4(bx.lx, bx.ly, bx.lz, bx.hx);
            sbox[threadIdx.x][1] = make_float4(bx.hy, bx.hz, 0.f, 0.f);
            const int cf[2] = {f, f + k}, cc[2] = {k, c - k};
            int ref[2];
#pragma unroll
            for (int sd = 0; sd < 2; ++sd) {
                if (cc[sd] <= kLeafMax && micro_leaf(gbox, gl, cf[sd], cc[sd], dd + 1, v.max_depth)) {
                    ref[sd] = leaf_ref(task.y + cf[sd], cc[sd]);
                } else {
                    ref[sd] = next++;
                    if (gl == 0) {
                        nodes[ref[sd]].ch.z = id;
                        nodes[ref[sd]].ch.w = dd + 1;
                    }
                }
            }
            if (gl == 0) {
                write_boxes(nodes[id], L, R);
                nodes[id].ch.x = ref[0];
                nodes[id].ch.y = ref[1];
            }
            // right first, so that the left child is built next
#pragma unroll
            for (int sd = 1; sd >= 0; --sd) {
                if (ref[sd] >= 0) {
                    if (gl == sp) {
                        s_range = cf[sd] | (cc[sd] << 8);
                        s_id = ref[sd];
                        s_depth = dd + 1;
                    }
                    ++sp;
                }
            }
            if (sp == 0)
                break;
            --sp;
            const int t = __shfl(s_range, sp, kGroup);
            id = __shfl(s_id, sp, kGroup);
            dd = __shfl(s_depth, sp, kGroup);
            f = t & 255;
            c = t >> 8;
        }
        if (gl < cnt)
            prim[task.y + gl] = pid;
        if (gl == 0) {
            // unused reserved ids: never referenced; a depth of -1 keeps refit away
            for (int h = next; h < task.x + cnt - 1; ++h) {
                Node &u = nodes[h];
                u.xy0 = u.xy1 = u.z01 = make_float4(0.f, 0.f, 0.f, 0.f);
                u.ch = make_int4(0, 0, -1, -1);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Where each environment's deferred tasks start in one list of all of them
// (exclusive scan of the per-environment counts; masked environments count
// none); off[n_envs] is the total.  One workgroup.
constexpr int kScanBlock = 1024;

__global__ __launch_bounds__(kScanBlock) void k_count_scan(BuildView v, const int32_t *count, int64_t *off)
{
    __shared__ int64_t s[kScanBlock];
    int64_t carry = 0;
    for (int c0 = 0; c0 < v.n_envs; c0 += kScanBlock) {
        const int e = c0 + threadIdx.x;
        const int64_t x = (e < v.n_envs && !masked_out(v, e)) ? count[e] : 0;
        s[threadIdx.x] = x;
        __syncthreads();
        for (int d = 1; d < kScanBlock; d <<= 1) {
            const int64_t y = (int)threadIdx.x >= d ? s[threadIdx.x - d] : 0;
            __syncthreads();
            s[threadIdx.x] += y;
            __syncthreads();
        }
        if (e < v.n_envs)
            off[e] = carry + s[threadIdx.x] - x;
        carry += s[kScanBlock - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        off[v.n_envs] = carry;
}

// K5c: leaf-ordered records and the inverse permutation, one thread per triangle.
__global__ __launch_bounds__(256) void k_gather(BuildView v)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= v.n_tris)
        return;
    const int e = v.tri_env[g];
    if (masked_out(v, e))
        return;
    const int64_t base = v.env_tri_off[e];
    const int i = (int)(g - base);
    const int id = v.prim[g];
    const float *w = v.world + 9 * (base + id);
    TriRec rec;
    rec.a = make_float4(w[0], w[1], w[2], w[3]);
    rec.b = make_float4(w[4], w[5], w[6], w[7]);
    rec.c = make_float4(w[8], __int_as_float(id), 0.f, 0.f);
    v.recs[g] = rec;
    v.pos_of[base + id] = i;
    const int2 src = v.tri_src[base + id];
    v.leaf_src[g] = make_int4(src.x, src.y, id, 0);
}

// ---------------------------------------------------------------------------
// K7: refit.  One workgroup per environment walks its nodes level by level,
// deepest first (the build groups node slots by depth, see k_level_order):
// each node
// takes the bounds of its leaf children from the records and of its internal
// children from their (already refitted) two child boxes.  All traffic stays
// inside one workgroup, so a barrier between levels is the only
// synchronisation.  min/max are exact, so the result equals the from-scratch
// bounds bit for bit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void leaf_box(const TriRec *recs, int ref, float b[6])
{
    const int code = ~ref;
    const int first = code >> 3, cnt = (code & 7) + 1;
    float lx = INFINITY, ly = INFINITY, lz = INFINITY, hx = -INFINITY, hy = -INFINITY, hz = -INFINITY;
    // The first kLeafMax records are loaded together (a missing one re-reads
    // the last record, which leaves the union unchanged): one memory round
    // trip per leaf instead of one per triangle.
    float4 ra[kLeafMax], rb[kLeafMax];
    float rc[kLeafMax];
#pragma unroll
    for (int k = 0; k < kLeafMax; ++k) {
        const TriRec *t = recs + first + (k < cnt ? k : cnt - 1);
        ra[k] = t->a;
        rb[k] = t->b;
        rc[k] = t->c.x;
    }
#pragma unroll
    for (int k = 0; k < kLeafMax; ++k) {
        lx = fminf(lx, fminf(fminf(ra[k].x, ra[k].w), rb[k].z));
        ly = fminf(ly, fminf(fminf(ra[k].y, rb[k].x), rb[k].w));
        lz = fminf(lz, fminf(fminf(ra[k].z, rb[k].y), rc[k]));
        hx = fmaxf(hx, fmaxf(fmaxf(ra[k].x, ra[k].w), rb[k].z));
        hy = fmaxf(hy, fmaxf(fmaxf(ra[k].y, rb[k].x), rb[k].w));
        hz = fmaxf(hz, fmaxf(fmaxf(ra[k].z, rb[k].y), rc[k]));
    }
    for (int k = kLeafMax; k < cnt; ++k) {  // larger leaves (the encoding admits 8)
        const TriRec r = recs[first + k];
        lx = fminf(lx, fminf(fminf(r.a.x, r.a.w), r.b.z));
        ly = fminf(ly, fminf(fminf(r.a.y, r.b.x), r.b.w));
        lz = fminf(lz, fminf(fminf(r.a.z, r.b.y), r.c.x));
        hx = fmaxf(hx, fmaxf(fmaxf(r.a.x, r.a.w), r.b.z));
        hy = fmaxf(hy, fmaxf(fmaxf(r.a.y, r.b.x), r.b.w));
        hz = fmaxf(hz, fmaxf(fmaxf(r.a.z, r.b.y), r.c.x));
    }
    b[0] = expand_lo(lx);
    b[1] = expand_hi(hx);
    b[2] = expand_lo(ly);
    b[3] = expand_hi(hy);
    b[4] = expand_lo(lz);
    b[5] = expand_hi(hz);
}

// Box of internal child c = union of its two (stored, already expanded) child
// boxes; expansion commutes with min/max, so this equals the expanded union.
__device__ __forceinline__ void node_box(const Node &c, float b[6])
{
    b[0] = fminf(c.xy0.x, c.xy1.x);
    b[1] = fmaxf(c.xy0.y, c.xy1.y);
    b[2] = fminf(c.xy0.z, c.xy1.z);
    b[3] = fmaxf(c.xy0.w, c.xy1.w);
    b[4] = fminf(c.z01.x, c.z01.z);
    b[5] = fmaxf(c.z01.y, c.z01.w);
}

constexpr int kRefitBlock = 256;

// K5d: group each environment's node slots by depth (counting sort in LDS;
// order within a level is irrelevant to the refit), so the refit's level
// passes touch only their own nodes.  Holes (depth -1) are left out.
__global__ __launch_bounds__(kRefitBlock) void k_level_order(BuildView v)
{
    const int e = blockIdx.x;
    if (masked_out(v, e))
        return;
    __shared__ int cnt[kLevels], pos[kLevels + 1];
    const int64_t base = node_base(v.env_tri_off[e], e);
    const int nn = v.env_nodes[e];
    const Node *nodes = v.nodes + base;
    for (int d = threadIdx.x; d < kLevels; d += kRefitBlock)
        cnt[d] = 0;
    __syncthreads();
    for (int m = threadIdx.x; m < nn; m += kRefitBlock) {
        const int d = nodes[m].ch.w;
        if (d >= 0 && d < kLevels)
            atomicAdd(&cnt[d], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int d = 0; d < kLevels; ++d) {
            pos[d] = acc;
            acc += cnt[d];
        }
        pos[kLevels] = acc;
    }
    __syncthreads();
    int32_t *off = v.level_off + (int64_t)e * (kLevels + 1);
    for (int d = threadIdx.x; d <= kLevels; d += kRefitBlock)
        off[d] = pos[d];
    __syncthreads();
    int32_t *out = v.level_nodes + base;
    for (int m = threadIdx.x; m < nn; m += kRefitBlock) {
        const int d = nodes[m].ch.w;
        if (d >= 0 && d < kLevels)
            out[atomicAdd(&pos[d], 1)] = m;
    }
}

__global__ __launch_bounds__(kRefitBlock) void k_refit(BuildView v)
{
    const int e = blockIdx.x;
    if (masked_out(v, e))
        return;
    const int64_t base = node_base(v.env_tri_off[e], e);
    Node *nodes = v.nodes + base;
    const int32_t *order = v.level_nodes + base;
    const int32_t *off = v.level_off + (int64_t)e * (kLevels + 1);
    const TriRec *recs = v.recs + v.env_tri_off[e];
    for (int level = kMaxNodeDepth; level >= 0; --level) {
        const int a = off[level], b = off[level + 1];
        if (a == b)
            continue;  // uniform: every thread reads the same offsets
        for (int i = a + threadIdx.x; i < b; i += kRefitBlock) {
            const int m = order[i];
            const int4 ch = nodes[m].ch;
            float b0[6], b1[6];
            if (ch.x < 0)
                leaf_box(recs, ch.x, b0);
            else
                node_box(nodes[ch.x], b0);
            if (ch.y < 0)
                leaf_box(recs, ch.y, b1);
            else
                node_box(nodes[ch.y], b1);
            Node &nd = nodes[m];
            nd.xy0 = make_float4(b0[0], b0[1], b0[2], b0[3]);
            nd.xy1 = make_float4(b1[0], b1[1], b1[2], b1[3]);
            nd.z01 = make_float4(b0[4], b0[5], b1[4], b1[5]);
        }
        __syncthreads();
    }
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// K7b: four-wide records (WideRec), one workgroup per environment, one
// thread per node slot.  Reads the node and its internal children; a slot
// that is a hole of the node numbering (depth -1) is skipped.
__global__ __launch_bounds__(kRefitBlock) void k_wide_fill(BuildView v)
{
    const int e = blockIdx.x;
    if (masked_out(v, e))
        return;
    const int64_t base = node_base(v.env_tri_off[e], e);
    const Node *nodes = v.nodes + base;
    WideRec *wide = v.wide + base;
    const int nn = v.env_nodes[e];
    for (int m = threadIdx.x; m < nn; m += kRefitBlock) {
        const Node nd = nodes[m];
        if (nd.ch.w < 0)
            continue;
        float lx[4], hx[4], ly[4], hy[4], lz[4], hz[4];
        int ref[4];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int c = i ? nd.ch.y : nd.ch.x;
            if (c >= 0) {
                const Node cn = nodes[c];
                lx[2 * i] = cn.xy0.x;
                hx[2 * i] = cn.xy0.y;
                ly[2 * i] = cn.xy0.z;
                hy[2 * i] = cn.xy0.w;
                lz[2 * i] = cn.z01.x;
                hz[2 * i] = cn.z01.y;
                lx[2 * i + 1] = cn.xy1.x;
                hx[2 * i + 1] = cn.xy1.y;
                ly[2 * i + 1] = cn.xy1.z;
                hy[2 * i + 1] = cn.xy1.w;
                lz[2 * i + 1] = cn.z01.z;
                hz[2 * i + 1] = cn.z01.w;
                ref[2 * i] = cn.ch.x;
                ref[2 * i + 1] = cn.ch.y;
            } else {
                const float4 xy = i ? nd.xy1 : nd.xy0;
                lx[2 * i] = xy.x;
                hx[2 * i] = xy.y;
                ly[2 * i] = xy.z;
                hy[2 * i] = xy.w;
                lz[2 * i] = i ? nd.z01.z : nd.z01.x;
                hz[2 * i] = i ? nd.z01.w : nd.z01.y;
                ref[2 * i] = c;
                // empty slot: a point at +infinity, which both slab tests reject
                lx[2 * i + 1] = ly[2 * i + 1] = lz[2 * i + 1] = INFINITY;
                hx[2 * i + 1] = hy[2 * i + 1] = hz[2 * i + 1] = INFINITY;
                ref[2 * i + 1] = kDoneRef;
            }
        }
        WideRec w;
        w.lox = make_float4(lx[0], lx[1], lx[2], lx[3]);
        w.hix = make_float4(hx[0], hx[1], hx[2], hx[3]);
        w.loy = make_float4(ly[0], ly[1], ly[2], ly[3]);
        w.hiy = make_float4(hy[0], hy[1], hy[2], hy[3]);
        w.loz = make_float4(lz[0], lz[1], lz[2], lz[3]);
        w.hiz = make_float4(hz[0], hz[1], hz[2], hz[3]);
        w.ref = make_int4(ref[0], ref[1], ref[2], ref[3]);
        w.pair = make_int4(nd.ch.x, nd.ch.y, 0, 0);
        wide[m] = w;
    }
}



// ---------------------------------------------------------------------------
// K6: linear BVH (builder RC_BUILD_LBVH), one workgroup per environment of
// kLeafMax + 1 .. kLbvhMax triangles.  Centroids are quantised to 10 bits per
// axis on a grid of cubic cells over the environment's centroid bounds (1024
// cells along the widest axis) and bit-interleaved (Morton order); a
// triangle whose box has a side above a quarter of the widest centroid
// extent also sets the key's top bit, so the large triangles (a ground
// plane, the walls of a room) form a subtree of their own beside the root
// instead of widening the boxes of every subtree their centroids fall in.
// The (code, triangle id) keys are sorted in LDS.  The tree is then built
// top-down, one level per step: a node over the sorted keys
// first .. last splits where the range's highest differing key bit changes
// (the split of the radix tree of Karras 2012, found by binary search on
// common prefix lengths), unless a subtree that deep could exceed
// kMaxNodeDepth, in which case it splits at the index median (the SAH
// builder's rule), so the depth bound always holds.  A node's id is its split
// position (the last key of its left part): unique, and deterministic
// whatever the order the level's ranges are processed in; ids that no node
// takes stay holes.  Bounds are left to the refit.  An environment outside
// the size range is flagged in sah_mask for the SAH kernels.
// ---------------------------------------------------------------------------
constexpr int kLbvhMax = 8192;  // 64 KB of sort keys + 16 KB of level lists in LDS (40 KB up to 4096)
static_assert(kLbvhMax <= 65536, "ranges are packed as two 16-bit key positions");

__device__ __forceinline__ uint32_t spread3(uint32_t x)  // bit b of a 10-bit value -> bit 3b
{
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ __forceinline__ uint32_t quant10(float c, float lo, float scale)
{
    const float q = (c - lo) * scale;
    return q >= 1023.0f ? 1023u : (q > 0.0f ? (uint32_t)q : 0u);
}

// One instance per LDS footprint: environments of LO + 1 .. MAXN triangles,
// NT threads (the larger footprint fits one workgroup per CU, so it takes
// more threads).  The FIRST instance also settles every environment no
// instance takes.
template <int MAXN, int LO, bool FIRST, int NT>
__global__ __launch_bounds__(NT) void k_lbvh(BuildView v, uint8_t *sah_mask)
{
    static_assert(MAXN <= kLbvhMax, "above the LBVH size limit");
    __shared__ uint64_t key[MAXN];
    // ranges of one level and of the next: (first, last) as 16-bit halves and
    // 2 * parent id + side (the root's parent is -1); a range holds at least
    // kLeafMax + 1 keys, so a level has at most MAXN / 5 of them
    constexpr int kList = MAXN / 5 + 1;
    __shared__ uint32_t wr[2][kList];
    __shared__ int wp[2][kList];
    __shared__ int wcnt[2];
    __shared__ float red[6][NT / 64];
    __shared__ int s_root;
    const int e = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = v.env_tri_off[e];
    const int n = (int)(v.env_tri_off[e + 1] - base);
    const bool want = !masked_out(v, e);
    if (!want || n <= LO || n > MAXN) {
        const bool lbvh_any = want && n > kLeafMax && n <= kLbvhMax;
        if (FIRST && tid == 0 && !lbvh_any)
            sah_mask[e] = want ? 1 : 0;
        return;
    }
    const float4 *blo = v.box_lo + base, *bhi = v.box_hi + base;
    // centroid bounds
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = tid; i < n; i += NT) {
        const float4 a = blo[i], b = bhi[i];
        const float c[3] = {0.5f * (a.x + b.x), 0.5f * (a.y + b.y), 0.5f * (a.z + b.z)};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], c[k]);
            hi[k] = fmaxf(hi[k], c[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        lo[k] = wave_min(lo[k]);
        hi[k] = wave_max(hi[k]);
        if (lane == 0) {
            red[k][wave] = lo[k];
            red[3 + k][wave] = hi[k];
        }
    }
    __syncthreads();
    float scale[3], ext = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float a = red[k][0], b = red[3 + k][0];
        for (int w = 1; w < NT / 64; ++w) {
            a = fminf(a, red[k][w]);
            b = fmaxf(b, red[3 + k][w]);
        }
        lo[k] = a;
        ext = fmaxf(ext, b - a);
    }
    // cubic cells: every axis quantised at the step of the widest one, so a
    // flat environment's first splits cut across its wide axes, not its height
#pragma unroll
    for (int k = 0; k < 3; ++k)
        scale[k] = ext > 0.0f ? 1024.0f / ext : 0.0f;
    const float big = 0.25f * ext;  // "large": a box side above a quarter of the widest centroid extent
    // keys, padded to a power of two with the largest key
    int P = 8;
    while (P < n)
        P <<= 1;
    for (int i = tid; i < P; i += NT) {
        uint64_t k64 = ~0ull;
        if (i < n) {
            const float4 a = blo[i], b = bhi[i];
            const float size = fmaxf(fmaxf(b.x - a.x, b.y - a.y), b.z - a.z);
            const uint32_t code = (spread3(quant10(0.5f * (a.x + b.x), lo[0], scale[0])) << 2) |
                                  (spread3(quant10(0.5f * (a.y + b.y), lo[1], scale[1])) << 1) |
                                  spread3(quant10(0.5f * (a.z + b.z), lo[2], scale[2])) |
                                  (size > big ? 0x80000000u : 0u);
            k64 = ((uint64_t)code << 32) | (uint32_t)i;
        }
        key[i] = k64;
    }
    __syncthreads();
    // bitonic sort: pair (i, i + j), i with bit j clear, ascending where bit k of i is clear
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = tid; t < P / 2; t += NT) {
                const int i = 2 * j * (t / j) + (t % j), m = i + j;
                const bool up = (i & k) == 0;
                const uint64_t a = key[i], b = key[m];
                if (up ? b < a : a < b) {
                    key[i] = b;
                    key[m] = a;
                }
            }
            __syncthreads();
        }
    }
    int32_t *prim = v.prim + base;
    for (int i = tid; i < n; i += NT)
        prim[i] = (int)(uint32_t)key[i];
    // top-down construction; delta = common prefix length of two keys
    Node *nodes = v.nodes + node_base(base, e);
    auto delta = [&](int a, int b) -> int { return __clzll(key[a] ^ key[b]); };
    for (int i = tid; i < n - 1; i += NT) {  // every id a hole until a node takes it
        Node &nd = nodes[i];
        nd.xy0 = nd.xy1 = nd.z01 = make_float4(0.f, 0.f, 0.f, 0.f);
        nd.ch = make_int4(0, 0, -1, -1);
    }
    if (tid == 0) {
        wr[0][0] = (uint32_t)(n - 1) << 16;  // keys 0 .. n - 1
        wp[0][0] = -2;                        // parent -1, side 0
        wcnt[0] = 1;
        wcnt[1] = 0;
    }
    __syncthreads();
    int cur = 0;
    for (int depth = 0; depth <= kMaxNodeDepth; ++depth) {
        const int cnt = wcnt[cur], nxt = cur ^ 1;
        if (cnt == 0)
            break;
        for (int t = tid; t < cnt; t += NT) {
            const int first = (int)(wr[cur][t] & 0xffffu), last = (int)(wr[cur][t] >> 16);
            const int pw = wp[cur][t], parent = pw >> 1, side = pw & 1;
            const int size = last - first + 1;
            int g;  // the left part ends at key g
            if (depth + levels_needed(size) - 1 >= v.max_depth) {
                g = first + size / 2 - 1;
            } else {
                const int dnode = delta(first, last);
                int lo = first, hi = last - 1;  // largest g with delta(first, g) > dnode
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (delta(first, mid) > dnode)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                g = lo;
            }
            Node &nd = nodes[g];
            nd.ch.z = parent;
            nd.ch.w = depth;
            if (parent < 0)
                s_root = g;
            else if (side == 0)
                nodes[parent].ch.x = g;
            else
                nodes[parent].ch.y = g;
            const int nl = g - first + 1, nr = last - g;
            if (nl > kLeafMax) {
                const int q = atomicAdd(&wcnt[nxt], 1);
                wr[nxt][q] = (uint32_t)first | ((uint32_t)g << 16);
                wp[nxt][q] = 2 * g;
            } else {
                nd.ch.x = leaf_ref(first, nl);
            }
            if (nr > kLeafMax) {
                const int q = atomicAdd(&wcnt[nxt], 1);
                wr[nxt][q] = (uint32_t)(g + 1) | ((uint32_t)last << 16);
                wp[nxt][q] = 2 * g + 1;
            } else {
                nd.ch.y = leaf_ref(g + 1, nr);
            }
        }
        __syncthreads();
        if (tid == 0)
            wcnt[cur] = 0;
        cur = nxt;
        __syncthreads();
    }
    if (tid == 0) {
        sah_mask[e] = 0;
        v.env_root[e] = s_root;
        v.env_nodes[e] = n - 1;
        v.env_micro[e] = 0;
    }
}

}  // namespace

hipError_t launch_transform(const BuildView &v, const int32_t *tri_list, int64_t n, bool to_recs, hipStream_t st)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_transform, dim3(blocks_for(n, 256)), dim3(256), 0, st, v, tri_list, n, (int)to_recs);
    return hipGetLastError();
}

hipError_t launch_transform_leaf(const BuildView &v, hipStream_t st)
{
    if (v.n_tris == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_transform_leaf, dim3(blocks_for(v.n_tris, 256)), dim3(256), 0, st, v);
    return hipGetLastError();
}

hipError_t launch_pose_snapshot(int64_t n_inst, const int32_t *inst_env, const uint8_t *dyn, const uint8_t *env_mask,
                                bool dyn_only, const float *src, float *dst, uint8_t *stale_env, hipStream_t st)
{
    if (n_inst == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pose_snapshot, dim3(blocks_for(n_inst, 256)), dim3(256), 0, st, n_inst, inst_env, dyn,
                       env_mask, (int)dyn_only, src, dst, stale_env);
    return hipGetLastError();
}

hipError_t launch_inst_prep(const InstPrep &p, hipStream_t st)
{
    if (p.n_inst == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_inst_prep, dim3(blocks_for(p.n_inst, 256)), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_move(int64_t n_inst, const float *T0, const float *vel, const uint8_t *dyn, int32_t step,
                       const int32_t *d_step, float dt, float *T, hipStream_t st)
{
    if (n_inst == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_move, dim3(blocks_for(n_inst, 256)), dim3(256), 0, st, n_inst, T0, vel, dyn, step, d_step,
                       dt, T);
    return hipGetLastError();
}

__global__ void k_bump(int32_t *d_step)
{
    if (threadIdx.x == 0)
        *d_step += 1;
}

hipError_t launch_bump(int32_t *d_step, hipStream_t st)
{
    hipLaunchKernelGGL(k_bump, dim3(1), dim3(64), 0, st, d_step);
    return hipGetLastError();
}

// Subtrees of at most kSmall primitives (k_build_local, one wavefront each),
// then the ranges of 5..kMicro primitives (k_build_micro), for the
// environments the view admits.
hipError_t launch_deferred(const BuildView &v, hipStream_t st)
{
    hipLaunchKernelGGL(k_count_scan, dim3(1), dim3(kScanBlock), 0, st, v, (const int32_t *)v.env_local, v.local_off);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess)
        return err;
    // persistent wavefronts; a deferred subtree holds > kMicro primitives (or is a whole environment)
    const int64_t tasks = v.n_tris / (kMicro + 1) + v.n_envs;
    hipLaunchKernelGGL(k_build_local, dim3((unsigned)(tasks < 8192 ? tasks : 8192)), dim3(64), 0, st, v);
    if ((err = hipGetLastError()) != hipSuccess)
        return err;
    hipLaunchKernelGGL(k_count_scan, dim3(1), dim3(kScanBlock), 0, st, v, (const int32_t *)v.env_micro, v.micro_off);
    if ((err = hipGetLastError()) != hipSuccess)
        return err;
    // persistent groups; every range holds >= 5 primitives, so there are at most n_tris / 5
    const int64_t groups = v.n_tris / 5 + 1;
    const int64_t blocks = (groups * kGroup + kMicroBlock - 1) / kMicroBlock;
    hipLaunchKernelGGL(k_build_micro, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(kMicroBlock), 0, st, v);
    return hipGetLastError();
}

hipError_t launch_build_sah(const BuildView &v, hipStream_t st)
{
    if (v.n_tris > 0) {
        hipLaunchKernelGGL(k_bounds, dim3(blocks_for(v.n_tris, 256)), dim3(256), 0, st, v);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess)
            return err;
    }
    if (v.n_envs == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_build_sah, dim3(v.n_envs), dim3(64), 0, st, v);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess || v.n_tris == 0)
        return err;
    if ((err = launch_deferred(v, st)) != hipSuccess)
        return err;
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(v.n_tris, 256)), dim3(256), 0, st, v);
    if ((err = hipGetLastError()) != hipSuccess)
        return err;
    hipLaunchKernelGGL(k_level_order, dim3(v.n_envs), dim3(kRefitBlock), 0, st, v);
    if ((err = hipGetLastError()) != hipSuccess)
        return err;
    return launch_wide_fill(v, st);
}

hipError_t launch_build_lbvh(const BuildView &v, uint8_t *sah_mask, hipStream_t st)
{
    if (v.n_envs == 0)
        return hipSuccess;
    if (v.n_tris > 0) {
        hipLaunchKernelGGL(k_bounds, dim3(blocks_for(v.n_tris, 256)), dim3(256), 0, st, v);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess)
            return err;
    }
    hipLaunchKernelGGL((k_lbvh<kLbvhMax / 2, kLeafMax, true, 256>), dim3(v.n_envs), dim3(256), 0, st, v, sah_mask);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess)
        return err;
    hipLaunchKernelGGL((k_lbvh<kLbvhMax, kLbvhMax / 2, false, 1024>), dim3(v.n_envs), dim3(1024), 0, st, v, sah_mask);
    if ((err = hipGetLastError()) != hipSuccess)
        return err;
    // the SAH kernels build exactly the environments flagged above
    BuildView vs = v;
    vs.env_mask = sah_mask;
    hipLaunchKernelGGL(k_build_sah, dim3(v.n_envs), dim3(64), 0, st, vs);
    if ((err = hipGetLastError()) != hipSuccess || v.n_tris == 0)
        return err;
    if ((err = launch_deferred(vs, st)) != hipSuccess)
        return err;
    // every requested environment: records in leaf order, level lists, bounds
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(v.n_tris, 256)), dim3(256), 0, st, v);
    if ((err = hipGetLastError()) != hipSuccess)
        return err;
    hipLaunchKernelGGL(k_level_order, dim3(v.n_envs), dim3(kRefitBlock), 0, st, v);
    if ((err = hipGetLastError()) != hipSuccess)
        return err;
    return launch_refit(v, st);
}

hipError_t launch_refit(const BuildView &v, hipStream_t st)
{
    if (v.n_envs == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_refit, dim3(v.n_envs), dim3(kRefitBlock), 0, st, v);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess || !v.wide)
        return err;
    return launch_wide_fill(v, st);
}

hipError_t launch_wide_fill(const BuildView &v, hipStream_t st)
{
    if (v.n_envs == 0 || !v.wide)
        return hipSuccess;
    hipLaunchKernelGGL(k_wide_fill, dim3(v.n_envs), dim3(kRefitBlock), 0, st, v);
    return hipGetLastError();
}

}  // namespace rc
