// rc_render.hip -- ray generation, BVH traversal and output kernels (gfx950).
//
// Paper, Sec. III-D: one ray per pixel (pinhole) or beam (LiDAR) is cast
// against the environment's transformed mesh; the sensor-to-hit distance is
// range, the distance from the image plane is depth, and segmentation, face
// index and hit point come from the same nearest hit.
//
// Arithmetic.  Traversal and triangle tests run in FP32.  Every FP32 test
// carries a forward error bound, so each decision is either certain (equal to
// the exact-arithmetic decision) or flagged uncertain; uncertain decisions,
// and the reported t of the final winner, are evaluated in FP64 on the same
// FP32 inputs (an adaptive-precision predicate).  Hence every render mode and
// every BVH returns the exact nearest hit up to FP64 rounding, with the
// lowest-id tie break, and all modes are bit-identical.
//
// Layout.  A wavefront (64 lanes) takes one tile of 64 rays of one sensor
// instance (4, 8, 16 or 32 columns by 16, 8, 4 or 2 rows, a tuning choice);
// a 256-lane workgroup holds four such tiles.  The traversal stack lives in
// LDS (kStack entries per lane, lane-interleaved).
#include "rc_common.hpp"

namespace rc {

namespace {

constexpr float kU = 0x1p-24f;              // unit roundoff
constexpr float kErr = 0x1p-17f;            // triple-product error factor (>= 48 u)
constexpr float kBoxGrow = 1.0f + 0x1p-20f;  // >= 1 + 4 gamma_3 (robust slab test)
constexpr int kBlock = 256;
// Render kernels are latency bound: ask for seven waves per SIMD (72 VGPRs),
// which the LDS stack also admits (on the LiDAR forest six waves measured
// 4 % slower than seven, and five 23 % slower than six).
#ifndef RC_MIN_WAVES
#define RC_MIN_WAVES 7
#endif
#define RC_WAVES_PER_EU __attribute__((amdgpu_waves_per_eu(RC_MIN_WAVES, 8)))
// Two-level scenes keep a second (object-space) ray in registers: four waves
// per SIMD (128 VGPRs).
#ifndef RC_MIN_WAVES_TWO
#define RC_MIN_WAVES_TWO 4
#endif
#define RC_WAVES_PER_EU_T __attribute__((amdgpu_waves_per_eu(TWO ? RC_MIN_WAVES_TWO : RC_MIN_WAVES, 8)))

struct Ray {
    static constexpr bool kObject = false;
    float ox, oy, oz;
    float dx, dy, dz;
    float ix, iy, iz;
    float knd;  // kErr * max|d_i|
    float tn, tf;
    // Plane constants of the single-octant slab test (slab_consts): axis a
    // enters a box at fma(near_a, i_a, cn_a) and leaves it at
    // fma(far_a, i_a, cf_a).
    float cnx, cny, cnz, cfx, cfy, cfz;
};

// cn_a / cf_a = -o_a i_a moved down / up by s_a = 3u |o_a i_a|.  With p the
// rounded product o_a i_a, the exact value of n i_a + cn_a is at most
// (n - o_a) i_a: the product's rounding (u |o_a i_a|) and the constant's own
// (u |p + s_a|) are covered by s_a; likewise the exit lies at or beyond
// (f - o_a) i_a.  The fused multiply-add then rounds once, so each plane's
// computed parameter is within one rounding (relative) of the
// subtract-multiply value's exact counterpart, and the same growth factor
// kBoxGrow keeps the test conservative.  An infinite or overflowing product
// (a zero direction component) makes the constants infinite or NaN: the
// plane parameters are then NaN or an infinity that cannot cull, and
// fminf / fmaxf ignore NaN operands, so that axis never rejects a box.
__device__ __forceinline__ float slab_slack(float p) { return (3.0f * kU) * fabsf(p); }

__device__ __forceinline__ void slab_consts(Ray &r)
{
    const float px = r.ox * r.ix, py = r.oy * r.iy, pz = r.oz * r.iz;
    const float sx = slab_slack(px), sy = slab_slack(py), sz = slab_slack(pz);
    r.cnx = -px - sx;
    r.cny = -py - sy;
    r.cnz = -pz - sz;
    r.cfx = -px + sx;
    r.cfy = -py + sy;
    r.cfz = -pz + sz;
}

__device__ __forceinline__ float uniform_f(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Unified wave-uniform view of one work item.
struct Tile {
    int s, env, W, H, kind, tiles_x, tw_shift;
    float hw, hh, scale, tn, tf;
    int64_t table_off, ray_base;
};

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Ray of (row, col) of sensor instance s.  Local direction: pinhole
// (1, -(col+1/2-W/2) s, -(row+1/2-H/2) s); lidar / table from the FP32
// direction table.  World direction i = fma(P_i0, dx, fma(P_i1, dy, P_i2 dz)).
__device__ __forceinline__ void local_dir(const SensorView &se, const Tile &t, int row, int col, float &lx, float &ly,
                                          float &lz)
{
    if (t.kind == 0) {
        lx = 1.0f;
        ly = -((((float)col + 0.5f) - t.hw) * t.scale);
        lz = -((((float)row + 0.5f) - t.hh) * t.scale);
    } else {
        const float *d = se.tables + 3 * (t.table_off + (int64_t)row * t.W + col);
        lx = d[0];
        ly = d[1];
        lz = d[2];
    }
}

__device__ __forceinline__ void gen_ray(const SensorView &se, const Tile &t, int row, int col, Ray &r)
{
    float lx, ly, lz;
    local_dir(se, t, row, col, lx, ly, lz);
    const float *P = se.pose + 12 * (int64_t)t.s;
    // the origin and the range are those of the tile's sensor instance:
    // wave-uniform, so they live in scalar registers
    r.ox = uniform_f(P[3]);
    r.oy = uniform_f(P[7]);
    r.oz = uniform_f(P[11]);
    r.dx = fmaf(P[0], lx, fmaf(P[1], ly, P[2] * lz));
    r.dy = fmaf(P[4], lx, fmaf(P[5], ly, P[6] * lz));
    r.dz = fmaf(P[8], lx, fmaf(P[9], ly, P[10] * lz));
    r.ix = 1.0f / r.dx;
    r.iy = 1.0f / r.dy;
    r.iz = 1.0f / r.dz;
    r.knd = kErr * fmaxf(fmaxf(fabsf(r.dx), fabsf(r.dy)), fabsf(r.dz));
    r.tn = uniform_f(t.tn);
    r.tf = uniform_f(t.tf);
    slab_consts(r);
}

__device__ __forceinline__ Tile load_tile(const SensorView &se, int2 item)
{
    Tile t;
    t.s = item.x;
    const int m = se.si_model[t.s];
    const SensorModel &M = se.models[m];
    t.env = se.si_env[t.s];
    t.W = M.W;
    t.H = M.H;
    t.kind = M.kind;
    t.tiles_x = M.tiles_x;
    t.tw_shift = M.tw_shift;
    t.hw = M.hw;
    t.hh = M.hh;
    t.scale = M.s;
    t.tn = M.tn;
    t.tf = M.tf;
    t.table_off = M.table_off;
    t.ray_base = se.ray_off[t.s];
    return t;
}

// ---------------------------------------------------------------------------
// Maximum and minimum of quiet operands.  fmaxf / fminf must quiet a
// signalling NaN, so the compiler re-quiets every operand it cannot prove to
// be an arithmetic result, and a loop-invariant limit (the ray's near limit,
// the current hit bound) costs one extra instruction per node visit.  Every
// operand here is an arithmetic result or a finite limit checked on the host,
// so the plain instructions give the same result: a NaN operand is ignored,
// as by fmaxf / fminf.  The operand `u` of the _u forms is read from a scalar
// register and must be wave-uniform.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float qmax3(float a, float b, float c)
{
    float d;
    asm("v_max3_f32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

__device__ __forceinline__ float qmin3(float a, float b, float c)
{
    float d;
    asm("v_min3_f32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

__device__ __forceinline__ float qmax_u(float a, float u)
{
    float d;
    asm("v_max_f32 %0, %1, %2" : "=v"(d) : "s"(u), "v"(a));
    return d;
}

__device__ __forceinline__ float qmin(float a, float b)
{
    float d;
    asm("v_min_f32 %0, %1, %2" : "=v"(d) : "v"(a), "v"(b));
    return d;
}

// ---------------------------------------------------------------------------
// Robust slab test (boxes are stored expanded outward by one float step).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool slab(const Ray &r, float lx, float hx, float ly, float hy, float lz, float hz,
                                     float tcap, float &tenter)
{
    const float t0x = (lx - r.ox) * r.ix, t1x = (hx - r.ox) * r.ix;
    const float t0y = (ly - r.oy) * r.iy, t1y = (hy - r.oy) * r.iy;
    const float t0z = (lz - r.oz) * r.iz, t1z = (hz - r.oz) * r.iz;
    const float tmin = qmax_u(qmax3(fminf(t0x, t1x), fminf(t0y, t1y), fminf(t0z, t1z)), r.tn);
    const float tmax = qmin(qmin3(fmaxf(t0x, t1x), fmaxf(t0y, t1y), fmaxf(t0z, t1z)), tcap);
    tenter = tmin;
    return tmin <= tmax * kBoxGrow;
}

// The same test when every lane of the wavefront has the same direction
// octant (bit a of OCT: the inverse direction component a has its sign bit
// set; OCT = kMixed selects the general test above).  The near plane of each
// axis is then known from the sign alone (the low plane for a non-negative
// inverse), so the min / max pairs of the general test reduce to a choice,
// and each plane costs one fused multiply-add with the ray's plane constants
// (slab_consts) instead of a subtraction and a multiplication.  Where the
// general test treats a plane the ray runs parallel to as a miss or a hit
// exactly, this one ignores the axis (see slab_consts); both are safe,
// because a stored box lies strictly outside its triangles' bounds (one float
// step), so such a ray cannot reach a triangle inside it.
constexpr int kMixed = 8;

template <int OCT>
__device__ __forceinline__ bool slab_oct(const Ray &r, float lx, float hx, float ly, float hy, float lz, float hz,
                                         float tcap, float &tenter)
{
    if constexpr (OCT == kMixed) {
        return slab(r, lx, hx, ly, hy, lz, hz, tcap, tenter);
    } else {
        const float nx = (OCT & 1) ? hx : lx, fx = (OCT & 1) ? lx : hx;
        const float ny = (OCT & 2) ? hy : ly, fy = (OCT & 2) ? ly : hy;
        const float nz = (OCT & 4) ? hz : lz, fz = (OCT & 4) ? lz : hz;
        const float tmin = qmax3(fmaf(nx, r.ix, r.cnx), fmaf(ny, r.iy, r.cny), qmax_u(fmaf(nz, r.iz, r.cnz), r.tn));
        const float tmax = qmin3(fmaf(fx, r.ix, r.cfx), fmaf(fy, r.iy, r.cfy), qmin(fmaf(fz, r.iz, r.cfz), tcap));
        tenter = tmin;
        return tmin <= tmax * kBoxGrow;
    }
}

// Raw buffer view of one environment's nodes or triangle records: the
// traversal's loads take a 32-bit byte offset per lane instead of 64-bit
// address arithmetic, and the hardware checks the range (a load past the
// view's size returns zeros).
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // descriptor dword 3 for untyped loads (gfx9 family)

__device__ __forceinline__ Rsrc buffer_view(const void *p, int64_t bytes)
{
    const uint32_t n = bytes < 0xffffffffll ? (uint32_t)bytes : 0xffffffffu;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)n, kRsrcWord3);
}
__device__ __forceinline__ float4 ldf4(Rsrc r, uint32_t off)
{
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
__device__ __forceinline__ int4 ldi4(Rsrc r, uint32_t off)
{
    return __builtin_bit_cast(int4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

// Octant shared by every active lane of the wavefront, else kMixed.
__device__ __forceinline__ int wave_octant(const Ray &r)
{
    const int o = (signbit(r.ix) ? 1 : 0) | (signbit(r.iy) ? 2 : 0) | (signbit(r.iz) ? 4 : 0);
    const int o0 = uniform(o);
    return __all(o == o0) ? o0 : kMixed;
}

// ---------------------------------------------------------------------------
// Moller-Trumbore with certified FP32 decisions.
//   e1 = v1 - v0, e2 = v2 - v0, T = o - v0, p = d x e2, q = T x e1,
//   det = e1.p, U = T.p, V = d.q, W = e2.q;  hit iff det != 0, U/det >= 0,
//   V/det >= 0, (U+V)/det <= 1 and near <= W/det <= far.
// Each triple product is within kErr * (product of the operands' max-norms)
// of its exact value.  Returns kReject / kAccept when certain, else kUnsure;
// on kAccept, [t - et, t + et] contains the exact t.
// ---------------------------------------------------------------------------
enum { kReject = 0, kAccept = 1, kUnsure = 2 };

template <class R>
__device__ __forceinline__ int mt32(const R &r, const float4 A, const float4 B, const float4 C, float tcap, float &t,
                                    float &et)
{
    const float e1x = A.w - A.x, e1y = B.x - A.y, e1z = B.y - A.z;
    const float e2x = B.z - A.x, e2y = B.w - A.y, e2z = C.x - A.z;
    const float Tx = r.ox - A.x, Ty = r.oy - A.y, Tz = r.oz - A.z;
    const float px = fmaf(r.dy, e2z, -(r.dz * e2y));
    const float py = fmaf(r.dz, e2x, -(r.dx * e2z));
    const float pz = fmaf(r.dx, e2y, -(r.dy * e2x));
    const float det = fmaf(e1x, px, fmaf(e1y, py, e1z * pz));
    const float qx = fmaf(Ty, e1z, -(Tz * e1y));
    const float qy = fmaf(Tz, e1x, -(Tx * e1z));
    const float qz = fmaf(Tx, e1y, -(Ty * e1x));
    const float U = fmaf(Tx, px, fmaf(Ty, py, Tz * pz));
    const float V = fmaf(r.dx, qx, fmaf(r.dy, qy, r.dz * qz));
    const float W = fmaf(e2x, qx, fmaf(e2y, qy, e2z * qz));
    const float n1 = fmaxf(fmaxf(fabsf(e1x), fabsf(e1y)), fabsf(e1z));
    const float n2 = fmaxf(fmaxf(fabsf(e2x), fabsf(e2y)), fabsf(e2z));
    float nT = fmaxf(fmaxf(fabsf(Tx), fabsf(Ty)), fabsf(Tz));
    if constexpr (R::kObject)
        nT += r.no;  // the ray's FP32 origin is a rounded one (ObjRay)
    const float kT = r.knd * nT;
    const float eD = r.knd * n1 * n2;
    const float eU = kT * n2;
    const float eV = kT * n1;
    const float eW = kErr * nT * n1 * n2;
    const float ad = fabsf(det);
    if (!(ad > 2.0f * eD))
        return kUnsure;
    const bool neg = det < 0.0f;
    const float sU = neg ? -U : U, sV = neg ? -V : V, sW = neg ? -W : W;
    if (sU < -eU || sV < -eV)
        return kReject;
    const float S = sU + sV;
    const float eS = eU + eV + eD + 4.0f * kU * (fabsf(sU) + fabsf(sV) + ad);
    if (S > ad + eS)
        return kReject;
    const float rcp = __builtin_amdgcn_rcpf(ad);
    t = sW * rcp;
    const float at = fabsf(t);
    et = 2.0f * fmaf(at, eD, eW) * rcp + 4.0f * kU * at;
    if (t + et < r.tn || t - et > tcap)
        return kReject;
    const bool sure = sU >= eU && sV >= eV && S <= ad - eS && t - et >= r.tn && t + et <= r.tf;
    return sure ? kAccept : kUnsure;
}

// FP64 evaluation of the same test on the same FP32 inputs.  Kept out of
// line (it runs only for uncertain tests and winners) and called by value so
// the ray stays in registers.
struct T64 {
    double t;
    int ok;
};

__device__ __noinline__ T64 mt64v(float ox, float oy, float oz, float dxf, float dyf, float dzf, float tn, float tf,
                                 float4 A, float4 B, float4 C)
{
    T64 res{0.0, 0};
    const double ax = A.x, ay = A.y, az = A.z;
    const double e1x = (double)A.w - ax, e1y = (double)B.x - ay, e1z = (double)B.y - az;
    const double e2x = (double)B.z - ax, e2y = (double)B.w - ay, e2z = (double)C.x - az;
    const double dx = dxf, dy = dyf, dz = dzf;
    const double px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
    double det = e1x * px + e1y * py + e1z * pz;
    if (det == 0.0)
        return res;
    const double Tx = (double)ox - ax, Ty = (double)oy - ay, Tz = (double)oz - az;
    const double qx = Ty * e1z - Tz * e1y, qy = Tz * e1x - Tx * e1z, qz = Tx * e1y - Ty * e1x;
    double U = Tx * px + Ty * py + Tz * pz;
    double V = dx * qx + dy * qy + dz * qz;
    double W = e2x * qx + e2y * qy + e2z * qz;
    if (det < 0.0) {
        det = -det;
        U = -U;
        V = -V;
        W = -W;
    }
    if (U < 0.0 || V < 0.0 || U + V > det)
        return res;
    res.t = W / det;
    res.ok = res.t >= (double)tn && res.t <= (double)tf;
    return res;
}

__device__ __forceinline__ bool mt64(const Ray &r, const float4 A, const float4 B, const float4 C, double &t)
{
    const T64 q = mt64v(r.ox, r.oy, r.oz, r.dx, r.dy, r.dz, r.tn, r.tf, A, B, C);
    t = q.t;
    return q.ok != 0;
}

struct Best {
    float lo, hi;  // bracket of the exact t of the current winner
    int pos;       // record index (-1: none)
    int id;        // environment-local triangle id
    bool have64;
    double t64;
    int inst = -1;  // two-level scenes: the winner's instance (pos indexes its mesh's records)
};

struct Stats {
    unsigned box, tri, fp64;
};

// Offer triangle record (A, B, C) at index pos to the running winner.
template <bool STATS>
__device__ __forceinline__ void offer(const Ray &r, const TriRec *__restrict__ recs, int pos, const float4 A,
                                     const float4 B, const float4 C, Best &b, Stats &st)
{
    float t, et;
    const int code = mt32(r, A, B, C, b.hi, t, et);
    if (code == kReject)
        return;
    if (code == kAccept && t + et < b.lo) {
        b.lo = t - et;
        b.hi = t + et;
        b.pos = pos;
        b.id = __float_as_int(C.y);
        b.have64 = false;
        return;
    }
    if (STATS)
        ++st.fp64;
    double tc;
    if (!mt64(r, A, B, C, tc))
        return;
    const int idc = __float_as_int(C.y);
    if (b.pos >= 0 && !b.have64) {
        const TriRec w = recs[b.pos];
        double tw;
        if (mt64(r, w.a, w.b, w.c, tw)) {
            b.t64 = tw;
            b.have64 = true;
        } else {
            b.pos = -1;  // cannot happen for a certain accept; drop it defensively
        }
    }
    if (b.pos < 0 || tc < b.t64 || (tc == b.t64 && idc < b.id)) {
        b.pos = pos;
        b.id = idc;
        b.t64 = tc;
        b.have64 = true;
        const float tf = (float)tc;
        b.lo = tf * (1.0f - 0x1p-23f);
        b.hi = tf * (1.0f + 0x1p-23f);
    }
}

// Stack-based traversal of one ray (nearest child first), in two phases per
// round so that the wavefront stays converged: phase 1 walks internal nodes
// and postpones the first leaf it meets (continuing down the tree until every
// active lane holds a leaf or finishes); phase 2 tests the postponed leaves.
constexpr int kDone = INT32_MIN;  // never a leaf reference

// Phase 1 of a round: walk internal nodes until this lane holds a leaf (or
// has finished) and every other active lane does too.
template <bool STATS, int OCT>
__device__ __forceinline__ void descend(const Ray &r, Rsrc nodes, int *stk, float tcap, int &sp, int &ref, int &leaf,
                                        Stats &st)
{
    while (ref >= 0) {
        const uint32_t off = (uint32_t)ref * (uint32_t)sizeof(Node);
        const float4 a = ldf4(nodes, off), c = ldf4(nodes, off + 16), z = ldf4(nodes, off + 32);
        const int4 ch = ldi4(nodes, off + 48);
        // Issue all four loads of the node before the first use: left alone,
        // the scheduler may start on the first box and send the last load
        // after waiting for the others, a second memory round trip per node.
        __builtin_amdgcn_sched_barrier(0);
        float t0, t1;
        const bool h0 = slab_oct<OCT>(r, a.x, a.y, a.z, a.w, z.x, z.y, tcap, t0);
        const bool h1 = slab_oct<OCT>(r, c.x, c.y, c.z, c.w, z.z, z.w, tcap, t1);
        if (STATS)
            st.box += 2;
        if (h0 && h1) {
            const bool first0 = t0 <= t1;
            stk[sp * kBlock] = first0 ? ch.y : ch.x;
            ++sp;
            ref = first0 ? ch.x : ch.y;
        } else if (h0 || h1) {
            ref = h0 ? ch.x : ch.y;
        } else {
            ref = sp > 0 ? stk[--sp * kBlock] : kDone;
        }
        if (ref < 0 && ref != kDone && leaf == kDone) {
            leaf = ref;
            ref = sp > 0 ? stk[--sp * kBlock] : kDone;
        }
        if (__all(leaf != kDone))
            break;
    }
}

__device__ __forceinline__ float comp(const float4 &v, int k)
{
    return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
}

// Phase 1 on the four-wide records (WideRec): one visit of internal node m
// tests the up to four boxes one level below m's children.  The nearer
// pair's nearer slot is visited next; the farther pair is pushed as one
// entry (m's child itself when both of its slots are hit, else the one slot
// hit), then the nearer pair's other slot.  Every path visit leaves on the
// stack at most as many entries as it descends levels of the binary tree, so
// the stack bound of the binary traversal (kMaxNodeDepth + 2) still holds.
// A popped child entry is visited through its own record, which tests the
// level below the boxes already passed: conservative, and the certified
// triangle tests make the result independent of the order.
template <bool STATS, int OCT>
__device__ __forceinline__ void descend_wide(const Ray &r, Rsrc wide, int *stk, float tcap, int &sp, int &ref,
                                             int &leaf, Stats &st)
{
    while (ref >= 0) {
        const uint32_t off = (uint32_t)ref * (uint32_t)sizeof(WideRec);
        const float4 lx = ldf4(wide, off), hx = ldf4(wide, off + 16), ly = ldf4(wide, off + 32);
        const float4 hy = ldf4(wide, off + 48), lz = ldf4(wide, off + 64), hz = ldf4(wide, off + 80);
        const int4 rf = ldi4(wide, off + 96);
        const int4 pr = ldi4(wide, off + 112);
        __builtin_amdgcn_sched_barrier(0);
        float t[4];
        bool h[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            h[k] = slab_oct<OCT>(r, comp(lx, k), comp(hx, k), comp(ly, k), comp(hy, k), comp(lz, k), comp(hz, k), tcap,
                                 t[k]);
        if (STATS)
            st.box += (rf.x != kDone) + (rf.y != kDone) + (rf.z != kDone) + (rf.w != kDone);
        // per pair: its nearer hit slot and whether both are hit
        const bool a0 = h[0] && (!h[1] || t[0] <= t[1]);
        const int nA = a0 ? rf.x : rf.y, oA = a0 ? rf.y : rf.x;
        const float tA = h[0] || h[1] ? (a0 ? t[0] : t[1]) : INFINITY;
        const bool bothA = h[0] && h[1], anyA = h[0] || h[1];
        const bool b0 = h[2] && (!h[3] || t[2] <= t[3]);
        const int nB = b0 ? rf.z : rf.w, oB = b0 ? rf.w : rf.z;
        const float tB = h[2] || h[3] ? (b0 ? t[2] : t[3]) : INFINITY;
        const bool bothB = h[2] && h[3], anyB = h[2] || h[3];
        const bool firstA = anyA && (!anyB || tA <= tB);
        const bool anyN = firstA ? anyA : anyB, anyF = firstA ? anyB : anyA;
        const bool bothN = firstA ? bothA : bothB, bothF = firstA ? bothB : bothA;
        const int near = firstA ? nA : nB, nfar = firstA ? oA : oB;
        const int fent = bothF ? (firstA ? pr.y : pr.x) : (firstA ? nB : nA);
        // (the depth argument above keeps sp <= kStack; the guards only make
        // an overflow impossible by construction)
        if (anyF && sp < kStack) {
            stk[sp * kBlock] = fent;
            ++sp;
        }
        if (bothN && sp < kStack) {
            stk[sp * kBlock] = nfar;
            ++sp;
        }
        if (anyN)
            ref = near;
        else
            ref = sp > 0 ? stk[--sp * kBlock] : kDone;
        if (ref < 0 && ref != kDone && leaf == kDone) {
            leaf = ref;
            ref = sp > 0 ? stk[--sp * kBlock] : kDone;
        }
        if (__all(leaf != kDone))
            break;
    }
}

// nodes: the binary node array, or with WIDE the four-wide records.
// The ray is updated in place: knd is set before each leaf phase and the slab
// constants are computed again after it, from opaque copies of the direction
// and its inverse, so neither stays in registers through the other phase
// (that keeps the kernel within the 72 registers of seven waves per SIMD).
template <bool STATS, bool WIDE>
__device__ __forceinline__ void traverse(Ray &r, Rsrc nodes, Rsrc rv, const TriRec *__restrict__ recs, int root,
                                         int *stk, Best &b, Stats &st)
{
    const int oct = wave_octant(r);
    int sp = 0;
    int ref = root;   // next node to visit (internal >= 0, leaf < 0) or kDone
    int leaf = kDone; // postponed leaf
    if (root < 0) {   // the whole tree is one leaf
        leaf = root;
        ref = kDone;
    }
    while (true) {
        switch (oct) {
        case 0:
            if constexpr (WIDE)
                descend_wide<STATS, 0>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            else
                descend<STATS, 0>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            break;
        case 1:
            if constexpr (WIDE)
                descend_wide<STATS, 1>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            else
                descend<STATS, 1>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            break;
        case 2:
            if constexpr (WIDE)
                descend_wide<STATS, 2>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            else
                descend<STATS, 2>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            break;
        case 3:
            if constexpr (WIDE)
                descend_wide<STATS, 3>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            else
                descend<STATS, 3>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            break;
        case 4:
            if constexpr (WIDE)
                descend_wide<STATS, 4>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            else
                descend<STATS, 4>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            break;
        case 5:
            if constexpr (WIDE)
                descend_wide<STATS, 5>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            else
                descend<STATS, 5>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            break;
        case 6:
            if constexpr (WIDE)
                descend_wide<STATS, 6>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            else
                descend<STATS, 6>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            break;
        case 7:
            if constexpr (WIDE)
                descend_wide<STATS, 7>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            else
                descend<STATS, 7>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            break;
        default:
            if constexpr (WIDE)
                descend_wide<STATS, kMixed>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            else
                descend<STATS, kMixed>(r, nodes, stk, b.hi, sp, ref, leaf, st);
            break;
        }
        {
            float ax = r.dx, ay = r.dy, az = r.dz;
            asm volatile("" : "+v"(ax), "+v"(ay), "+v"(az));
            r.knd = kErr * fmaxf(fmaxf(fabsf(ax), fabsf(ay)), fabsf(az));
        }
        while (leaf != kDone) {
            const int code = ~leaf;
            const int first = code >> 3, cnt = (code & 7) + 1;
            for (int k = 0; k < cnt; ++k) {
                const uint32_t off = (uint32_t)(first + k) * (uint32_t)sizeof(TriRec);
                const float4 ta = ldf4(rv, off), tb = ldf4(rv, off + 16), tc = ldf4(rv, off + 32);
                if (STATS)
                    ++st.tri;
                offer<STATS>(r, recs, first + k, ta, tb, tc, b, st);
            }
            if (ref < 0 && ref != kDone) {
                leaf = ref;
                ref = sp > 0 ? stk[--sp * kBlock] : kDone;
            } else {
                leaf = kDone;
            }
        }
        if (ref == kDone)
            break;
        asm volatile("" : "+v"(r.ix), "+v"(r.iy), "+v"(r.iz));
        slab_consts(r);
    }
}

// ---------------------------------------------------------------------------
// Two-level scenes.  The world ray walks the environment's top level (instance
// boxes); at a top-level leaf it enters each instance's frame and walks the
// bottom level of that instance's mesh, with the same certified tests.
//
// The object-space ray is O = M (o - p), D = M d in FP64 (M the FP64 inverse
// of the pose's linear part), which is the exact ray in the mesh's frame up
// to FP64 rounding; the FP32 ray (o', d') the tests run on is O, D rounded, so
// each component is within u of it.  The tests stay conservative for the
// exact ray by widening: the bottom-level boxes by 2u (|o'_a| + far |d'_a|)
// per axis (a point of the exact ray at t <= far lies that close to the same
// point of the FP32 ray), and the triangle tests' error bounds by using
// max|T| + max|o'| for the norm of T = o' - v0 (the rounding of o' and d'
// adds at most 12u times the products the bounds already cover with
// kErr = 128u against the 48u of the FP32 evaluation).  Uncertain tests and
// the winner's t are evaluated in FP64 on O and D.  Results therefore equal
// the exact nearest hit on the moved meshes (each mesh under its pose, not
// rounded to FP32) up to FP64 rounding, with the lowest environment-local
// triangle id winning ties.
// ---------------------------------------------------------------------------
struct ObjRay {
    static constexpr bool kObject = true;
    float ox, oy, oz;
    float dx, dy, dz;
    float ix, iy, iz;
    float knd;  // kErr * max|d'_i|
    float no;   // max|o'_i|
    float tn, tf;
    float cnx, cny, cnz, cfx, cfy, cfz;  // widened plane constants (slab_obj)
};

// The 12 FP64 inverse-pose entries of instance inst (InstView::inv) through a
// range-checked view.
__device__ __forceinline__ void load_inv(Rsrc inv, int inst, double (&M)[12])
{
    const uint32_t off = (uint32_t)inst * 96u;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int4 v = ldi4(inv, off + 16u * k);
        M[2 * k] = __hiloint2double(v.y, v.x);
        M[2 * k + 1] = __hiloint2double(v.w, v.z);
    }
}

__device__ __forceinline__ void obj_ray(const Ray &r, const double (&M)[12], ObjRay &q)
{
    const double wx = (double)r.ox - M[3], wy = (double)r.oy - M[7], wz = (double)r.oz - M[11];
    const double dx = r.dx, dy = r.dy, dz = r.dz;
    q.ox = (float)(M[0] * wx + M[1] * wy + M[2] * wz);
    q.oy = (float)(M[4] * wx + M[5] * wy + M[6] * wz);
    q.oz = (float)(M[8] * wx + M[9] * wy + M[10] * wz);
    q.dx = (float)(M[0] * dx + M[1] * dy + M[2] * dz);
    q.dy = (float)(M[4] * dx + M[5] * dy + M[6] * dz);
    q.dz = (float)(M[8] * dx + M[9] * dy + M[10] * dz);
    q.ix = 1.0f / q.dx;
    q.iy = 1.0f / q.dy;
    q.iz = 1.0f / q.dz;
    q.knd = kErr * fmaxf(fmaxf(fabsf(q.dx), fabsf(q.dy)), fabsf(q.dz));
    q.no = fmaxf(fmaxf(fabsf(q.ox), fabsf(q.oy)), fabsf(q.oz));
    q.tn = r.tn;
    q.tf = r.tf;
    // plane parameter p_a = o'_a i_a: slab_consts' 3u |p_a| for the product's
    // and the constant's rounding, plus the widening 2u (|o'_a| + far |d'_a|)
    // |i_a| <= 2u (|p_a| + far) (1 + u)^2, each taken twice
    const float px = q.ox * q.ix, py = q.oy * q.iy, pz = q.oz * q.iz;
    const float ft = (4.0f * kU) * q.tf;
    const float sx = fmaf(8.0f * kU, fabsf(px), ft), sy = fmaf(8.0f * kU, fabsf(py), ft),
                sz = fmaf(8.0f * kU, fabsf(pz), ft);
    q.cnx = -px - sx;
    q.cny = -py - sy;
    q.cnz = -pz - sz;
    q.cfx = -px + sx;
    q.cfy = -py + sy;
    q.cfz = -pz + sz;
}

// Slab test of the object-space ray, the near plane of each axis chosen per
// lane by the sign of the inverse direction (slab_oct's test with the widened
// constants).
__device__ __forceinline__ bool slab_obj(const ObjRay &q, float lx, float hx, float ly, float hy, float lz, float hz,
                                         float tcap, float &tenter)
{
    const bool sx = signbit(q.ix), sy = signbit(q.iy), sz = signbit(q.iz);
    const float nx = sx ? hx : lx, fx = sx ? lx : hx;
    const float ny = sy ? hy : ly, fy = sy ? ly : hy;
    const float nz = sz ? hz : lz, fz = sz ? lz : hz;
    const float tmin = fmaxf(fmaxf(fmaf(nx, q.ix, q.cnx), fmaf(ny, q.iy, q.cny)), fmaxf(fmaf(nz, q.iz, q.cnz), q.tn));
    const float tmax = fminf(fminf(fmaf(fx, q.ix, q.cfx), fmaf(fy, q.iy, q.cfy)), fminf(fmaf(fz, q.iz, q.cfz), tcap));
    tenter = tmin;
    return tmin <= tmax * kBoxGrow;
}

// FP64 Moller-Trumbore of the exact object-space ray (O, D recomputed from
// the world ray and the instance's inverse) against one record; out of line
// like mt64v.
__device__ __noinline__ T64 mt64obj(float ox, float oy, float oz, float dxf, float dyf, float dzf, float tn, float tf,
                                    Rsrc inv, int inst, float4 A, float4 B, float4 C)
{
    T64 res{0.0, 0};
    double M[12];
    load_inv(inv, inst, M);
    const double wx = (double)ox - M[3], wy = (double)oy - M[7], wz = (double)oz - M[11];
    const double Ox = M[0] * wx + M[1] * wy + M[2] * wz;
    const double Oy = M[4] * wx + M[5] * wy + M[6] * wz;
    const double Oz = M[8] * wx + M[9] * wy + M[10] * wz;
    const double dx = M[0] * (double)dxf + M[1] * (double)dyf + M[2] * (double)dzf;
    const double dy = M[4] * (double)dxf + M[5] * (double)dyf + M[6] * (double)dzf;
    const double dz = M[8] * (double)dxf + M[9] * (double)dyf + M[10] * (double)dzf;
    const double ax = A.x, ay = A.y, az = A.z;
    const double e1x = (double)A.w - ax, e1y = (double)B.x - ay, e1z = (double)B.y - az;
    const double e2x = (double)B.z - ax, e2y = (double)B.w - ay, e2z = (double)C.x - az;
    const double px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
    double det = e1x * px + e1y * py + e1z * pz;
    if (det == 0.0 || !(det == det))
        return res;
    const double Tx = Ox - ax, Ty = Oy - ay, Tz = Oz - az;
    const double qx = Ty * e1z - Tz * e1y, qy = Tz * e1x - Tx * e1z, qz = Tx * e1y - Ty * e1x;
    double U = Tx * px + Ty * py + Tz * pz;
    double V = dx * qx + dy * qy + dz * qz;
    double W = e2x * qx + e2y * qy + e2z * qz;
    if (det < 0.0) {
        det = -det;
        U = -U;
        V = -V;
        W = -W;
    }
    if (U < 0.0 || V < 0.0 || U + V > det)
        return res;
    res.t = W / det;
    res.ok = res.t >= (double)tn && res.t <= (double)tf;
    return res;
}

// Range-checked views of a two-level scene's shared arrays (wave-uniform:
// one descriptor each, per-lane 32-bit offsets).
struct TwoViews {
    Rsrc bnodes, brecs, inv, info;
};

__device__ __forceinline__ TwoViews two_views(const InstView &iv)
{
    TwoViews v;
    v.bnodes = buffer_view(iv.bnodes, iv.bnode_count * (int64_t)sizeof(Node));
    v.brecs = buffer_view(iv.brecs, iv.brec_count * (int64_t)sizeof(TriRec));
    v.inv = buffer_view(iv.inv, iv.n_inst * 96);
    v.info = buffer_view(iv.inst_info, iv.n_inst * 16);
    return v;
}

__device__ __forceinline__ void ld_rec(Rsrc recs, int pos, float4 &a, float4 &b, float4 &c)
{
    const uint32_t off = (uint32_t)pos * (uint32_t)sizeof(TriRec);
    a = ldf4(recs, off);
    b = ldf4(recs, off + 16);
    c = ldf4(recs, off + 32);
}

// Offer record pos (mesh records) of instance inst, environment-local id
// idc, to the running winner.
template <bool STATS>
__device__ __forceinline__ void offer_obj(const Ray &r, const ObjRay &q, const TwoViews &tv, int inst, int pos,
                                         int idc, const float4 A, const float4 B, const float4 C, Best &b, Stats &st)
{
    float t, et;
    const int code = mt32(q, A, B, C, b.hi, t, et);
    if (code == kReject)
        return;
    if (code == kAccept && t + et < b.lo) {
        b.lo = t - et;
        b.hi = t + et;
        b.pos = pos;
        b.id = idc;
        b.inst = inst;
        b.have64 = false;
        return;
    }
    if (STATS)
        ++st.fp64;
    const T64 c = mt64obj(r.ox, r.oy, r.oz, r.dx, r.dy, r.dz, r.tn, r.tf, tv.inv, inst, A, B, C);
    if (!c.ok)
        return;
    if (b.pos >= 0 && !b.have64) {
        float4 wa, wb, wc;
        ld_rec(tv.brecs, b.pos, wa, wb, wc);
        const T64 cw = mt64obj(r.ox, r.oy, r.oz, r.dx, r.dy, r.dz, r.tn, r.tf, tv.inv, b.inst, wa, wb, wc);
        if (cw.ok) {
            b.t64 = cw.t;
            b.have64 = true;
        } else {
            b.pos = -1;  // cannot happen for a certain accept; drop it defensively
        }
    }
    if (b.pos < 0 || c.t < b.t64 || (c.t == b.t64 && idc < b.id)) {
        b.pos = pos;
        b.id = idc;
        b.inst = inst;
        b.t64 = c.t;
        b.have64 = true;
        const float tf = (float)c.t;
        b.lo = tf * (1.0f - 0x1p-23f);
        b.hi = tf * (1.0f + 0x1p-23f);
    }
}

// Bottom level of one instance; the stack entries above sp0 are this walk's.
template <bool STATS>
__device__ __forceinline__ void walk_instance(const Ray &r, const InstView &iv, const TwoViews &tv, int inst, int *stk,
                                              int sp0, Best &b, Stats &st)
{
    const int4 info = ldi4(tv.info, (uint32_t)inst * 16u);
    const int m = info.x;
    int ref = iv.broot[m];
    if (ref == kEmptyRoot)
        return;
    ObjRay q;
    {
        double M[12];
        load_inv(tv.inv, inst, M);
        obj_ray(r, M, q);
    }
    const int64_t rb = iv.mesh_tri_off[m];
    const uint32_t nbase = (uint32_t)node_base(rb, m) * (uint32_t)sizeof(Node);
    int sp = sp0;
    while (true) {
        if (ref >= 0) {
            const uint32_t off = nbase + (uint32_t)ref * (uint32_t)sizeof(Node);
            const float4 a = ldf4(tv.bnodes, off), c = ldf4(tv.bnodes, off + 16), z = ldf4(tv.bnodes, off + 32);
            const int4 ch = ldi4(tv.bnodes, off + 48);
            __builtin_amdgcn_sched_barrier(0);
            float t0, t1;
            const bool h0 = slab_obj(q, a.x, a.y, a.z, a.w, z.x, z.y, b.hi, t0);
            const bool h1 = slab_obj(q, c.x, c.y, c.z, c.w, z.z, z.w, b.hi, t1);
            if (STATS)
                st.box += 2;
            if (h0 && h1) {
                const bool first0 = t0 <= t1;
                stk[sp * kBlock] = first0 ? ch.y : ch.x;
                ++sp;
                ref = first0 ? ch.x : ch.y;
            } else if (h0 || h1) {
                ref = h0 ? ch.x : ch.y;
            } else {
                ref = sp > sp0 ? stk[--sp * kBlock] : kDone;
            }
        } else if (ref == kDone) {
            break;
        } else {
            const int code = ~ref;
            const int first = code >> 3, cnt = (code & 7) + 1;
            for (int k = 0; k < cnt; ++k) {
                const int pos = (int)rb + first + k;
                float4 ra, rbb, rc;
                ld_rec(tv.brecs, pos, ra, rbb, rc);
                if (STATS)
                    ++st.tri;
                offer_obj<STATS>(r, q, tv, inst, pos, info.y + __float_as_int(rc.y), ra, rbb, rc, b, st);
            }
            ref = sp > sp0 ? stk[--sp * kBlock] : kDone;
        }
    }
}

// Top level of environment env with the world ray.
template <bool STATS>
__device__ __forceinline__ void traverse_two(const Ray &r, const InstView &iv, int env, int *stk, Best &b, Stats &st)
{
    int ref = iv.troot[env];
    if (ref == kEmptyRoot)
        return;
    const int64_t ib = iv.inst_off[env];
    const int64_t n_inst = iv.inst_off[env + 1] - ib;
    const int64_t tb = node_base(ib, env);
    const Rsrc tnodes = buffer_view(iv.tnodes + tb, (node_base(ib + n_inst, env + 1) - tb) * (int64_t)sizeof(Node));
    const Rsrc trecs = buffer_view(iv.trecs + ib, n_inst * (int64_t)sizeof(TriRec));
    const TwoViews tv = two_views(iv);
    int sp = 0;
    while (true) {
        while (ref >= 0) {
            const uint32_t off = (uint32_t)ref * (uint32_t)sizeof(Node);
            const float4 a = ldf4(tnodes, off), c = ldf4(tnodes, off + 16), z = ldf4(tnodes, off + 32);
            const int4 ch = ldi4(tnodes, off + 48);
            __builtin_amdgcn_sched_barrier(0);
            float t0, t1;
            const bool h0 = slab(r, a.x, a.y, a.z, a.w, z.x, z.y, b.hi, t0);
            const bool h1 = slab(r, c.x, c.y, c.z, c.w, z.z, z.w, b.hi, t1);
            if (STATS)
                st.box += 2;
            if (h0 && h1) {
                const bool first0 = t0 <= t1;
                stk[sp * kBlock] = first0 ? ch.y : ch.x;
                ++sp;
                ref = first0 ? ch.x : ch.y;
            } else if (h0 || h1) {
                ref = h0 ? ch.x : ch.y;
            } else {
                ref = sp > 0 ? stk[--sp * kBlock] : kDone;
            }
        }
        if (ref == kDone)
            break;
        const int code = ~ref;
        const int first = code >> 3, cnt = (code & 7) + 1;
        ref = sp > 0 ? stk[--sp * kBlock] : kDone;
        for (int k = 0; k < cnt; ++k) {
            // the instance's own world box (the record's triangle (lo, hi, lo)):
            // the object-space setup and walk only for an instance the ray meets
            const uint32_t roff = (uint32_t)(first + k) * (uint32_t)sizeof(TriRec);
            const float4 ra = ldf4(trecs, roff), rb = ldf4(trecs, roff + 16), rc = ldf4(trecs, roff + 32);
            float te;
            if (STATS)
                ++st.box;
            if (slab(r, ra.x, ra.w, ra.y, rb.x, ra.z, rb.y, b.hi, te))
                walk_instance<STATS>(r, iv, tv, (int)ib + __float_as_int(rc.y), stk, sp, b, st);
        }
    }
}

// Final outputs of one ray from the winner (FP64 t, re-evaluated if the
// winner was accepted in FP32; hit = o + t d).
// Output pairing of the persistent form (kPairFlag).  A 16-column tile row
// covers half of a 128-byte line of depth (and of segmentation); its
// horizontal neighbour, the next tile of the same pop, covers the other half.
// The first tile of such a pair (kPairFirst) parks its depth and segmentation
// in the lane's LDS slot and the second (kPairSecond) stores both tiles'
// values together, so that each line is written whole instead of in two
// halves tens of microseconds apart (when L2 has often written the first
// half back already).
constexpr int kPairNone = 0, kPairFirst = 1, kPairSecond = 2;

// The first tile's parked values, stored one pair width to the left of the
// second tile's position idx (same rows, same sensor instance).  Ordinary
// stores: the two halves of each line now reach L2 together and leave it as
// one line (streaming stores of the two halves measured 45 % more bytes
// written than the outputs).
__device__ __forceinline__ void flush_pair(const OutView &o, int64_t idx, const int2 *slot)
{
    const int2 v = *slot;
    if (o.depth)
        o.depth[idx - kPairCols] = __int_as_float(v.x);
    if (o.seg)
        o.seg[idx - kPairCols] = v.y;
}

__device__ __forceinline__ void write_out(const OutView &o, const SceneView &sc, const SensorView &se, const Tile &tl,
                                          int row, int col, const Ray &r, const TriRec *__restrict__ recs, Best &b,
                                          int pair = kPairNone, int2 *slot = nullptr)
{
    const int env = tl.env;
    const int64_t r_local = (int64_t)row * tl.W + col;
    float depth = -1.0f, hx = __builtin_nanf(""), hy = hx, hz = hx;
    int seg = -1, tri = -1;
    double t = 0.0;
    if (b.pos >= 0) {
        t = b.t64;
        if (!b.have64) {
            t = 0.5 * ((double)b.lo + (double)b.hi);
            if (recs) {
                const TriRec w = recs[b.pos];
                double tw;
                if (mt64(r, w.a, w.b, w.c, tw))
                    t = tw;
            }
        }
        depth = (float)t;
        hx = (float)((double)r.ox + t * (double)r.dx);
        hy = (float)((double)r.oy + t * (double)r.dy);
        hz = (float)((double)r.oz + t * (double)r.dz);
        tri = b.id;
        // two-level scenes: the winner's instance (a global index) carries the label
        seg = sc.inst.tnodes ? sc.inst.inst_seg[b.inst] : sc.tri_seg[sc.env_tri_off[env] + b.id];
    }
    if (o.depth_tab) {  // per-request buffers (served batches)
        float *dp = o.depth_tab[tl.s];
        int32_t *sp = o.seg_tab[tl.s];
        int32_t *tp = o.tri_tab[tl.s];
        float *hp = o.hit_tab[tl.s];
        if (dp)
            __builtin_nontemporal_store(depth, dp + r_local);
        if (sp)
            __builtin_nontemporal_store(seg, sp + r_local);
        if (tp)
            __builtin_nontemporal_store(tri, tp + r_local);
        if (hp) {
            __builtin_nontemporal_store(hx, hp + 3 * r_local + 0);
            __builtin_nontemporal_store(hy, hp + 3 * r_local + 1);
            __builtin_nontemporal_store(hz, hp + 3 * r_local + 2);
        }
        return;
    }
    // the sensor instance's first ray, loaded here: kept from load_tile it
    // would occupy two vector registers across the traversal (spilled)
    int s2 = tl.s;
    asm volatile("" : "+s"(s2));
    const int64_t idx = se.ray_off[s2] + r_local;
    // Outside a pair, streaming stores (here and for served requests above):
    // a tile row fills only part of a 128-byte line, and the neighbouring tile
    // that completes the line is rendered tens of microseconds later, by when
    // L2 has often written the half-dirty line back; output lines are never
    // read here, so they bypass the cache.
    if (pair == kPairFirst) {
        *slot = make_int2(__float_as_int(depth), seg);
    } else if (pair == kPairSecond) {
        flush_pair(o, idx, slot);
        if (o.depth)
            o.depth[idx] = depth;
        if (o.seg)
            o.seg[idx] = seg;
    } else {
        if (o.depth)
            __builtin_nontemporal_store(depth, o.depth + idx);
        if (o.seg)
            __builtin_nontemporal_store(seg, o.seg + idx);
    }
    if (o.tri)
        __builtin_nontemporal_store(tri, o.tri + idx);
    if (o.hit) {
        __builtin_nontemporal_store(hx, o.hit + 3 * idx + 0);
        __builtin_nontemporal_store(hy, o.hit + 3 * idx + 1);
        __builtin_nontemporal_store(hz, o.hit + 3 * idx + 2);
    }
}

// One 64-ray tile per wavefront; pair: the tile's role in an output pair.
template <bool STATS, bool TWO, bool WIDE>
__device__ __forceinline__ void render_tile(const SceneView &sc, const SensorView &se, const OutView &o, int2 item,
                                            int *stk, Stats &st, int pair = kPairNone, int2 *slot = nullptr)
{
    const Tile t = load_tile(se, item);
    const int lane = threadIdx.x & 63;
    const int tile = item.y;
    const int ty = tile / t.tiles_x, tx = tile - ty * t.tiles_x;
    const int tw = 1 << t.tw_shift;
    const int row = ty * (64 >> t.tw_shift) + (lane >> t.tw_shift), col = tx * tw + (lane & (tw - 1));
    if (row >= t.H || col >= t.W) {
        // past the right edge, the first tile's lane may still hold a value
        if (pair == kPairSecond && row < t.H && col - kPairCols < t.W)
            flush_pair(o, se.ray_off[t.s] + (int64_t)row * t.W + col, slot);
        return;
    }
    Ray r;
    gen_ray(se, t, row, col, r);
    Best b{r.tf, r.tf, -1, -1, false, 0.0};
    const TriRec *recs = nullptr;
    if constexpr (TWO) {
        traverse_two<STATS>(r, sc.inst, t.env, stk, b, st);
        if (b.pos >= 0 && !b.have64) {  // the winner's t in FP64 on the exact object-space ray
            const TwoViews tv = two_views(sc.inst);
            float4 wa, wb, wc;
            ld_rec(tv.brecs, b.pos, wa, wb, wc);
            const T64 c = mt64obj(r.ox, r.oy, r.oz, r.dx, r.dy, r.dz, r.tn, r.tf, tv.inv, b.inst, wa, wb, wc);
            b.t64 = c.ok ? c.t : 0.5 * ((double)b.lo + (double)b.hi);
            b.have64 = true;
        }
    } else {
        const int64_t base = sc.env_tri_off[t.env], end = sc.env_tri_off[t.env + 1];
        const int64_t nb = node_base(base, t.env), nn = node_base(end, t.env + 1) - nb;
        const Rsrc nodes = WIDE ? buffer_view(sc.wide + nb, nn * (int64_t)sizeof(WideRec))
                                : buffer_view(sc.nodes + nb, nn * (int64_t)sizeof(Node));
        recs = sc.recs + base;
        const Rsrc rv = buffer_view(recs, (end - base) * (int64_t)sizeof(TriRec));
        const int root = sc.env_root[t.env];
        if (root != kEmptyRoot)
            traverse<STATS, WIDE>(r, nodes, rv, recs, root, stk, b, st);
    }
    // The output position is recomputed here from the lane: the empty asm
    // hides that it equals the one above, so the compiler does not keep
    // address arithmetic alive (spilled) across the traversal.
    int lane2 = lane;
    asm volatile("" : "+v"(lane2));
    const int row2 = ty * (64 >> t.tw_shift) + (lane2 >> t.tw_shift), col2 = tx * tw + (lane2 & (tw - 1));
    write_out(o, sc, se, t, row2, col2, r, recs, b, pair, slot);
}

// Blocks are dealt round-robin to the 8 XCDs; map them so that each XCD walks
// a contiguous range of work (neighbouring tiles share an environment's BVH
// in that XCD's L2).
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb)
{
    const int64_t q = nb >> 3, rem = nb & 7, x = b & 7;
    return x * q + (x < rem ? x : rem) + (b >> 3);
}

template <bool TWO, bool WIDE>
__global__ __launch_bounds__(kBlock) RC_WAVES_PER_EU_T void k_render_flat(SceneView sc, SensorView se, OutView o, int64_t item_begin,
                                                        int64_t n_items)
{
    __shared__ int s_stack[(TWO ? kStackTwo : kStack) * kBlock];
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t k = lb * (kBlock / 64) + uniform(threadIdx.x >> 6);
    if (k >= n_items)
        return;
    Stats st{0, 0, 0};
    render_tile<false, TWO, WIDE>(sc, se, o, se.items[item_begin + k], s_stack + threadIdx.x, st);
}

template <bool TWO, bool WIDE>
__global__ __launch_bounds__(kBlock) RC_WAVES_PER_EU_T void k_render_stats(SceneView sc, SensorView se, OutView o, int64_t n_items,
                                                         unsigned long long *counters)
{
    __shared__ int s_stack[(TWO ? kStackTwo : kStack) * kBlock];
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t k = lb * (kBlock / 64) + uniform(threadIdx.x >> 6);
    if (k >= n_items)
        return;
    Stats st{0, 0, 0};
    render_tile<true, TWO, WIDE>(sc, se, o, se.items[k], s_stack + threadIdx.x, st);
    unsigned box = st.box, tri = st.tri, f64 = st.fp64;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        box += __shfl_xor(box, off, 64);
        tri += __shfl_xor(tri, off, 64);
        f64 += __shfl_xor(f64, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&counters[0], (unsigned long long)box);
        atomicAdd(&counters[1], (unsigned long long)tri);
        atomicAdd(&counters[2], (unsigned long long)f64);
    }
}

// Persistent form: every wavefront pops `chunk` tiles at a time from its
// XCD's queue and, once that is empty, from the other queues in turn.
template <bool TWO, bool WIDE>
__global__ __launch_bounds__(kBlock) RC_WAVES_PER_EU_T void k_render_batched(SceneView sc, SensorView se, OutView o,
                                                                           QueueView q)
{
    __shared__ int s_stack[(TWO ? kStackTwo : kStack) * kBlock];
    __shared__ int2 s_pair[kBlock];
    const int lane = threadIdx.x & 63;
    int qi = blockIdx.x & (kQueues - 1);
    Stats st{0, 0, 0};
    const bool pairs = o.depth_tab == nullptr && (o.depth || o.seg);
    for (int exhausted = 0; exhausted < kQueues;) {
        unsigned int base = 0;
        if (lane == 0)
            base = atomicAdd(q.head + qi * kQueueStride, (unsigned int)q.chunk);
        base = (unsigned int)uniform((int)base);
        const int64_t b = q.off[qi] + (int64_t)base, e = q.off[qi + 1];
        if (b >= e) {
            qi = (qi + 1) & (kQueues - 1);
            ++exhausted;
            continue;
        }
        const int64_t stop = b + q.chunk < e ? b + q.chunk : e;
        int mode = kPairNone;
        for (int64_t k = b; k < stop; ++k) {
            int2 it = q.items[k];
            const bool first = (it.y & kPairFlag) != 0;
            it.y &= ~kPairFlag;
            mode = mode == kPairFirst ? kPairSecond : (pairs && first && k + 1 < stop ? kPairFirst : kPairNone);
            render_tile<false, TWO, WIDE>(sc, se, o, it, s_stack + threadIdx.x, st, mode, s_pair + threadIdx.x);
        }
    }
}

// Reference path: every triangle of the environment, original order.
__global__ __launch_bounds__(kBlock) void k_render_brute(SceneView sc, SensorView se, OutView o, int64_t n_items)
{
    const int64_t k = (int64_t)blockIdx.x * (kBlock / 64) + uniform(threadIdx.x >> 6);
    if (k >= n_items)
        return;
    const int2 item = se.items[k];
    const Tile t = load_tile(se, item);
    const int lane = threadIdx.x & 63;
    const int ty = item.y / t.tiles_x, tx = item.y - ty * t.tiles_x;
    const int tw = 1 << t.tw_shift;
    const int row = ty * (64 >> t.tw_shift) + (lane >> t.tw_shift), col = tx * tw + (lane & (tw - 1));
    if (row >= t.H || col >= t.W)
        return;
    Ray r;
    gen_ray(se, t, row, col, r);
    Best b{r.tf, r.tf, -1, -1, false, 0.0};
    Stats st{0, 0, 0};
    const int64_t base = sc.env_tri_off[t.env];
    const int n = (int)(sc.env_tri_off[t.env + 1] - base);
    // records in original order are built on the fly from the world array;
    // the winner is re-read through the same path, so pos indexes world tris
    const float *w = sc.world + 9 * base;
    for (int i = 0; i < n; ++i) {
        const float *q = w + 9 * i;
        const float4 A = make_float4(q[0], q[1], q[2], q[3]);
        const float4 B = make_float4(q[4], q[5], q[6], q[7]);
        const float4 C = make_float4(q[8], __int_as_float(i), 0.f, 0.f);
        float tt, et;
        const int code = mt32(r, A, B, C, b.hi, tt, et);
        if (code == kReject)
            continue;
        if (code == kAccept && tt + et < b.lo) {
            b.lo = tt - et;
            b.hi = tt + et;
            b.pos = i;
            b.id = i;
            b.have64 = false;
            continue;
        }
        double tc;
        if (!mt64(r, A, B, C, tc))
            continue;
        if (b.pos >= 0 && !b.have64) {
            const float *p = w + 9 * b.pos;
            double tw;
            if (mt64(r, make_float4(p[0], p[1], p[2], p[3]), make_float4(p[4], p[5], p[6], p[7]),
                     make_float4(p[8], 0.f, 0.f, 0.f), tw)) {
                b.t64 = tw;
                b.have64 = true;
            } else {
                b.pos = -1;
            }
        }
        if (b.pos < 0 || tc < b.t64 || (tc == b.t64 && i < b.id)) {
            b.pos = i;
            b.id = i;
            b.t64 = tc;
            b.have64 = true;
            const float tf = (float)tc;
            b.lo = tf * (1.0f - 0x1p-23f);
            b.hi = tf * (1.0f + 0x1p-23f);
        }
    }
    if (b.pos >= 0 && !b.have64) {
        const float *p = w + 9 * b.pos;
        double tw;
        if (mt64(r, make_float4(p[0], p[1], p[2], p[3]), make_float4(p[4], p[5], p[6], p[7]),
                 make_float4(p[8], 0.f, 0.f, 0.f), tw)) {
            b.t64 = tw;
            b.have64 = true;
        }
    }
    (void)st;
    write_out(o, sc, se, t, row, col, r, nullptr, b);
}

struct alignas(4) UV {
    float u, v;
};

// Further data types of the nearest hit: unit normal facing the sensor,
// barycentric (u, v), sensor-frame point t * local direction, global vertex
// ids.  One FP64 Moller-Trumbore solve on the winner's FP32 world vertices
// gives all of them: its t = W / det is the render's FP64 t bit for bit (the
// same expressions in the same order; negating both W and det, as the
// render's test does, leaves the quotient unchanged), u and v take one
// reciprocal of det, the normal one reciprocal of its length.  g: global
// original-order triangle index, -1 on a miss (NaN outputs, vertex ids -1).
// Each output is one vector store per ray, so a wavefront writes whole
// contiguous runs; the (u, v) pair goes out as UV, aligned to four bytes like
// the float buffer it lands in (HIP's float2 would assume eight).
__device__ __forceinline__ void write_extras(const OutView &o, const SceneView &sc, int64_t g, int64_t idx,
                                             const Ray &r, float lx, float ly, float lz)
{
    const float nan = __builtin_nanf("");
    float3 nrm = make_float3(nan, nan, nan), pt = nrm;
    UV uv{nan, nan};
    int3 vid = make_int3(-1, -1, -1);
    if (g >= 0) {
        const float *w = sc.world + 9 * g;
        const double ax = w[0], ay = w[1], az = w[2];
        const double e1x = (double)w[3] - ax, e1y = (double)w[4] - ay, e1z = (double)w[5] - az;
        const double e2x = (double)w[6] - ax, e2y = (double)w[7] - ay, e2z = (double)w[8] - az;
        const double dx = r.dx, dy = r.dy, dz = r.dz;
        const double px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
        const double det = e1x * px + e1y * py + e1z * pz;
        const double Tx = (double)r.ox - ax, Ty = (double)r.oy - ay, Tz = (double)r.oz - az;
        const double qx = Ty * e1z - Tz * e1y, qy = Tz * e1x - Tx * e1z, qz = Tx * e1y - Ty * e1x;
        const double U = Tx * px + Ty * py + Tz * pz;
        const double V = dx * qx + dy * qy + dz * qz;
        const double W = e2x * qx + e2y * qy + e2z * qz;
        const double t = W / det;
        const double rdet = 1.0 / det;
        uv = UV{(float)(U * rdet), (float)(V * rdet)};
        pt = make_float3((float)(t * (double)lx), (float)(t * (double)ly), (float)(t * (double)lz));
        double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
        double rl = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
        if (nx * dx + ny * dy + nz * dz > 0.0)
            rl = -rl;
        nrm = make_float3((float)(nx * rl), (float)(ny * rl), (float)(nz * rl));
        if (o.vert) {
            const int32_t *pv = sc.proto_tri + 3 * (int64_t)sc.tri_src[g].y;
            vid = make_int3(pv[0], pv[1], pv[2]);
        }
    }
    if (o.normal)
        *reinterpret_cast<float3 *>(o.normal + 3 * idx) = nrm;
    if (o.bary)
        *reinterpret_cast<UV *>(o.bary + 2 * idx) = uv;
    if (o.point)
        *reinterpret_cast<float3 *>(o.point + 3 * idx) = pt;
    if (o.vert)
        *reinterpret_cast<int3 *>(o.vert + 3 * idx) = vid;
}

// Second pass for the further data types: one wavefront per 64-ray tile
// reads the winner's id from the tri output and writes the requested
// buffers.  Kept apart from the traversal kernels so that they carry none of
// its registers.
__global__ __launch_bounds__(kBlock) void k_hit_extras(SceneView sc, SensorView se, OutView o, int64_t n_items)
{
    const int64_t k = xcd_remap(blockIdx.x, gridDim.x) * (kBlock / 64) + uniform(threadIdx.x >> 6);
    if (k >= n_items)
        return;
    const int2 item = se.items[k];
    const Tile t = load_tile(se, item);
    const int lane = threadIdx.x & 63;
    const int ty = item.y / t.tiles_x, tx = item.y - ty * t.tiles_x;
    const int tw = 1 << t.tw_shift;
    const int row = ty * (64 >> t.tw_shift) + (lane >> t.tw_shift), col = tx * tw + (lane & (tw - 1));
    if (row >= t.H || col >= t.W)
        return;
    const int64_t idx = t.ray_base + (int64_t)row * t.W + col;
    const int id = o.tri[idx];  // in flight while the ray is generated
    Ray r;
    gen_ray(se, t, row, col, r);
    float lx, ly, lz;
    local_dir(se, t, row, col, lx, ly, lz);
    write_extras(o, sc, id >= 0 ? sc.env_tri_off[t.env] + id : -1, idx, r, lx, ly, lz);
}


// ---------------------------------------------------------------------------
// Stereo shadows: the segment from each hit point back to the stereo pair's
// second camera.  Any-hit traversal (stops at the first triangle that meets
// the segment), with the same conservative boxes and certified FP32 decisions
// resolved in FP64 as the nearest-hit search, so the answer is the exact one
// up to FP64 rounding.
// ---------------------------------------------------------------------------
constexpr float kShadowS0 = 0x1p-13f;  // lower end of the segment parameter

// Any-hit traversal in the two phases of the nearest-hit search (internal
// nodes until every active lane holds a leaf, then the leaves), with the
// node loop specialised on the wavefront's direction octant; a lane that
// finds an occluder stops.  The answer does not depend on the order.
__device__ __forceinline__ bool any_hit(Ray &r, Rsrc nodes, Rsrc rv, int root, int *stk)
{
    const int oct = wave_octant(r);
    Stats st{0, 0, 0};
    int sp = 0;
    int ref = root;
    int leaf = kDone;
    if (root < 0) {
        leaf = root;
        ref = kDone;
    }
    bool hit = false;
    while (true) {
        switch (oct) {
        case 0: descend<false, 0>(r, nodes, stk, r.tf, sp, ref, leaf, st); break;
        case 1: descend<false, 1>(r, nodes, stk, r.tf, sp, ref, leaf, st); break;
        case 2: descend<false, 2>(r, nodes, stk, r.tf, sp, ref, leaf, st); break;
        case 3: descend<false, 3>(r, nodes, stk, r.tf, sp, ref, leaf, st); break;
        case 4: descend<false, 4>(r, nodes, stk, r.tf, sp, ref, leaf, st); break;
        case 5: descend<false, 5>(r, nodes, stk, r.tf, sp, ref, leaf, st); break;
        case 6: descend<false, 6>(r, nodes, stk, r.tf, sp, ref, leaf, st); break;
        case 7: descend<false, 7>(r, nodes, stk, r.tf, sp, ref, leaf, st); break;
        default: descend<false, kMixed>(r, nodes, stk, r.tf, sp, ref, leaf, st); break;
        }
        {  // as in traverse: knd for the leaf phase only
            float ax = r.dx, ay = r.dy, az = r.dz;
            asm volatile("" : "+v"(ax), "+v"(ay), "+v"(az));
            r.knd = kErr * fmaxf(fmaxf(fabsf(ax), fabsf(ay)), fabsf(az));
        }
        while (leaf != kDone) {
            const int code = ~leaf;
            const int first = code >> 3, cnt = (code & 7) + 1;
            for (int k = 0; k < cnt && !hit; ++k) {
                const uint32_t off = (uint32_t)(first + k) * (uint32_t)sizeof(TriRec);
                const float4 ta = ldf4(rv, off), tb = ldf4(rv, off + 16), tc = ldf4(rv, off + 32);
                float tt, et;
                const int d = mt32(r, ta, tb, tc, r.tf, tt, et);
                double t64;
                hit = d == kAccept || (d == kUnsure && mt64(r, ta, tb, tc, t64));
            }
            if (hit) {
                leaf = ref = kDone;
            } else if (ref < 0 && ref != kDone) {
                leaf = ref;
                ref = sp > 0 ? stk[--sp * kBlock] : kDone;
            } else {
                leaf = kDone;
            }
        }
        if (ref == kDone)
            break;
        asm volatile("" : "+v"(r.ix), "+v"(r.iy), "+v"(r.iz));  // slab constants for the next node phase
        slab_consts(r);
    }
    return hit;
}

// One wavefront per 64-ray tile: the hit point p = o + t d (FP64 t of the
// winner read from the tri output, rounded as the hit output is), the second
// centre c2 = pose applied to the baseline (FP32, the transform's fma order),
// the segment p + s (c2 - p), s in [kShadowS0, 1].
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_stereo_shadow(SceneView sc,
                                                                                                   SensorView se,
                                                                                                   OutView o,
                                                                                                   int64_t n_items)
{
    __shared__ int s_stack[kStack * kBlock];
    // each XCD walks a contiguous range of tiles (environments stay in one L2)
    const int64_t k = xcd_remap(blockIdx.x, gridDim.x) * (kBlock / 64) + uniform(threadIdx.x >> 6);
    if (k >= n_items)
        return;
    const int2 item = se.items[k];
    const Tile t = load_tile(se, item);
    const int lane = threadIdx.x & 63;
    const int ty = item.y / t.tiles_x, tx = item.y - ty * t.tiles_x;
    const int tw = 1 << t.tw_shift;
    const int row = ty * (64 >> t.tw_shift) + (lane >> t.tw_shift), col = tx * tw + (lane & (tw - 1));
    if (row >= t.H || col >= t.W)
        return;
    const int64_t idx = t.ray_base + (int64_t)row * t.W + col;
    const SensorModel &M = se.models[se.si_model[t.s]];
    const int id = o.tri[idx];
    uint8_t hidden = 0;
    const int root = sc.env_root[t.env];
    if (M.stereo && id >= 0 && root != kEmptyRoot) {
        Ray r;
        gen_ray(se, t, row, col, r);
        const int64_t base = sc.env_tri_off[t.env];
        const float *w = sc.world + 9 * (base + id);
        const float4 A = make_float4(w[0], w[1], w[2], w[3]), B = make_float4(w[4], w[5], w[6], w[7]),
                     C = make_float4(w[8], 0.f, 0.f, 0.f);
        double tt;
        if (!mt64(r, A, B, C, tt))
            tt = 0.5 * ((double)r.tn + (double)r.tf);  // unreachable for a certified winner
        const float px = (float)((double)r.ox + tt * (double)r.dx);
        const float py = (float)((double)r.oy + tt * (double)r.dy);
        const float pz = (float)((double)r.oz + tt * (double)r.dz);
        const float *P = se.pose + 12 * (int64_t)t.s;
        const float cx = fmaf(P[0], M.sb[0], fmaf(P[1], M.sb[1], fmaf(P[2], M.sb[2], P[3])));
        const float cy = fmaf(P[4], M.sb[0], fmaf(P[5], M.sb[1], fmaf(P[6], M.sb[2], P[7])));
        const float cz = fmaf(P[8], M.sb[0], fmaf(P[9], M.sb[1], fmaf(P[10], M.sb[2], P[11])));
        Ray s;
        s.ox = px;
        s.oy = py;
        s.oz = pz;
        s.dx = cx - px;
        s.dy = cy - py;
        s.dz = cz - pz;
        s.ix = 1.0f / s.dx;
        s.iy = 1.0f / s.dy;
        s.iz = 1.0f / s.dz;
        s.knd = kErr * fmaxf(fmaxf(fabsf(s.dx), fabsf(s.dy)), fabsf(s.dz));
        s.tn = kShadowS0;
        s.tf = 1.0f;
        slab_consts(s);
        const int64_t end = sc.env_tri_off[t.env + 1];
        const int64_t nb = node_base(base, t.env);
        const Rsrc nodes = buffer_view(sc.nodes + nb, (node_base(end, t.env + 1) - nb) * (int64_t)sizeof(Node));
        const Rsrc rv = buffer_view(sc.recs + base, (end - base) * (int64_t)sizeof(TriRec));
        hidden = any_hit(s, nodes, rv, root, s_stack + threadIdx.x) ? 1 : 0;
    }
    o.shadow[idx] = hidden;
}

__global__ __launch_bounds__(256) void k_debug_rays(SensorView se, int32_t s, int64_t n,
                                                    const int64_t *__restrict__ ray_idx, float *o, float *d)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const Tile t = load_tile(se, make_int2(s, 0));
    const int64_t ri = ray_idx[i];
    const int row = (int)(ri / t.W), col = (int)(ri % t.W);
    Ray r;
    gen_ray(se, t, row, col, r);
    o[3 * i] = r.ox;
    o[3 * i + 1] = r.oy;
    o[3 * i + 2] = r.oz;
    d[3 * i] = r.dx;
    d[3 * i + 1] = r.dy;
    d[3 * i + 2] = r.dz;
}

__global__ void k_fill_u32(unsigned int *p, int64_t n, unsigned int value)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = value;
}

inline unsigned blocks_for(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_render_flat(const SceneView &sc, const SensorView &se, const OutView &o, int64_t item_begin,
                              int64_t n_items, hipStream_t st)
{
    if (n_items == 0)
        return hipSuccess;
    const dim3 grid(blocks_for(n_items, kBlock / 64));
    if (sc.inst.tnodes)
        hipLaunchKernelGGL((k_render_flat<true, false>), grid, dim3(kBlock), 0, st, sc, se, o, item_begin, n_items);
    else if (sc.wide)
        hipLaunchKernelGGL((k_render_flat<false, true>), grid, dim3(kBlock), 0, st, sc, se, o, item_begin, n_items);
    else
        hipLaunchKernelGGL((k_render_flat<false, false>), grid, dim3(kBlock), 0, st, sc, se, o, item_begin, n_items);
    return hipGetLastError();
}

int batched_blocks_per_cu(bool two_level)
{
    int per_cu = 0;
    const hipError_t e =
        two_level ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_render_batched<true, false>, kBlock, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_render_batched<false, false>, kBlock, 0);
    if (e != hipSuccess || per_cu < 1)
        per_cu = 1;
    return per_cu;
}

hipError_t launch_render_batched(const SceneView &sc, const SensorView &se, const OutView &o, const QueueView &q,
                                 int grid, hipStream_t st)
{
    if (q.off[kQueues] == 0)
        return hipSuccess;
    if (q.chunk < 1)  // a pop must take at least one tile, or the queue never drains
        return hipErrorInvalidValue;
    hipError_t err = launch_fill_u32(q.head, kQueues * kQueueStride, 0u, st);
    if (err != hipSuccess)
        return err;
    if (sc.inst.tnodes)
        hipLaunchKernelGGL((k_render_batched<true, false>), dim3(grid), dim3(kBlock), 0, st, sc, se, o, q);
    else if (sc.wide)
        hipLaunchKernelGGL((k_render_batched<false, true>), dim3(grid), dim3(kBlock), 0, st, sc, se, o, q);
    else
        hipLaunchKernelGGL((k_render_batched<false, false>), dim3(grid), dim3(kBlock), 0, st, sc, se, o, q);
    return hipGetLastError();
}

hipError_t launch_hit_extras(const SceneView &sc, const SensorView &se, const OutView &o, int64_t n_items,
                             hipStream_t st)
{
    if (n_items == 0 || !(o.normal || o.bary || o.point || o.vert))
        return hipSuccess;
    hipLaunchKernelGGL(k_hit_extras, dim3((unsigned)((n_items + kBlock / 64 - 1) / (kBlock / 64))), dim3(kBlock), 0,
                       st, sc, se, o, n_items);
    return hipGetLastError();
}

hipError_t launch_stereo_shadow(const SceneView &sc, const SensorView &se, const OutView &o, int64_t n_items,
                                hipStream_t st)
{
    if (n_items == 0 || !o.shadow)
        return hipSuccess;
    hipLaunchKernelGGL(k_stereo_shadow, dim3((unsigned)((n_items + kBlock / 64 - 1) / (kBlock / 64))), dim3(kBlock),
                       0, st, sc, se, o, n_items);
    return hipGetLastError();
}

hipError_t launch_render_brute(const SceneView &sc, const SensorView &se, const OutView &o, int64_t n_items,
                               hipStream_t st)
{
    if (n_items == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_render_brute, dim3(blocks_for(n_items, kBlock / 64)), dim3(kBlock), 0, st, sc, se, o,
                       n_items);
    return hipGetLastError();
}

hipError_t launch_render_stats(const SceneView &sc, const SensorView &se, const OutView &o, int64_t n_items,
                               unsigned long long *counters, hipStream_t st)
{
    if (n_items == 0)
        return hipSuccess;
    const dim3 grid(blocks_for(n_items, kBlock / 64));
    if (sc.inst.tnodes)
        hipLaunchKernelGGL((k_render_stats<true, false>), grid, dim3(kBlock), 0, st, sc, se, o, n_items, counters);
    else if (sc.wide)
        hipLaunchKernelGGL((k_render_stats<false, true>), grid, dim3(kBlock), 0, st, sc, se, o, n_items, counters);
    else
        hipLaunchKernelGGL((k_render_stats<false, false>), grid, dim3(kBlock), 0, st, sc, se, o, n_items, counters);
    return hipGetLastError();
}

hipError_t launch_debug_rays(const SensorView &se, int32_t s, int64_t n, const int64_t *ray_idx, float *o, float *d,
                             hipStream_t st)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_debug_rays, dim3(blocks_for(n, 256)), dim3(256), 0, st, se, s, n, ray_idx, o, d);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned int *p, int64_t n, unsigned int value, hipStream_t st)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, value);
    return hipGetLastError();
}

}  // namespace rc
