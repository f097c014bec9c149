// rc_build.hip -- transform, BVH build and refit kernels (gfx950).
//
// Paper, Sec. III-D: every sub-mesh of environment i is moved by its own
// transform and a BVH is computed over the transformed mesh; the paper
// rebuilds it when static environments are randomised.  Here the build is a
// binned surface-area-heuristic builder with one wavefront per environment
// (all environments in one launch), plus a bottom-up refit on the fixed
// topology for moving instances.
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

__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

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

// K8: constant-velocity motion of dynamic instances.
__global__ __launch_bounds__(256) void k_move(int64_t n, const float *__restrict__ T0, const float *__restrict__ vel,
                                              const uint8_t *__restrict__ dyn, int32_t step, float dt,
                                              float *__restrict__ T)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float sdt = (float)step * dt;
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

// K2: per-triangle bounds and centroid (build scratch).
__global__ __launch_bounds__(256) void k_bounds(BuildView v)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= v.n_tris)
        return;
    const float *w = v.world + 9 * g;
    const float lx = fminf(fminf(w[0], w[3]), w[6]), hx = fmaxf(fmaxf(w[0], w[3]), w[6]);
    const float ly = fminf(fminf(w[1], w[4]), w[7]), hy = fmaxf(fmaxf(w[1], w[4]), w[7]);
    const float lz = fminf(fminf(w[2], w[5]), w[8]), hz = fmaxf(fmaxf(w[2], w[5]), w[8]);
    v.box_lo[g] = make_float4(lx, ly, lz, 0.f);
    v.box_hi[g] = make_float4(hx, hy, hz, 0.f);
    v.cen[g] = make_float4(0.5f * (lx + hx), 0.5f * (ly + hy), 0.5f * (lz + hz), 0.f);
}

// ---------------------------------------------------------------------------
// K5: binned SAH build, one wavefront (64 lanes) per environment.
// Tasks are processed depth first (left child next), node ids are assigned
// when a task is popped, so the left child of node i is node i+1.  Splits are
// stable partitions of the primitive list, so the build is deterministic.
// A node whose subtree could exceed kMaxNodeDepth is split at the index median
// (balanced), which bounds the traversal stack.
// ---------------------------------------------------------------------------
constexpr int kTaskCap = kMaxNodeDepth + 4;

struct WaveBox {
    float lx, ly, lz, hx, hy, hz;
};

__device__ __forceinline__ WaveBox reduce_boxes(const BuildView &v, const int32_t *prim, int64_t base, int b, int e,
                                                int lane)
{
    float lx = INFINITY, ly = INFINITY, lz = INFINITY, hx = -INFINITY, hy = -INFINITY, hz = -INFINITY;
    for (int i = b + lane; i < e; i += 64) {
        const int p = prim[i];
        const float4 lo = v.box_lo[base + p], hi = v.box_hi[base + p];
        lx = fminf(lx, lo.x);
        ly = fminf(ly, lo.y);
        lz = fminf(lz, lo.z);
        hx = fmaxf(hx, hi.x);
        hy = fmaxf(hy, hi.y);
        hz = fmaxf(hz, hi.z);
    }
    return WaveBox{wave_min(lx), wave_min(ly), wave_min(lz), wave_max(hx), wave_max(hy), wave_max(hz)};
}

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

__global__ __launch_bounds__(64) void k_build_sah(BuildView v)
{
    const int e = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t base = v.env_tri_off[e];
    const int n = (int)(v.env_tri_off[e + 1] - base);
    int32_t *prim = v.prim + base;
    int32_t *tmp = v.tmp + base;
    Node *nodes = v.nodes + base;

    __shared__ int s_cnt[3 * kBins];
    __shared__ int s_lo[3 * kBins * 3];
    __shared__ int s_hi[3 * kBins * 3];
    __shared__ int s_tp[kTaskCap], s_ts[kTaskCap], s_tb[kTaskCap], s_te[kTaskCap], s_td[kTaskCap];

    for (int i = lane; i < n; i += 64)
        prim[i] = i;
    int n_nodes = 0;
    if (n == 0) {
        if (lane == 0) {
            v.env_root[e] = kEmptyRoot;
            v.env_nodes[e] = 0;
        }
        return;
    }
    __syncthreads();
    if (n <= kLeafMax) {
        if (lane == 0)
            v.env_root[e] = leaf_ref(0, n);
    } else {
        int sp = 0;
        s_tp[0] = -1;
        s_ts[0] = 0;
        s_tb[0] = 0;
        s_te[0] = n;
        s_td[0] = 0;
        sp = 1;
        __syncthreads();
        while (sp > 0) {
            --sp;
            const int parent = s_tp[sp], side = s_ts[sp], b = s_tb[sp], en = s_te[sp], depth = s_td[sp];
            const int cnt = en - b;
            const int id = n_nodes++;
            if (lane == 0) {
                if (parent < 0)
                    v.env_root[e] = id;
                else if (side == 0)
                    nodes[parent].ch.x = id;
                else
                    nodes[parent].ch.y = id;
                nodes[id].ch.z = parent;
                nodes[id].ch.w = 0;
            }
            // centroid bounds
            float cl0 = INFINITY, cl1 = INFINITY, cl2 = INFINITY, ch0 = -INFINITY, ch1 = -INFINITY, ch2 = -INFINITY;
            for (int i = b + lane; i < en; i += 64) {
                const float4 c = v.cen[base + prim[i]];
                cl0 = fminf(cl0, c.x);
                cl1 = fminf(cl1, c.y);
                cl2 = fminf(cl2, c.z);
                ch0 = fmaxf(ch0, c.x);
                ch1 = fmaxf(ch1, c.y);
                ch2 = fmaxf(ch2, c.z);
            }
            const float cmin[3] = {wave_min(cl0), wave_min(cl1), wave_min(cl2)};
            const float cmax[3] = {wave_max(ch0), wave_max(ch1), wave_max(ch2)};
            float scale[3];
            bool usable = false;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float ext = cmax[a] - cmin[a];
                scale[a] = ext > 0.f ? (float)kBins / ext : 0.f;
                usable |= ext > 0.f;
            }
            const bool forced = depth + levels_needed(cnt) - 1 >= kMaxNodeDepth;

            int mid = -1, best_axis = -1, best_k = -1;
            WaveBox L{}, R{};
            if (usable && !forced) {
                for (int j = lane; j < 3 * kBins; j += 64) {
                    s_cnt[j] = 0;
                    s_lo[3 * j] = s_lo[3 * j + 1] = s_lo[3 * j + 2] = f2o(INFINITY);
                    s_hi[3 * j] = s_hi[3 * j + 1] = s_hi[3 * j + 2] = f2o(-INFINITY);
                }
                __syncthreads();
                for (int i = b + lane; i < en; i += 64) {
                    const int p = prim[i];
                    const float4 c = v.cen[base + p], lo = v.box_lo[base + p], hi = v.box_hi[base + p];
                    const float cc[3] = {c.x, c.y, c.z};
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        if (scale[a] == 0.f)
                            continue;
                        const int j = a * kBins + bin_of(cc[a], cmin[a], scale[a]);
                        atomicAdd(&s_cnt[j], 1);
                        atomicMin(&s_lo[3 * j + 0], f2o(lo.x));
                        atomicMin(&s_lo[3 * j + 1], f2o(lo.y));
                        atomicMin(&s_lo[3 * j + 2], f2o(lo.z));
                        atomicMax(&s_hi[3 * j + 0], f2o(hi.x));
                        atomicMax(&s_hi[3 * j + 1], f2o(hi.y));
                        atomicMax(&s_hi[3 * j + 2], f2o(hi.z));
                    }
                }
                __syncthreads();
                // evaluate 3 x (kBins-1) split planes, one per lane
                float cost = INFINITY;
                int nl = 0;
                WaveBox bl{INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
                WaveBox br = bl;
                if (lane < 3 * (kBins - 1)) {
                    const int a = lane / (kBins - 1), k = lane % (kBins - 1);
                    if (scale[a] != 0.f) {
                        int nr = 0;
                        for (int j = 0; j < kBins; ++j) {
                            const int q = a * kBins + j;
                            const int c = s_cnt[q];
                            if (c == 0)
                                continue;
                            WaveBox &B = j <= k ? bl : br;
                            B.lx = fminf(B.lx, o2f(s_lo[3 * q]));
                            B.ly = fminf(B.ly, o2f(s_lo[3 * q + 1]));
                            B.lz = fminf(B.lz, o2f(s_lo[3 * q + 2]));
                            B.hx = fmaxf(B.hx, o2f(s_hi[3 * q]));
                            B.hy = fmaxf(B.hy, o2f(s_hi[3 * q + 1]));
                            B.hz = fmaxf(B.hz, o2f(s_hi[3 * q + 2]));
                            if (j <= k)
                                nl += c;
                            else
                                nr += c;
                        }
                        if (nl > 0 && nr > 0)
                            cost = half_area(bl.lx, bl.ly, bl.lz, bl.hx, bl.hy, bl.hz) * (float)nl +
                                   half_area(br.lx, br.ly, br.lz, br.hx, br.hy, br.hz) * (float)nr;
                    }
                }
                // argmin over lanes, ties to the lower lane
                float bc = cost;
                int bw = lane;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    const float oc = __shfl_xor(bc, o, 64);
                    const int ow = __shfl_xor(bw, o, 64);
                    if (oc < bc || (oc == bc && ow < bw)) {
                        bc = oc;
                        bw = ow;
                    }
                }
                if (bc < INFINITY) {
                    best_axis = bw / (kBins - 1);
                    best_k = bw % (kBins - 1);
                    const int nL = __shfl(nl, bw, 64);
                    L = WaveBox{__shfl(bl.lx, bw, 64), __shfl(bl.ly, bw, 64), __shfl(bl.lz, bw, 64),
                                __shfl(bl.hx, bw, 64), __shfl(bl.hy, bw, 64), __shfl(bl.hz, bw, 64)};
                    R = WaveBox{__shfl(br.lx, bw, 64), __shfl(br.ly, bw, 64), __shfl(br.lz, bw, 64),
                                __shfl(br.hx, bw, 64), __shfl(br.hy, bw, 64), __shfl(br.hz, bw, 64)};
                    mid = b + nL;
                    // stable partition into tmp, then copy back
                    int lc = 0, rc = 0;
                    const float cm = cmin[best_axis], sc = scale[best_axis];
                    for (int c0 = b; c0 < en; c0 += 64) {
                        const int i = c0 + lane;
                        const bool valid = i < en;
                        const int p = valid ? prim[i] : 0;
                        float cc = 0.f;
                        if (valid) {
                            const float4 c = v.cen[base + p];
                            cc = best_axis == 0 ? c.x : (best_axis == 1 ? c.y : c.z);
                        }
                        const bool left = valid && bin_of(cc, cm, sc) <= best_k;
                        const uint64_t m = __ballot(left);
                        const uint64_t below = lane == 0 ? 0ull : (m & (~0ull >> (64 - lane)));
                        const int rank = __popcll(below);
                        const int nvalid = min(64, en - c0);
                        if (left)
                            tmp[b + lc + rank] = p;
                        else if (valid)
                            tmp[mid + rc + (lane - rank)] = p;
                        const int cl = __popcll(m);
                        lc += cl;
                        rc += nvalid - cl;
                    }
                    __syncthreads();
                    for (int i = b + lane; i < en; i += 64)
                        prim[i] = tmp[i];
                    __syncthreads();
                }
            }
            if (mid < 0) {  // index-median split (forced depth bound or no usable plane)
                mid = b + cnt / 2;
                L = reduce_boxes(v, prim, base, b, mid, lane);
                R = reduce_boxes(v, prim, base, mid, en, lane);
            }
            // write the node's child boxes (expanded outward by one step)
            if (lane == 0) {
                Node &nd = nodes[id];
                nd.xy0 = make_float4(expand_lo(L.lx), expand_hi(L.hx), expand_lo(L.ly), expand_hi(L.hy));
                nd.xy1 = make_float4(expand_lo(R.lx), expand_hi(R.hx), expand_lo(R.ly), expand_hi(R.hy));
                nd.z01 = make_float4(expand_lo(L.lz), expand_hi(L.hz), expand_lo(R.lz), expand_hi(R.hz));
                const int nl = mid - b, nr = en - mid;
                if (nl <= kLeafMax)
                    nd.ch.x = leaf_ref(b, nl);
                if (nr <= kLeafMax)
                    nd.ch.y = leaf_ref(mid, nr);
            }
            const int nl = mid - b, nr = en - mid;
            // push right then left so that the left child is popped next
            if (nr > kLeafMax) {
                s_tp[sp] = id;
                s_ts[sp] = 1;
                s_tb[sp] = mid;
                s_te[sp] = en;
                s_td[sp] = depth + 1;
                ++sp;
            }
            if (nl > kLeafMax) {
                s_tp[sp] = id;
                s_ts[sp] = 0;
                s_tb[sp] = b;
                s_te[sp] = mid;
                s_td[sp] = depth + 1;
                ++sp;
            }
            __syncthreads();
        }
    }
    if (lane == 0)
        v.env_nodes[e] = n_nodes;
    __syncthreads();
    // leaf-ordered records and the inverse permutation
    for (int i = lane; i < n; i += 64) {
        const int id = prim[i];
        const float *w = v.world + 9 * (base + id);
        TriRec rec;
        rec.a = make_float4(w[0], w[1], w[2], w[3]);
        rec.b = make_float4(w[4], w[5], w[6], w[7]);
        rec.c = make_float4(w[8], __int_as_float(id), 0.f, 0.f);
        v.recs[base + i] = rec;
        v.pos_of[base + id] = i;
    }
}

// ---------------------------------------------------------------------------
// K7: refit.  One thread per internal node: it writes the boxes of its leaf
// children, then arrives at its own counter; every completed node writes its
// box (union of its two child boxes) into its parent and arrives there.  The
// last arrival (internal children + the node's own thread) completes a node
// and carries on upward.  min/max are exact, so the result does not depend on
// the arrival order and equals the from-scratch bounds bit for bit.  Counters
// are returned to zero by the thread that completes the node.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float ld_f(const float *p)
{
    return __int_as_float(__hip_atomic_load((const int *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

__device__ __forceinline__ void leaf_box(const TriRec *recs, int ref, float b[6])
{
    const int code = ~ref;
    const int first = code >> 3, cnt = (code & 7) + 1;
    float lx = INFINITY, ly = INFINITY, lz = INFINITY, hx = -INFINITY, hy = -INFINITY, hz = -INFINITY;
    for (int k = 0; k < cnt; ++k) {
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

__device__ __forceinline__ void store_child_box(Node *nd, int side, const float b[6])
{
    float *xy = side == 0 ? &nd->xy0.x : &nd->xy1.x;
    xy[0] = b[0];
    xy[1] = b[1];
    xy[2] = b[2];
    xy[3] = b[3];
    float *z = &nd->z01.x + 2 * side;
    z[0] = b[4];
    z[1] = b[5];
}

__global__ __launch_bounds__(256) void k_refit(BuildView v)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= v.n_tris)
        return;
    const int e = v.tri_env[g];
    const int64_t base = v.env_tri_off[e];
    const int m = (int)(g - base);
    if (m >= v.env_nodes[e])
        return;
    Node *nodes = v.nodes + base;
    const TriRec *recs = v.recs + base;
    int32_t *cnt = v.refit_cnt + base;

    const int4 ch = nodes[m].ch;
    float b[6];
    if (ch.x < 0) {
        leaf_box(recs, ch.x, b);
        store_child_box(&nodes[m], 0, b);
    }
    if (ch.y < 0) {
        leaf_box(recs, ch.y, b);
        store_child_box(&nodes[m], 1, b);
    }
    __threadfence();
    int cur = m;
    int pending = (ch.x >= 0) + (ch.y >= 0);
    if (atomicAdd(&cnt[cur], 1) != pending)
        return;
    while (true) {
        __threadfence();
        cnt[cur] = 0;
        const int parent = nodes[cur].ch.z;
        if (parent < 0)
            break;
        const float *xy0 = &nodes[cur].xy0.x, *xy1 = &nodes[cur].xy1.x, *z01 = &nodes[cur].z01.x;
        float u[6];
        u[0] = fminf(ld_f(xy0 + 0), ld_f(xy1 + 0));
        u[1] = fmaxf(ld_f(xy0 + 1), ld_f(xy1 + 1));
        u[2] = fminf(ld_f(xy0 + 2), ld_f(xy1 + 2));
        u[3] = fmaxf(ld_f(xy0 + 3), ld_f(xy1 + 3));
        u[4] = fminf(ld_f(z01 + 0), ld_f(z01 + 2));
        u[5] = fmaxf(ld_f(z01 + 1), ld_f(z01 + 3));
        const int4 pch = nodes[parent].ch;
        store_child_box(&nodes[parent], pch.x == cur ? 0 : 1, u);
        __threadfence();
        pending = (pch.x >= 0) + (pch.y >= 0);
        if (atomicAdd(&cnt[parent], 1) != pending)
            break;
        cur = parent;
    }
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_transform(const BuildView &v, const int32_t *tri_list, int64_t n, bool to_recs, hipStream_t st)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_transform, dim3(blocks_for(n, 256)), dim3(256), 0, st, v, tri_list, n, (int)to_recs);
    return hipGetLastError();
}

hipError_t launch_move(int64_t n_inst, const float *T0, const float *vel, const uint8_t *dyn, int32_t step, float dt,
                       float *T, hipStream_t st)
{
    if (n_inst == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_move, dim3(blocks_for(n_inst, 256)), dim3(256), 0, st, n_inst, T0, vel, dyn, step, dt, T);
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
    return hipGetLastError();
}

hipError_t launch_refit(const BuildView &v, hipStream_t st)
{
    if (v.n_tris == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_refit, dim3(blocks_for(v.n_tris, 256)), dim3(256), 0, st, v);
    return hipGetLastError();
}

}  // namespace rc
