/*
 * rc_oracle.c -- brute-force CPU oracle for batched ray-cast rendering.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP renderer.
 *
 * What it computes (paper, Sec. III-D "Exteroceptive Sensors"):
 *   - each environment's mesh is the union of its sub-meshes, each moved by
 *     its own transform (world vertex = A[:, :3] v + A[:, 3]);
 *   - one ray is cast per pixel (pinhole camera) or per beam (LiDAR) from the
 *     sensor origin;
 *   - the reported value is the distance from the image plane for cameras
 *     (depth) and the sensor-to-hit distance for LiDARs (range).
 * The paper builds a BVH only to accelerate this query; the result is the
 * nearest intersection over *every* triangle of the environment, which is
 * what this file computes, triangle by triangle, with no acceleration
 * structure.
 *
 * Precision: the vertex transform and the ray directions are FP32 with a
 * fixed fused-multiply-add order (the renderer's input precision); the
 * intersection itself is evaluated in FP64 on those FP32 values.  A second
 * transform (orc_transform64) keeps the moved vertices in FP64, unrounded,
 * for renderers that intersect each sub-mesh in its own frame; orc_cast64
 * runs the same search on those.
 *
 * Readings where the paper is silent (numbered as in the design notes):
 *   near/far is an interval on the ray parameter t (closed); triangles are
 *   two-sided; no epsilon in the determinant test (reject det == 0 only);
 *   equal t is resolved by the lower environment-local triangle id; misses
 *   report t = -1, triangle -1.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#define ORC_API __attribute__((visibility("default")))

/* classification bits (per ray) */
#define ORC_HIT 1
#define ORC_B_BARY 2      /* winner's barycentric margin <= 1e-4 */
#define ORC_B_GAP 4       /* another candidate within 1e-4 relative depth */
#define ORC_B_RANGE 8     /* winner within 1e-4 relative of near or far */
#define ORC_B_GRAZE 16    /* |cos| between ray and winner normal < 1e-3 */
#define ORC_B_NEARMISS 32 /* miss ray with a near-miss candidate */

static const double MARGIN = 1e-4;
static const double GRAZE = 1e-3;

/* ---------------------------------------------------------------------- */
/* Sub-mesh transform: one world triangle per entry.                        */
/* corner_xyz: [n][9] prototype coordinates of the triangle's 3 corners      */
/* inst_T:     [n_inst][12] row-major 3x4 affine;  tri_inst: [n] instance    */
/* out:        [n][9] world coordinates                                      */
/* ---------------------------------------------------------------------- */
ORC_API void orc_transform(int64_t n, const float *corner_xyz, const int32_t *tri_inst,
                           const float *inst_T, float *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const float *A = inst_T + 12 * (int64_t)tri_inst[i];
        for (int c = 0; c < 3; ++c) {
            const float x = corner_xyz[9 * i + 3 * c + 0];
            const float y = corner_xyz[9 * i + 3 * c + 1];
            const float z = corner_xyz[9 * i + 3 * c + 2];
            for (int r = 0; r < 3; ++r) {
                const float *row = A + 4 * r;
                out[9 * i + 3 * c + r] = fmaf(row[0], x, fmaf(row[1], y, fmaf(row[2], z, row[3])));
            }
        }
    }
}

/* ---------------------------------------------------------------------- */
/* The same sub-mesh transform evaluated in FP64 and not rounded to FP32:   */
/* out = A[:, :3] v + A[:, 3] for the FP32 pose A and prototype vertex v,   */
/* as sums of FP64 products ((A_r0 x + A_r1 y) + A_r2 z) + A_r3.  This is   */
/* the moved mesh of Sec. III-D (each sub-mesh's base mesh composed with    */
/* its own transform) to FP64 accuracy, which is what a renderer that       */
/* moves rays into each sub-mesh's frame instead of moving the vertices     */
/* intersects.                                                              */
/* ---------------------------------------------------------------------- */
ORC_API void orc_transform64(int64_t n, const float *corner_xyz, const int32_t *tri_inst,
                             const float *inst_T, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const float *A = inst_T + 12 * (int64_t)tri_inst[i];
        for (int c = 0; c < 3; ++c) {
            const double x = corner_xyz[9 * i + 3 * c + 0];
            const double y = corner_xyz[9 * i + 3 * c + 1];
            const double z = corner_xyz[9 * i + 3 * c + 2];
            for (int r = 0; r < 3; ++r) {
                const float *row = A + 4 * r;
                out[9 * i + 3 * c + r] = (((double)row[0] * x + (double)row[1] * y) + (double)row[2] * z) +
                                         (double)row[3];
            }
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Constant-velocity instance motion: for every instance with dyn != 0 the   */
/* translation column becomes fma(v, float(step) * dt, c0) (FP32), where c0  */
/* is the translation at step 0; the linear part is unchanged.               */
/* ---------------------------------------------------------------------- */
ORC_API void orc_move(int64_t n_inst, const float *T0, const float *vel, const uint8_t *dyn,
                      int32_t step, float dt, float *T)
{
    const float sdt = (float)step * dt;
    for (int64_t i = 0; i < n_inst; ++i) {
        for (int k = 0; k < 12; ++k)
            T[12 * i + k] = T0[12 * i + k];
        if (dyn[i])
            for (int r = 0; r < 3; ++r)
                T[12 * i + 4 * r + 3] = fmaf(vel[3 * i + r], sdt, T0[12 * i + 4 * r + 3]);
    }
}

/* ---------------------------------------------------------------------- */
/* Ray generation.                                                          */
/* kind 0 pinhole: ray r = row*W + col; pixel centre (col+1/2, row+1/2),      */
/*   row 0 at the top; square pixels with focal length (W/2)/tan(hfov/2);    */
/*   local direction (1, -(col+1/2-W/2)*s, -(row+1/2-H/2)*s), s = 1/f, so    */
/*   the forward component is exactly 1 and t is depth.                      */
/* kind 1 LiDAR: ray r = ch*W + az with W azimuths and H channels;           */
/*   elevation vmax - ch*(vmax-vmin)/(H-1) (channel 0 on top), azimuth       */
/*   hmin + az*(hmax-hmin)/W counter-clockwise from +x; unit direction, so   */
/*   t is range.                                                             */
/* kind 2 table: local direction = table[r].                                 */
/* World ray: origin = pose column 3, dir_i = A_i0 dx + A_i1 dy + A_i2 dz.   */
/* ---------------------------------------------------------------------- */
ORC_API void orc_rays(int32_t kind, int32_t W, int32_t H, float hfov, float vmin, float vmax,
                      float hmin, float hmax, const float *table, const float *pose,
                      int64_t n, const int64_t *ray_idx, float *o, float *d, float *dl_out)
{
    const float s = (float)(tan((double)hfov * 0.5) / ((double)W * 0.5));
    for (int64_t i = 0; i < n; ++i) {
        const int64_t r = ray_idx[i];
        float dl[3];
        if (kind == 0) {
            const int64_t row = r / W, col = r % W;
            const float hw = (float)W * 0.5f, hh = (float)H * 0.5f;
            dl[0] = 1.0f;
            dl[1] = -((((float)col + 0.5f) - hw) * s);
            dl[2] = -((((float)row + 0.5f) - hh) * s);
        } else if (kind == 1) {
            const int64_t ch = r / W, az = r % W;
            const double el = H > 1 ? (double)vmax - (double)ch * ((double)vmax - (double)vmin) / (double)(H - 1)
                                    : (double)vmax;
            const double a = (double)hmin + (double)az * ((double)hmax - (double)hmin) / (double)W;
            dl[0] = (float)(cos(el) * cos(a));
            dl[1] = (float)(cos(el) * sin(a));
            dl[2] = (float)sin(el);
        } else {
            dl[0] = table[3 * r + 0];
            dl[1] = table[3 * r + 1];
            dl[2] = table[3 * r + 2];
        }
        for (int k = 0; k < 3; ++k) {
            const float *row = pose + 4 * k;
            o[3 * i + k] = row[3];
            d[3 * i + k] = fmaf(row[0], dl[0], fmaf(row[1], dl[1], row[2] * dl[2]));
            if (dl_out)
                dl_out[3 * i + k] = dl[k];
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Nearest hit by exhaustive search.                                        */
/* tris:     [N][9] world triangles (FP32; FP64 for orc_cast64),            */
/*           environment e owns the env-local                                */
/*           triangles tris[env_off[e] .. env_off[e+1])                      */
/* per ray:  env, origin o[3], direction d[3], near, far (FP32)              */
/* outputs (all [n_rays], hit as [n][3]): t (-1 on miss), tri (env-local,    */
/*   -1 on miss), u, v, hit point o + t d, bary margin, depth margin,        */
/*   grazing cosine, classification bits.                                    */
/* ---------------------------------------------------------------------- */
typedef struct {
    double t;
    int64_t id;
} orc_cand;

static int cand_less(double ta, int64_t ia, double tb, int64_t ib)
{
    return ta < tb || (ta == tb && ia < ib);
}

/* Corner coordinates of triangle k: from the FP32 array when it is given,  */
/* else from the FP64 one.                                                  */
static void tri_corners(const float *t32, const double *t64, int64_t k, double v[9])
{
    for (int j = 0; j < 9; ++j)
        v[j] = t32 ? (double)t32[9 * k + j] : t64[9 * k + j];
}

static void cast_rays(const float *tris32, const double *tris64, const int64_t *env_off, int64_t n_rays,
                      const int32_t *ray_env, const float *o, const float *d,
                      const float *nearv, const float *farv, int32_t nthreads,
                      double *t_out, int32_t *tri_out, double *u_out, double *v_out,
                      double *hit_out, double *mb_out, double *md_out, double *g_out,
                      int32_t *cls_out)
{
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t r = 0; r < n_rays; ++r) {
        const int32_t e = ray_env[r];
        const double ox = o[3 * r], oy = o[3 * r + 1], oz = o[3 * r + 2];
        const double dx = d[3 * r], dy = d[3 * r + 1], dz = d[3 * r + 2];
        const double tn = nearv[r], tf = farv[r];
        const double lo = tn * (1.0 - MARGIN), hi = tf * (1.0 + MARGIN);

        double bt = INFINITY, bu = 0, bv = 0;
        int64_t bid = -1;
        /* the two smallest (t, id) among loose candidates */
        orc_cand c1 = {INFINITY, -1}, c2 = {INFINITY, -1};

        const int64_t base = env_off[e], n = env_off[e + 1] - env_off[e];
        for (int64_t k = 0; k < n; ++k) {
            double T[9];
            tri_corners(tris32, tris64, base + k, T);
            const double ax = T[0], ay = T[1], az = T[2];
            const double e1x = T[3] - ax, e1y = T[4] - ay, e1z = T[5] - az;
            const double e2x = T[6] - ax, e2y = T[7] - ay, e2z = T[8] - az;
            /* p = d x e2, det = e1 . p */
            const double px = dy * e2z - dz * e2y;
            const double py = dz * e2x - dx * e2z;
            const double pz = dx * e2y - dy * e2x;
            const double det = e1x * px + e1y * py + e1z * pz;
            if (det == 0.0)
                continue;
            const double inv = 1.0 / det;
            const double sx = ox - ax, sy = oy - ay, sz = oz - az;
            const double u = (sx * px + sy * py + sz * pz) * inv;
            /* q = s x e1 */
            const double qx = sy * e1z - sz * e1y;
            const double qy = sz * e1x - sx * e1z;
            const double qz = sx * e1y - sy * e1x;
            const double v = (dx * qx + dy * qy + dz * qz) * inv;
            const double t = (e2x * qx + e2y * qy + e2z * qz) * inv;
            const double w = 1.0 - u - v;
            const double m = fmin(u, fmin(v, w));
            if (m >= -MARGIN && t >= lo && t <= hi) {
                if (cand_less(t, k, c1.t, c1.id)) {
                    c2 = c1;
                    c1.t = t;
                    c1.id = k;
                } else if (cand_less(t, k, c2.t, c2.id)) {
                    c2.t = t;
                    c2.id = k;
                }
            }
            if (u >= 0.0 && v >= 0.0 && u + v <= 1.0 && t >= tn && t <= tf) {
                if (cand_less(t, k, bt, bid)) {
                    bt = t;
                    bid = k;
                    bu = u;
                    bv = v;
                }
            }
        }

        int32_t cls = 0;
        if (bid >= 0) {
            cls |= ORC_HIT;
            t_out[r] = bt;
            tri_out[r] = (int32_t)bid;
            u_out[r] = bu;
            v_out[r] = bv;
            hit_out[3 * r + 0] = ox + bt * dx;
            hit_out[3 * r + 1] = oy + bt * dy;
            hit_out[3 * r + 2] = oz + bt * dz;
            const double mb = fmin(bu, fmin(bv, 1.0 - bu - bv));
            /* nearest other candidate: c1 unless c1 is the winner itself */
            const orc_cand other = (c1.id == bid) ? c2 : c1;
            double md = fmin((bt - tn) / bt, (tf - bt) / bt);
            if (other.id >= 0)
                md = fmin(md, (other.t - bt) / bt);
            /* grazing cosine |n.d| / (|n| |d|) */
            double T[9];
            tri_corners(tris32, tris64, base + bid, T);
            const double e1x = T[3] - T[0], e1y = T[4] - T[1], e1z = T[5] - T[2];
            const double e2x = T[6] - T[0], e2y = T[7] - T[1], e2z = T[8] - T[2];
            const double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
            const double g = fabs(nx * dx + ny * dy + nz * dz) /
                             (sqrt(nx * nx + ny * ny + nz * nz) * sqrt(dx * dx + dy * dy + dz * dz));
            mb_out[r] = mb;
            md_out[r] = md;
            g_out[r] = g;
            if (mb <= MARGIN)
                cls |= ORC_B_BARY;
            if (other.id >= 0 && (other.t - bt) / bt <= MARGIN)
                cls |= ORC_B_GAP;
            if ((bt - tn) / bt <= MARGIN || (tf - bt) / bt <= MARGIN)
                cls |= ORC_B_RANGE;
            if (g < GRAZE)
                cls |= ORC_B_GRAZE;
        } else {
            t_out[r] = -1.0;
            tri_out[r] = -1;
            u_out[r] = v_out[r] = 0.0;
            hit_out[3 * r + 0] = hit_out[3 * r + 1] = hit_out[3 * r + 2] = NAN;
            mb_out[r] = md_out[r] = g_out[r] = NAN;
            if (c1.id >= 0)
                cls |= ORC_B_NEARMISS;
        }
        cls_out[r] = cls;
    }
}

ORC_API void orc_cast(const float *tris, const int64_t *env_off, int64_t n_rays,
                      const int32_t *ray_env, const float *o, const float *d,
                      const float *nearv, const float *farv, int32_t nthreads,
                      double *t_out, int32_t *tri_out, double *u_out, double *v_out,
                      double *hit_out, double *mb_out, double *md_out, double *g_out,
                      int32_t *cls_out)
{
    cast_rays(tris, NULL, env_off, n_rays, ray_env, o, d, nearv, farv, nthreads, t_out, tri_out, u_out, v_out,
              hit_out, mb_out, md_out, g_out, cls_out);
}

/* The same search over FP64 world triangles (orc_transform64).             */
ORC_API void orc_cast64(const double *tris, const int64_t *env_off, int64_t n_rays,
                        const int32_t *ray_env, const float *o, const float *d,
                        const float *nearv, const float *farv, int32_t nthreads,
                        double *t_out, int32_t *tri_out, double *u_out, double *v_out,
                        double *hit_out, double *mb_out, double *md_out, double *g_out,
                        int32_t *cls_out)
{
    cast_rays(NULL, tris, env_off, n_rays, ray_env, o, d, nearv, farv, nthreads, t_out, tri_out, u_out, v_out,
              hit_out, mb_out, md_out, g_out, cls_out);
}

/* ---------------------------------------------------------------------- */
/* Further data types of a hit (Sec. III-D: surface normals and point       */
/* clouds come from the same intersection).  For ray r with winner tri[r]  */
/* (env-local, -1 on a miss) of environment ray_env[r]:                     */
/*   normal: the cross product (v1 - v0) x (v2 - v0) of the winner's world  */
/*           vertices in FP64, divided by its length and negated when it    */
/*           points along the ray (positive dot product with d), so that it */
/*           faces the sensor;                                              */
/*   point:  the hit in the sensor frame, t times the ray's local direction */
/*           (the sensor pose maps it to o + t d).                          */
/* Both rounded to FP32 once; NaN on a miss.                                */
/* ---------------------------------------------------------------------- */
ORC_API void orc_extras(const float *tris, const int64_t *env_off, int64_t n, const int32_t *ray_env,
                        const int32_t *tri, const float *d, const float *dl, const double *t,
                        float *normal, float *point)
{
    for (int64_t r = 0; r < n; ++r) {
        if (tri[r] < 0) {
            for (int k = 0; k < 3; ++k) {
                normal[3 * r + k] = NAN;
                point[3 * r + k] = NAN;
            }
            continue;
        }
        const float *v = tris + 9 * (env_off[ray_env[r]] + tri[r]);
        double e1[3], e2[3], nv[3];
        for (int k = 0; k < 3; ++k) {
            e1[k] = (double)v[3 + k] - (double)v[k];
            e2[k] = (double)v[6 + k] - (double)v[k];
        }
        nv[0] = e1[1] * e2[2] - e1[2] * e2[1];
        nv[1] = e1[2] * e2[0] - e1[0] * e2[2];
        nv[2] = e1[0] * e2[1] - e1[1] * e2[0];
        const double len = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
        const double along = nv[0] * (double)d[3 * r] + nv[1] * (double)d[3 * r + 1] + nv[2] * (double)d[3 * r + 2];
        const double sgn = along > 0.0 ? -1.0 : 1.0;
        for (int k = 0; k < 3; ++k) {
            normal[3 * r + k] = (float)(sgn * nv[k] / len);
            point[3 * r + k] = (float)(t[r] * (double)dl[3 * r + k]);
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Stereo shadows (Sec. III-D): a pixel seen by the rendered camera is      */
/* invalid when the second camera of the stereo pair cannot see the same    */
/* point, i.e. when the segment from the hit point back to the second       */
/* camera's centre meets the environment.  For ray r with winner win[r]     */
/* (env-local, -1 on a miss: not tested) and FP32 hit point p[r]:           */
/*   c2: the second centre, pose applied to the baseline b in the sensor    */
/*       frame, coordinate k = fma(P_k0, b0, fma(P_k1, b1, fma(P_k2, b2,    */
/*       P_k3))) in FP32 (the vertex transform's order);                    */
/*   D = c2 - p in FP32;                                                    */
/*   occluded iff a triangle of the environment meets p + s D at some s in  */
/*       [SHADOW_S0, 1] (FP64 Moller-Trumbore on the FP32 inputs, two-      */
/*       sided, only det == 0 rejects).  SHADOW_S0 keeps the surface around */
/*       p (the winner and its neighbours meet the segment at s ~ 0, within */
/*       the rounding of p) from shadowing itself.                          */
/* cls: bit 1 occluded; bit 2 borderline: neither a triangle that occludes  */
/* with margin (all barycentrics > MARGIN, s in [2 S0, 1 - MARGIN],         */
/* grazing cosine >= GRAZE) nor the absence of loose candidates             */
/* (barycentrics >= -MARGIN, s in [S0 / 2, 1 + MARGIN]).                    */
/* ---------------------------------------------------------------------- */
#define SHADOW_S0 0x1p-13 /* 1.22e-4, exact in FP32 and FP64 */

ORC_API void orc_shadow(const float *tris, const int64_t *env_off, int64_t n, const int32_t *ray_env,
                        const int32_t *win, const float *p, const float *pose, const float *b, int32_t nthreads,
                        uint8_t *occ_out, int32_t *cls_out)
{
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t r = 0; r < n; ++r) {
        occ_out[r] = 0;
        cls_out[r] = 0;
        if (win[r] < 0)
            continue;
        const float *P = pose + 12 * r;
        const float *B = b + 3 * r;
        float D32[3];
        for (int k = 0; k < 3; ++k) {
            const float c2 = fmaf(P[4 * k + 0], B[0], fmaf(P[4 * k + 1], B[1], fmaf(P[4 * k + 2], B[2], P[4 * k + 3])));
            D32[k] = c2 - p[3 * r + k];
        }
        const double ox = p[3 * r], oy = p[3 * r + 1], oz = p[3 * r + 2];
        const double dx = D32[0], dy = D32[1], dz = D32[2];
        const double dn = sqrt(dx * dx + dy * dy + dz * dz);
        int occluded = 0, robust_occ = 0, loose = 0;
        const int64_t base = env_off[ray_env[r]], cnt = env_off[ray_env[r] + 1] - base;
        for (int64_t k = 0; k < cnt; ++k) {
            const float *T = tris + 9 * (base + k);
            const double ax = T[0], ay = T[1], az = T[2];
            const double e1x = (double)T[3] - ax, e1y = (double)T[4] - ay, e1z = (double)T[5] - az;
            const double e2x = (double)T[6] - ax, e2y = (double)T[7] - ay, e2z = (double)T[8] - az;
            const double px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
            const double det = e1x * px + e1y * py + e1z * pz;
            if (det == 0.0)
                continue;
            const double inv = 1.0 / det;
            const double sx = ox - ax, sy = oy - ay, sz = oz - az;
            const double u = (sx * px + sy * py + sz * pz) * inv;
            const double qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
            const double v = (dx * qx + dy * qy + dz * qz) * inv;
            const double t = (e2x * qx + e2y * qy + e2z * qz) * inv;
            const double m = fmin(u, fmin(v, 1.0 - u - v));
            if (u >= 0.0 && v >= 0.0 && u + v <= 1.0 && t >= SHADOW_S0 && t <= 1.0)
                occluded = 1;
            if (m >= -MARGIN && t >= 0.5 * SHADOW_S0 && t <= 1.0 + MARGIN)
                loose = 1;
            if (m > MARGIN && t >= 2.0 * SHADOW_S0 && t <= 1.0 - MARGIN) {
                const double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
                const double g = fabs(nx * dx + ny * dy + nz * dz) / (sqrt(nx * nx + ny * ny + nz * nz) * dn);
                if (g >= GRAZE)
                    robust_occ = 1;
            }
        }
        occ_out[r] = (uint8_t)occluded;
        cls_out[r] = occluded | ((robust_occ || !loose) ? 0 : 2);
    }
}
