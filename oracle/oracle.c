/*
 * Oracle: plain, slow FP64 reference for the multi-camera depth path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the bench's CPU
 * baseline may load this library.  It shares no code with the GPU renderer.
 *
 * What it computes (paper Sec. 3.2.2 and Algorithm 1, "Multi-Depth Ray
 * Casting Kernel"): for every environment e, camera c and pixel (x, y), the
 * closest intersection of the camera ray with the union of the posed robot
 * link meshes and the shared static terrain, clipped by the far plane; plus
 * the sensor model the paper names (latency, noise, dropout: Sec. 1 and
 * Sec. 4.1; dropout and noise parameters in Table 6).
 *
 * Every ray is tested against every triangle (brute force) in FP64, with the
 * FP32 inputs promoted exactly.  The intersection formula is the classic
 * edge/cross-product form (Moller & Trumbore 1997), closed triangles, two
 * sided, accepted for ray parameter lambda > 0.
 *
 * Readings of the paper used here (it is silent on them):
 *  - ray: r = ((x + 0.5 - cx)/fx, (y + 0.5 - cy)/fy, 1) in the optical frame
 *    (x right, y down, z forward), D = R(q_c) r unnormalised, o = p_c, so the
 *    ray parameter lambda IS planar (optical-z) depth; range depth is
 *    lambda * |r| (Algorithm 1's scale m, made implicit).
 *  - quaternions are (x, y, z, w), normalised before use, rotate local->world.
 *  - bodies are queried in their local frames: o_b = R_b^T (o - t_b),
 *    d_b = R_b^T d (Sec. 3.2.2); the parameter lambda is frame independent.
 *  - result = lexicographic minimum of (lambda, inst, tri) over hits with
 *    depth <= far; links have inst = b in [0, B), the terrain inst = B.  This
 *    is Algorithm 1's query order (bodies first, then terrain) with a strict
 *    bound.  No hit: depth = far, inst = tri = -1.
 *  - flags (ambiguous within FP32 resolution, counted and checked weakly):
 *    EDGE  some candidate at lambda <= lambda* + 1e-4 m has min barycentric
 *          in [-1e-6, 1e-6];
 *    FAR   a hit with |depth* - far| <= 1e-5 m, or a miss that passes a
 *          surface in (far, far + 1e-5 m];
 *    TIE   another hit surface within 1e-5 m (depth) of the closest one.
 *  - candidates (what a weak check may accept for a flagged ray): every
 *    triangle with lambda > 0, lambda <= lambda* + 1e-4 m (lambda_far + 1e-4 m
 *    for a miss), depth <= far + 1e-5 m and min barycentric >= -1e-6, the K
 *    nearest in increasing depth (ties in input order: links, then terrain).
 *  - a triangle is closed: min barycentric >= -1e-12 counts as a hit (FP64
 *    rounding allowance; such rays are in the EDGE band anyway).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EDGE 1
#define ORC_FAR 2
#define ORC_TIE 4

#define EDGE_BARY 1e-6
#define EDGE_DEPTH 1e-4
#define FAR_BAND 1e-5
#define TIE_BAND 1e-5
/* A triangle is closed: it is hit when its min barycentric is >= -CLOSED_EPS.
 * The allowance covers FP64 rounding, so that a ray running exactly along a
 * shared edge cannot slip between the two triangles that share it. */
#define CLOSED_EPS 1e-12

typedef struct { double x, y, z; } v3;

static v3 v3f(const float* p) { v3 r = {p[0], p[1], p[2]}; return r; }
static v3 sub(v3 a, v3 b) { v3 r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 cross(v3 a, v3 b) {
    v3 r = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
    return r;
}

/* Rotation matrix (row major) of the normalised quaternion (x, y, z, w). */
static void quat_to_mat(const float* q4, double R[9]) {
    double x = q4[0], y = q4[1], z = q4[2], w = q4[3];
    double n = sqrt(x * x + y * y + z * z + w * w);
    x /= n; y /= n; z /= n; w /= n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - z * w);     R[2] = 2 * (x * z + y * w);
    R[3] = 2 * (x * y + z * w);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - x * w);
    R[6] = 2 * (x * z - y * w);     R[7] = 2 * (y * z + x * w);     R[8] = 1 - 2 * (x * x + y * y);
}

static v3 mat_mul(const double R[9], v3 v) {
    v3 r = {R[0] * v.x + R[1] * v.y + R[2] * v.z,
            R[3] * v.x + R[4] * v.y + R[5] * v.z,
            R[6] * v.x + R[7] * v.y + R[8] * v.z};
    return r;
}

static v3 mat_tmul(const double R[9], v3 v) {
    v3 r = {R[0] * v.x + R[3] * v.y + R[6] * v.z,
            R[1] * v.x + R[4] * v.y + R[7] * v.z,
            R[2] * v.x + R[5] * v.y + R[8] * v.z};
    return r;
}

/* Ray/plane of one triangle: returns 0 when the ray is parallel to its plane,
 * or when the triangle has zero area (its edges are parallel: no interior, so
 * no ray meets it; tested on the cross product of the edges, which is exact
 * for single-precision vertices).
 * *lam = ray parameter of the plane crossing, *mb = min barycentric there. */
static int tri_plane(v3 o, v3 d, const float* t9, double* lam, double* mb) {
    v3 p0 = v3f(t9), p1 = v3f(t9 + 3), p2 = v3f(t9 + 6);
    v3 e1 = sub(p1, p0), e2 = sub(p2, p0);
    v3 n = cross(e1, e2);
    if (n.x == 0.0 && n.y == 0.0 && n.z == 0.0) return 0;
    v3 P = cross(d, e2);
    double det = dot(e1, P);
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    v3 T = sub(o, p0);
    double u = dot(T, P) * inv;
    v3 Q = cross(T, e1);
    double v = dot(d, Q) * inv;
    double w = 1.0 - u - v;
    *lam = dot(e2, Q) * inv;
    double m = u < v ? u : v;
    *mb = m < w ? m : w;
    return 1;
}

typedef struct {
    const float* terrain; int64_t n_terrain;
    const float* link_tri; const int64_t* link_off; int n_links;
    const float* link_pos; const float* link_quat;  /* [E][B][3], [E][B][4] */
    const float* cam_pos; const float* cam_quat; const float* intr; /* [E][C][*] */
    const double* cam64;  /* optional [E][C][16]: R row-major [9], p [3], fx, fy, cx, cy */
    int E, C, W, H;
    double far; int depth_mode; /* 0 planar, 1 range */
} scene_t;

/* Camera ray of pixel index p in [E][C][H][W]; returns the depth scale. */
static double make_ray(const scene_t* s, int64_t p, v3* o, v3* d, int* env) {
    int64_t x = p % s->W, y = (p / s->W) % s->H;
    int64_t ec = p / ((int64_t)s->W * s->H);
    double R[9], fx, fy, cx, cy;
    if (s->cam64) {  /* a camera given in FP64 (e.g. after randomisation) */
        const double* c = s->cam64 + 16 * ec;
        for (int k = 0; k < 9; ++k) R[k] = c[k];
        fx = c[12]; fy = c[13]; cx = c[14]; cy = c[15];
    } else {
        const float* K = s->intr + 4 * ec;
        fx = K[0]; fy = K[1]; cx = K[2]; cy = K[3];
        quat_to_mat(s->cam_quat + 4 * ec, R);
    }
    v3 r = {((double)x + 0.5 - cx) / fx, ((double)y + 0.5 - cy) / fy, 1.0};
    *d = mat_mul(R, r);
    if (s->cam64) {
        const double* c = s->cam64 + 16 * ec;
        v3 po = {c[9], c[10], c[11]};
        *o = po;
    } else {
        *o = v3f(s->cam_pos + 3 * ec);
    }
    *env = (int)(ec / s->C);
    return s->depth_mode == 1 ? sqrt(dot(r, r)) : 1.0;
}

typedef struct { double lam; int inst; int tri; } hit_t;

static int lex_less(double lam, int inst, int tri, const hit_t* h) {
    if (lam != h->lam) return lam < h->lam;
    if (inst != h->inst) return inst < h->inst;
    return tri < h->tri;
}

/* A link pose that places the mesh nowhere: a non-finite position or
 * quaternion component, or a zero quaternion.  Algorithm 1 assumes valid
 * poses; the reading here is that such a link is absent from its environment
 * (no triangle of it is ever hit), while the other links and the terrain are
 * unaffected. */
static int pose_ok(const float* t3, const float* q4) {
    for (int i = 0; i < 3; ++i)
        if (!isfinite(t3[i])) return 0;
    double n2 = 0.0;
    for (int i = 0; i < 4; ++i) {
        if (!isfinite(q4[i])) return 0;
        n2 += (double)q4[i] * q4[i];
    }
    return n2 > 0.0;
}

/* Body k of a ray: link k (k < B) in its local frame, or the terrain (k == B)
 * in the world frame.  Gives the ray in that frame and the triangle list. */
static void body_ray(const scene_t* s, int env, int k, v3 o, v3 d, v3* ro, v3* rd,
                     const float** tris, int64_t* ntri) {
    if (k < s->n_links) {
        double Rb[9];
        int64_t eb = (int64_t)env * s->n_links + k;
        if (!pose_ok(s->link_pos + 3 * eb, s->link_quat + 4 * eb)) {
            *ro = o;
            *rd = d;
            *tris = s->link_tri;
            *ntri = 0;
            return;
        }
        quat_to_mat(s->link_quat + 4 * eb, Rb);
        v3 tb = v3f(s->link_pos + 3 * eb);
        *ro = mat_tmul(Rb, sub(o, tb));
        *rd = mat_tmul(Rb, d);
        *tris = s->link_tri + 9 * s->link_off[k];
        *ntri = s->link_off[k + 1] - s->link_off[k];
    } else {
        *ro = o;
        *rd = d;
        *tris = s->terrain;
        *ntri = s->n_terrain;
    }
}

static void render_ray(const scene_t* s, int64_t p, double* depth, int32_t* inst_o,
                       int32_t* tri_o, int32_t* flags, int32_t* cand, double* cand_d, int K) {
    v3 o, d; int env;
    double m = make_ray(s, p, &o, &d, &env);
    double lam_far = s->far / m;
    hit_t best = {INFINITY, -1, -1};
    /* pass 1: the closest hit */
    for (int k = 0; k <= s->n_links; ++k) {
        v3 ro, rd; const float* tris; int64_t nt;
        body_ray(s, env, k, o, d, &ro, &rd, &tris, &nt);
        for (int64_t t = 0; t < nt; ++t) {
            double lam, mb;
            if (tri_plane(ro, rd, tris + 9 * t, &lam, &mb) && mb >= -CLOSED_EPS && lam > 0.0 &&
                lam <= lam_far && lex_less(lam, k, (int)t, &best)) {
                best.lam = lam; best.inst = k; best.tri = (int)t;
            }
        }
    }
    double dstar = best.inst >= 0 ? best.lam * m : s->far;
    *depth = dstar;
    *inst_o = best.inst;
    *tri_o = best.tri;
    /* pass 2: ambiguity flags and the candidates a weak check may accept */
    int f = 0, nc = 0;
    double lam_lim = (best.inst >= 0 ? best.lam : lam_far) + EDGE_DEPTH / m;
    for (int q = 0; q < K; ++q) { cand[2 * q] = -1; cand[2 * q + 1] = -1; cand_d[q] = NAN; }
    /* the far band: the closest hit lies within FAR_BAND of the far plane, or a
     * miss passes a surface just beyond it (hit or miss then hinges on FP32
     * rounding); a miss with no surface near the far plane is not flagged */
    if (best.inst >= 0 && fabs(dstar - s->far) <= FAR_BAND) f |= ORC_FAR;
    for (int k = 0; k <= s->n_links; ++k) {
        v3 ro, rd; const float* tris; int64_t nt;
        body_ray(s, env, k, o, d, &ro, &rd, &tris, &nt);
        for (int64_t t = 0; t < nt; ++t) {
            double lam, mb;
            if (!tri_plane(ro, rd, tris + 9 * t, &lam, &mb) || !(lam > 0.0) || lam > lam_lim ||
                lam * m > s->far + FAR_BAND || mb < -EDGE_BARY)
                continue;
            int is_best = (k == best.inst && (int)t == best.tri);
            if (best.inst < 0 && lam * m > s->far) f |= ORC_FAR;
            if (mb <= EDGE_BARY) f |= ORC_EDGE;
            if (!is_best && mb >= -CLOSED_EPS && best.inst >= 0 && fabs(lam - best.lam) * m <= TIE_BAND)
                f |= ORC_TIE;
            /* keep the K nearest candidates, sorted by depth */
            double dd = lam * m;
            int pos = nc < K ? nc : K;
            while (pos > 0 && cand_d[pos - 1] > dd) {
                if (pos < K) {
                    cand_d[pos] = cand_d[pos - 1];
                    cand[2 * pos] = cand[2 * pos - 2];
                    cand[2 * pos + 1] = cand[2 * pos - 1];
                }
                --pos;
            }
            if (pos < K) { cand_d[pos] = dd; cand[2 * pos] = k; cand[2 * pos + 1] = (int)t; }
            if (nc < K) ++nc;
        }
    }
    *flags = f;
}

/*
 * oracle_render: depth, inst, tri and flags for the listed pixels.
 * rays: linear indices into [E][C][H][W] (n of them), or NULL for all pixels.
 * cand [n][K][2] / cand_depth [n][K]: nearest candidates (any ray), -1/NaN pad.
 * cam64: NULL, or FP64 cameras [E][C][16] (R row-major, p, fx, fy, cx, cy)
 * that replace cam_pos / cam_quat / intr.
 * Returns 0, or -1 on bad arguments.
 */
/* Host threads of the parallel loops (timing of the oracle only). */
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int oracle_get_threads(void) { return omp_get_max_threads(); }

int oracle_render(const float* terrain, int64_t n_terrain,
                  const float* link_tri, const int64_t* link_off, int n_links,
                  const float* link_pos, const float* link_quat,
                  const float* cam_pos, const float* cam_quat, const float* intr,
                  int E, int C, int W, int H, double far, int depth_mode,
                  const int64_t* rays, int64_t n,
                  double* depth, int32_t* inst, int32_t* tri, int32_t* flags,
                  int32_t* cand, double* cand_depth, int K, const double* cam64) {
    if (E < 0 || C < 0 || W < 0 || H < 0 || n_links < 0 || n_terrain < 0 || K < 1) return -1;
    scene_t s = {terrain, n_terrain, link_tri, link_off, n_links, link_pos, link_quat,
                 cam_pos, cam_quat, intr, cam64, E, C, W, H, far, depth_mode};
    int64_t total = (int64_t)E * C * H * W;
    if (rays == NULL) n = total;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        int64_t p = rays ? rays[i] : i;
        if (p < 0 || p >= total) { depth[i] = NAN; inst[i] = tri[i] = -2; flags[i] = 0; continue; }
        render_ray(&s, p, depth + i, inst + i, tri + i, flags + i, cand + 2 * K * i,
                   cand_depth + K * i, K);
    }
    return 0;
}

/*
 * oracle_heightmap: the privileged height map of the paper's terrain experts
 * (Sec. 3.1: a local grid of 1.6 m x 1.0 m at 0.1 m around the robot).  For
 * env e and grid point (i, j), i < nx along the heading, j < ny to the left:
 * local (gx, gy) = ((i - (nx - 1) / 2) dx, (j - (ny - 1) / 2) dy), world
 * (x, y) = base_xy + Rz(yaw) (gx, gy); a vertical ray from z = base_z + top
 * down to depth; the closest terrain hit (closed triangles) gives
 * heights[e][j][i] = (base_z + top - t) - base_z; no hit gives `miss`.  FP64.
 */
void oracle_heightmap(const float* terrain, int64_t n_terrain, const float* base_pos,
                      const float* base_yaw, int E, int nx, int ny, double dx, double dy,
                      double top, double depth, double miss, double* heights) {
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < (int64_t)E * nx * ny; ++q) {
        int e = (int)(q / ((int64_t)nx * ny));
        int j = (int)((q / nx) % ny), i = (int)(q % nx);
        double gx = (i - 0.5 * (nx - 1)) * dx, gy = (j - 0.5 * (ny - 1)) * dy;
        double c = cos((double)base_yaw[e]), sn = sin((double)base_yaw[e]);
        v3 o = {base_pos[3 * e] + c * gx - sn * gy, base_pos[3 * e + 1] + sn * gx + c * gy,
                base_pos[3 * e + 2] + top};
        v3 d = {0.0, 0.0, -1.0};
        double best = INFINITY;
        for (int64_t t = 0; t < n_terrain; ++t) {
            double lam, mb;
            if (tri_plane(o, d, terrain + 9 * t, &lam, &mb) && mb >= -CLOSED_EPS && lam > 0.0 &&
                lam <= depth && lam < best)
                best = lam;
        }
        heights[q] = best < INFINITY ? top - best : miss;
    }
}

/* ------------------------------------------------------------------------
 * Counter-based generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
 * Multipliers 0xD2511F53 and 0xCD9E8D57, key increments 0x9E3779B9 and
 * 0xBB67AE85 (golden ratio and sqrt(3)-1 in 0.32 fixed point).
 * ---------------------------------------------------------------------- */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------
 * Sensor model (latency, noise, dropout; Sec. 1, Sec. 4.1, Table 6).
 *
 * Readings: a capture at step s of pixel p of camera uid u draws
 *   w = Philox(ctr = (p, u, s_lo32, (s_hi16 << 16) | 0), key = seed);
 * drop <=> w0 < floor(p_drop * 2^32); Gaussian g by Box-Muller from
 * u1 = ((w1 >> 8) + 1) 2^-24 in (0, 1] and u2 = (w2 >> 8) 2^-24;
 * z' = hit ? z + (sigma_abs + sigma_rel z) g : far; z'' = clamp(z', near, far);
 * capture = drop ? fill : z''.  The latency of camera u at output step s is
 *   k = lat_min + ((w0 * (lat_max - lat_min + 1)) >> 32) with
 *   w = Philox(ctr = (0xFFFFFFFF, u, s_lo32, (s_hi16 << 16) | 1));
 * the output at step s is the capture of step max(s - k, s0), where s0 is the
 * first step of the sequence.  Noise and dropout belong to the capture, so a
 * frame shown late keeps the noise it was captured with.
 * ---------------------------------------------------------------------- */
#define POST_NOISE 1u
#define POST_DROPOUT 2u
#define POST_LATENCY 4u

typedef struct {
    uint64_t seed;
    float sigma_abs, sigma_rel, p_drop, near_, far_, fill;
    int32_t lat_min, lat_max;
    uint32_t flags;
} post_params_t;

static uint64_t drop_threshold(float p) {
    double t = floor((double)p * 4294967296.0);
    if (!(t > 0.0)) return 0;
    if (t > 4294967296.0) return 4294967296ull;
    return (uint64_t)t;
}

int oracle_latency(const post_params_t* pp, uint32_t cam_uid, uint64_t step) {
    if (!(pp->flags & POST_LATENCY)) return 0;
    uint32_t key[2] = {(uint32_t)pp->seed, (uint32_t)(pp->seed >> 32)};
    uint32_t ctr[4] = {0xFFFFFFFFu, cam_uid, (uint32_t)step,
                       (uint32_t)(((step >> 32) & 0xFFFFu) << 16) | 1u};
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    uint64_t span = (uint64_t)(pp->lat_max - pp->lat_min + 1);
    return pp->lat_min + (int)(((uint64_t)w[0] * span) >> 32);
}

static double capture(const post_params_t* pp, float z, int32_t inst, uint32_t pix,
                      uint32_t cam_uid, uint64_t step, uint8_t* dropped) {
    uint32_t key[2] = {(uint32_t)pp->seed, (uint32_t)(pp->seed >> 32)};
    uint32_t ctr[4] = {pix, cam_uid, (uint32_t)step, (uint32_t)(((step >> 32) & 0xFFFFu) << 16)};
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    int drop = (pp->flags & POST_DROPOUT) && ((uint64_t)w[0] < drop_threshold(pp->p_drop));
    double zz;
    if (inst >= 0) {
        double g = 0.0;
        if (pp->flags & POST_NOISE) {
            double u1 = ((double)(w[1] >> 8) + 1.0) * 0x1p-24;
            double u2 = (double)(w[2] >> 8) * 0x1p-24;
            g = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
        }
        zz = (double)z + ((double)pp->sigma_abs + (double)pp->sigma_rel * (double)z) * g;
    } else {
        zz = (double)pp->far_;
    }
    if (zz < pp->near_) zz = pp->near_;
    if (zz > pp->far_) zz = pp->far_;
    *dropped = (uint8_t)drop;
    return drop ? (double)pp->fill : zz;
}

/*
 * oracle_post: the sensor model over a sequence of S rendered frames.
 * depth/inst [S][N] with N = E*C*H*W for steps s0 .. s0+S-1; cam_uid [E*C]
 * (NULL: e*C + c).  Outputs out [S][N], drop [S][N] (the mask of the capture
 * shown) and lat [S][E*C].
 */
int oracle_post(const float* depth, const int32_t* inst, int E, int C, int H, int W, int S,
                uint64_t s0, const uint32_t* cam_uid, const post_params_t* pp,
                double* out, uint8_t* drop, uint8_t* lat) {
    if (E < 0 || C < 0 || H < 0 || W < 0 || S < 0) return -1;
    if ((pp->flags & POST_LATENCY) && (pp->lat_min < 0 || pp->lat_max < pp->lat_min)) return -1;
    int64_t N = (int64_t)E * C * H * W, HW = (int64_t)H * W;
    for (int si = 0; si < S; ++si) {
        uint64_t s = s0 + (uint64_t)si;
        #pragma omp parallel for schedule(static)
        for (int64_t ec = 0; ec < (int64_t)E * C; ++ec) {
            uint32_t u = cam_uid ? cam_uid[ec] : (uint32_t)ec;
            int k = oracle_latency(pp, u, s);
            lat[(int64_t)si * E * C + ec] = (uint8_t)k;
            uint64_t src = (s >= s0 + (uint64_t)k) ? s - (uint64_t)k : s0;
            int64_t fi = (int64_t)(src - s0);
            for (int64_t pix = 0; pix < HW; ++pix) {
                int64_t p = ec * HW + pix;
                uint8_t dm;
                out[(int64_t)si * N + p] = capture(pp, depth[fi * N + p], inst[fi * N + p],
                                                   (uint32_t)pix, u, src, &dm);
                drop[(int64_t)si * N + p] = dm;
            }
        }
    }
    return 0;
}
