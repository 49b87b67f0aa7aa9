// Multi-camera depth ray casting (Algorithm 1, Sec. 3.2.2).
//
// One lane casts one pixel ray; a 64-lane wavefront covers an 8x8 pixel tile
// of one camera image, so its rays are coherent and its camera, environment
// and top-level hierarchy are uniform.  Per ray:
//   1. ray generation in FP64 (r = K^-1 [x + 0.5, y + 0.5, 1], d = R(q_c) r,
//      o = p_c), rounded to an FP32 direction plus its FP32 residual; the ray
//      parameter is planar depth, so Algorithm 1's scale m is 1 (or |r| for
//      range depth);
//   2. robot bodies: the environment's top-level hierarchy over link
//      instances; at an instance the ray goes to the link frame,
//      o_b = R_b^T (o - t_b), d_b = R_b^T d, and the link hierarchy is
//      traversed under the current bound (early termination);
//   3. terrain: its hierarchy under the bound left by the bodies;
//   4. output of depth, instance id and triangle id.
// Traversal is stackless: a 64-bit trail records, per level, whether the
// other child is still pending; backtracking climbs parent links stored in
// the node records and jumps to the stored sibling.  Children are visited
// nearest first.  Ray/triangle tests are the watertight shear test of Woop,
// Benthin and Wald (2013) in FP32; a test whose edge functions are too close
// to zero to be decided in FP32 is repeated in FP64 from the FP64 ray (full
// rate on CDNA), so hit decisions agree with exact arithmetic except for
// rays within ~1e-12 of an edge.
#include <algorithm>

#include "rc_internal.h"

#pragma clang fp contract(off)

namespace rc {

namespace {

constexpr int kChunk = 8;  // tiles a wavefront of the batched launch takes at a time

struct TileCfg {
    int tw, th, rpl;  // tile width and height (tw * th = 64), tiles per wavefront
};
// Error bounds of the FP32 triangle test (u = 2^-24).  The decision and the
// depth are taken in FP32 only when they cannot differ from exact arithmetic
// on the exact (FP64) ray; otherwise the exact pass repeats the test in FP64.
// With p = v - o, P = max |p| over the vertices' coordinates, (X, Y) the
// sheared vertex coordinates and S = sum |X| + |Y|:
//  - in the world frame each computed X or Y is within e = 8u P + u |X| of
//    its exact value (rounding of v - o and of the shear product, the FP32
//    ray direction and the hardware reciprocal in the shear constant: 5u);
//    a rounded ray origin (randomised cameras) adds twice its rounding;
//  - in a link frame (R rounded once from FP64, the link-frame ray computed in
//    FP64 from the exact pixel ray and rounded once) each direction component
//    is within 1.87u |d_b| and each origin component within 1.87u |o_b| of
//    exact (max norms), so the shear constant is within 7u and
//    e <= u |X| + 10u P + 3.74u |o_b|;
//  - an edge function U = C_x B_y - C_y B_x then errs by at most
//    u |U| + 1.25u S^2 + 8u P S (in the world frame), so every edge function
//    is within thr = 4u (|U| + |V| + |W|) + S (2u S + k_P P + e_O) of exact,
//    with k_P = 16u (world) or 32u (link frame) and e_O the origin term
//    (16u |o_b| in the link frame), each at least twice its bound.
// A certain hit's depth t is the height Z of the triangle's plane over the
// ray in sheared coordinates; vertex errors of e in X and Y move it by about
// |grad Z|_1 e, grad Z = -(n_x, n_y) / n_z for the plane's normal n in
// sheared coordinates (n_z = det), and FP32 keeps the depth only when that is
// below kDepthTol (a fifth of the depth bar, which also covers the rounding
// of Z itself, a few ulp of t).  A triangle seen almost edge-on (grazing
// incidence) or a sliver has tiny edge functions but not tiny errors; these
// bounds, not a margin relative to the edge functions alone, keep its
// decisions and depths exact.
constexpr float kU = 5.9604644775390625e-08f;  // 2^-24
constexpr float kTerrainKP = 16.0f * kU;
constexpr float kLinkKP = 32.0f * kU;
constexpr float kLinkKO = 16.0f * kU;         // per unit of |o_b| (max norm)
constexpr float kDepthTol = 2.0e-5f;          // a fifth of the 1e-4 m depth bar

struct Slab {  // box-test form of a ray: t = b * (1/d) - o * (1/d)
    float ix, iy, iz, oix, oiy, oiz;
};

struct Shear {  // rows of the watertight shear: x' = m1.(v-o), y' = m2.(v-o), z' = m3.(v-o)
    float m1x, m1y, m1z, m2x, m2y, m2z, m3x, m3y, m3z;
};

// Reciprocals of ray quantities use the hardware reciprocal (about 1 ulp): box
// tests are covered by the boxes' outward padding, and every triangle test of
// a ray uses the same shear, so decisions stay consistent across edges.
__device__ __forceinline__ float safe_inv(float d) {
    float a = fabsf(d) < 1e-20f ? copysignf(1e-20f, d) : d;
    return __builtin_amdgcn_rcpf(a);
}

__device__ __forceinline__ Slab make_slab(float ox, float oy, float oz, float dx, float dy, float dz) {
    Slab s;
    s.ix = safe_inv(dx); s.iy = safe_inv(dy); s.iz = safe_inv(dz);
    s.oix = ox * s.ix; s.oiy = oy * s.iy; s.oiz = oz * s.iz;
    return s;
}

// Woop, Benthin, Wald (2013): kz = dominant axis of d, (kx, ky) the next two
// (swapped when d[kz] < 0), Sx = d[kx]/d[kz], Sy = d[ky]/d[kz], Sz = 1/d[kz].
__device__ __forceinline__ Shear make_shear(float dx, float dy, float dz) {
    float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
    int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    float dk = kz == 0 ? dx : (kz == 1 ? dy : dz);
    if (dk < 0.0f) { int t = kx; kx = ky; ky = t; }
    float dkx = kx == 0 ? dx : (kx == 1 ? dy : dz);
    float dky = ky == 0 ? dx : (ky == 1 ? dy : dz);
    float sz = __builtin_amdgcn_rcpf(dk);
    float sx = dkx * sz, sy = dky * sz;
    Shear m;
    m.m1x = (kx == 0) ? 1.0f : (kz == 0 ? -sx : 0.0f);
    m.m1y = (kx == 1) ? 1.0f : (kz == 1 ? -sx : 0.0f);
    m.m1z = (kx == 2) ? 1.0f : (kz == 2 ? -sx : 0.0f);
    m.m2x = (ky == 0) ? 1.0f : (kz == 0 ? -sy : 0.0f);
    m.m2y = (ky == 1) ? 1.0f : (kz == 1 ? -sy : 0.0f);
    m.m2z = (ky == 2) ? 1.0f : (kz == 2 ? -sy : 0.0f);
    m.m3x = kz == 0 ? sz : 0.0f;
    m.m3y = kz == 1 ? sz : 0.0f;
    m.m3z = kz == 2 ? sz : 0.0f;
    return m;
}

// Slab test of one box (lo.x, hi.x, lo.y, hi.y, lo.z, hi.z) over [0, tmax].
// OCT >= 0: the signs of (1/dx, 1/dy, 1/dz) are known (bit k set: axis k
// negative), so the near and far planes are known and no min/max pairs are
// needed; fma is monotonic, so the result equals the general form bit for bit.
template <int OCT = -1>
__device__ __forceinline__ bool slab(float lx, float hx, float ly, float hy, float lz, float hz,
                                     const Slab& r, float tmax, float& tn) {
    float a, b;
    if (OCT < 0) {
        float tx0 = __fmaf_rn(lx, r.ix, -r.oix), tx1 = __fmaf_rn(hx, r.ix, -r.oix);
        float ty0 = __fmaf_rn(ly, r.iy, -r.oiy), ty1 = __fmaf_rn(hy, r.iy, -r.oiy);
        float tz0 = __fmaf_rn(lz, r.iz, -r.oiz), tz1 = __fmaf_rn(hz, r.iz, -r.oiz);
        a = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
        b = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), tmax));
    } else {
        const float nx = (OCT & 1) ? hx : lx, fx = (OCT & 1) ? lx : hx;
        const float ny = (OCT & 2) ? hy : ly, fy = (OCT & 2) ? ly : hy;
        const float nz = (OCT & 4) ? hz : lz, fz = (OCT & 4) ? lz : hz;
        a = fmaxf(fmaxf(__fmaf_rn(nx, r.ix, -r.oix), __fmaf_rn(ny, r.iy, -r.oiy)),
                  fmaxf(__fmaf_rn(nz, r.iz, -r.oiz), 0.0f));
        b = fminf(fminf(__fmaf_rn(fx, r.ix, -r.oix), __fmaf_rn(fy, r.iy, -r.oiy)),
                  fminf(__fmaf_rn(fz, r.iz, -r.oiz), tmax));
    }
    tn = a;
    return a <= b;
}

// Box test of a ray going straight down from (r.oix, r.oiy, r.oiz) (the
// vertical rays of the height map): containment in x and y, then the z range
// over [0, tmax].  Exact in FP32 against the padded boxes.
__device__ __forceinline__ bool vslab(float lx, float hx, float ly, float hy, float lz, float hz,
                                      const Slab& r, float tmax, float& tn) {
    tn = fmaxf(r.oiz - hz, 0.0f);
    return (lx <= r.oix) & (r.oix <= hx) & (ly <= r.oiy) & (r.oiy <= hy) & (tn <= fminf(r.oiz - lz, tmax));
}

__device__ __forceinline__ int slab_octant(const Slab& r) {
    return (r.ix < 0.0f ? 1 : 0) | (r.iy < 0.0f ? 2 : 0) | (r.iz < 0.0f ? 4 : 0);
}

// FP64 watertight test of one triangle; closed triangle, both sides; hit at t > 0.
__device__ __forceinline__ bool tri_test64(const float* __restrict__ v, const double o[3],
                                           const double d[3], double& t) {
    double ax = fabs(d[0]), ay = fabs(d[1]), az = fabs(d[2]);
    int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    if (d[kz] < 0.0) { int s = kx; kx = ky; ky = s; }
    double sz = 1.0 / d[kz];
    double sx = d[kx] * sz, sy = d[ky] * sz;
    double X[3], Y[3], Z[3];
    for (int k = 0; k < 3; ++k) {
        double p[3] = {(double)v[3 * k] - o[0], (double)v[3 * k + 1] - o[1], (double)v[3 * k + 2] - o[2]};
        X[k] = p[kx] - sx * p[kz];
        Y[k] = p[ky] - sy * p[kz];
        Z[k] = sz * p[kz];
    }
    double U = X[2] * Y[1] - Y[2] * X[1];
    double V = X[0] * Y[2] - Y[0] * X[2];
    double W = X[1] * Y[0] - Y[1] * X[0];
    bool in = (U >= 0.0 && V >= 0.0 && W >= 0.0) || (U <= 0.0 && V <= 0.0 && W <= 0.0);
    double det = U + V + W;
    if (!in || det == 0.0) return false;
    t = (U * Z[0] + V * Z[1] + W * Z[2]) / det;
    return t > 0.0;
}

__device__ __forceinline__ void quat_mat64(const float* __restrict__ q, double R[9]) {
    double x = q[0], y = q[1], z = q[2], w = q[3];
    double n = sqrt(x * x + y * y + z * z + w * w);
    x /= n; y /= n; z /= n; w /= n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - z * w); R[2] = 2 * (x * z + y * w);
    R[3] = 2 * (x * y + z * w); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - x * w);
    R[6] = 2 * (x * z - y * w); R[7] = 2 * (y * z + x * w); R[8] = 1 - 2 * (x * x + y * y);
}

// A camera's FP64 ray basis (16 doubles, written once per launch by
// k_cam_prep from the camera's centre p_c, quaternion q_c (optical -> world)
// and intrinsics (fx, fy, cx, cy)): R(q_c) row-major [9], p_c [3], 1/fx, 1/fy,
// cx, cy.
struct CamRef {
    const double* b;
};
constexpr int kCamBasis = 16;

__device__ __forceinline__ void cam_basis(const float* pos, const float* quat, const float* intr,
                                          double* b) {
    double R[9];
    quat_mat64(quat, R);
    for (int k = 0; k < 9; ++k) b[k] = R[k];
    b[9] = pos[0]; b[10] = pos[1]; b[11] = pos[2];
    b[12] = 1.0 / (double)intr[0];
    b[13] = 1.0 / (double)intr[1];
    b[14] = intr[2];
    b[15] = intr[3];
}

// FP64 camera ray of pixel (x, y): o = p_c, d = R(q_c) K^-1 [x+.5, y+.5, 1].
__device__ __forceinline__ void pixel_ray64(const CamRef& cam, int x, int y, double o[3],
                                            double d[3], double& rx, double& ry) {
    const double* b = cam.b;
    rx = ((double)x + 0.5 - b[14]) * b[12];
    ry = ((double)y + 0.5 - b[15]) * b[13];
    d[0] = b[0] * rx + b[1] * ry + b[2];
    d[1] = b[3] * rx + b[4] * ry + b[5];
    d[2] = b[6] * rx + b[7] * ry + b[8];
    o[0] = b[9]; o[1] = b[10]; o[2] = b[11];
}

// The exact-decision path: rebuild the pixel's FP64 ray (and its FP64 link-frame
// ray for link >= 0) and repeat the triangle test in FP64.  Rarely taken, so it
// recomputes everything instead of keeping an FP64 ray live in registers.
__device__ __noinline__ bool refine(const float* __restrict__ v, const double* cam, int x, int y,
                                    int link, int e, int n_links,
                                    const float* __restrict__ link_pos,
                                    const float* __restrict__ link_quat, double* t) {
    double o[3], d[3], rx, ry;
    pixel_ray64(CamRef{cam}, x, y, o, d, rx, ry);
    if (link >= 0) {
        const int64_t eb = (int64_t)e * n_links + link;
        double R[9];
        quat_mat64(link_quat + 4 * eb, R);
        const float* p = link_pos + 3 * eb;
        double q[3] = {o[0] - (double)p[0], o[1] - (double)p[1], o[2] - (double)p[2]};
        double lo[3], ld[3];
        for (int k = 0; k < 3; ++k) {
            lo[k] = R[k] * q[0] + R[3 + k] * q[1] + R[6 + k] * q[2];
            ld[k] = R[k] * d[0] + R[3 + k] * d[1] + R[6 + k] * d[2];
        }
        return tri_test64(v, lo, ld, *t);
    }
    return tri_test64(v, o, d, *t);
}

struct Hit {
    float tmax;    // current bound = ray parameter of the best hit so far
    uint64_t key;  // (inst << 32) | tri of the best hit, ~0 for none
    float tu;      // fast pass: smallest ray parameter of an FP32-undecided test
};

struct PixelRef {  // what the exact-decision path needs to rebuild the ray
    CamRef cam;
    const float* link_pos;
    const float* link_quat;
    int x, y, e, n_links;
    uint2* cand;  // fast pass: this lane's two LDS slots for FP32-undecided triangles
    float eo;     // 4 x the rounding of the FP32 ray origin (0 when it is exact)
};

// FP32-undecided triangles the fast pass keeps per ray (in LDS), for the exact
// pass to decide in FP64 without re-casting the ray.  A slot holds
// (id, bits of the plane distance); id = (link + 1) << kLeafBits | leaf, link
// + 1 = 0 for the terrain.  A ray with more undecided triangles near its hit
// than slots is re-cast in full.
constexpr uint32_t kNoCand = 0xFFFFFFFFu;
constexpr int kLeafBits = 25;
constexpr int kCandSlots = 2;
// an undecided plane farther than the bound times this cannot matter (covers
// the FP32 error of its distance)
constexpr float kUndecidedSlack = 1.0f + 1.0f / 1024.0f;

// Per-ray work counters of the diagnostic render (rc_render_counts): node
// records whose child boxes a lane reads, triangles tested, link instances
// entered.  NoCount compiles to nothing in the production kernels.
struct NoCount {
    static constexpr bool kOn = false;
    __device__ __forceinline__ void node() {}
    __device__ __forceinline__ void tri() {}
    __device__ __forceinline__ void inst() {}
    __device__ __forceinline__ uint32_t nodes() const { return 0; }
    __device__ __forceinline__ void link_nodes(uint32_t) {}
};
struct RayCount {
    static constexpr bool kOn = true;
    uint32_t n = 0, t = 0, i = 0, l = 0;  // l: node records of link hierarchies (part of n)
    __device__ __forceinline__ void node() { ++n; }
    __device__ __forceinline__ void tri() { ++t; }
    __device__ __forceinline__ void inst() { ++i; }
    __device__ __forceinline__ uint32_t nodes() const { return n; }
    __device__ __forceinline__ void link_nodes(uint32_t k) { l += k; }
};

// Test one triangle (leaf-order record v) against the ray (origin o, shear m).
// FP32 decides when all three edge functions clearly share a sign (hit) or
// clearly disagree (miss).  Otherwise the fast pass keeps the triangle for the
// exact pass (an LDS slot, or the ray is re-cast if they are full), which
// repeats the test in FP64.  The hit distance is T * rcp(det) (a couple of
// ulp; the same expression in both passes), the input triangle id is read
// only for an accepted hit.
// Zero-area triangles never get here: the hierarchy builder makes them
// unreachable (their edge functions would be rounding residues of one sign).
template <bool EXACT>
__device__ __forceinline__ void tri_test(const float* __restrict__ v,
                                         const int32_t* __restrict__ tri_ids, uint32_t inst,
                                         float ox, float oy, float oz, const Shear& m, float k_p,
                                         float e_o,
                                         Hit& h, const PixelRef& px, int link, int leaf) {
    const float p0x = v[0] - ox, p0y = v[1] - oy, p0z = v[2] - oz;
    const float p1x = v[3] - ox, p1y = v[4] - oy, p1z = v[5] - oz;
    const float p2x = v[6] - ox, p2y = v[7] - oy, p2z = v[8] - oz;
    const float Ax = __fmaf_rn(m.m1z, p0z, __fmaf_rn(m.m1y, p0y, m.m1x * p0x));
    const float Ay = __fmaf_rn(m.m2z, p0z, __fmaf_rn(m.m2y, p0y, m.m2x * p0x));
    const float Bx = __fmaf_rn(m.m1z, p1z, __fmaf_rn(m.m1y, p1y, m.m1x * p1x));
    const float By = __fmaf_rn(m.m2z, p1z, __fmaf_rn(m.m2y, p1y, m.m2x * p1x));
    const float Cx = __fmaf_rn(m.m1z, p2z, __fmaf_rn(m.m1y, p2y, m.m1x * p2x));
    const float Cy = __fmaf_rn(m.m2z, p2z, __fmaf_rn(m.m2y, p2y, m.m2x * p2x));
    const float U = __fmaf_rn(Cx, By, -(Cy * Bx));
    const float V = __fmaf_rn(Ax, Cy, -(Ay * Cx));
    const float W = __fmaf_rn(Bx, Ay, -(By * Ax));
    const float P = fmaxf(fmaxf(fmaxf(fmaxf(fabsf(p0x), fabsf(p0y)), fmaxf(fabsf(p0z), fabsf(p1x))),
                                fmaxf(fmaxf(fabsf(p1y), fabsf(p1z)), fmaxf(fabsf(p2x), fabsf(p2y)))),
                          fabsf(p2z));
    const float S = ((fabsf(Ax) + fabsf(Ay)) + (fabsf(Bx) + fabsf(By))) + (fabsf(Cx) + fabsf(Cy));
    const float inner = __fmaf_rn(S, 2.0f * kU, __fmaf_rn(P, k_p, e_o));  // twice the X, Y error
    const float thr = __fmaf_rn(fabsf(U) + fabsf(V) + fabsf(W), 4.0f * kU, S * inner);
    const float lo = fminf(fminf(U, V), W), hi = fmaxf(fmaxf(U, V), W);
    if ((lo < -thr) & (hi > thr)) return;  // certainly outside
    // certain hit only when all three clear the margin with the same sign
    const bool sure = (thr > 0.0f) & ((lo > thr) | (hi < -thr));
    // FP32 also gives the depth of a certain hit unless the triangle is seen
    // almost edge-on (the depth bound above); then the exact pass computes it
    bool fp32 = sure;
    float t = 0.0f, det = 0.0f;
    if (!EXACT || sure) {
        const float Az = __fmaf_rn(m.m3z, p0z, __fmaf_rn(m.m3y, p0y, m.m3x * p0x));
        const float Bz = __fmaf_rn(m.m3z, p1z, __fmaf_rn(m.m3y, p1y, m.m3x * p1x));
        const float Cz = __fmaf_rn(m.m3z, p2z, __fmaf_rn(m.m3y, p2y, m.m3x * p2x));
        det = U + V + W;
        const float T = __fmaf_rn(W, Cz, __fmaf_rn(V, Bz, U * Az));
        t = T * __builtin_amdgcn_rcpf(det);
        if (sure) {
            const float dX1 = Bx - Ax, dY1 = By - Ay, dZ1 = Bz - Az;
            const float dX2 = Cx - Ax, dY2 = Cy - Ay, dZ2 = Cz - Az;
            const float gx = __fmaf_rn(dY1, dZ2, -(dZ1 * dY2));
            const float gy = __fmaf_rn(dZ1, dX2, -(dX1 * dZ2));
            fp32 = (fabsf(gx) + fabsf(gy)) * (0.5f * inner) <= kDepthTol * fabsf(det);
        }
    }
    if (!fp32) {
        if (EXACT) {
            double t64;
            if (!refine(v, px.cam.b, px.x, px.y, link, px.e, px.n_links,
                        px.link_pos, px.link_quat, &t64))
                return;
            t = (float)t64;
        } else {
            // undecided in FP32 (the test, or the depth of a certain hit): keep
            // the triangle for the exact pass unless its plane is behind the
            // origin (well conditioned) or beyond the bound
            const bool cond = !sure && fabsf(det) > thr;
            if (cond && t < -1e-3f) return;
            const float tu = (cond && t > 0.0f) ? t : 0.0f;
            const float lim = h.tmax * kUndecidedSlack;
            if (tu > lim) return;
            if ((uint32_t)leaf < (1u << kLeafBits)) {
                const uint32_t id = ((uint32_t)(link + 1) << kLeafBits) | (uint32_t)leaf;
                for (int k = 0; k < kCandSlots; ++k) {
                    const uint2 c = px.cand[k];  // a slot is free if empty or out of reach now
                    if (c.x == kNoCand || __uint_as_float(c.y) > lim) {
                        px.cand[k] = make_uint2(id, __float_as_uint(tu));
                        return;
                    }
                }
            }
            h.tu = fminf(h.tu, tu);  // no free slot: the ray will be re-cast in full
            return;
        }
    }
    if (t > 0.0f && t <= h.tmax) {
        const uint64_t key = ((uint64_t)inst << 32) | (uint32_t)tri_ids[leaf];
        const bool upd = t < h.tmax || key < h.key;
        h.tmax = upd ? t : h.tmax;
        h.key = upd ? key : h.key;
    }
}

// Per-lane nearest-first traversal of the subtree at `start` of a hierarchy
// of n_nodes records and n_prim leaves; `leaf(i)` handles leaf i.  A 64-bit
// trail marks, per level below the start, whether the far child is still
// pending.  With a short stack (stk: this lane's column of an LDS array,
// kStack entries, stride kLanes), the pending far children of the shallowest
// kStack such levels are kept there, so backtracking is a pop; a pending level
// beyond them is reached by climbing the parent links stored in the records,
// which is also the whole mechanism without a stack.  Indices are range
// checked and the loop is bounded (a valid hierarchy needs fewer than
// 2 n_nodes + 2 steps), so a corrupt hierarchy ends the ray instead of
// faulting or spinning.
constexpr int kStack = kWalkStack;
constexpr int kLanes = 64 * kWavesPerBlock;

template <int OCT = -1, bool VERT = false, typename Cnt, typename Leaf>
__device__ __forceinline__ void traverse(const Node* __restrict__ nodes, int n_nodes, int n_prim,
                                         const Slab& r, Hit& h, Cnt& cnt, Leaf&& leaf,
                                         int start = 0, uint32_t* stk = nullptr) {
    uint64_t trail = 0;
    int cur = start;
    int sp = 0;  // far children kept on the stack (the shallowest pending levels)
    int budget = 2 * n_nodes + 2;
    for (;;) {
        if ((unsigned)cur >= (unsigned)n_nodes || --budget < 0) return;
        const float4* np = reinterpret_cast<const float4*>(nodes + cur);
        const float4 q0 = np[0], q1 = np[1], q2 = np[2];
        const int4 q3 = reinterpret_cast<const int4*>(np)[3];
        cnt.node();
        float tn0, tn1;
        bool h0 = VERT ? vslab(q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, r, h.tmax, tn0)
                       : slab<OCT>(q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, r, h.tmax, tn0);
        bool h1 = VERT ? vslab(q1.z, q1.w, q2.x, q2.y, q2.z, q2.w, r, h.tmax, tn1)
                       : slab<OCT>(q1.z, q1.w, q2.x, q2.y, q2.z, q2.w, r, h.tmax, tn1);
        const int c0 = q3.x, c1 = q3.y;
        // non-short-circuit forms: mask arithmetic instead of branches
        h0 = h0 & ((c0 >= 0) | ((unsigned)~c0 < (unsigned)n_prim));
        h1 = h1 & ((c1 >= 0) | ((unsigned)~c1 < (unsigned)n_prim));
        const bool l0 = h0 & (c0 < 0), l1 = h1 & (c1 < 0);
        if (l0 || l1) {  // leaf children first, nearest first
            const bool swap = l0 && l1 && tn1 < tn0;
            const int la = (l0 && !swap) ? ~c0 : ~c1;
            const int lb = (l0 && l1) ? (swap ? ~c0 : ~c1) : -1;
            const float tb = swap ? tn0 : tn1;
            for (int k = 0; k < 2; ++k) {
                const int lf = k == 0 ? la : lb;
                if (lf < 0 || (k == 1 && tb > h.tmax)) break;
                leaf(lf);
            }
        }
        const bool g0 = h0 & !l0 & (tn0 <= h.tmax);
        const bool g1 = h1 & !l1 & (tn1 <= h.tmax);
        if (g0 && g1) {
            const bool first1 = tn1 < tn0;
            trail = (trail << 1) | 1ull;
            cur = first1 ? c1 : c0;
            if (stk && sp < kStack) stk[kLanes * sp++] = (uint32_t)(first1 ? c0 : c1);
            continue;
        }
        if (g0 || g1) {
            trail <<= 1;
            cur = g0 ? c0 : c1;
            continue;
        }
        if (trail == 0ull) return;
        if (stk && __popcll(trail) == sp) {  // the deepest pending level is on the stack
            trail = (trail >> __builtin_ctzll(trail)) ^ 1ull;
            cur = (int)stk[kLanes * --sp];
            continue;
        }
        // climb to the deepest level whose other child is pending
        int par = q3.z, sib = q3.w;
        for (;;) {
            if (trail & 1ull) {
                trail ^= 1ull;
                cur = sib;
                break;
            }
            trail >>= 1;
            if ((unsigned)par >= (unsigned)n_nodes || --budget < 0) return;
            const int4 pq = reinterpret_cast<const int4*>(nodes + par)[3];
            par = pq.z;
            sib = pq.w;
        }
    }
}

// The fast pass's terrain walk, over the 4-wide records (kWideRec): per lane,
// nearest first, with the triangle tests gathered across the wavefront.
// A visit tests the record's four boxes at once.  Leaf slots that the ray
// reaches are parked (the record's index and a slot mask) and the lane pauses;
// the internal slots it reaches are ordered by entry distance, the nearest
// entered next and the others pushed farthest first on the lane's LDS stack.
// The wavefront tests the parked leaves of all its lanes in one pass once the
// lanes still walking are at most a quarter of the live ones (or none), so a
// pass of the triangle test serves many lanes rather than the few that reached
// a leaf at the same step.  A paused lane's next record was chosen under the
// bound it had before its leaves were tested; the children of that record are
// tested under the tightened bound.  Every step moves a walking lane (the
// budget bounds these) or empties the parked slots, so the loop ends.  A push
// onto a full stack (cap entries) is dropped and marks the ray (h.tu = 0): the
// fast pass's exact pass then re-casts it in full, and the height map walks
// the column again over the binary records, so no result depends on the
// stack's depth; the exact pass's own walks get a stack that cannot overflow.
constexpr int kGatherNum = 3, kGatherDen = 4;  // test once parked >= 3/4 of live lanes
// The exact pass's full re-casts walk the 4-wide records with a stack that
// cannot overflow: a path from the root visits at most kMaxDepth / 2 + 1
// records and each leaves at most three slots pending.
constexpr int kExactStack = 104;
static_assert(kExactStack >= 3 * (kMaxDepth / 2 + 1), "exact-pass stack too short");

template <int OCT, bool VERT = false, typename Cnt, typename Leaf>
__device__ __forceinline__ void traverse4(const float4* __restrict__ wide, int n_nodes, int n_prim,
                                          const Slab& r, Hit& h, Cnt& cnt, Leaf&& leaf, int start,
                                          uint32_t* stk, int cap) {
    int cur = start;
    int sp = 0;
    int budget = 2 * n_nodes + 2;
    int pn = 0;       // record whose leaf slots are parked
    uint32_t pm = 0;  // parked slot mask
    bool walk = true;
    for (;;) {
        if (walk && pm == 0u) {
            if ((unsigned)cur >= (unsigned)n_nodes || --budget < 0) {
                walk = false;
            } else {
                const float4* np = wide + kWideRec * (int64_t)cur;
                const float4 xl = np[0], xh = np[1], yl = np[2], yh = np[3], zl = np[4], zh = np[5];
                const int4 ch = *reinterpret_cast<const int4*>(np + 6);
                cnt.node();
                float tn[4];
                bool hit[4];
                if constexpr (VERT) {  // the height map's vertical columns
                    hit[0] = vslab(xl.x, xh.x, yl.x, yh.x, zl.x, zh.x, r, h.tmax, tn[0]);
                    hit[1] = vslab(xl.y, xh.y, yl.y, yh.y, zl.y, zh.y, r, h.tmax, tn[1]);
                    hit[2] = vslab(xl.z, xh.z, yl.z, yh.z, zl.z, zh.z, r, h.tmax, tn[2]);
                    hit[3] = vslab(xl.w, xh.w, yl.w, yh.w, zl.w, zh.w, r, h.tmax, tn[3]);
                } else {
                    hit[0] = slab<OCT>(xl.x, xh.x, yl.x, yh.x, zl.x, zh.x, r, h.tmax, tn[0]);
                    hit[1] = slab<OCT>(xl.y, xh.y, yl.y, yh.y, zl.y, zh.y, r, h.tmax, tn[1]);
                    hit[2] = slab<OCT>(xl.z, xh.z, yl.z, yh.z, zl.z, zh.z, r, h.tmax, tn[2]);
                    hit[3] = slab<OCT>(xl.w, xh.w, yl.w, yh.w, zl.w, zh.w, r, h.tmax, tn[3]);
                }
                const int c[4] = {ch.x, ch.y, ch.z, ch.w};
                uint32_t lm = 0;
                float d[4];
                int e[4];
                for (int k = 0; k < 4; ++k) {
                    const bool lf = hit[k] & (c[k] < 0) & ((unsigned)~c[k] < (unsigned)n_prim);
                    lm |= (lf ? 1u : 0u) << k;
                    d[k] = hit[k] & (c[k] >= 0) ? tn[k] : INFINITY;
                    e[k] = c[k];
                }
                pm = lm;
                pn = cur;
                // sorting network on (distance, child): nearest in slot 0
                auto cx = [&](int i, int j) {
                    const bool sw = d[j] < d[i];
                    const float di = d[i], dj = d[j];
                    const int ei = e[i], ej = e[j];
                    d[i] = sw ? dj : di;
                    d[j] = sw ? di : dj;
                    e[i] = sw ? ej : ei;
                    e[j] = sw ? ei : ej;
                };
                cx(0, 1); cx(2, 3); cx(0, 2); cx(1, 3); cx(1, 2);
                if (d[0] < INFINITY) {
                    for (int k = 3; k >= 1; --k) {
                        if (d[k] < INFINITY) {
                            if (sp < cap) stk[kLanes * sp++] = (uint32_t)e[k];
                            else h.tu = 0.0f;
                        }
                    }
                    cur = e[0];
                } else if (sp == 0) {
                    walk = false;
                } else {
                    cur = (int)stk[kLanes * --sp];
                }
            }
        }
        const bool parked = pm != 0u;
        const uint64_t P = __ballot(parked);
        const uint64_t Wk = __ballot(walk && !parked);
        if (P != 0ull &&
            (Wk == 0ull || __popcll(P) * kGatherDen >= __popcll(P | Wk) * kGatherNum)) {
            if (parked) {
                const int4 ch = *reinterpret_cast<const int4*>(wide + kWideRec * (int64_t)pn + 6);
                while (pm) {
                    const int k = __builtin_ctz(pm);
                    pm &= pm - 1u;
                    leaf(~(k == 0 ? ch.x : (k == 1 ? ch.y : (k == 2 ? ch.z : ch.w))));
                }
            }
        }
        if (!walk && pm == 0u) return;
    }
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni_f(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Enter link b of env e: take the ray to the link frame (o_b = R_b^T (o - t_b),
// d_b = R_b^T d) and traverse the link's hierarchy under the current bound.
template <bool EXACT, typename Cnt>
__device__ __forceinline__ void enter_link(const RenderLaunch& a, int e, int b, float ox, float oy,
                                           float oz, float dx, float dy, float dz, Hit& h,
                                           const PixelRef& px, Cnt& cnt, uint32_t* stk) {
    cnt.inst();
    const InstXform X = a.xf[(int64_t)e * a.n_links + b];
    // the link-frame ray in FP64 from the exact pixel ray, rounded once: each
    // component is then within 1.87u of the exact one (max norm; R is rounded
    // from FP64 as well), which is what the link-frame error bound uses
    double o64[3], d64[3], rx, ry;
    pixel_ray64(px.cam, px.x, px.y, o64, d64, rx, ry);
    const double qx = o64[0] - (double)X.t[0], qy = o64[1] - (double)X.t[1], qz = o64[2] - (double)X.t[2];
    float lox = (float)((double)X.m[0] * qx + (double)X.m[1] * qy + (double)X.m[2] * qz);
    float loy = (float)((double)X.m[3] * qx + (double)X.m[4] * qy + (double)X.m[5] * qz);
    float loz = (float)((double)X.m[6] * qx + (double)X.m[7] * qy + (double)X.m[8] * qz);
    if constexpr (!EXACT) {  // the fast pass's wavefront shares one camera, so one o_b
        lox = uni_f(lox);
        loy = uni_f(loy);
        loz = uni_f(loz);
    }
    const float ldx = (float)((double)X.m[0] * d64[0] + (double)X.m[1] * d64[1] + (double)X.m[2] * d64[2]);
    const float ldy = (float)((double)X.m[3] * d64[0] + (double)X.m[4] * d64[1] + (double)X.m[5] * d64[2]);
    const float ldz = (float)((double)X.m[6] * d64[0] + (double)X.m[7] * d64[1] + (double)X.m[8] * d64[2]);
    (void)ox; (void)oy; (void)oz; (void)dx; (void)dy; (void)dz;
    const Slab ls = make_slab(lox, loy, loz, ldx, ldy, ldz);
    const Shear lm = make_shear(ldx, ldy, ldz);
    // origin term of the link-frame error bound (grows with |o_b|)
    const float e_o = fmaxf(fmaxf(fabsf(lox), fabsf(loy)), fabsf(loz)) * kLinkKO;
    const LinkMeta M = a.link_meta[b];
    const float* __restrict__ tris = a.link_tris + M.tri_base;
    const int32_t* __restrict__ ids = a.link_tri_id + M.id_base;
    const uint32_t n0 = cnt.nodes();
    traverse(a.link_nodes + M.node_base, M.n_tri > 1 ? M.n_tri - 1 : 1, M.n_tri, ls, h, cnt, [&](int i) {
        cnt.tri();
        tri_test<EXACT>(tris + 9 * (int64_t)i, ids, (uint32_t)b, lox, loy, loz, lm, kLinkKP, e_o, h,
                        px, b, i);
    }, 0, stk);
    cnt.link_nodes(cnt.nodes() - n0);
}

// Schedule variants of the fast pass (bits of MODE).
constexpr int kPacketTerrain = 1;  // walk the terrain as a wavefront packet
constexpr int kFlatBodies = 2;     // cull links against the wavefront's cone instead of the top level

// Wavefront reductions by DPP lane moves (no LDS round trips; all 64 lanes
// must be active): shifts within each row of 16 lanes leave the row's result
// in its last lane, two row broadcasts carry those on to lane 63, whose value
// is returned to every lane as a scalar.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, ROWS, 0xF, false));
}
template <typename Op>
__device__ __forceinline__ float wave_reduce(float v, Op op) {
    v = op(v, dpp_mov<0x111, 0xF>(v));  // row_shr:1
    v = op(v, dpp_mov<0x112, 0xF>(v));  // row_shr:2
    v = op(v, dpp_mov<0x114, 0xF>(v));  // row_shr:4
    v = op(v, dpp_mov<0x118, 0xF>(v));  // row_shr:8
    v = op(v, dpp_mov<0x142, 0xA>(v));  // row_bcast:15 into rows 1 and 3
    v = op(v, dpp_mov<0x143, 0xC>(v));  // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ float wave_sum(float v) {
    return wave_reduce(v, [](float x, float y) { return x + y; });
}
__device__ __forceinline__ float wave_min(float v) {
    return wave_reduce(v, [](float x, float y) { return fminf(x, y); });
}
__device__ __forceinline__ float wave_max(float v) {
    return wave_reduce(v, [](float x, float y) { return fmaxf(x, y); });
}

// World bounding sphere of link b of env e, written by the top-level build:
// the centre of its local (padded) box under the pose, the box's
// half-diagonal as radius, widened by 1% + 1 mm so FP32 rounding cannot cull
// a reachable link.
__device__ __forceinline__ void link_sphere(const RenderLaunch& a, int e, int b, float& cx, float& cy,
                                            float& cz, float& rad) {
    const float4 S = *reinterpret_cast<const float4*>(a.xf[(int64_t)e * a.n_links + b].s);
    cx = S.x;
    cy = S.y;
    cz = S.z;
    rad = S.w;
}

// One pixel ray: robot bodies first, then the terrain under their bound
// (Algorithm 1's query order).  WAVE: the wavefront shares the environment
// and walks its top-level hierarchy together (trail and node records are
// wave-uniform, in scalar registers; a node is entered if any lane's ray hits
// it, a link only by the lanes whose rays hit its box) - or, with
// kFlatBodies, tests every link's bounding sphere against the cone of its
// rays (one link per lane) and visits the survivors one by one, entering a
// link where the lane's ray segment passes its sphere.  Otherwise each lane
// walks the top level alone.
template <bool EXACT, bool WAVE, int MODE, typename Cnt>
__device__ __forceinline__ Hit cast_ray(const RenderLaunch& a, const CamRef& cam, int e, int x, int y,
                                        float bound, uint2* cand, uint32_t* stk,
                                        Cnt& cnt) {
    double o64[3], d64[3], rx, ry;
    pixel_ray64(cam, x, y, o64, d64, rx, ry);
    float ox = (float)o64[0], oy = (float)o64[1], oz = (float)o64[2];
    if constexpr (WAVE) {  // one camera per wavefront: its origin lives in scalar registers
        ox = uni_f(ox);
        oy = uni_f(oy);
        oz = uni_f(oz);
    }
    const float dx = (float)d64[0], dy = (float)d64[1], dz = (float)d64[2];
    const double scale = a.depth_mode == RC_DEPTH_RANGE ? sqrt(rx * rx + ry * ry + 1.0) : 1.0;
    Hit h;
    h.tmax = fminf(a.depth_mode == RC_DEPTH_RANGE ? (float)((double)a.far_plane / scale) : a.far_plane,
                   bound);
    h.key = ~0ull;
    h.tu = INFINITY;
    // a rounded origin (randomised cameras) moves every sheared coordinate by
    // up to twice its rounding
    const double r_o = fmax(fmax(fabs(o64[0] - (double)ox), fabs(o64[1] - (double)oy)),
                            fabs(o64[2] - (double)oz));
    const PixelRef px{cam, a.link_pos, a.link_quat, x, y, e, a.n_links, cand, (float)(4.0 * r_o)};

    if (a.n_links > 0) {
        const int n_rec = a.n_links > 1 ? a.n_links - 1 : 1;
        const Node* __restrict__ tl = a.tlas + (int64_t)e * n_rec;
        if (!WAVE) {
            // one lane alone (the exact pass): every link's bounding sphere
            // against the lane's segment [o, o + tmax d]; the result does not
            // depend on the order, since hits are ranked by (depth, inst, tri)
            const float dd = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
            for (int b = 0; b < a.n_links; ++b) {
                float sx, sy, sz, sr;
                link_sphere(a, e, b, sx, sy, sz, sr);
                const float wx = sx - ox, wy = sy - oy, wz = sz - oz;
                const float tc = fminf(fmaxf(__fmaf_rn(wz, dz, __fmaf_rn(wy, dy, wx * dx)) *
                                                 __builtin_amdgcn_rcpf(dd), 0.0f),
                                       h.tmax);
                const float qx = __fmaf_rn(-tc, dx, wx), qy = __fmaf_rn(-tc, dy, wy),
                            qz = __fmaf_rn(-tc, dz, wz);
                if (__fmaf_rn(qz, qz, __fmaf_rn(qy, qy, qx * qx)) <= sr * sr)
                    enter_link<EXACT>(a, e, b, ox, oy, oz, dx, dy, dz, h, px, cnt, nullptr);
            }
        } else if (MODE & kFlatBodies) {
            // cone of the wavefront's rays (common apex o): unit axis and the
            // cosine of its half-angle, widened for rounding
            const float il = rsqrtf(__fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx)));
            const float nx = dx * il, ny = dy * il, nz = dz * il;
            float ax = wave_sum(nx), ay = wave_sum(ny), az = wave_sum(nz);
            const float al = sqrtf(__fmaf_rn(az, az, __fmaf_rn(ay, ay, ax * ax)));
            float cmin = -1.0f;
            if (al > 1e-3f) {
                ax /= al; ay /= al; az /= al;
                cmin = wave_min(__fmaf_rn(nz, az, __fmaf_rn(ny, ay, nx * ax))) - 1e-4f;
            }
            const float smin = sqrtf(fmaxf(0.0f, 1.0f - cmin * cmin));
            // lane b: world bounding sphere of link b (local box centre under
            // the pose, half-diagonal radius with a margin) against the cone;
            // the survivors' spheres are rebuilt from wave-uniform loads below
            const int lane = threadIdx.x & 63;
            bool keep = false;
            if (lane < a.n_links) {
                float cx, cy, cz, rad;
                link_sphere(a, e, lane, cx, cy, cz, rad);
                const float vx = cx - ox, vy = cy - oy, vz = cz - oz;
                const float along = __fmaf_rn(vz, az, __fmaf_rn(vy, ay, vx * ax));
                const float v2 = __fmaf_rn(vz, vz, __fmaf_rn(vy, vy, vx * vx));
                const float perp = sqrtf(fmaxf(0.0f, v2 - along * along));
                keep = cmin <= -1.0f || __fmaf_rn(perp, cmin, -along * smin) <= rad;
            }
            uint64_t todo = __ballot(keep);
            while (todo) {  // wave-uniform loop over the surviving links
                const int b = uni(__builtin_ctzll(todo));
                todo &= todo - 1ull;
                float sx, sy, sz, sr;
                link_sphere(a, e, b, sx, sy, sz, sr);
                // closest point of the lane's segment [o, o + tmax d] to the centre
                const float wx = sx - ox, wy = sy - oy, wz = sz - oz;
                const float dd = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
                const float tc = fminf(fmaxf(__fmaf_rn(wz, dz, __fmaf_rn(wy, dy, wx * dx)) *
                                                 __builtin_amdgcn_rcpf(dd), 0.0f),
                                       h.tmax);
                const float qx = __fmaf_rn(-tc, dx, wx), qy = __fmaf_rn(-tc, dy, wy),
                            qz = __fmaf_rn(-tc, dz, wz);
                if (__fmaf_rn(qz, qz, __fmaf_rn(qy, qy, qx * qx)) <= sr * sr)
                    enter_link<EXACT>(a, e, b, ox, oy, oz, dx, dy, dz, h, px, cnt, stk);
            }
        } else {
            // 64-bit trail: a Karras hierarchy over 64 instances can be deeper
            // than 32 levels when Morton codes tie
            uint64_t trail = 0;
            int cur = 0;
            int budget = 2 * n_rec + 2;
            for (;;) {
                cur = uni(cur);
                if ((unsigned)cur >= (unsigned)n_rec || --budget < 0) break;
                const Node N = tl[cur];
                cnt.node();
                const Slab ws = make_slab(ox, oy, oz, dx, dy, dz);
                float tn0, tn1;
                bool h0 = slab(N.b0[0], N.b0[1], N.b0[2], N.b0[3], N.b0[4], N.b0[5], ws, h.tmax, tn0);
                bool h1 = slab(N.b1[0], N.b1[1], N.b1[2], N.b1[3], N.b1[4], N.b1[5], ws, h.tmax, tn1);
                const int c0 = N.c0, c1 = N.c1;
                h0 = h0 && (c0 >= 0 || (unsigned)~c0 < (unsigned)a.n_links);
                h1 = h1 && (c1 >= 0 || (unsigned)~c1 < (unsigned)a.n_links);
                for (int k = 0; k < 2; ++k) {  // instance children
                    const int c = k == 0 ? c0 : c1;
                    const bool hk = k == 0 ? h0 : h1;
                    if (c >= 0 || __ballot(hk) == 0ull) continue;
                    if (hk) enter_link<EXACT>(a, e, ~c, ox, oy, oz, dx, dy, dz, h, px, cnt, stk);
                }
                const bool g0 = c0 >= 0 && h0 && tn0 <= h.tmax;
                const bool g1 = c1 >= 0 && h1 && tn1 <= h.tmax;
                const uint64_t G0 = __ballot(g0), G1 = __ballot(g1);
                if (G0 && G1) {
                    const int want1 = __popcll(__ballot(g1 && (!g0 || tn1 < tn0)));
                    const int want0 = __popcll(__ballot(g0 && (!g1 || tn0 <= tn1)));
                    trail = (trail << 1) | 1ull;
                    cur = want1 > want0 ? c1 : c0;
                    continue;
                }
                if (G0 || G1) {
                    trail <<= 1;
                    cur = G0 ? c0 : c1;
                    continue;
                }
                int par = N.parent, sib = N.sibling;
                bool done = false;
                for (;;) {
                    if (trail == 0ull) { done = true; break; }
                    if (trail & 1ull) { trail ^= 1ull; cur = sib; break; }
                    trail >>= 1;
                    par = uni(par);
                    if ((unsigned)par >= (unsigned)n_rec || --budget < 0) { done = true; break; }
                    sib = tl[par].sibling;
                    par = tl[par].parent;
                }
                if (done) break;
            }
        }
    }
    {
        // Terrain entry: the wavefront's rays can only reach points inside the
        // box F of their segments [o, o + tmax d].  Walking down from the root
        // while exactly one child box overlaps F skips subtrees no lane can
        // reach; the lanes then traverse from that node on their own.
        int entry = 0;
        bool reach = true;
        if (WAVE) {
            const float ex = ox + h.tmax * dx, ey = oy + h.tmax * dy, ez = oz + h.tmax * dz;
            float f[6] = {fminf(ox, ex), fmaxf(ox, ex), fminf(oy, ey), fmaxf(oy, ey),
                          fminf(oz, ez), fmaxf(oz, ez)};
            for (int k = 0; k < 6; ++k) f[k] = (k & 1) ? wave_max(f[k]) : wave_min(f[k]);
            for (int guard = 0; guard < 64; ++guard) {
                const Node& N = a.terrain_nodes[entry];
                cnt.node();
                const bool o0 = N.b0[0] <= f[1] && N.b0[1] >= f[0] && N.b0[2] <= f[3] &&
                                N.b0[3] >= f[2] && N.b0[4] <= f[5] && N.b0[5] >= f[4];
                const bool o1 = N.b1[0] <= f[1] && N.b1[1] >= f[0] && N.b1[2] <= f[3] &&
                                N.b1[3] >= f[2] && N.b1[4] <= f[5] && N.b1[5] >= f[4];
                if (o0 && o1) break;
                if (!o0 && !o1) { reach = false; break; }
                const int c = o0 ? N.c0 : N.c1;
                if (c < 0 || c >= a.n_terrain - 1) break;
                entry = c;
            }
        }
        if (reach) {
            const Slab ws = make_slab(ox, oy, oz, dx, dy, dz);
            const Shear wm = make_shear(dx, dy, dz);
            const int n_nodes = a.n_terrain > 1 ? a.n_terrain - 1 : 1;
            auto leaf = [&](int i) {
                cnt.tri();
                tri_test<EXACT>(a.terrain_tris + 9 * (int64_t)i, a.terrain_tri_id,
                                (uint32_t)a.n_links, ox, oy, oz, wm, kTerrainKP, px.eo, h, px, -1, i);
            };
            if (!(MODE & kPacketTerrain)) {
                // the fast pass walks the 4-wide records, with the octant's
                // specialised box tests when the wavefront's rays share one
                // direction octant (the common case for a tile); the exact
                // pass's lanes walk the binary records alone
                const int oct = slab_octant(ws);
                const int oct0 = uni(oct);
                if (WAVE && !EXACT && __ballot(oct != oct0) == 0ull) {
                    switch (oct0) {
#define RC_OCT(K) \
    case K:                                                                                      \
        traverse4<K>(a.terrain_wide, n_nodes, a.n_terrain, ws, h, cnt, leaf, entry, stk, a.wide_stack); \
        break;
                        RC_OCT(0) RC_OCT(1) RC_OCT(2) RC_OCT(3) RC_OCT(4) RC_OCT(5) RC_OCT(6) RC_OCT(7)
#undef RC_OCT
                    }
                } else if (WAVE && !EXACT) {
                    traverse4<-1>(a.terrain_wide, n_nodes, a.n_terrain, ws, h, cnt, leaf, entry, stk,
                                  a.wide_stack);
                } else if (EXACT && stk) {
                    traverse4<-1>(a.terrain_wide, n_nodes, a.n_terrain, ws, h, cnt, leaf, entry, stk,
                                  kExactStack);
                } else {
                    traverse(a.terrain_nodes, n_nodes, a.n_terrain, ws, h, cnt, leaf, entry, stk);
                }
            } else {
                // Packet form: the wavefront walks the terrain hierarchy together
                // (node index, trail and records wave-uniform); a child is
                // entered if any lane's ray reaches it within that lane's bound,
                // the nearer child first by vote.
                uint64_t trail = 0;
                int cur = entry;
                int budget = 2 * n_nodes + 2;
                for (;;) {
                    cur = uni(cur);
                    if ((unsigned)cur >= (unsigned)n_nodes || --budget < 0) break;
                    const Node N = a.terrain_nodes[cur];
                    cnt.node();
                    float tn0, tn1;
                    bool h0 = slab(N.b0[0], N.b0[1], N.b0[2], N.b0[3], N.b0[4], N.b0[5], ws, h.tmax, tn0);
                    bool h1 = slab(N.b1[0], N.b1[1], N.b1[2], N.b1[3], N.b1[4], N.b1[5], ws, h.tmax, tn1);
                    const int c0 = N.c0, c1 = N.c1;
                    h0 = h0 && (c0 >= 0 || (unsigned)~c0 < (unsigned)a.n_terrain);
                    h1 = h1 && (c1 >= 0 || (unsigned)~c1 < (unsigned)a.n_terrain);
                    const bool l0 = h0 && c0 < 0, l1 = h1 && c1 < 0;
                    if (l0 || l1) {  // leaf children, nearest first
                        const bool swap = l0 && l1 && tn1 < tn0;
                        const int la = (l0 && !swap) ? ~c0 : ~c1;
                        const int lb = (l0 && l1) ? (swap ? ~c0 : ~c1) : -1;
                        const float tb = swap ? tn0 : tn1;
                        leaf(la);
                        if (lb >= 0 && tb <= h.tmax) leaf(lb);
                    }
                    const bool g0 = c0 >= 0 && h0 && tn0 <= h.tmax;
                    const bool g1 = c1 >= 0 && h1 && tn1 <= h.tmax;
                    const uint64_t G0 = __ballot(g0), G1 = __ballot(g1);
                    if (G0 && G1) {
                        const int want1 = __popcll(__ballot(g1 && (!g0 || tn1 < tn0)));
                        const int want0 = __popcll(__ballot(g0 && (!g1 || tn0 <= tn1)));
                        trail = (trail << 1) | 1ull;
                        cur = want1 > want0 ? c1 : c0;
                        continue;
                    }
                    if (G0 || G1) {
                        trail <<= 1;
                        cur = G0 ? c0 : c1;
                        continue;
                    }
                    int par = N.parent, sib = N.sibling;
                    bool done = false;
                    for (;;) {
                        if (trail == 0ull) { done = true; break; }
                        if (trail & 1ull) { trail ^= 1ull; cur = sib; break; }
                        trail >>= 1;
                        par = uni(par);
                        if ((unsigned)par >= (unsigned)n_nodes || --budget < 0) { done = true; break; }
                        sib = a.terrain_nodes[par].sibling;
                        par = a.terrain_nodes[par].parent;
                    }
                    if (done) break;
                }
            }
        }
    }
    return h;
}

// Output of one ray: planar depth is the ray parameter; range depth scales it
// by |K^-1 [x + .5, y + .5, 1]| (recomputed here rather than kept live).
__device__ __forceinline__ void write_out(const RenderLaunch& a, int64_t p, const Hit& h,
                                          const CamRef& cam, int x, int y) {
    const bool hit = h.key != ~0ull;
    float depth = h.tmax;
    if (a.depth_mode == RC_DEPTH_RANGE) {
        const double rx = ((double)x + 0.5 - cam.b[14]) * cam.b[12];
        const double ry = ((double)y + 0.5 - cam.b[15]) * cam.b[13];
        depth = (float)((double)h.tmax * sqrt(rx * rx + ry * ry + 1.0));
    }
    a.depth[p] = hit ? depth : a.far_plane;
    if (a.inst) a.inst[p] = hit ? (int32_t)(h.key >> 32) : -1;
    if (a.tri) a.tri[p] = hit ? (int32_t)(uint32_t)h.key : -1;
}

// Camera `index` of the launch: (env * n_cam + cam) in the plain form, the
// descriptor's index in the batched form.
__device__ __forceinline__ CamRef launch_cam(const RenderLaunch& a, int64_t index) {
    return CamRef{a.cam_basis + kCamBasis * index};
}

// Perception randomisation of one camera basis b (the draws and the rules are
// stated with rc_cam_rand): offset = a (2u - 1), u = (w >> 8) 2^-24.
__device__ __forceinline__ double rand_offset(uint32_t w, float half) {
    return (double)half * (2.0 * ((double)(w >> 8) * 5.9604644775390625e-08) - 1.0);
}

__device__ void cam_randomize(const rc_cam_rand& p, uint32_t uid, double* b) {
    const uint32_t k0 = (uint32_t)p.seed, k1 = (uint32_t)(p.seed >> 32);
    const uint32_t e_lo = (uint32_t)p.epoch, e_hi = (uint32_t)((p.epoch >> 32) & 0xFFFFull) << 16;
    const uint4 w2 = philox4x32_10(make_uint4(uid, 0xFFFFFFFEu, e_lo, e_hi | 2u), k0, k1);
    const uint4 w3 = philox4x32_10(make_uint4(uid, 0xFFFFFFFEu, e_lo, e_hi | 3u), k0, k1);
    const double t[3] = {rand_offset(w2.x, p.trans_m[0]), rand_offset(w2.y, p.trans_m[1]),
                         rand_offset(w2.z, p.trans_m[2])};
    const double deg = 3.14159265358979323846 / 180.0;
    const double ph = rand_offset(w2.w, p.euler_deg[0]) * deg;
    const double th = rand_offset(w3.x, p.euler_deg[1]) * deg;
    const double ps = rand_offset(w3.y, p.euler_deg[2]) * deg;
    // translation in the camera's own frame
    for (int r = 0; r < 3; ++r) b[9 + r] += b[3 * r] * t[0] + b[3 * r + 1] * t[1] + b[3 * r + 2] * t[2];
    // R Rx(ph) Ry(th) Rz(ps)
    const double cx = cos(ph), sx = sin(ph), cy = cos(th), sy = sin(th), cz = cos(ps), sz = sin(ps);
    const double M[9] = {cy * cz, -cy * sz, sy,
                         sx * sy * cz + cx * sz, -sx * sy * sz + cx * cz, -sx * cy,
                         -cx * sy * cz + sx * sz, cx * sy * sz + sx * cz, cx * cy};
    double R[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            R[3 * r + c] = b[3 * r] * M[c] + b[3 * r + 1] * M[3 + c] + b[3 * r + 2] * M[6 + c];
    for (int k = 0; k < 9; ++k) b[k] = R[k];
    if (p.dfov_deg != 0.0f) {  // both axes: f' = c / tan(atan(c / f) + dfov / 2)
        const double half = 0.5 * rand_offset(w3.z, p.dfov_deg) * deg;
        const double fx = 1.0 / b[12], fy = 1.0 / b[13];
        b[12] = tan(atan(b[14] / fx) + half) / b[14];
        b[13] = tan(atan(b[15] / fy) + half) / b[15];
    }
}

// Ray bases of every camera of the launch (randomised when asked); `zero`:
// the exact-pass counters to reset first (plain form), or NULL.
__global__ void k_cam_prep(RenderLaunch a, int64_t n, uint32_t* zero) {
    if (zero && blockIdx.x == 0 && threadIdx.x == 0) zero[0] = zero[1] = 0u;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double* b = a.cam_basis + kCamBasis * i;
        uint32_t uid;
        if (a.desc) {
            const rc_cam_desc& D = a.desc[i];
            cam_basis(D.pos, D.quat, D.intr, b);
            uid = D.cam_uid;
        } else {
            cam_basis(a.cam_pos + 3 * i, a.cam_quat + 4 * i, a.intr + 4 * i, b);
            uid = (uint32_t)i;
        }
        if (a.cam_rand_on) cam_randomize(a.cam_rand, uid, b);
    }
}

// Cast the rpl stacked tw x th sub-tiles of one wavefront tile of an image
// (width x height, env e, camera `cam`, output pixels from `out0`); lanes
// past the image edge trace a copy of an edge pixel (so wave-wide reductions
// see only real rays) and write nothing.  Rays whose closest hit could hinge
// on FP32-undecided triangles go to the exact pass: with the certain hit
// found here and the (at most two) undecided triangles to decide in FP64 at
// the front of its list, or, with more, to be re-cast in full (from the back
// of the list, starting from the certain hit's bound).
template <int RPL, int MODE, typename Cnt = NoCount>
__device__ __forceinline__ void cast_tile(const RenderLaunch& a, const TileCfg& c, const CamRef& cam,
                                          int e, uint32_t cam_index, int width, int height,
                                          int64_t out0, int tx, int ty) {
    const int lane = threadIdx.x & 63;
    const int span_h = c.th * RPL;
    const int xt = tx * c.tw + (lane % c.tw);
    __shared__ uint2 s_cand[kLanes * kCandSlots];
    __shared__ uint32_t s_stack[kLanes * kStack];
    uint2* cand = s_cand + kCandSlots * threadIdx.x;
    uint32_t* stk = s_stack + threadIdx.x;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int y0 = ty * span_h + r * c.th;
        if (y0 >= height) break;  // wave-uniform
        const int yt = y0 + lane / c.tw;
        const bool valid = xt < width && yt < height;
        const int x = xt < width ? xt : width - 1;
        const int y = yt < height ? yt : height - 1;
        Cnt cnt;
        for (int k = 0; k < kCandSlots; ++k) cand[k].x = kNoCand;
        const Hit h = cast_ray<false, true, MODE>(a, cam, e, x, y, INFINITY, cand, stk, cnt);
        if (!valid) continue;
        const int64_t p = out0 + (int64_t)y * width + x;
        write_out(a, p, h, cam, x, y);
        if constexpr (Cnt::kOn)
            reinterpret_cast<uint4*>(a.counts)[p] = make_uint4(cnt.n, cnt.t, cnt.i, cnt.l);
        const float lim = h.tmax * kUndecidedSlack;
        const uint4 head = make_uint4((uint32_t)p, cam_index, (uint32_t)x | ((uint32_t)y << 16),
                                      __float_as_uint(h.tmax));
        if (h.tu <= lim) {  // re-cast in full
            const uint32_t slot = atomicAdd(a.exact_count + 1, 1u);
            if ((int64_t)slot < a.exact_cap) a.exact_list[2 * (a.exact_cap - 1 - slot)] = head;
        } else {
            const uint2 c0 = cand[0], c1 = cand[1];
            const uint32_t i0 = (c0.x != kNoCand && __uint_as_float(c0.y) <= lim) ? c0.x : kNoCand;
            const uint32_t i1 = (c1.x != kNoCand && __uint_as_float(c1.y) <= lim) ? c1.x : kNoCand;
            if (i0 != kNoCand || i1 != kNoCand) {
                const uint32_t slot = atomicAdd(a.exact_count, 1u);
                if ((int64_t)slot < a.exact_cap) {
                    a.exact_list[2 * (int64_t)slot] = head;
                    a.exact_list[2 * (int64_t)slot + 1] =
                        make_uint4((uint32_t)h.key, (uint32_t)(h.key >> 32), i0, i1);
                }
            }
        }
    }
}

// Fast pass over the plain [env][cam][H][W] layout, one wavefront tile.
// XCD-aware order: hardware deals blocks round-robin over the 8 XCDs.  The
// logical tiles go out in chunks of kXcdChunk consecutive tiles, chunk g to
// XCD g mod 8, so neighbouring environments share terrain nodes in one XCD's
// L2 while every XCD keeps a share of the whole launch to its end (192 tiles,
// two environments' four 64x48 images: 2% faster than one contiguous run per
// XCD; 24 tiles lose the L2 reuse).  Block bid of a grid of 8 * xcd_blocks(n)
// blocks maps to logical tile xcd_logical(bid); those >= n do nothing.
constexpr int64_t kXcdChunk = 192;

__device__ __forceinline__ int64_t xcd_logical(int64_t bid) {
    const int64_t j = bid >> 3;
    return ((j / kXcdChunk) * 8 + (bid & 7)) * kXcdChunk + (j % kXcdChunk);
}

inline int64_t xcd_blocks(int64_t n_logical) {
    return ((n_logical + 7) / 8 + kXcdChunk - 1) / kXcdChunk * kXcdChunk;
}

template <int RPL, int MODE, typename Cnt>
__device__ __forceinline__ void plain_tile(const RenderLaunch& a, const TileCfg& c, int64_t n_logical,
                                           int64_t per_xcd) {
    const int64_t lb = xcd_logical(blockIdx.x);
    if (lb >= n_logical) return;
    const int64_t tile = (int64_t)uni((int)(lb * kWavesPerBlock)) + uni(threadIdx.x >> 6);
    const int span_h = c.th * c.rpl;
    const int tiles_x = (a.width + c.tw - 1) / c.tw;
    const int tiles_y = (a.height + span_h - 1) / span_h;
    const int64_t tiles_img = (int64_t)tiles_x * tiles_y;
    const int64_t ec = tile / tiles_img;
    if (ec >= (int64_t)a.n_env * a.n_cam) return;
    const int tin = (int)(tile - ec * tiles_img);
    cast_tile<RPL, MODE, Cnt>(a, c, launch_cam(a, ec), (int)(ec / a.n_cam), (uint32_t)ec, a.width, a.height,
                        ec * (int64_t)a.width * a.height, tin % tiles_x, tin / tiles_x);
}

// Fast pass.  WAVES asks the compiler for at least that many resident
// wavefronts per SIMD (fewer registers per lane, maybe a few spills); MODE
// selects the body culling and terrain walk variants.  The autotuner picks
// them and the tile schedule.
template <int WAVES, int RPL, int MODE>
__global__ void __launch_bounds__(64 * kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(WAVES, 8)))
k_render(RenderLaunch a, TileCfg c, int64_t n_logical, int64_t per_xcd) {
    plain_tile<RPL, MODE, NoCount>(a, c, n_logical, per_xcd);
}

// The fast pass with per-ray work counters (diagnostic render).
template <int MODE>
__global__ void __launch_bounds__(64 * kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(6, 8)))
k_render_counts(RenderLaunch a, TileCfg c, int64_t n_logical, int64_t per_xcd) {
    plain_tile<1, MODE, RayCount>(a, c, n_logical, per_xcd);
}

// Batched uneven form, setup: validate each camera descriptor, count its
// tiles, prefix-sum them (one block) and reset the work counter, the exact
// list and the status word.  An invalid descriptor gets no tiles and sets
// bit 0 of *status.
__global__ void __launch_bounds__(1024) k_batch_prep(RenderLaunch a, TileCfg c, uint32_t* tile_start,
                                                     uint32_t* queues, uint32_t* status) {
    __shared__ uint32_t sums[1024];
    if (threadIdx.x == 0) *status = 0u;
    const int n = a.n_desc;
    const int chunk = (n + 1023) / 1024;
    const int b = threadIdx.x * chunk, e = min(b + chunk, n);
    uint32_t local = 0;
    bool bad = false;
    for (int d = b; d < e; ++d) {
        const rc_cam_desc& D = a.desc[d];
        const bool ok = D.env >= 0 && D.env < a.n_env && D.width >= 1 && D.height >= 1 &&
                        D.width <= a.max_width && D.height <= a.max_height &&
                        (int64_t)D.out_offset + (int64_t)D.width * D.height <= a.n_pixels;
        bad |= !ok;
        const int span_h = c.th * c.rpl;
        local += ok ? (uint32_t)(((D.width + c.tw - 1) / c.tw) * ((D.height + span_h - 1) / span_h)) : 0u;
    }
    sums[threadIdx.x] = local;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t add = threadIdx.x >= (unsigned)off ? sums[threadIdx.x - off] : 0u;
        __syncthreads();
        sums[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = sums[threadIdx.x] - local;
    for (int d = b; d < e; ++d) {
        tile_start[d] = run;
        const rc_cam_desc& D = a.desc[d];
        const bool ok = D.env >= 0 && D.env < a.n_env && D.width >= 1 && D.height >= 1 &&
                        D.width <= a.max_width && D.height <= a.max_height &&
                        (int64_t)D.out_offset + (int64_t)D.width * D.height <= a.n_pixels;
        const int span_h = c.th * c.rpl;
        run += ok ? (uint32_t)(((D.width + c.tw - 1) / c.tw) * ((D.height + span_h - 1) / span_h)) : 0u;
    }
    if (threadIdx.x == 1023) tile_start[n] = sums[1023];
    if (threadIdx.x == 0) queues[0] = 0u;
    if (threadIdx.x == 0) a.exact_count[0] = a.exact_count[1] = 0u;
    if (bad) atomicOr(status, 1u);
}

// Batched uneven form: one persistent launch.  Each wavefront takes chunks
// of kChunk consecutive tiles from one work counter (consecutive tiles are
// neighbouring pixels of one camera, so a chunk's rays share cache lines on
// the XCD that runs it) until the tiles run out; the tile table maps a tile
// to its camera descriptor by binary search.
template <int WAVES, int RPL, int MODE>
__global__ void __launch_bounds__(64 * kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(WAVES, 8)))
k_render_batched(RenderLaunch a, TileCfg c, const uint32_t* __restrict__ tile_start,
                 uint32_t* queue) {
    const int lane = threadIdx.x & 63;
    const uint32_t n_tiles = tile_start[a.n_desc];
    for (;;) {
        uint32_t t0 = 0;
        if (lane == 0) t0 = atomicAdd(queue, (uint32_t)kChunk);
        t0 = (uint32_t)uni((int)__shfl(t0, 0, 64));
        if (t0 >= n_tiles) break;
        const uint32_t t1 = min(t0 + (uint32_t)kChunk, n_tiles);
        for (uint32_t tile = t0; tile < t1; ++tile) {
            // the descriptor owning this tile: last d with tile_start[d] <= tile
            int lo = 0, hi = a.n_desc - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (tile_start[mid] <= tile) lo = mid; else hi = mid - 1;
            }
            const int d = uni(lo);
            const rc_cam_desc* D = a.desc + d;
            const int width = D->width;
            const int tiles_x = (width + c.tw - 1) / c.tw;
            const int tin = (int)(tile - tile_start[d]);
            cast_tile<RPL, MODE>(a, c, launch_cam(a, d), D->env, (uint32_t)d, width, D->height,
                                   (int64_t)D->out_offset, tin % tiles_x, tin / tiles_x);
        }
    }
}

// Batched uneven form, flat launch: wavefront (camera d, tile k) of a
// camera-major grid sized for the largest image; tiles past a camera's own
// count exit at once.  No loop around the tile, so no state is carried
// between tiles (the persistent form's loop costs registers).
template <int WAVES, int RPL, int MODE>
__global__ void __launch_bounds__(64 * kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(WAVES, 8)))
k_render_flat(RenderLaunch a, TileCfg c, const uint32_t* __restrict__ tile_start, int tiles_per_cam,
              int64_t n_logical, int64_t per_xcd) {
    const int64_t lb = xcd_logical(blockIdx.x);
    if (lb >= n_logical) return;
    const int64_t w = (int64_t)uni((int)(lb * kWavesPerBlock)) + uni(threadIdx.x >> 6);
    const int d = (int)(w / tiles_per_cam);
    const int k = (int)(w - (int64_t)d * tiles_per_cam);
    if (d >= a.n_desc) return;
    const uint32_t n_own = tile_start[d + 1] - tile_start[d];  // 0 for an invalid descriptor
    if ((uint32_t)k >= n_own) return;
    const rc_cam_desc* D = a.desc + d;
    const int width = D->width;
    const int tiles_x = (width + c.tw - 1) / c.tw;
    cast_tile<RPL, MODE>(a, c, launch_cam(a, d), D->env, (uint32_t)d, width, D->height,
                         (int64_t)D->out_offset, k % tiles_x, k / tiles_x);
}

// Exact pass.  If the list overflowed, every pixel is re-cast.
__device__ __forceinline__ void entry_cam(const RenderLaunch& a, uint32_t cam_index, CamRef& cam,
                                          int& e) {
    if (a.desc) {
        const rc_cam_desc* D = a.desc + cam_index;
        cam = launch_cam(a, cam_index);
        e = D->env;
    } else {
        cam = launch_cam(a, cam_index);
        e = (int)(cam_index / (uint32_t)a.n_cam);
    }
}

// Full re-cast of one ray with FP64 decisions for undecided triangles.
__device__ __forceinline__ void exact_one(const RenderLaunch& a, int64_t p, uint32_t cam_index, int x,
                                          int y, float bound, uint32_t* stk) {
    CamRef cam;
    int e;
    entry_cam(a, cam_index, cam, e);
    NoCount none;
    const Hit h = cast_ray<true, false, 0>(a, cam, e, x, y, bound, nullptr, stk, none);
    write_out(a, p, h, cam, x, y);
}

// Decide a listed ray's undecided triangles in FP64 and merge them with the
// fast pass's certain hit (same order as the traversal: ray parameter, then
// (inst, tri)).
__device__ __forceinline__ void resolve_one(const RenderLaunch& a, const uint4 head, const uint4 rest) {
    CamRef cam;
    int e;
    entry_cam(a, head.y, cam, e);
    const int x = (int)(head.z & 0xFFFFu), y = (int)(head.z >> 16);
    Hit h;
    h.tmax = __uint_as_float(head.w);
    h.key = ((uint64_t)rest.y << 32) | rest.x;
    h.tu = INFINITY;
    for (int k = 0; k < kCandSlots; ++k) {
        const uint32_t id = k == 0 ? rest.z : rest.w;
        if (id == kNoCand) continue;
        const int link = (int)(id >> kLeafBits) - 1;
        const int leaf = (int)(id & ((1u << kLeafBits) - 1u));
        const float* v;
        int32_t tri_id;
        uint32_t inst;
        if (link < 0) {
            if (leaf >= a.n_terrain) continue;
            v = a.terrain_tris + 9 * (int64_t)leaf;
            tri_id = a.terrain_tri_id[leaf];
            inst = (uint32_t)a.n_links;
        } else {
            if (link >= a.n_links) continue;
            const LinkMeta M = a.link_meta[link];
            if (leaf >= M.n_tri) continue;
            v = a.link_tris + M.tri_base + 9 * (int64_t)leaf;
            tri_id = a.link_tri_id[M.id_base + leaf];
            inst = (uint32_t)link;
        }
        double t64;
        if (!refine(v, cam.b, x, y, link, e, a.n_links, a.link_pos,
                    a.link_quat, &t64))
            continue;
        const float t = (float)t64;
        if (!(t > 0.0f) || t > h.tmax) continue;
        const uint64_t key = ((uint64_t)inst << 32) | (uint32_t)tri_id;
        if (t < h.tmax || key < h.key) {
            h.tmax = t;
            h.key = key;
        }
    }
    write_out(a, head.x, h, cam, x, y);
}


static_assert(kLanes == 64, "the exact pass indexes its stack with a 64-lane stride");
__global__ void __launch_bounds__(64) k_render_exact(RenderLaunch a, const uint32_t* tile_start) {
    __shared__ uint32_t s_xstack[64 * kExactStack];
    uint32_t* stk = s_xstack + threadIdx.x;
    const uint32_t n_res = a.exact_count[0], n_full = a.exact_count[1];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((int64_t)n_res + n_full <= a.exact_cap) {
        for (int64_t i = gid; i < (int64_t)n_res; i += stride)
            resolve_one(a, a.exact_list[2 * i], a.exact_list[2 * i + 1]);
        // full re-casts: one ray per wavefront, so no wavefront waits on the
        // slowest of many divergent traversals
        if ((threadIdx.x & 63) == 0) {
            for (int64_t j = gid >> 6; j < (int64_t)n_full; j += stride >> 6) {
                const uint4 it = a.exact_list[2 * (a.exact_cap - 1 - j)];
                exact_one(a, it.x, it.y, (int)(it.z & 0xFFFFu), (int)(it.z >> 16),
                          __uint_as_float(it.w), stk);
            }
        }
        return;
    }
    // overflow: re-cast every pixel exactly
    if (!a.desc) {
        const int64_t hw = (int64_t)a.width * a.height;
        for (int64_t p = gid; p < a.n_pixels; p += stride) {
            const int64_t ec = p / hw;
            const int pin = (int)(p - ec * hw);
            exact_one(a, p, (uint32_t)ec, pin % a.width, pin / a.width, INFINITY, stk);
        }
    } else {
        for (int d = 0; d < a.n_desc; ++d) {
            const rc_cam_desc& D = a.desc[d];
            if (tile_start[d + 1] == tile_start[d]) continue;  // invalid descriptor
            const int64_t np = (int64_t)D.width * D.height;
            for (int64_t q = gid; q < np; q += stride)
                exact_one(a, (int64_t)D.out_offset + q, (uint32_t)d, (int)(q % D.width),
                          (int)(q / D.width), INFINITY, stk);
        }
    }
}

// Privileged height map (the terrain experts' local grid, Sec. 3.1): one
// vertical ray per grid point, from base_z + top down to `depth`, against the
// terrain hierarchy (its 4-wide records); every triangle test is the FP64
// watertight test (closed triangles), so a point on a shared edge or vertex
// finds its surface.
__global__ void __launch_bounds__(kLanes) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_heightmap(HeightLaunch hl) {
    __shared__ uint32_t s_stack[kLanes * kStack];
    const int64_t n = (int64_t)hl.n_env * hl.nx * hl.ny;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const int e = (int)(q / ((int64_t)hl.nx * hl.ny));
        const int j = (int)((q / hl.nx) % hl.ny), i = (int)(q % hl.nx);
        const double gx = (i - 0.5 * (hl.nx - 1)) * (double)hl.dx;
        const double gy = (j - 0.5 * (hl.ny - 1)) * (double)hl.dy;
        const double c = cos((double)hl.base_yaw[e]), s = sin((double)hl.base_yaw[e]);
        const double o64[3] = {(double)hl.base_pos[3 * e] + c * gx - s * gy,
                               (double)hl.base_pos[3 * e + 1] + s * gx + c * gy,
                               (double)hl.base_pos[3 * e + 2] + (double)hl.top};
        const double d64[3] = {0.0, 0.0, -1.0};
        Slab r;  // vertical form: the FP32 origin only
        r.ix = r.iy = r.iz = 0.0f;
        r.oix = (float)o64[0];
        r.oiy = (float)o64[1];
        r.oiz = (float)o64[2];
        Hit h;
        h.tmax = hl.depth;
        h.key = ~0ull;
        h.tu = INFINITY;
        double best = INFINITY;
        NoCount none;
        auto leaf = [&](int leaf) {
            const float* v = hl.tris + 9 * (int64_t)leaf;
            double t;
            if (tri_test64(v, o64, d64, t) && t <= (double)hl.depth && t < best) {
                best = t;
                // the FP32 bound must not cut below the FP64 hit
                h.tmax = nextafterf((float)t, INFINITY);
            }
        };
        const int n_int = hl.n_prim > 1 ? hl.n_prim - 1 : 1;
        traverse4<-1, true>(hl.wide, n_int, hl.n_prim, r, h, none, leaf, 0, s_stack + threadIdx.x,
                            hl.wide_stack);
        // a dropped push (full stack) left subtrees unvisited: walk the binary
        // records, whose trail has no such limit, for that column (the hits
        // found so far stand; the bound only prunes)
        if (h.tu == 0.0f)
            traverse<-1, true>(hl.nodes, n_int, hl.n_prim, r, h, none, leaf, 0, s_stack + threadIdx.x);
        hl.heights[q] = best < INFINITY ? (float)((double)hl.top - best) : hl.miss;
    }
}

}  // namespace

hipError_t launch_heightmap(const HeightLaunch& hl, hipStream_t s) {
    const int64_t n = (int64_t)hl.n_env * hl.nx * hl.ny;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + kLanes - 1) / kLanes, 65535);
    hipLaunchKernelGGL(k_heightmap, dim3(blocks), dim3(kLanes), 0, s, hl);
    return hipGetLastError();
}

// Kernel variant index: 100 * mode + 10 * waves + tiles per wavefront.
#define RC_MODE_VARIANTS(X, M) X(6, 1, M) X(6, 2, M) X(7, 1, M) X(7, 2, M) X(8, 1, M) X(8, 2, M)
#define RC_VARIANTS(X) \
    RC_MODE_VARIANTS(X, 0) RC_MODE_VARIANTS(X, 1) RC_MODE_VARIANTS(X, 2) RC_MODE_VARIANTS(X, 3)

static int cfg_mode(const RenderCfg& cfg) {
    return (cfg.terrain_packet ? kPacketTerrain : 0) | (cfg.bodies_flat ? kFlatBodies : 0);
}
static int variant(const RenderCfg& cfg, int rpl) {
    return 100 * cfg_mode(cfg) + 10 * cfg.waves + rpl;
}

hipError_t launch_render(const RenderLaunch& a, const RenderCfg& cfg, hipStream_t s) {
    // the counting variant casts one tile per wavefront
    TileCfg c{cfg.tile_w, cfg.tile_h, a.counts ? 1 : cfg.rays_per_lane};
    const int span_h = c.th * c.rpl;
    const int tiles_x = (a.width + c.tw - 1) / c.tw;
    const int tiles_y = (a.height + span_h - 1) / span_h;
    const int64_t tiles = (int64_t)a.n_env * a.n_cam * tiles_x * tiles_y;
    const int64_t n_logical = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t per_xcd = xcd_blocks(n_logical);
    const dim3 grid((unsigned)(per_xcd * 8)), block(64 * kWavesPerBlock);
    const int64_t n_cams = (int64_t)a.n_env * a.n_cam;
    // one camera per lane, 64-lane blocks: a short FP64 chain per camera, so
    // spread the cameras over many compute units; it also resets the exact-pass
    // counters
    hipLaunchKernelGGL(k_cam_prep, dim3((unsigned)std::min<int64_t>((n_cams + 63) / 64, 16384)),
                       dim3(64), 0, s, a, n_cams, a.exact_count);
    if (a.ev_begin) hipEventRecord(a.ev_begin, s);
    if (a.counts) {
        switch (cfg_mode(cfg)) {
#define RC_COUNT(M)                                                                             \
    case M:                                                                                    \
        hipLaunchKernelGGL((k_render_counts<M>), grid, block, 0, s, a, c, n_logical, per_xcd); \
        break;
            RC_COUNT(0) RC_COUNT(1) RC_COUNT(2) RC_COUNT(3)
#undef RC_COUNT
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (variant(cfg, c.rpl)) {
#define RC_PLAIN(W, R, P)                                                                      \
    case 100 * P + 10 * W + R:                                                      \
        hipLaunchKernelGGL((k_render<W, R, P>), grid, block, 0, s, a, c, n_logical, per_xcd); \
        break;
            RC_VARIANTS(RC_PLAIN)
#undef RC_PLAIN
            default: return hipErrorInvalidValue;
        }
    }
    if (a.ev_end) hipEventRecord(a.ev_end, s);
    hipLaunchKernelGGL(k_render_exact, dim3(4096), dim3(64), 0, s, a, (const uint32_t*)nullptr);
    return hipGetLastError();
}

hipError_t launch_render_batched(const RenderLaunch& a, const RenderCfg& cfg, uint32_t* tile_start,
                                 uint32_t* queues, uint32_t* status, int persistent_blocks,
                                 hipStream_t s) {
    TileCfg c{cfg.tile_w, cfg.tile_h, cfg.rays_per_lane};
    hipLaunchKernelGGL(k_batch_prep, dim3(1), dim3(1024), 0, s, a, c, tile_start, queues, status);
    hipLaunchKernelGGL(k_cam_prep, dim3((unsigned)std::min<int64_t>((a.n_desc + 63) / 64, 16384)),
                       dim3(64), 0, s, a, (int64_t)a.n_desc, (uint32_t*)nullptr);
    if (a.ev_begin) hipEventRecord(a.ev_begin, s);
    const dim3 block(64 * kWavesPerBlock);
    if (cfg.persistent) {
        const dim3 grid((unsigned)persistent_blocks);
        switch (variant(cfg, c.rpl)) {
#define RC_BATCH(W, R, P)                                                                          \
    case 100 * P + 10 * W + R:                                                          \
        hipLaunchKernelGGL((k_render_batched<W, R, P>), grid, block, 0, s, a, c, tile_start, queues); \
        break;
            RC_VARIANTS(RC_BATCH)
#undef RC_BATCH
            default: return hipErrorInvalidValue;
        }
    } else {
        const int span_h = c.th * c.rpl;
        const int tiles_per_cam = ((a.max_width + c.tw - 1) / c.tw) * ((a.max_height + span_h - 1) / span_h);
        const int64_t waves = (int64_t)a.n_desc * tiles_per_cam;
        const int64_t n_logical = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
        const int64_t per_xcd = xcd_blocks(n_logical);
        const dim3 grid((unsigned)(per_xcd * 8));
        switch (variant(cfg, c.rpl)) {
#define RC_FLAT(W, R, P)                                                                         \
    case 100 * P + 10 * W + R:                                                         \
        hipLaunchKernelGGL((k_render_flat<W, R, P>), grid, block, 0, s, a, c,                    \
                           (const uint32_t*)tile_start, tiles_per_cam, n_logical, per_xcd);      \
        break;
            RC_VARIANTS(RC_FLAT)
#undef RC_FLAT
            default: return hipErrorInvalidValue;
        }
    }
    if (a.ev_end) hipEventRecord(a.ev_end, s);
    hipLaunchKernelGGL(k_render_exact, dim3(4096), dim3(64), 0, s, a, (const uint32_t*)tile_start);
    return hipGetLastError();
}

bool render_cfg_ok(const RenderCfg& c) {
    return c.tile_w >= 1 && c.tile_h >= 1 && c.tile_w * c.tile_h == 64 &&
           (c.rays_per_lane == 1 || c.rays_per_lane == 2) &&
           (c.waves == 6 || c.waves == 7 || c.waves == 8) &&
           (c.terrain_packet == 0 || c.terrain_packet == 1) && (c.bodies_flat == 0 || c.bodies_flat == 1) &&
           (c.persistent == 0 || c.persistent == 1);
}

}  // namespace rc
