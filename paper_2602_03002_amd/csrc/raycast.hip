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
#include "rc_internal.h"

#pragma clang fp contract(off)

namespace rc {

namespace {

constexpr int kTile = 8;             // 8 x 8 pixels per wavefront
constexpr int kWavesPerBlock = 4;
constexpr float kEdgeRel = 1.0f / 256.0f;  // FP32 edge decision margin (relative)

struct TRay {
    float ox, oy, oz;     // origin
    float ix, iy, iz;     // 1 / d (components clamped away from 0)
    float oix, oiy, oiz;  // o * (1 / d)
    float m1x, m1y, m1z;  // shear rows: x' = m1 . (v - o), y' = m2 . (v - o),
    float m2x, m2y, m2z;  //              z' = m3 . (v - o)
    float m3x, m3y, m3z;
};

struct Ray64 {  // world ray: o exact (float), d = (dx, dy, dz) + (lx, ly, lz)
    float ox, oy, oz, dx, dy, dz, lx, ly, lz;
};

__device__ __forceinline__ float safe_inv(float d) {
    float a = fabsf(d) < 1e-20f ? copysignf(1e-20f, d) : d;
    return 1.0f / a;
}

__device__ __forceinline__ void make_tray(float ox, float oy, float oz, float dx, float dy,
                                          float dz, TRay& r) {
    r.ox = ox; r.oy = oy; r.oz = oz;
    r.ix = safe_inv(dx); r.iy = safe_inv(dy); r.iz = safe_inv(dz);
    r.oix = ox * r.ix; r.oiy = oy * r.iy; r.oiz = oz * r.iz;
    float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
    int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    float dk = kz == 0 ? dx : (kz == 1 ? dy : dz);
    if (dk < 0.0f) { int t = kx; kx = ky; ky = t; }
    float dkx = kx == 0 ? dx : (kx == 1 ? dy : dz);
    float dky = ky == 0 ? dx : (ky == 1 ? dy : dz);
    float sz = 1.0f / dk;
    float sx = dkx * sz, sy = dky * sz;
    r.m1x = (kx == 0) ? 1.0f : (kz == 0 ? -sx : 0.0f);
    r.m1y = (kx == 1) ? 1.0f : (kz == 1 ? -sx : 0.0f);
    r.m1z = (kx == 2) ? 1.0f : (kz == 2 ? -sx : 0.0f);
    r.m2x = (ky == 0) ? 1.0f : (kz == 0 ? -sy : 0.0f);
    r.m2y = (ky == 1) ? 1.0f : (kz == 1 ? -sy : 0.0f);
    r.m2z = (ky == 2) ? 1.0f : (kz == 2 ? -sy : 0.0f);
    r.m3x = kz == 0 ? sz : 0.0f;
    r.m3y = kz == 1 ? sz : 0.0f;
    r.m3z = kz == 2 ? sz : 0.0f;
}

// Slab test of one box (lo.x, hi.x, lo.y, hi.y, lo.z, hi.z) over (0, tmax].
__device__ __forceinline__ bool slab(float lx, float hx, float ly, float hy, float lz, float hz,
                                     const TRay& r, float tmax, float& tn) {
    float tx0 = __fmaf_rn(lx, r.ix, -r.oix), tx1 = __fmaf_rn(hx, r.ix, -r.oix);
    float ty0 = __fmaf_rn(ly, r.iy, -r.oiy), ty1 = __fmaf_rn(hy, r.iy, -r.oiy);
    float tz0 = __fmaf_rn(lz, r.iz, -r.oiz), tz1 = __fmaf_rn(hz, r.iz, -r.oiz);
    float a = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
    float b = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), tmax));
    tn = a;
    return a <= b;
}

// FP64 watertight test of one triangle against an FP64 ray; closed triangle,
// both sides; returns whether it is hit at t > 0 and sets t.
__device__ __noinline__ bool tri_test64(const float* __restrict__ v, double ox, double oy, double oz,
                                        double dx, double dy, double dz, double& t) {
    double ax = fabs(dx), ay = fabs(dy), az = fabs(dz);
    int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    double d[3] = {dx, dy, dz};
    if (d[kz] < 0.0) { int s = kx; kx = ky; ky = s; }
    double sz = 1.0 / d[kz];
    double sx = d[kx] * sz, sy = d[ky] * sz;
    double o[3] = {ox, oy, oz};
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

// FP64 ray of `link` in env `e` (or the world ray for link < 0).
__device__ __noinline__ bool refine(const float* __restrict__ v, const Ray64& w, int link, int e,
                                    int n_links, const float* __restrict__ link_pos,
                                    const float* __restrict__ link_quat, double& t) {
    double ox = w.ox, oy = w.oy, oz = w.oz;
    double dx = (double)w.dx + (double)w.lx, dy = (double)w.dy + (double)w.ly,
           dz = (double)w.dz + (double)w.lz;
    if (link >= 0) {
        const int64_t eb = (int64_t)e * n_links + link;
        const float* q = link_quat + 4 * eb;
        const float* p = link_pos + 3 * eb;
        double x = q[0], y = q[1], z = q[2], ww = q[3];
        double n = sqrt(x * x + y * y + z * z + ww * ww);
        x /= n; y /= n; z /= n; ww /= n;
        double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - z * ww), 2 * (x * z + y * ww),
                       2 * (x * y + z * ww), 1 - 2 * (x * x + z * z), 2 * (y * z - x * ww),
                       2 * (x * z - y * ww), 2 * (y * z + x * ww), 1 - 2 * (x * x + y * y)};
        double px = ox - (double)p[0], py = oy - (double)p[1], pz = oz - (double)p[2];
        double lox = R[0] * px + R[3] * py + R[6] * pz;
        double loy = R[1] * px + R[4] * py + R[7] * pz;
        double loz = R[2] * px + R[5] * py + R[8] * pz;
        double ldx = R[0] * dx + R[3] * dy + R[6] * dz;
        double ldy = R[1] * dx + R[4] * dy + R[7] * dz;
        double ldz = R[2] * dx + R[5] * dy + R[8] * dz;
        return tri_test64(v, lox, loy, loz, ldx, ldy, ldz, t);
    }
    return tri_test64(v, ox, oy, oz, dx, dy, dz, t);
}

struct Hit {
    float tmax;          // current bound = depth parameter of the best hit so far
    uint64_t key;        // (inst << 32) | tri of the best hit, ~0 for none
};

// Test leaf `leaf` of a hierarchy whose leaf-order triangles start at `tris`.
__device__ __forceinline__ void leaf_tri(const float* __restrict__ tris,
                                         const int32_t* __restrict__ ids, int leaf, uint32_t inst,
                                         const TRay& r, Hit& h, const Ray64& w, int link, int e,
                                         int n_links, const float* __restrict__ link_pos,
                                         const float* __restrict__ link_quat) {
    const float* v = tris + 9 * (int64_t)leaf;
    float p0x = v[0] - r.ox, p0y = v[1] - r.oy, p0z = v[2] - r.oz;
    float p1x = v[3] - r.ox, p1y = v[4] - r.oy, p1z = v[5] - r.oz;
    float p2x = v[6] - r.ox, p2y = v[7] - r.oy, p2z = v[8] - r.oz;
    float Ax = __fmaf_rn(r.m1z, p0z, __fmaf_rn(r.m1y, p0y, r.m1x * p0x));
    float Ay = __fmaf_rn(r.m2z, p0z, __fmaf_rn(r.m2y, p0y, r.m2x * p0x));
    float Bx = __fmaf_rn(r.m1z, p1z, __fmaf_rn(r.m1y, p1y, r.m1x * p1x));
    float By = __fmaf_rn(r.m2z, p1z, __fmaf_rn(r.m2y, p1y, r.m2x * p1x));
    float Cx = __fmaf_rn(r.m1z, p2z, __fmaf_rn(r.m1y, p2y, r.m1x * p2x));
    float Cy = __fmaf_rn(r.m2z, p2z, __fmaf_rn(r.m2y, p2y, r.m2x * p2x));
    float U = __fmaf_rn(Cx, By, -(Cy * Bx));
    float V = __fmaf_rn(Ax, Cy, -(Ay * Cx));
    float W = __fmaf_rn(Bx, Ay, -(By * Ax));
    float thr = (fabsf(U) + fabsf(V) + fabsf(W)) * kEdgeRel;
    bool neg = (U < -thr) || (V < -thr) || (W < -thr);
    bool pos = (U > thr) || (V > thr) || (W > thr);
    if (neg && pos) return;  // certain miss
    float t;
    bool sure = !(neg && pos) && ((U >= thr && V >= thr && W >= thr) ||
                                  (U <= -thr && V <= -thr && W <= -thr)) && thr > 0.0f;
    if (sure) {
        float Az = __fmaf_rn(r.m3z, p0z, __fmaf_rn(r.m3y, p0y, r.m3x * p0x));
        float Bz = __fmaf_rn(r.m3z, p1z, __fmaf_rn(r.m3y, p1y, r.m3x * p1x));
        float Cz = __fmaf_rn(r.m3z, p2z, __fmaf_rn(r.m3y, p2y, r.m3x * p2x));
        float det = U + V + W;
        float T = __fmaf_rn(W, Cz, __fmaf_rn(V, Bz, U * Az));
        t = T / det;
    } else {
        double t64;
        if (!refine(v, w, link, e, n_links, link_pos, link_quat, t64)) return;
        t = (float)t64;
    }
    if (!(t > 0.0f) || t > h.tmax) return;
    uint64_t key = ((uint64_t)inst << 32) | (uint32_t)ids[leaf];
    if (t < h.tmax || key < h.key) {
        h.tmax = t;
        h.key = key;
    }
}

// Stackless nearest-first traversal of one hierarchy of n_nodes records and
// n_prim leaves.  `leaf(i)` handles leaf i.  Indices are range-checked and the
// loop is bounded (a valid hierarchy needs fewer than 2 n_nodes + 2 steps),
// so a corrupt hierarchy ends the ray instead of faulting or spinning.
template <typename Leaf>
__device__ __forceinline__ void traverse(const Node* __restrict__ nodes, int n_nodes, int n_prim,
                                         const TRay& r, Hit& h, Leaf&& leaf) {
    uint64_t trail = 0;
    int cur = 0;
    int budget = 2 * n_nodes + 2;
    for (;;) {
        if ((unsigned)cur >= (unsigned)n_nodes || --budget < 0) return;
        const float4* np = reinterpret_cast<const float4*>(nodes + cur);
        float4 q0 = np[0], q1 = np[1], q2 = np[2];
        int4 q3 = reinterpret_cast<const int4*>(np)[3];
        float tn0, tn1;
        bool h0 = slab(q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, r, h.tmax, tn0);
        bool h1 = slab(q1.z, q1.w, q2.x, q2.y, q2.z, q2.w, r, h.tmax, tn1);
        const int c0 = q3.x, c1 = q3.y;
        h0 = h0 && (c0 >= 0 || (unsigned)~c0 < (unsigned)n_prim);
        h1 = h1 && (c1 >= 0 || (unsigned)~c1 < (unsigned)n_prim);
        const bool l0 = h0 && c0 < 0, l1 = h1 && c1 < 0;
        if (l0 || l1) {
            if (l0 && l1) {
                const bool first1 = tn1 < tn0;
                leaf(first1 ? ~c1 : ~c0);
                if ((first1 ? tn0 : tn1) <= h.tmax) leaf(first1 ? ~c0 : ~c1);
            } else {
                leaf(l0 ? ~c0 : ~c1);
            }
        }
        const bool g0 = h0 && !l0 && tn0 <= h.tmax;
        const bool g1 = h1 && !l1 && tn1 <= h.tmax;
        if (g0 && g1) {
            trail = (trail << 1) | 1ull;
            cur = (tn1 < tn0) ? c1 : c0;
            continue;
        }
        if (g0 || g1) {
            trail <<= 1;
            cur = g0 ? c0 : c1;
            continue;
        }
        // backtrack to the deepest level whose other child is pending
        int par = q3.z, sib = q3.w;
        for (;;) {
            if (trail == 0ull) return;
            if (trail & 1ull) {
                trail ^= 1ull;
                cur = sib;
                break;
            }
            trail >>= 1;
            if ((unsigned)par >= (unsigned)n_nodes || --budget < 0) return;
            int4 pq = reinterpret_cast<const int4*>(nodes + par)[3];
            par = pq.z;
            sib = pq.w;
        }
    }
}

__global__ void __launch_bounds__(256) k_render(RenderLaunch a, int64_t n_logical, int64_t per_xcd) {
    // XCD-aware order: hardware deals blocks round-robin over the 8 XCDs, so
    // give each XCD a contiguous run of tiles (neighbouring environments share
    // terrain nodes in that XCD's L2).
    const int64_t bid = blockIdx.x;
    const int64_t lb = (bid & 7) * per_xcd + (bid >> 3);
    if (lb >= n_logical) return;
    const int lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)__builtin_amdgcn_readfirstlane((int)(lb * kWavesPerBlock)) +
                         __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tiles_x = (a.width + kTile - 1) / kTile;
    const int tiles_y = (a.height + kTile - 1) / kTile;
    const int64_t tiles_img = (int64_t)tiles_x * tiles_y;
    const int64_t ec = tile / tiles_img;
    if (ec >= (int64_t)a.n_env * a.n_cam) return;
    const int tin = (int)(tile - ec * tiles_img);
    const int x = (tin % tiles_x) * kTile + (lane & 7);
    const int y = (tin / tiles_x) * kTile + (lane >> 3);
    if (x >= a.width || y >= a.height) return;
    const int e = (int)(ec / a.n_cam);

    // 1. ray generation in FP64
    const float* K = a.intr + 4 * ec;
    const float* qc = a.cam_quat + 4 * ec;
    const float* pc = a.cam_pos + 3 * ec;
    double rx = ((double)x + 0.5 - (double)K[2]) / (double)K[0];
    double ry = ((double)y + 0.5 - (double)K[3]) / (double)K[1];
    double qx = qc[0], qy = qc[1], qz = qc[2], qw = qc[3];
    double qn = sqrt(qx * qx + qy * qy + qz * qz + qw * qw);
    qx /= qn; qy /= qn; qz /= qn; qw /= qn;
    double dx = (1 - 2 * (qy * qy + qz * qz)) * rx + 2 * (qx * qy - qz * qw) * ry + 2 * (qx * qz + qy * qw);
    double dy = 2 * (qx * qy + qz * qw) * rx + (1 - 2 * (qx * qx + qz * qz)) * ry + 2 * (qy * qz - qx * qw);
    double dz = 2 * (qx * qz - qy * qw) * rx + 2 * (qy * qz + qx * qw) * ry + (1 - 2 * (qx * qx + qy * qy));
    Ray64 w;
    w.ox = pc[0]; w.oy = pc[1]; w.oz = pc[2];
    w.dx = (float)dx; w.dy = (float)dy; w.dz = (float)dz;
    w.lx = (float)(dx - (double)w.dx);
    w.ly = (float)(dy - (double)w.dy);
    w.lz = (float)(dz - (double)w.dz);
    const double scale = a.depth_mode == RC_DEPTH_RANGE ? sqrt(rx * rx + ry * ry + 1.0) : 1.0;
    Hit h;
    h.tmax = (float)((double)a.far_plane / scale);
    h.key = ~0ull;

    TRay r;
    // 2. robot bodies through the environment's top-level hierarchy
    if (a.n_links > 0) {
        make_tray(w.ox, w.oy, w.oz, w.dx, w.dy, w.dz, r);
        const int n_rec = a.n_links > 1 ? a.n_links - 1 : 1;
        const Node* tl = a.tlas + (int64_t)e * n_rec;
        traverse(tl, n_rec, a.n_links, r, h, [&](int b) {
            const InstXform X = a.xf[(int64_t)e * a.n_links + b];
            const float px = w.ox - X.t[0], py = w.oy - X.t[1], pz = w.oz - X.t[2];
            const float lox = __fmaf_rn(X.m[2], pz, __fmaf_rn(X.m[1], py, X.m[0] * px));
            const float loy = __fmaf_rn(X.m[5], pz, __fmaf_rn(X.m[4], py, X.m[3] * px));
            const float loz = __fmaf_rn(X.m[8], pz, __fmaf_rn(X.m[7], py, X.m[6] * px));
            const float ldx = __fmaf_rn(X.m[2], w.dz, __fmaf_rn(X.m[1], w.dy, X.m[0] * w.dx));
            const float ldy = __fmaf_rn(X.m[5], w.dz, __fmaf_rn(X.m[4], w.dy, X.m[3] * w.dx));
            const float ldz = __fmaf_rn(X.m[8], w.dz, __fmaf_rn(X.m[7], w.dy, X.m[6] * w.dx));
            TRay lr;
            make_tray(lox, loy, loz, ldx, ldy, ldz, lr);
            const LinkMeta M = a.link_meta[b];
            const float* tris = a.link_tris + M.tri_base;
            const int32_t* ids = a.link_tri_id + M.id_base;
            traverse(a.link_nodes + M.node_base, M.n_tri > 1 ? M.n_tri - 1 : 1, M.n_tri, lr, h,
                     [&](int leafi) {
                leaf_tri(tris, ids, leafi, (uint32_t)b, lr, h, w, b, e, a.n_links, a.link_pos,
                         a.link_quat);
            });
        });
    }
    // 3. terrain under the bound left by the bodies
    make_tray(w.ox, w.oy, w.oz, w.dx, w.dy, w.dz, r);
    traverse(a.terrain_nodes, a.n_terrain > 1 ? a.n_terrain - 1 : 1, a.n_terrain, r, h,
             [&](int leafi) {
        leaf_tri(a.terrain_tris, a.terrain_tri_id, leafi, (uint32_t)a.n_links, r, h, w, -1, e,
                 a.n_links, a.link_pos, a.link_quat);
    });

    // 4. output D[e, c, y, x]
    const int64_t p = ec * (int64_t)a.width * a.height + (int64_t)y * a.width + x;
    const bool hit = h.key != ~0ull;
    a.depth[p] = hit ? (float)((double)h.tmax * scale) : a.far_plane;
    if (a.inst) a.inst[p] = hit ? (int32_t)(h.key >> 32) : -1;
    if (a.tri) a.tri[p] = hit ? (int32_t)(uint32_t)h.key : -1;
}

}  // namespace

hipError_t launch_render(const RenderLaunch& a, hipStream_t s) {
    const int tiles_x = (a.width + kTile - 1) / kTile;
    const int tiles_y = (a.height + kTile - 1) / kTile;
    const int64_t tiles = (int64_t)a.n_env * a.n_cam * tiles_x * tiles_y;
    const int64_t n_logical = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t per_xcd = (n_logical + 7) / 8;
    hipLaunchKernelGGL(k_render, dim3((unsigned)(per_xcd * 8)), dim3(64 * kWavesPerBlock), 0, s, a,
                       n_logical, per_xcd);
    return hipGetLastError();
}

}  // namespace rc
