// Per-environment top-level hierarchy over the robot's link instances,
// rebuilt from the link poses on every render (the poses change each step).
//
// One 64-lane wavefront builds one environment: lane b handles instance b
// (its world box from the link's local root box under (t_b, q_b), the
// transform M = R_b^T used to take rays into the link frame, Sec. 3.2.2, and
// the world bounding sphere the fast pass culls links with);
// the wave ranks the 30-bit Morton codes of the box centres by counting
// (keys broken by instance index), builds the Karras hierarchy from the
// ranked keys, and boxes every internal node as the union of its leaf range.
// Everything stays in LDS; no atomics, so the result is deterministic.
//
// A link whose pose is not finite (or whose quaternion is zero) is absent from
// its environment for this render: its transform places it at
// the far point (identity rotation, t = 1e30) and its instance box and
// sphere (radius 0) are that point, so no ray reaches it; the other links and
// the terrain are unaffected.  When the renderer culls links by their
// bounding spheres (the default schedule) it never walks the top level, and
// only the transforms and spheres are written.
#include "rc_internal.h"

#pragma clang fp contract(off)

namespace rc {

namespace {

constexpr int kWaves = 4;

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    uint32_t x = v & 0x3FFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ __forceinline__ int tdelta(const uint32_t* k, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    uint32_t a = k[i], b = k[j];
    if (a != b) return __clz((int)(a ^ b));
    return 32 + __clz((int)((uint32_t)i ^ (uint32_t)j));
}

__global__ void __launch_bounds__(256)
k_tlas(const float* __restrict__ link_pos, const float* __restrict__ link_quat, int n_env, int B,
       const LinkMeta* __restrict__ meta, Node* __restrict__ tlas, InstXform* __restrict__ xf,
       int with_nodes) {
    __shared__ float sbox[kWaves][kMaxLinks][6];
    __shared__ float nbox[kWaves][kMaxLinks][6];
    __shared__ uint32_t skey[kWaves][kMaxLinks];
    __shared__ int32_t sidx[kWaves][kMaxLinks];
    __shared__ int32_t npar[kWaves][kMaxLinks];
    __shared__ int32_t nsib[kWaves][kMaxLinks];
    __shared__ int32_t nch[kWaves][kMaxLinks][2];

    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int e = blockIdx.x * kWaves + w;
    const bool env_ok = e < n_env;
    const bool inst_ok = env_ok && lane < B;
    const int n_rec = B > 1 ? B - 1 : 1;

    float box[6] = {0, 0, 0, 0, 0, 0};
    float cw[3] = {0, 0, 0};
    bool pose_ok = false;  // an instance with a usable pose
    if (inst_ok) {
        const int64_t eb = (int64_t)e * B + lane;
        const float* q = link_quat + 4 * eb;
        const float* t = link_pos + 3 * eb;
        const double qx = q[0], qy = q[1], qz = q[2], qw = q[3];
        const double nn = sqrt(qx * qx + qy * qy + qz * qz + qw * qw);
        pose_ok = isfinite(t[0]) && isfinite(t[1]) && isfinite(t[2]) && nn > 0.0 && isfinite(nn);
        if (!pose_ok) {
            InstXform X;
            for (int k = 0; k < 9; ++k) X.m[k] = (k % 4 == 0) ? 1.0f : 0.0f;
            X.t[0] = X.t[1] = X.t[2] = kFarBox;
            X.s[0] = X.s[1] = X.s[2] = kFarBox;
            X.s[3] = 0.0f;
            xf[eb] = X;
            for (int k = 0; k < 6; ++k) box[k] = kFarBox;
        }
    }
    if (pose_ok) {
        const int64_t eb = (int64_t)e * B + lane;
        const float* q = link_quat + 4 * eb;
        const float* t = link_pos + 3 * eb;
        // the rotation in FP64, rounded once: each FP32 entry is within half an
        // ulp of the exact R(q_b), which bounds the error of the FP32 link-frame
        // rays the renderer's triangle margins account for
        double qx = q[0], qy = q[1], qz = q[2], qw = q[3];
        const double nn = sqrt(qx * qx + qy * qy + qz * qz + qw * qw);
        qx /= nn; qy /= nn; qz /= nn; qw /= nn;
        float R[9];
        R[0] = (float)(1.0 - 2.0 * (qy * qy + qz * qz));
        R[1] = (float)(2.0 * (qx * qy - qz * qw));
        R[2] = (float)(2.0 * (qx * qz + qy * qw));
        R[3] = (float)(2.0 * (qx * qy + qz * qw));
        R[4] = (float)(1.0 - 2.0 * (qx * qx + qz * qz));
        R[5] = (float)(2.0 * (qy * qz - qx * qw));
        R[6] = (float)(2.0 * (qx * qz - qy * qw));
        R[7] = (float)(2.0 * (qy * qz + qx * qw));
        R[8] = (float)(1.0 - 2.0 * (qx * qx + qy * qy));
        InstXform X;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) X.m[3 * r + c] = R[3 * c + r];
        X.t[0] = t[0]; X.t[1] = t[1]; X.t[2] = t[2];
        {
            // world bounding sphere: the local (padded) box's centre under the
            // pose, its half-diagonal widened by 1% + 1 mm so that FP32
            // rounding cannot cull a reachable link
            const float* rb = meta[lane].root;
            const float lx = 0.5f * (rb[0] + rb[1]), ly = 0.5f * (rb[2] + rb[3]),
                        lz = 0.5f * (rb[4] + rb[5]);
            const float hx = 0.5f * (rb[1] - rb[0]), hy = 0.5f * (rb[3] - rb[2]),
                        hz = 0.5f * (rb[5] - rb[4]);
            X.s[0] = __fmaf_rn(X.m[6], lz, __fmaf_rn(X.m[3], ly, X.m[0] * lx)) + X.t[0];
            X.s[1] = __fmaf_rn(X.m[7], lz, __fmaf_rn(X.m[4], ly, X.m[1] * lx)) + X.t[1];
            X.s[2] = __fmaf_rn(X.m[8], lz, __fmaf_rn(X.m[5], ly, X.m[2] * lx)) + X.t[2];
            X.s[3] = sqrtf(__fmaf_rn(hz, hz, __fmaf_rn(hy, hy, hx * hx))) * 1.01f + 1e-3f;
        }
        xf[eb] = X;
        const float* rb = meta[lane].root;
        for (int a = 0; a < 3; ++a) {
            float c = 0.0f;
            float h = 0.0f;
            for (int k = 0; k < 3; ++k) {
                float lc = (rb[2 * k] + rb[2 * k + 1]) * 0.5f;
                float lh = (rb[2 * k + 1] - rb[2 * k]) * 0.5f;
                c = c + R[3 * a + k] * lc;
                h = h + fabsf(R[3 * a + k]) * lh;
            }
            cw[a] = c + t[a];
            float pad = fabsf(cw[a]) * kInstPadRel + kInstPadAbs;
            box[2 * a] = cw[a] - h - pad;
            box[2 * a + 1] = cw[a] + h + pad;
        }
    }
    if (!with_nodes) return;  // uniform over the block
    // centre bounds of this environment's instances (wave reduction)
    float cmin[3], cmax[3];
    for (int a = 0; a < 3; ++a) {
        cmin[a] = pose_ok ? cw[a] : INFINITY;
        cmax[a] = pose_ok ? cw[a] : -INFINITY;
        for (int off = 32; off >= 1; off >>= 1) {
            cmin[a] = fminf(cmin[a], __shfl_xor(cmin[a], off, 64));
            cmax[a] = fmaxf(cmax[a], __shfl_xor(cmax[a], off, 64));
        }
    }
    uint32_t key = 0xFFFFFFFFu;  // absent instances sort last
    if (pose_ok) {
        uint32_t q[3];
        for (int a = 0; a < 3; ++a) {
            float ext = cmax[a] - cmin[a];
            float s = ext > 0.0f ? __fdiv_rn(1024.0f, ext) : 0.0f;
            float f = fminf(fmaxf((cw[a] - cmin[a]) * s, 0.0f), 1023.0f);
            q[a] = (uint32_t)f;
        }
        key = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    }
    // rank by (key, instance index)
    int rank = 0;
    for (int j = 0; j < B; ++j) {
        uint32_t kj = __shfl(key, j, 64);
        rank += (kj < key || (kj == key && j < lane)) ? 1 : 0;
    }
    if (inst_ok) {
        skey[w][rank] = key;
        sidx[w][rank] = lane;
        for (int k = 0; k < 6; ++k) sbox[w][rank][k] = box[k];
    }
    __syncthreads();

    if (env_ok && B > 1 && lane < B - 1) {
        const uint32_t* K = skey[w];
        const int i = lane;
        int d = (tdelta(K, B, i, i + 1) - tdelta(K, B, i, i - 1)) > 0 ? 1 : -1;
        int dmin = tdelta(K, B, i, i - d);
        int lmax = 2;
        while (tdelta(K, B, i, i + lmax * d) > dmin) lmax <<= 1;
        int l = 0;
        for (int t = lmax >> 1; t >= 1; t >>= 1)
            if (tdelta(K, B, i, i + (l + t) * d) > dmin) l += t;
        int j = i + l * d;
        int dnode = tdelta(K, B, i, j);
        int s = 0;
        for (int div = 2;; div <<= 1) {
            int t = (l + div - 1) / div;
            if (tdelta(K, B, i, i + (s + t) * d) > dnode) s += t;
            if (t <= 1) break;
        }
        int g = i + s * d + (d < 0 ? -1 : 0);
        int lo = i < j ? i : j, hi = i < j ? j : i;
        int c0 = (lo == g) ? ~sidx[w][g] : g;
        int c1 = (hi == g + 1) ? ~sidx[w][g + 1] : g + 1;
        nch[w][i][0] = c0;
        nch[w][i][1] = c1;
        if (c0 >= 0) { npar[w][c0] = i; nsib[w][c0] = c1; }
        if (c1 >= 0) { npar[w][c1] = i; nsib[w][c1] = c0; }
        if (i == 0) { npar[w][0] = -1; nsib[w][0] = -1; }
        float u[6] = {INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY};
        for (int k = lo; k <= hi; ++k)
            for (int a = 0; a < 3; ++a) {
                u[2 * a] = fminf(u[2 * a], sbox[w][k][2 * a]);
                u[2 * a + 1] = fmaxf(u[2 * a + 1], sbox[w][k][2 * a + 1]);
            }
        for (int k = 0; k < 6; ++k) nbox[w][i][k] = u[k];
    }
    __syncthreads();

    if (!env_ok) return;
    Node* out = tlas + (int64_t)e * n_rec;
    if (B == 1) {
        if (lane == 0) {
            Node P;
            for (int k = 0; k < 6; ++k) { P.b0[k] = sbox[w][0][k]; P.b1[k] = kFarBox; }
            P.c0 = ~0; P.c1 = ~0; P.parent = -1; P.sibling = -1;
            out[0] = P;
        }
        return;
    }
    if (lane < B - 1) {
        const int i = lane;
        Node P;
        int c[2] = {nch[w][i][0], nch[w][i][1]};
        for (int h = 0; h < 2; ++h) {
            float* dst = h == 0 ? P.b0 : P.b1;
            // a leaf's ref holds the instance id; find its sorted slot for the box
            const float* src;
            if (c[h] >= 0) {
                src = nbox[w][c[h]];
            } else {
                int inst = ~c[h];
                int slot = 0;
                for (int k = 0; k < B; ++k) slot = (sidx[w][k] == inst) ? k : slot;
                src = sbox[w][slot];
            }
            for (int k = 0; k < 6; ++k) dst[k] = src[k];
        }
        P.c0 = c[0]; P.c1 = c[1]; P.parent = npar[w][i]; P.sibling = nsib[w][i];
        out[i] = P;
    }
}

}  // namespace

hipError_t launch_tlas_build(const float* link_pos, const float* link_quat, int n_env, int n_links,
                             const LinkMeta* meta, Node* tlas, InstXform* xf, bool with_nodes,
                             hipStream_t s) {
    unsigned blocks = (unsigned)((n_env + kWaves - 1) / kWaves);
    hipLaunchKernelGGL(k_tlas, dim3(blocks), dim3(64 * kWaves), 0, s, link_pos, link_quat, n_env,
                       n_links, meta, tlas, xf, with_nodes ? 1 : 0);
    return hipGetLastError();
}

}  // namespace rc
