// Sensor model: latency, Gaussian noise and per-pixel dropout (the paper names
// these three effects in Sec. 1 and Sec. 4.1 and gives dropout and noise
// parameters in Table 6), fused in one pass over the rendered frame.
//
// Random numbers come from Philox4x32-10 (Salmon et al., SC'11), a
// counter-based generator, so every draw is a pure function of (seed, pixel,
// camera uid, capture step): no generator state is stored, and a request's
// draws do not depend on how it is batched with others.  The ring buffer
// keeps the last max_latency + 1 captures per pixel on the device.
#include "rc_internal.h"

#pragma clang fp contract(off)

namespace rc {

namespace {

__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ uint32_t step_hi(uint64_t s) {
    return (uint32_t)(((s >> 32) & 0xFFFFull) << 16);
}

// Sensor model of packed pixel p: pixel `pix` of its image, camera `uid`.
__device__ __forceinline__ void post_pixel(const PostLaunch& a, int64_t p, uint32_t pix, uint32_t uid,
                                           uint8_t* lat_slot) {
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const uint64_t s = a.step;

    // capture of this step
    const float z = a.depth_in[p];
    const bool hit = a.inst_in ? (a.inst_in[p] >= 0) : (z < a.far_plane);
    const uint4 wd = philox10(make_uint4(pix, uid, (uint32_t)s, step_hi(s)), k0, k1);
    const bool drop = (a.flags & RC_POST_DROPOUT) && ((uint64_t)wd.x < a.drop_thr);
    float zz;
    if (hit) {
        float g = 0.0f;
        if (a.flags & RC_POST_NOISE) {
            const float u1 = (float)((wd.y >> 8) + 1u) * 5.9604644775390625e-08f;  // 2^-24
            const float u2 = (float)(wd.z >> 8) * 5.9604644775390625e-08f;
            g = sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
        }
        zz = z + (a.sigma_abs + a.sigma_rel * z) * g;
    } else {
        zz = a.far_plane;
    }
    zz = fminf(fmaxf(zz, a.near_plane), a.far_plane);
    const float cap = drop ? a.fill : zz;
    a.ring[(int64_t)(s % (uint64_t)a.ring_len) * a.n_pix + p] = cap;

    // frame shown at this step
    int k = 0;
    if (a.flags & RC_POST_LATENCY) {
        const uint4 wl = philox10(make_uint4(0xFFFFFFFFu, uid, (uint32_t)s, step_hi(s) | 1u), k0, k1);
        const uint64_t span = (uint64_t)(a.lat_max - a.lat_min + 1);
        k = a.lat_min + (int)(((uint64_t)wl.x * span) >> 32);
    }
    const uint64_t src = (s - a.s0 >= (uint64_t)k) ? s - (uint64_t)k : a.s0;
    float out = cap;
    bool out_drop = drop;
    if (src != s) {
        out = a.ring[(int64_t)(src % (uint64_t)a.ring_len) * a.n_pix + p];
        if (a.drop_out) {
            const uint4 wo = philox10(make_uint4(pix, uid, (uint32_t)src, step_hi(src)), k0, k1);
            out_drop = (a.flags & RC_POST_DROPOUT) && ((uint64_t)wo.x < a.drop_thr);
        }
    }
    a.depth_out[p] = out;
    if (a.drop_out) a.drop_out[p] = out_drop ? 1 : 0;
    if (lat_slot && pix == 0) *lat_slot = (uint8_t)k;
}

// Plain layout [env][cam][height][width]: one thread per pixel.
__global__ void __launch_bounds__(256) k_post(PostLaunch a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n_pix) return;
    const int64_t hw = (int64_t)a.height * a.width;
    const int64_t ec = p / hw;
    const uint32_t pix = (uint32_t)(p - ec * hw);
    const uint32_t uid = a.cam_uid ? a.cam_uid[ec] : (uint32_t)ec;
    post_pixel(a, p, pix, uid, a.lat_out ? a.lat_out + ec : nullptr);
}

// Packed batch: block row x = camera, the blocks of a row stride over its pixels.
__global__ void __launch_bounds__(256) k_post_batched(PostLaunch a, const rc_cam_desc* desc) {
    const rc_cam_desc D = desc[blockIdx.x];
    const int64_t np = (int64_t)D.width * D.height;
    if (D.width < 1 || D.height < 1 || (int64_t)D.out_offset + np > a.n_pix) return;
    for (int64_t q = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; q < np;
         q += (int64_t)gridDim.y * blockDim.x)
        post_pixel(a, (int64_t)D.out_offset + q, (uint32_t)q, D.cam_uid,
                   a.lat_out ? a.lat_out + blockIdx.x : nullptr);
}

}  // namespace

hipError_t launch_post(const PostLaunch& a, hipStream_t s) {
    const unsigned blocks = (unsigned)((a.n_pix + 255) / 256);
    hipLaunchKernelGGL(k_post, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_post_batched(const PostLaunch& a, const rc_cam_desc* desc, int n_desc,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_post_batched, dim3((unsigned)n_desc, 8), dim3(256), 0, s, a, desc);
    return hipGetLastError();
}

}  // namespace rc
