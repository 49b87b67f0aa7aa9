// Sensor model: latency, Gaussian noise and per-pixel dropout (the paper names
// these three effects in Sec. 1 and Sec. 4.1 and gives dropout and noise
// parameters in Table 6), fused in one pass over the rendered frame.
//
// Random numbers come from Philox4x32-10 (Salmon et al., SC'11), a
// counter-based generator, so every draw is a pure function of (seed, pixel,
// camera uid, capture step): no generator state is stored, and a request's
// draws do not depend on how it is batched with others.  The ring buffer
// keeps the last max_latency + 1 captures per pixel on the device.
#include <algorithm>

#include "rc_internal.h"

#pragma clang fp contract(off)

namespace rc {

namespace {

__device__ __forceinline__ uint32_t step_hi(uint64_t s) {
    return (uint32_t)(((s >> 32) & 0xFFFFull) << 16);
}

// Latency (frames) of camera `uid` at this step: one draw per (camera, step).
__device__ __forceinline__ int latency_draw(const PostLaunch& a, uint32_t uid) {
    if (!(a.flags & RC_POST_LATENCY)) return 0;
    const uint64_t s = a.step;
    const uint4 wl = philox4x32_10(make_uint4(0xFFFFFFFFu, uid, (uint32_t)s, step_hi(s) | 1u),
                              (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
    const uint64_t span = (uint64_t)(a.lat_max - a.lat_min + 1);
    return a.lat_min + (int)(((uint64_t)wl.x * span) >> 32);
}

// Random side masking: columns masked on each side of the images of env
// `env` (0 for mode none), drawn once per env and mask epoch.
__device__ __forceinline__ int side_mask_cols(const PostLaunch& a, int env, int width) {
    if (!(a.flags & RC_POST_SIDEMASK)) return 0;
    const int type = a.mask_type ? min((int)a.mask_type[env], 3) : 0;
    const uint32_t e_hi = (uint32_t)((a.mask_epoch >> 32) & 0xFFFFull) << 16;
    const uint4 w = philox4x32_10(make_uint4((uint32_t)env, 0xFFFFFFFDu, (uint32_t)a.mask_epoch, e_hi | 4u),
                                  (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
    const float u = (float)(w.x >> 8) * 5.9604644775390625e-08f;  // 2^-24
    const float* pk = a.mask_p[type];
    if (u < pk[0]) return 0;
    const int mode = u < pk[0] + pk[1] ? 0 : 1;
    const float band = a.mask_frac[mode] * (float)width;
    return (int)floorf(band + 0.5f);
}

// The draw of pixel `pix` of camera `uid` at this step.
__device__ __forceinline__ uint4 pixel_draw(const PostLaunch& a, uint32_t pix, uint32_t uid) {
    return philox4x32_10(make_uint4(pix, uid, (uint32_t)a.step, step_hi(a.step)), (uint32_t)a.seed,
                         (uint32_t)(a.seed >> 32));
}

// Capture of one pixel at this step: noise on hits, clamp to [near, far],
// dropout (the capture is then the fill value).
__device__ __forceinline__ float capture(const PostLaunch& a, float z, bool hit, const uint4& wd,
                                         bool& drop) {
    drop = (a.flags & RC_POST_DROPOUT) && ((uint64_t)wd.x < a.drop_thr);
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
    return drop ? a.fill : zz;
}

// Frames back to the capture shown at this step: max(s - k, s0) (k < ring_len).
__device__ __forceinline__ int delay(const PostLaunch& a, int k) {
    return (a.step - a.s0 >= (uint64_t)k) ? k : (int)(a.step - a.s0);
}

// Side masking: is column x masked, and the fill from word 3 of the draw.
__device__ __forceinline__ bool masked_col(uint32_t pix, int mask_m, int width) {
    const int x = (int)(pix % (uint32_t)width);
    return x < mask_m || x >= width - mask_m;
}
__device__ __forceinline__ float mask_fill(const PostLaunch& a, const uint4& wd) {
    const float u = (float)(wd.w >> 8) * 5.9604644775390625e-08f;
    return __fmaf_rn(a.far_plane - a.near_plane, u, a.near_plane);
}

// Sensor model of packed pixel p: pixel `pix` of its image (width `width`),
// camera `uid`, whose latency at this step is k frames; mask_m side columns
// of the image are masked.
__device__ __forceinline__ void post_pixel(const PostLaunch& a, int64_t p, uint32_t pix, uint32_t uid,
                                           int k, int mask_m, int width) {
    const float z = a.depth_in[p];
    const bool hit = a.inst_in ? (a.inst_in[p] >= 0) : (z < a.far_plane);
    const uint4 wd = pixel_draw(a, pix, uid);
    if (a.words_out) a.words_out[p] = wd;
    bool drop;
    const float cap = capture(a, z, hit, wd, drop);
    const int64_t here = (int64_t)a.slot * a.n_pix + p;
    a.ring[here] = cap;
    a.ring_drop[here] = drop ? 1 : 0;

    const int d = delay(a, k);
    float out = cap;
    bool out_drop = drop;
    if (d > 0) {
        const int slot = a.slot >= d ? a.slot - d : a.slot - d + a.ring_len;
        const int64_t there = (int64_t)slot * a.n_pix + p;
        out = a.ring[there];
        out_drop = a.ring_drop[there] != 0;
    }
    if (mask_m > 0 && masked_col(pix, mask_m, width)) {  // random side masking of the frame shown
        out = mask_fill(a, wd);
        out_drop = false;
    }
    a.depth_out[p] = out;
    if (a.drop_out) a.drop_out[p] = out_drop ? 1 : 0;
}

// The same for four consecutive pixels p .. p+3 of one image (p a multiple of
// 4, arrays aligned for 16-byte and 4-byte accesses): wide loads and stores,
// four independent draws per thread.
__device__ __forceinline__ void post_quad(const PostLaunch& a, int64_t p, uint32_t pix, uint32_t uid,
                                          int k, int mask_m, int width) {
    const float4 z4 = *reinterpret_cast<const float4*>(a.depth_in + p);
    const float z[4] = {z4.x, z4.y, z4.z, z4.w};
    int4 i4 = make_int4(0, 0, 0, 0);
    if (a.inst_in) i4 = *reinterpret_cast<const int4*>(a.inst_in + p);
    const int id[4] = {i4.x, i4.y, i4.z, i4.w};
    uint4 wd[4];
    float cap[4];
    uint32_t bits = 0u;
    for (int j = 0; j < 4; ++j) {
        wd[j] = pixel_draw(a, pix + (uint32_t)j, uid);
        if (a.words_out) a.words_out[p + j] = wd[j];
        const bool hit = a.inst_in ? (id[j] >= 0) : (z[j] < a.far_plane);
        bool drop;
        cap[j] = capture(a, z[j], hit, wd[j], drop);
        bits |= (drop ? 1u : 0u) << (8 * j);
    }
    const int64_t here = (int64_t)a.slot * a.n_pix + p;
    *reinterpret_cast<float4*>(a.ring + here) = make_float4(cap[0], cap[1], cap[2], cap[3]);
    *reinterpret_cast<uint32_t*>(a.ring_drop + here) = bits;

    const int d = delay(a, k);
    float out[4] = {cap[0], cap[1], cap[2], cap[3]};
    uint32_t obits = bits;
    if (d > 0) {
        const int slot = a.slot >= d ? a.slot - d : a.slot - d + a.ring_len;
        const int64_t there = (int64_t)slot * a.n_pix + p;
        const float4 o4 = *reinterpret_cast<const float4*>(a.ring + there);
        out[0] = o4.x; out[1] = o4.y; out[2] = o4.z; out[3] = o4.w;
        obits = *reinterpret_cast<const uint32_t*>(a.ring_drop + there);
    }
    if (mask_m > 0) {
        for (int j = 0; j < 4; ++j) {
            if (masked_col(pix + (uint32_t)j, mask_m, width)) {
                out[j] = mask_fill(a, wd[j]);
                obits &= ~(0xFFu << (8 * j));
            }
        }
    }
    *reinterpret_cast<float4*>(a.depth_out + p) = make_float4(out[0], out[1], out[2], out[3]);
    if (a.drop_out) *reinterpret_cast<uint32_t*>(a.drop_out + p) = obits;
}

// Plain layout [env][cam][height][width]: block row x = image (env, cam), the
// blocks of a row stride over its pixels.
// QUAD: four pixels per thread (the image size a multiple of 4).
template <bool QUAD>
__global__ void __launch_bounds__(256) k_post(PostLaunch a) {
    const int64_t ec = blockIdx.x;
    const int64_t hw = (int64_t)a.height * a.width;
    const uint32_t uid = a.cam_uid ? a.cam_uid[ec] : (uint32_t)ec;
    const int k = latency_draw(a, uid);
    const int mask_m = side_mask_cols(a, (int)(ec / a.n_cam), a.width);
    if (a.lat_out && blockIdx.y == 0 && threadIdx.x == 0) a.lat_out[ec] = (uint8_t)k;
    const int64_t n = QUAD ? hw / 4 : hw;
    for (int64_t q = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.y * blockDim.x) {
        if (QUAD) post_quad(a, ec * hw + 4 * q, (uint32_t)(4 * q), uid, k, mask_m, a.width);
        else post_pixel(a, ec * hw + q, (uint32_t)q, uid, k, mask_m, a.width);
    }
}

// Packed batch: block row x = camera descriptor, the blocks of a row stride
// over its pixels.
__global__ void __launch_bounds__(256) k_post_batched(PostLaunch a, const rc_cam_desc* desc) {
    const rc_cam_desc D = desc[blockIdx.x];
    const int64_t np = (int64_t)D.width * D.height;
    if (D.width < 1 || D.height < 1 || (int64_t)D.out_offset + np > a.n_pix) return;
    const int k = latency_draw(a, D.cam_uid);
    const int mask_m = D.env >= 0 ? side_mask_cols(a, D.env, D.width) : 0;
    if (a.lat_out && blockIdx.y == 0 && threadIdx.x == 0) a.lat_out[blockIdx.x] = (uint8_t)k;
    for (int64_t q = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; q < np;
         q += (int64_t)gridDim.y * blockDim.x)
        post_pixel(a, (int64_t)D.out_offset + q, (uint32_t)q, D.cam_uid, k, mask_m, D.width);
}

// Block pooling of rendered frames (the paper feeds its policy 240x135 depth
// downsampled to 48x27, Sec. 4.1): output pixel (oy, ox) is the mean depth of
// the hit pixels of its f x f block, summed in row-major order, or far when
// none of them hit.  Grid: x over the output pixels of an image, y over images.
__global__ void __launch_bounds__(256) k_downsample(const float* __restrict__ depth,
                                                    const int32_t* __restrict__ inst, int64_t n_img,
                                                    int H, int W, int f, float far_plane,
                                                    float* __restrict__ out) {
    const int Ho = H / f, Wo = W / f;
    const int per = Ho * Wo;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= per) return;
    const int oy = q / Wo, ox = q - oy * Wo;
    for (int64_t img = blockIdx.y; img < n_img; img += gridDim.y) {
        const int64_t base = img * H * W + (int64_t)(oy * f) * W + (int64_t)ox * f;
        float sum = 0.0f;
        int cnt = 0;
        for (int dy = 0; dy < f; ++dy)
            for (int dx = 0; dx < f; ++dx) {
                const int64_t p = base + (int64_t)dy * W + dx;
                const float z = depth[p];
                const bool hit = inst ? inst[p] >= 0 : z < far_plane;
                if (hit) {
                    sum += z;
                    ++cnt;
                }
            }
        out[img * per + q] = cnt ? sum / (float)cnt : far_plane;
    }
}

}  // namespace

hipError_t launch_downsample(const float* depth, const int32_t* inst, int64_t n_img, int H, int W,
                             int f, float far_plane, float* out, hipStream_t s) {
    const int per = (H / f) * (W / f);
    const unsigned gy = (unsigned)std::min<int64_t>(n_img, 65535);
    hipLaunchKernelGGL(k_downsample, dim3((unsigned)((per + 255) / 256), gy), dim3(256), 0, s, depth,
                       inst, n_img, H, W, f, far_plane, out);
    return hipGetLastError();
}

hipError_t launch_post(const PostLaunch& a, hipStream_t s) {
    const int64_t hw = (int64_t)a.height * a.width;
    auto al = [](const void* q, uintptr_t m) { return ((uintptr_t)q & (m - 1)) == 0; };
    const bool quad = hw % 4 == 0 && al(a.depth_in, 16) && al(a.inst_in, 16) && al(a.ring, 16) &&
                      al(a.depth_out, 16) && al(a.ring_drop, 4) && al(a.drop_out, 4);
    const int64_t items = quad ? hw / 4 : hw;
    const unsigned per_image = (unsigned)std::min<int64_t>((items + 255) / 256, 1024);
    const dim3 grid((unsigned)((int64_t)a.n_env * a.n_cam), per_image);
    if (quad) hipLaunchKernelGGL(k_post<true>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_post<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_post_batched(const PostLaunch& a, const rc_cam_desc* desc, int n_desc,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_post_batched, dim3((unsigned)n_desc, 8), dim3(256), 0, s, a, desc);
    return hipGetLastError();
}

}  // namespace rc
