// Internal declarations shared by the HIP sources of librc (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <string>

#include "../../include/rc.h"

namespace rc {

// Node record, 64 bytes: two child boxes (lo.x, hi.x, lo.y, hi.y, lo.z, hi.z),
// then child0, child1, parent, sibling.  child >= 0: internal node; child < 0:
// leaf ~child.  A BVH over n >= 2 leaves has n - 1 records (root = 0); over one
// leaf it has one record whose second box is a point at (1e30, 1e30, 1e30),
// beyond any far plane.  The same far point stands for a child subtree that
// holds only zero-area triangles.
struct alignas(16) Node {
    float b0[6];
    float b1[6];
    int32_t c0, c1, parent, sibling;
};
static_assert(sizeof(Node) == 64, "node record is one 64-byte line");

// 4-wide record of binary node n (the fast pass's terrain walk): n's two
// children, each internal one replaced by its own two children, so one record
// spans two levels.  Slot-major float4 columns: lo.x, hi.x, lo.y, hi.y, lo.z,
// hi.z (one lane per slot), then the four child words (>= 0 internal node,
// < 0 leaf ~i) and one float4 of padding: 128 bytes, two cache lines.  An
// unused slot has the far-point box.
constexpr int kWideRec = 8;

// Entries of the per-lane LDS stack of the hierarchy walks.
constexpr int kWalkStack = 16;

// Per-link hierarchy directory entry (device), 64 bytes.
// Bases are element offsets from the start of the robot workspace.
struct alignas(16) LinkMeta {
    int32_t node_base;  // in 64-byte node records
    int32_t tri_base;   // in floats: first float of the link's leaf-order triangles
    int32_t id_base;    // in int32: first input index of the link's leaves
    int32_t n_tri;
    float root[6];      // padded box of the whole mesh (lo.x, hi.x, lo.y, ...)
    int32_t pad1[6];
};
static_assert(sizeof(LinkMeta) == 64, "link directory entry is 64 bytes");

// Instance transform written by the top-level build: M = R^T (row-major),
// t = link position; o_local = M (o - t), d_local = M d; s = the link's world
// bounding sphere (centre, radius) for the fast pass's cone and segment culls.
struct alignas(16) InstXform {
    float m[9];
    float t[3];
    float s[4];
};
static_assert(sizeof(InstXform) == 64, "instance transform is 64 bytes");

// Wavefronts per block of the ray-cast kernels.  One: a block keeps its LDS and
// its slot until its slowest wavefront ends, and the fast pass's wavefronts
// differ widely in length, so single-wavefront blocks free their resources as
// soon as each one is done (7% faster than four per block, 3% than two).
constexpr int kWavesPerBlock = 1;

constexpr int kMaxLinks = 64;
constexpr int kMaxDepth = 64;          // bits in the traversal trail
constexpr float kFarBox = 1.0e30f;               // the unreachable box (a far point)
constexpr float kMaxFar = 1.0e20f;               // largest far plane: rays end far short of kFarBox
constexpr float kPadRel = 9.5367431640625e-07f;  // 2^-20, outward box padding
constexpr float kPadAbs = 1.0e-5f;               // metres
constexpr float kInstPadRel = 9.5367431640625e-07f;
constexpr float kInstPadAbs = 1.0e-4f;

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Byte layout of one hierarchy inside a workspace.
struct BvhLayout {
    int64_t n_prim = 0, n_nodes = 0;
    size_t nodes = 0, wide = 0, tris = 0, tri_id = 0, keys = 0;
    // build scratch
    size_t keys_alt = 0, vals = 0, vals_alt = 0, prim_box = 0, flags = 0, leaf_parent = 0,
           hist = 0, partial = 0, cbounds = 0, depth = 0, end = 0;
    int64_t n_blocks_sort = 0, n_blocks_red = 0;
};

BvhLayout bvh_layout(int64_t n, size_t base);

// Binned-SAH binary hierarchy over n host triangles (sah_build.hip): writes
// max(n - 1, 1) records (16 words each), the triangles in leaf order and
// their ids (ids_in[p], or p when ids_in is NULL); returns the depth of the
// deepest record (root 0), or -1 for n < 1.  tris_out must not alias tri.
int32_t sah_build_host(const float* tri, int64_t n, const int32_t* ids_in, float* rec, float* tris_out,
                       int32_t* ids_out);
// 4-wide records of a built binary hierarchy (as the builders write them).
hipError_t launch_collapse4(const Node* nodes, int64_t n_nodes, float4* out, hipStream_t s);

// Host-side launchers (each returns a hipError_t of its enqueue).
hipError_t launch_blas_build(const float* tri, int64_t n, char* ws, const BvhLayout& L,
                             hipStream_t s);
// with_nodes = false: only the instance transforms (the renderer's sphere
// culling never walks the top level)
hipError_t launch_tlas_build(const float* link_pos, const float* link_quat, int n_env,
                             int n_links, const LinkMeta* meta, Node* tlas, InstXform* xf,
                             bool with_nodes, hipStream_t s);

struct RenderLaunch {
    const Node* terrain_nodes;
    const float4* terrain_wide;  // 4-wide records, kWideRec float4 each, indexed like terrain_nodes
    int wide_stack;              // stack entries the 4-wide walk may use (1..kWalkStack)
    const float* terrain_tris;
    const int32_t* terrain_tri_id;
    const Node* link_nodes;
    const float* link_tris;
    const int32_t* link_tri_id;
    const LinkMeta* link_meta;
    const Node* tlas;
    const InstXform* xf;
    const float* link_pos;
    const float* link_quat;
    const float* cam_pos;
    const float* cam_quat;
    const float* intr;
    float* depth;
    int32_t* inst;
    int32_t* tri;
    // Rays the fast pass hands to the exact pass: [0] rays whose undecided
    // triangles are listed (entries from the front), [1] rays to re-cast in
    // full (entries from the back).  An entry is two uint4: (pixel, camera
    // index, x | y << 16, bits of the fast pass's bound) and, for the first
    // kind, (certain hit key low, high, two triangle ids or ~0).
    uint32_t* exact_count;
    uint4* exact_list;
    int64_t exact_cap;  // entries
    double* cam_basis;        // workspace: FP64 ray basis of every camera (16 doubles each)
    rc_cam_rand cam_rand;     // perception randomisation of the cameras (if cam_rand_on)
    int cam_rand_on;
    const rc_cam_desc* desc;  // batched form: camera descriptors (NULL: plain layout)
    int n_desc;
    int max_width, max_height;  // batched form: largest image a descriptor may have
    hipEvent_t ev_begin, ev_end;  // optional events around the fast-pass kernel
    int64_t n_pixels;         // output pixels
    uint32_t* counts = nullptr;  // diagnostic: per-ray (nodes, triangles, instances, 0), uint4
    int n_env, n_cam, width, height, n_links, depth_mode, n_terrain;
    float far_plane;
};
// Launch schedule of the fast pass (chosen by the autotuner).
// Defaults: the schedule measured fastest at 4096 envs x 2 cameras x 64x48.
struct RenderCfg {
    int tile_w = 8, tile_h = 8;  // pixels per wavefront tile, tile_w * tile_h = 64
    int rays_per_lane = 1;       // tiles each wavefront casts, stacked vertically
    int waves = 6;               // resident wavefronts per SIMD asked of the compiler (6, 7, 8)
    int persistent = 0;          // batched form: persistent work-queue launch (1) or flat grid (0)
    int terrain_packet = 0;      // terrain walked per lane (0) or as a wavefront packet (1)
    int bodies_flat = 1;         // links found by the top-level walk (0) or by cone culling (1)
};
bool render_cfg_ok(const RenderCfg& c);
// One word per schedule (fields of 8 bits each), so a schedule can be read and
// replaced atomically.
inline uint64_t pack_cfg(const RenderCfg& c) {
    return (uint64_t)(c.tile_w & 0xFF) | (uint64_t)(c.tile_h & 0xFF) << 8 |
           (uint64_t)(c.rays_per_lane & 0xFF) << 16 | (uint64_t)(c.waves & 0xFF) << 24 |
           (uint64_t)(c.persistent & 0xFF) << 32 | (uint64_t)(c.terrain_packet & 0xFF) << 40 |
           (uint64_t)(c.bodies_flat & 0xFF) << 48;
}
inline RenderCfg unpack_cfg(uint64_t v) {
    RenderCfg c;
    c.tile_w = (int)(v & 0xFF);
    c.tile_h = (int)((v >> 8) & 0xFF);
    c.rays_per_lane = (int)((v >> 16) & 0xFF);
    c.waves = (int)((v >> 24) & 0xFF);
    c.persistent = (int)((v >> 32) & 0xFF);
    c.terrain_packet = (int)((v >> 40) & 0xFF);
    c.bodies_flat = (int)((v >> 48) & 0xFF);
    return c;
}

struct HeightLaunch {
    const Node* nodes;
    const float4* wide;  // 4-wide records of the same hierarchy
    int wide_stack;      // stack entries the 4-wide walk may use (1..kWalkStack)
    const float* tris;
    int n_prim;
    const float* base_pos;  // [n_env][3]
    const float* base_yaw;  // [n_env]
    int n_env, nx, ny;
    float dx, dy, top, depth, miss;
    float* heights;  // [n_env][ny][nx]
};
hipError_t launch_heightmap(const HeightLaunch& hl, hipStream_t s);
hipError_t launch_render(const RenderLaunch& a, const RenderCfg& cfg, hipStream_t s);
hipError_t launch_render_batched(const RenderLaunch& a, const RenderCfg& cfg, uint32_t* tile_start,
                                 uint32_t* queues, uint32_t* status, int persistent_blocks,
                                 hipStream_t s);

struct PostLaunch {
    const float* depth_in;
    const int32_t* inst_in;
    const uint32_t* cam_uid;
    float* ring;         // [L][n_pix] captures
    uint8_t* ring_drop;  // [L][n_pix] their dropout masks
    float* depth_out;
    uint8_t* drop_out;
    uint8_t* lat_out;
    int64_t n_pix;
    int n_env, n_cam, height, width, ring_len;
    int slot;  // ring slot of this step: step mod ring_len
    uint64_t step, s0;
    uint64_t seed;
    uint64_t drop_thr;  // floor(p_drop * 2^32) in [0, 2^32]
    float sigma_abs, sigma_rel, near_plane, far_plane, fill;
    int lat_min, lat_max;
    uint32_t flags;
    float mask_frac[2];
    float mask_p[4][3];
    uint64_t mask_epoch;
    const uint8_t* mask_type;
    uint4* words_out = nullptr;  // debug: the raw Philox words of each pixel's draw
};
hipError_t launch_post(const PostLaunch& a, hipStream_t s);
hipError_t launch_downsample(const float* depth, const int32_t* inst, int64_t n_img, int H, int W,
                             int f, float far_plane, float* out, hipStream_t s);
hipError_t launch_post_batched(const PostLaunch& a, const rc_cam_desc* desc, int n_desc,
                               hipStream_t s);

void set_error(const std::string& msg);

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplications, with key increments 0x9E3779B9 and 0xBB67AE85.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit multiply gives both halves of each product
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Serving-loop helpers (api.hip): workspace bytes of a batched render whose
// exact-pass list is sized for cap_rays rays, and its enqueue.
size_t batched_ws_bytes(const rc_scene* scene, int64_t n_env, int64_t n_desc, int64_t cap_rays);
rc_status enqueue_batched(const rc_scene* scene, const rc_batch_args* a, int64_t cap_rays, void* ws,
                          size_t ws_bytes, hipStream_t s);
int scene_links(const rc_scene* scene);
bool scene_ready(const rc_scene* scene);

}  // namespace rc
