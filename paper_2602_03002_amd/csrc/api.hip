// C-ABI of librc: argument validation, workspace layout and kernel launches.
// Every entry point validates on the host before it enqueues anything and
// turns HIP failures into RC_ERR_DEVICE with a message for rc_last_error().
#include "rc_internal.h"

#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

struct rc_scene {
    char* ws = nullptr;
    rc::BvhLayout terrain;
    int32_t terrain_depth = 0;
    // robot
    char* robot_ws = nullptr;
    int32_t n_links = 0;
    size_t meta_off = 0;
    std::vector<rc::BvhLayout> links;
    std::vector<int32_t> link_depth;
    // Fast-pass schedules of rc_render and rc_render_batched, packed into one
    // word each: rc_autotune and rc_set_render_config may replace them while
    // renders run on other threads, and each render reads one whole schedule.
    // entries of the per-lane stack the fast pass's 4-wide terrain walk may
    // use (rc_set_walk_stack_limit; fewer only to test the overflow path)
    std::atomic<int32_t> wide_stack{rc::kWalkStack};
    std::atomic<uint64_t> cfg_word{rc::pack_cfg(rc::RenderCfg())};
    std::atomic<uint64_t> cfg_batched_word{rc::pack_cfg(rc::RenderCfg())};
    rc::RenderCfg cfg() const { return rc::unpack_cfg(cfg_word.load(std::memory_order_acquire)); }
    rc::RenderCfg cfg_batched() const {
        return rc::unpack_cfg(cfg_batched_word.load(std::memory_order_acquire));
    }
    void set_cfg(bool batched, const rc::RenderCfg& c) {
        (batched ? cfg_batched_word : cfg_word).store(rc::pack_cfg(c), std::memory_order_release);
    }
};

struct rc_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct rc_post {
    int32_t n_env, n_cam, height, width, max_latency;
    bool packed;
    int64_t n_pix;
    float* ring;         // [L][n_pix] captures
    uint8_t* ring_drop;  // [L][n_pix] dropout mask of each capture
    bool started;
    uint64_t s0, last;
};

namespace rc {

static thread_local std::string g_error;

void set_error(const std::string& msg) { g_error = msg; }

namespace {

rc_status fail(rc_status st, const std::string& msg) {
    set_error(msg);
    return st;
}

rc_status hip_fail(hipError_t e, const char* what) {
    return fail(RC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool aligned(const void* p, size_t a = 256) { return ((uintptr_t)p % a) == 0; }

// Robot workspace: link directory, its upload table, then one hierarchy per link.
size_t robot_layout(const int64_t* off, int32_t n, std::vector<BvhLayout>* out, size_t* meta_off,
                    size_t* table_off) {
    size_t o = 0;
    *meta_off = o;
    o = align_up(o + (size_t)kMaxLinks * sizeof(LinkMeta));
    *table_off = o;
    o = align_up(o + (size_t)kMaxLinks * 4 * sizeof(int64_t));
    if (out) out->clear();
    for (int32_t b = 0; b < n; ++b) {
        BvhLayout L = bvh_layout(off[b + 1] - off[b], o);
        if (out) out->push_back(L);
        o = L.end;
    }
    return o;
}

__global__ void k_link_meta(const char* base, LinkMeta* meta, const int64_t* table, int n) {
    // table[b] = {node byte offset, tri byte offset, id byte offset, n_tri}, from `base`
    int b = threadIdx.x;
    if (b >= n) return;
    const int64_t* t = table + 4 * b;
    LinkMeta M;
    M.node_base = (int32_t)(t[0] / (int64_t)sizeof(Node));
    M.tri_base = (int32_t)(t[1] / 4);
    M.id_base = (int32_t)(t[2] / 4);
    M.n_tri = (int32_t)t[3];
    const Node* root = reinterpret_cast<const Node*>(base + t[0]);
    // union of the root record's boxes, leaving out the far point (a single
    // leaf's second box, or a subtree of zero-area triangles)
    const bool use0 = root->b0[0] != kFarBox;
    const bool use1 = M.n_tri > 1 && root->b1[0] != kFarBox;
    for (int a = 0; a < 3; ++a) {
        float lo = kFarBox, hi = kFarBox;
        if (use0) { lo = root->b0[2 * a]; hi = root->b0[2 * a + 1]; }
        if (use1) {
            lo = use0 ? fminf(lo, root->b1[2 * a]) : root->b1[2 * a];
            hi = use0 ? fmaxf(hi, root->b1[2 * a + 1]) : root->b1[2 * a + 1];
        }
        M.root[2 * a] = lo;
        M.root[2 * a + 1] = hi;
    }
    for (int k = 0; k < 6; ++k) M.pad1[k] = 0;
    meta[b] = M;
}

}  // namespace
}  // namespace rc

using namespace rc;

extern "C" {

int32_t rc_version(void) { return 10100; }

const char* rc_status_string(rc_status st) {
    switch (st) {
        case RC_OK: return "ok";
        case RC_ERR_INVALID_ARG: return "invalid argument";
        case RC_ERR_WORKSPACE: return "workspace too small or misaligned";
        case RC_ERR_DEVICE: return "device error";
        case RC_ERR_STATE: return "call out of order";
        case RC_ERR_UNSUPPORTED: return "unsupported input";
        default: return "unknown status";
    }
}

const char* rc_last_error(void) { return g_error.c_str(); }

rc_status rc_scene_size(int64_t n_tri, size_t* ws_bytes) {
    if (!ws_bytes) return fail(RC_ERR_INVALID_ARG, "rc_scene_size: ws_bytes is NULL");
    if (n_tri < 1 || n_tri > (int64_t)0x7FFFFFFE)
        return fail(RC_ERR_INVALID_ARG, "rc_scene_size: n_tri must be in [1, 2^31 - 2]");
    *ws_bytes = bvh_layout(n_tri, 0).end;
    return RC_OK;
}

rc_status rc_scene_create(const float* tri, int64_t n_tri, void* ws, size_t ws_bytes,
                          rc_stream stream, rc_scene** out) {
    if (!out) return fail(RC_ERR_INVALID_ARG, "rc_scene_create: out is NULL");
    if (!tri || !ws) return fail(RC_ERR_INVALID_ARG, "rc_scene_create: NULL pointer");
    if (n_tri < 1 || n_tri > (int64_t)0x7FFFFFFE)
        return fail(RC_ERR_INVALID_ARG, "rc_scene_create: n_tri must be in [1, 2^31 - 2]");
    BvhLayout L = bvh_layout(n_tri, 0);
    if (ws_bytes < L.end || !aligned(ws))
        return fail(RC_ERR_WORKSPACE, "rc_scene_create: workspace needs " + std::to_string(L.end) +
                                          " bytes, 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_blas_build(tri, n_tri, (char*)ws, L, s);
    if (e != hipSuccess) return hip_fail(e, "rc_scene_create: build");
    int32_t depth = 0;
    e = hipMemcpyAsync(&depth, (char*)ws + L.depth, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "rc_scene_create: depth check");
    if (depth > kMaxDepth)
        return fail(RC_ERR_UNSUPPORTED, "rc_scene_create: hierarchy depth " + std::to_string(depth) +
                                            " exceeds 64");
    rc_scene* sc = new (std::nothrow) rc_scene();
    if (!sc) return fail(RC_ERR_DEVICE, "rc_scene_create: out of host memory");
    sc->ws = (char*)ws;
    sc->terrain = L;
    sc->terrain_depth = depth;
    *out = sc;
    return RC_OK;
}

// Binned-SAH rebuild of one hierarchy whose arrays start at `base` (layout L).
static rc_status rebuild_sah_one(char* base, const BvhLayout& L, int32_t* depth_out, hipStream_t s,
                                 const char* who) {
    const int64_t n = L.n_prim, m = L.n_nodes;
    std::vector<float> tri((size_t)n * 9), tri_out((size_t)n * 9), rec((size_t)m * 16);
    std::vector<int32_t> ids((size_t)n), ids_out((size_t)n);
    // the leaf-order triangles and their input ids hold the whole mesh
    hipError_t e = hipMemcpyAsync(tri.data(), base + L.tris, (size_t)n * 36, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ids.data(), base + L.tri_id, (size_t)n * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, (std::string(who) + ": read back").c_str());
    const int32_t depth = sah_build_host(tri.data(), n, ids.data(), rec.data(), tri_out.data(),
                                         ids_out.data());
    if (depth < 0) return fail(RC_ERR_STATE, std::string(who) + ": empty hierarchy");
    if (depth > kMaxDepth)
        return fail(RC_ERR_UNSUPPORTED, std::string(who) + ": hierarchy depth " + std::to_string(depth) +
                                            " exceeds 64 (hierarchy unchanged)");
    e = hipMemcpyAsync(base + L.nodes, rec.data(), (size_t)m * 64, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(base + L.tris, tri_out.data(), (size_t)n * 36, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(base + L.tri_id, ids_out.data(), (size_t)n * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_collapse4((const Node*)(base + L.nodes), m, (float4*)(base + L.wide), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host arrays end with this call
    if (e != hipSuccess) return hip_fail(e, (std::string(who) + ": upload").c_str());
    *depth_out = depth;
    return RC_OK;
}

rc_status rc_scene_rebuild_sah(rc_scene* scene, int32_t which, rc_stream stream) {
    if (!scene) return fail(RC_ERR_INVALID_ARG, "rc_scene_rebuild_sah: NULL scene");
    if (which < 1 || which > 3) return fail(RC_ERR_INVALID_ARG, "rc_scene_rebuild_sah: which must be 1, 2 or 3");
    hipStream_t s = (hipStream_t)stream;
    if (which & 1) {
        int32_t d = 0;
        const rc_status st = rebuild_sah_one(scene->ws, scene->terrain, &d, s, "rc_scene_rebuild_sah (terrain)");
        if (st != RC_OK) return st;
        scene->terrain_depth = d;
    }
    if (which & 2) {
        for (int32_t b = 0; b < scene->n_links; ++b) {
            int32_t d = 0;
            const rc_status st = rebuild_sah_one(scene->robot_ws, scene->links[b], &d, s,
                                                 "rc_scene_rebuild_sah (link)");
            if (st != RC_OK) return st;
            scene->link_depth[b] = d;
        }
    }
    return RC_OK;
}

rc_status rc_sah_build_host(const float* tri, int64_t n_tri, float* records, float* tris_out,
                            int32_t* ids_out, int32_t* depth) {
    if (!tri || !records || !tris_out || !ids_out || !depth)
        return fail(RC_ERR_INVALID_ARG, "rc_sah_build_host: NULL pointer");
    if (n_tri < 1 || n_tri > (int64_t)0x7FFFFFFE)
        return fail(RC_ERR_INVALID_ARG, "rc_sah_build_host: n_tri must be in [1, 2^31 - 2]");
    if (tri == tris_out) return fail(RC_ERR_INVALID_ARG, "rc_sah_build_host: tris_out aliases tri");
    *depth = sah_build_host(tri, n_tri, nullptr, records, tris_out, ids_out);
    return RC_OK;
}

rc_status rc_scene_destroy(rc_scene* scene) {
    delete scene;
    return RC_OK;
}

static rc_status check_offsets(const int64_t* off, int32_t n, const char* who) {
    if (n < 0 || n > kMaxLinks)
        return fail(RC_ERR_INVALID_ARG, std::string(who) + ": n_links must be in [0, 64]");
    if (n == 0) return RC_OK;
    if (!off) return fail(RC_ERR_INVALID_ARG, std::string(who) + ": tri_offset is NULL");
    if (off[0] != 0) return fail(RC_ERR_INVALID_ARG, std::string(who) + ": tri_offset[0] != 0");
    for (int32_t b = 0; b < n; ++b) {
        if (off[b + 1] - off[b] < 1)
            return fail(RC_ERR_INVALID_ARG, std::string(who) + ": every link needs >= 1 triangle");
        if (off[b + 1] - off[b] > (int64_t)0x7FFFFFFE)
            return fail(RC_ERR_INVALID_ARG, std::string(who) + ": link mesh too large");
    }
    return RC_OK;
}

rc_status rc_robot_size(const int64_t* tri_offset, int32_t n_links, size_t* ws_bytes) {
    if (!ws_bytes) return fail(RC_ERR_INVALID_ARG, "rc_robot_size: ws_bytes is NULL");
    rc_status st = check_offsets(tri_offset, n_links, "rc_robot_size");
    if (st != RC_OK) return st;
    size_t meta_off, table_off;
    *ws_bytes = robot_layout(tri_offset, n_links, nullptr, &meta_off, &table_off);
    return RC_OK;
}

rc_status rc_robot_meshes(rc_scene* scene, const float* link_tri, const int64_t* tri_offset,
                          int32_t n_links, void* ws, size_t ws_bytes, rc_stream stream) {
    if (!scene) return fail(RC_ERR_INVALID_ARG, "rc_robot_meshes: scene is NULL");
    rc_status st = check_offsets(tri_offset, n_links, "rc_robot_meshes");
    if (st != RC_OK) return st;
    if (n_links == 0) {
        scene->n_links = 0;
        scene->robot_ws = nullptr;
        scene->links.clear();
        scene->link_depth.clear();
        return RC_OK;
    }
    if (!link_tri || !ws) return fail(RC_ERR_INVALID_ARG, "rc_robot_meshes: NULL pointer");
    std::vector<BvhLayout> Ls;
    size_t meta_off, table_off;
    size_t need = robot_layout(tri_offset, n_links, &Ls, &meta_off, &table_off);
    if (ws_bytes < need || !aligned(ws))
        return fail(RC_ERR_WORKSPACE, "rc_robot_meshes: workspace needs " + std::to_string(need) +
                                          " bytes, 256-byte aligned");
    if (need > (size_t)0x7FFFFFFF)
        return fail(RC_ERR_UNSUPPORTED, "rc_robot_meshes: link meshes too large");
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)ws;
    hipError_t e = hipSuccess;
    for (int32_t b = 0; b < n_links && e == hipSuccess; ++b)
        e = launch_blas_build(link_tri + 9 * tri_offset[b], Ls[b].n_prim, base, Ls[b], s);
    if (e != hipSuccess) return hip_fail(e, "rc_robot_meshes: build");
    // directory: offsets relative to the start of the robot workspace
    std::vector<int64_t> table(4 * (size_t)n_links);
    for (int32_t b = 0; b < n_links; ++b) {
        table[4 * b + 0] = (int64_t)Ls[b].nodes;
        table[4 * b + 1] = (int64_t)Ls[b].tris;
        table[4 * b + 2] = (int64_t)Ls[b].tri_id;
        table[4 * b + 3] = Ls[b].n_prim;
    }
    int64_t* dtable = (int64_t*)(base + table_off);
    e = hipMemcpyAsync(dtable, table.data(), table.size() * sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_link_meta, dim3(1), dim3(kMaxLinks), 0, s, (const char*)base,
                           (LinkMeta*)(base + meta_off), (const int64_t*)dtable, n_links);
        e = hipGetLastError();
    }
    std::vector<int32_t> depth(n_links);
    for (int32_t b = 0; b < n_links && e == hipSuccess; ++b)
        e = hipMemcpyAsync(&depth[b], base + Ls[b].depth, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "rc_robot_meshes: directory");
    for (int32_t b = 0; b < n_links; ++b)
        if (depth[b] > kMaxDepth)
            return fail(RC_ERR_UNSUPPORTED, "rc_robot_meshes: link hierarchy deeper than 64");
    scene->robot_ws = base;
    scene->n_links = n_links;
    scene->meta_off = meta_off;
    scene->links = Ls;
    scene->link_depth = depth;
    return RC_OK;
}

// Render workspace: top-level records and instance transforms (with links),
// the exact pass's counter and bounded list, and for the batched form the
// tile table, the eight per-XCD queue counters (64 bytes apart) and a status word.
struct RenderWs {
    size_t xf, count, list, tiles, queues, status, cams, end;
    int64_t cap;
};

// n_cams: cameras of the launch (n_env * n_cam, or the descriptors); their ray
// bases come last, so the offsets before them depend on n_env, n_pixels and
// n_desc only.
static RenderWs render_layout(int64_t n_env, int64_t n_pixels, int32_t n_links, int64_t n_desc,
                              int64_t n_cams, int64_t cap_rays = -1) {
    RenderWs L;
    size_t o = 0;
    if (n_links > 0) {
        const int64_t n_rec = n_links > 1 ? n_links - 1 : 1;
        o = align_up((size_t)n_env * n_rec * sizeof(Node));
        L.xf = o;
        o = align_up(o + (size_t)n_env * n_links * sizeof(InstXform));
    } else {
        L.xf = 0;
    }
    L.count = o;  // two uint32 counters
    o = align_up(o + 8);
    // a bounded list of 32-byte entries (a pixel in 16 typically suffices by
    // far); on overflow the exact pass re-casts every pixel
    const int64_t basis = cap_rays >= 0 ? cap_rays : n_pixels;
    L.cap = basis / 16 > 4096 ? basis / 16 : 4096;
    L.list = o;
    o = align_up(o + (size_t)L.cap * 32);
    L.tiles = o;
    o = align_up(o + (size_t)(n_desc > 0 ? n_desc + 1 : 1) * 4);
    L.queues = o;
    o = align_up(o + 8 * 64);
    L.status = o;
    o = align_up(o + 4);
    L.cams = o;
    o = align_up(o + (size_t)n_cams * 16 * sizeof(double));
    L.end = o;
    return L;
}

static bool render_dims_ok(int32_t n_env, int32_t n_cam, int32_t width, int32_t height) {
    if (n_env < 1 || n_cam < 1 || width < 1 || height < 1 || width > 65535 || height > 65535)
        return false;
    const int64_t n_rays = (int64_t)n_env * n_cam * width * height;
    return n_rays <= (int64_t)0xFFFFFFFF;
}

rc_status rc_render_size(const rc_scene* scene, int32_t n_env, int32_t n_cam, int32_t width,
                         int32_t height, size_t* ws_bytes) {
    if (!scene || !ws_bytes) return fail(RC_ERR_INVALID_ARG, "rc_render_size: NULL pointer");
    if (!render_dims_ok(n_env, n_cam, width, height))
        return fail(RC_ERR_INVALID_ARG, "rc_render_size: sizes must be >= 1, width and height "
                                        "<= 65535, at most 2^32 - 1 rays");
    *ws_bytes = render_layout(n_env, (int64_t)n_env * n_cam * width * height, scene->n_links, 0,
                              (int64_t)n_env * n_cam).end;
    return RC_OK;
}

static void fill_scene(const rc_scene* scene, RenderLaunch& L) {
    L.terrain_nodes = (const Node*)(scene->ws + scene->terrain.nodes);
    L.terrain_wide = (const float4*)(scene->ws + scene->terrain.wide);
    L.wide_stack = scene->wide_stack.load(std::memory_order_acquire);
    L.terrain_tris = (const float*)(scene->ws + scene->terrain.tris);
    L.terrain_tri_id = (const int32_t*)(scene->ws + scene->terrain.tri_id);
    L.link_nodes = (const Node*)scene->robot_ws;
    L.link_tris = (const float*)scene->robot_ws;
    L.link_tri_id = (const int32_t*)scene->robot_ws;
    L.link_meta = scene->robot_ws ? (const LinkMeta*)(scene->robot_ws + scene->meta_off) : nullptr;
    L.n_links = scene->n_links;
    L.n_terrain = (int)scene->terrain.n_prim;
}

static bool cam_rand_ok(const rc_cam_rand* r) {
    if (!r) return true;
    for (int k = 0; k < 3; ++k)
        if (!(r->trans_m[k] >= 0.0f) || !std::isfinite(r->trans_m[k]) || !(r->euler_deg[k] >= 0.0f) ||
            !std::isfinite(r->euler_deg[k]))
            return false;
    return r->dfov_deg >= 0.0f && r->dfov_deg < 90.0f;
}

static void set_cam_rand(RenderLaunch& L, const rc_cam_rand* r) {
    L.cam_rand_on = r ? 1 : 0;
    if (r) L.cam_rand = *r;
    else std::memset(&L.cam_rand, 0, sizeof(L.cam_rand));
}

static rc_status prep_plain(const rc_scene* scene, const rc_render_args* a, void* ws,
                            size_t ws_bytes, RenderLaunch& L, const char* who,
                            int64_t cap_rays = -1) {
    const std::string w(who);
    if (!scene || !a) return fail(RC_ERR_INVALID_ARG, w + ": NULL scene or args");
    if (!scene->ws) return fail(RC_ERR_STATE, w + ": scene has no terrain");
    if (!render_dims_ok(a->n_env, a->n_cam, a->width, a->height))
        return fail(RC_ERR_INVALID_ARG, w + ": sizes must be >= 1, width and height <= 65535, "
                                            "at most 2^32 - 1 rays");
    if (!a->cam_pos || !a->cam_quat || !a->intr || !a->depth)
        return fail(RC_ERR_INVALID_ARG, w + ": cam_pos, cam_quat, intr and depth are required");
    if (scene->n_links > 0 && (!a->link_pos || !a->link_quat))
        return fail(RC_ERR_INVALID_ARG, w + ": link_pos and link_quat are required with links");
    if (!(a->far_plane > 0.0f) || !(a->far_plane <= kMaxFar))
        return fail(RC_ERR_INVALID_ARG, w + ": far_plane must be in (0, 1e20]");
    if (a->depth_mode != RC_DEPTH_PLANAR && a->depth_mode != RC_DEPTH_RANGE)
        return fail(RC_ERR_INVALID_ARG, w + ": unknown depth_mode");
    if (!cam_rand_ok(a->cam_rand))
        return fail(RC_ERR_INVALID_ARG, w + ": camera randomisation ranges must be finite and "
                                            ">= 0, dfov_deg < 90");
    const int64_t n_rays = (int64_t)a->n_env * a->n_cam * a->width * a->height;
    const RenderWs W = render_layout(a->n_env, n_rays, scene->n_links, 0, (int64_t)a->n_env * a->n_cam,
                                     cap_rays);
    if (!ws || ws_bytes < W.end || !aligned(ws))
        return fail(RC_ERR_WORKSPACE, w + ": workspace needs " + std::to_string(W.end) +
                                          " bytes, 256-byte aligned");
    fill_scene(scene, L);
    L.tlas = scene->n_links > 0 ? (const Node*)ws : nullptr;
    L.xf = scene->n_links > 0 ? (const InstXform*)((char*)ws + W.xf) : nullptr;
    L.link_pos = a->link_pos;
    L.link_quat = a->link_quat;
    L.cam_pos = a->cam_pos;
    L.cam_quat = a->cam_quat;
    L.intr = a->intr;
    L.depth = a->depth;
    L.inst = a->inst;
    L.tri = a->tri;
    L.n_env = a->n_env;
    L.n_cam = a->n_cam;
    L.width = a->width;
    L.height = a->height;
    L.depth_mode = a->depth_mode;
    L.far_plane = a->far_plane;
    L.exact_count = (uint32_t*)((char*)ws + W.count);
    L.exact_list = (uint4*)((char*)ws + W.list);
    L.exact_cap = W.cap;
    L.cam_basis = (double*)((char*)ws + W.cams);
    set_cam_rand(L, a->cam_rand);
    L.ev_begin = a->timing ? (hipEvent_t)a->timing[0] : nullptr;
    L.ev_end = a->timing ? (hipEvent_t)a->timing[1] : nullptr;
    L.desc = nullptr;
    L.n_desc = 0;
    L.max_width = a->width;
    L.max_height = a->height;
    L.n_pixels = n_rays;
    return RC_OK;
}

static hipError_t run_plain(const rc_scene* scene, const RenderLaunch& L, void* ws,
                            const RenderCfg& cfg, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (scene->n_links > 0)
        e = launch_tlas_build(L.link_pos, L.link_quat, L.n_env, scene->n_links, L.link_meta,
                              (Node*)ws, (InstXform*)L.xf, !cfg.bodies_flat, s);
    if (e == hipSuccess) e = launch_render(L, cfg, s);
    return e;
}

rc_status rc_render(const rc_scene* scene, const rc_render_args* a, void* ws, size_t ws_bytes,
                    rc_stream stream) {
    RenderLaunch L;
    rc_status st = prep_plain(scene, a, ws, ws_bytes, L, "rc_render");
    if (st != RC_OK) return st;
    hipError_t e = run_plain(scene, L, ws, scene->cfg(), (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rc_render: launch");
    return RC_OK;
}

rc_status rc_render_counts(const rc_scene* scene, const rc_render_args* a, uint32_t* counts,
                           void* ws, size_t ws_bytes, rc_stream stream) {
    if (!counts || !aligned(counts, 16))
        return fail(RC_ERR_INVALID_ARG, "rc_render_counts: counts must be a 16-byte aligned device pointer");
    RenderLaunch L;
    rc_status st = prep_plain(scene, a, ws, ws_bytes, L, "rc_render_counts");
    if (st != RC_OK) return st;
    L.counts = counts;
    hipError_t e = run_plain(scene, L, ws, scene->cfg(), (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rc_render_counts: launch");
    return RC_OK;
}

// ---- render without a caller workspace ----
//
// rc_render_noalloc takes its workspace from `scratch`, a device array of this
// file that the loader allocates once per GPU with the library's code object.
// In host code the array's name stands for a host-side shadow, not a device
// address: its address on the current device comes from hipGetSymbolAddress,
// taken once per device at that device's first call and kept here.

constexpr size_t kNoallocBytes = (size_t)32 << 20;
// exact-pass list of the no-allocation form: 2^17 entries (4 MiB); a render
// that hands more rays to the exact pass re-casts every pixel exactly
constexpr int64_t kNoallocListRays = (int64_t)16 << 17;
constexpr int kNoallocDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kNoallocDevices] = {};

static rc_status scratch_of_current_device(void** out, const char* who) {
    const std::string w(who);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, who);
    if (dev < 0 || dev >= kNoallocDevices)
        return fail(RC_ERR_UNSUPPORTED, w + ": device index beyond " + std::to_string(kNoallocDevices));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, who);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RC_OK;
}

rc_status rc_render_noalloc(const rc_scene* scene, const rc_render_args* a, rc_stream stream) {
    const char* who = "rc_render_noalloc";
    if (!scene || !a) return fail(RC_ERR_INVALID_ARG, "rc_render_noalloc: NULL scene or args");
    if (!render_dims_ok(a->n_env, a->n_cam, a->width, a->height))
        return fail(RC_ERR_INVALID_ARG, "rc_render_noalloc: sizes must be >= 1, width and height "
                                        "<= 65535, at most 2^32 - 1 rays");
    const int64_t n_rays = (int64_t)a->n_env * a->n_cam * a->width * a->height;
    const int64_t cap = n_rays < kNoallocListRays ? n_rays : kNoallocListRays;
    const size_t need = render_layout(a->n_env, n_rays, scene->n_links, 0,
                                      (int64_t)a->n_env * a->n_cam, cap).end;
    if (need > kNoallocBytes)
        return fail(RC_ERR_WORKSPACE, "rc_render_noalloc: this render needs " + std::to_string(need) +
                                          " bytes of scratch, the static scratch holds " +
                                          std::to_string(kNoallocBytes) + " (use rc_render)");
    void* ws = nullptr;
    rc_status st = scratch_of_current_device(&ws, who);
    if (st != RC_OK) return st;
    RenderLaunch L;
    st = prep_plain(scene, a, ws, kNoallocBytes, L, who, cap);
    if (st != RC_OK) return st;
    hipError_t e = run_plain(scene, L, ws, scene->cfg(), (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rc_render_noalloc: launch");
    return RC_OK;
}

// ---- batched form ----

static bool batch_dims_ok(int32_t n_env, int32_t n_desc, int64_t n_pixels) {
    return n_env >= 1 && n_desc >= 1 && n_desc <= (1 << 24) && n_pixels >= 1 &&
           n_pixels <= (int64_t)0xFFFFFFFF;
}

rc_status rc_render_batched_size(const rc_scene* scene, int32_t n_env, int32_t n_desc,
                                 int64_t n_pixels, size_t* ws_bytes) {
    if (!scene || !ws_bytes) return fail(RC_ERR_INVALID_ARG, "rc_render_batched_size: NULL pointer");
    if (!batch_dims_ok(n_env, n_desc, n_pixels))
        return fail(RC_ERR_INVALID_ARG, "rc_render_batched_size: need n_env >= 1, 1 <= n_desc <= "
                                        "2^24, 1 <= n_pixels <= 2^32 - 1");
    *ws_bytes = render_layout(n_env, n_pixels, scene->n_links, n_desc, n_desc).end;
    return RC_OK;
}

static int persistent_blocks(const RenderCfg& cfg) {
    // compute units of the current device, asked once per device (a function-
    // local array of atomics: concurrent first calls may both ask, and agree)
    static std::atomic<int> cus_of[64];
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64) {
        cus = cus_of[dev].load(std::memory_order_relaxed);
        if (cus == 0) {
            int n = 0;
            cus = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
                          n > 0 ? n : 256;
            cus_of[dev].store(cus, std::memory_order_relaxed);
        }
    }
    // `waves` resident wavefronts per SIMD, 4 SIMDs per CU, kWavesPerBlock per block
    int b = cus * 4 * cfg.waves / kWavesPerBlock;
    return (b + 7) / 8 * 8;
}

static rc_status prep_batched(const rc_scene* scene, const rc_batch_args* a, void* ws,
                              size_t ws_bytes, RenderLaunch& L, RenderWs& W, const char* who,
                              int64_t cap_rays = -1) {
    const std::string w(who);
    if (!scene || !a) return fail(RC_ERR_INVALID_ARG, w + ": NULL scene or args");
    if (!scene->ws) return fail(RC_ERR_STATE, w + ": scene has no terrain");
    if (!batch_dims_ok(a->n_env, a->n_desc, a->n_pixels))
        return fail(RC_ERR_INVALID_ARG, w + ": need n_env >= 1, 1 <= n_desc <= 2^24, "
                                            "1 <= n_pixels <= 2^32 - 1");
    if (!a->desc || !a->depth) return fail(RC_ERR_INVALID_ARG, w + ": desc and depth are required");
    if (a->max_width < 1 || a->max_width > 65535 || a->max_height < 1 || a->max_height > 65535)
        return fail(RC_ERR_INVALID_ARG, w + ": max_width and max_height must be in [1, 65535]");
    if (scene->n_links > 0 && (!a->link_pos || !a->link_quat))
        return fail(RC_ERR_INVALID_ARG, w + ": link_pos and link_quat are required with links");
    if (!(a->far_plane > 0.0f) || !(a->far_plane <= kMaxFar))
        return fail(RC_ERR_INVALID_ARG, w + ": far_plane must be in (0, 1e20]");
    if (a->depth_mode != RC_DEPTH_PLANAR && a->depth_mode != RC_DEPTH_RANGE)
        return fail(RC_ERR_INVALID_ARG, w + ": unknown depth_mode");
    if (!cam_rand_ok(a->cam_rand))
        return fail(RC_ERR_INVALID_ARG, w + ": camera randomisation ranges must be finite and "
                                            ">= 0, dfov_deg < 90");
    W = render_layout(a->n_env, a->n_pixels, scene->n_links, a->n_desc, a->n_desc, cap_rays);
    if (!ws || ws_bytes < W.end || !aligned(ws))
        return fail(RC_ERR_WORKSPACE, w + ": workspace needs " + std::to_string(W.end) +
                                          " bytes, 256-byte aligned");
    fill_scene(scene, L);
    L.tlas = scene->n_links > 0 ? (const Node*)ws : nullptr;
    L.xf = scene->n_links > 0 ? (const InstXform*)((char*)ws + W.xf) : nullptr;
    L.link_pos = a->link_pos;
    L.link_quat = a->link_quat;
    L.cam_pos = L.cam_quat = L.intr = nullptr;
    L.depth = a->depth;
    L.inst = a->inst;
    L.tri = a->tri;
    L.n_env = a->n_env;
    L.n_cam = 1;
    L.width = L.height = 1;
    L.depth_mode = a->depth_mode;
    L.far_plane = a->far_plane;
    L.exact_count = (uint32_t*)((char*)ws + W.count);
    L.exact_list = (uint4*)((char*)ws + W.list);
    L.exact_cap = W.cap;
    L.cam_basis = (double*)((char*)ws + W.cams);
    set_cam_rand(L, a->cam_rand);
    L.ev_begin = a->timing ? (hipEvent_t)a->timing[0] : nullptr;
    L.ev_end = a->timing ? (hipEvent_t)a->timing[1] : nullptr;
    L.desc = a->desc;
    L.n_desc = a->n_desc;
    L.max_width = a->max_width;
    L.max_height = a->max_height;
    L.n_pixels = a->n_pixels;
    return RC_OK;
}

static hipError_t run_batched(const rc_scene* scene, const RenderLaunch& L, void* ws,
                              const RenderWs& W, const RenderCfg& cfg, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (scene->n_links > 0)
        e = launch_tlas_build(L.link_pos, L.link_quat, L.n_env, scene->n_links, L.link_meta,
                              (Node*)ws, (InstXform*)L.xf, !cfg.bodies_flat, s);
    if (e == hipSuccess)
        e = launch_render_batched(L, cfg, (uint32_t*)((char*)ws + W.tiles),
                                  (uint32_t*)((char*)ws + W.queues), (uint32_t*)((char*)ws + W.status),
                                  persistent_blocks(cfg), s);
    return e;
}

rc_status rc_render_batched(const rc_scene* scene, const rc_batch_args* a, void* ws,
                            size_t ws_bytes, rc_stream stream) {
    RenderLaunch L;
    RenderWs W;
    rc_status st = prep_batched(scene, a, ws, ws_bytes, L, W, "rc_render_batched");
    if (st != RC_OK) return st;
    hipError_t e = run_batched(scene, L, ws, W, scene->cfg_batched(), (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rc_render_batched: launch");
    return RC_OK;
}

rc_status rc_render_batched_status(const rc_scene* scene, const rc_batch_args* a, const void* ws,
                                   uint32_t* status, int64_t* exact_rays, rc_stream stream) {
    if (!scene || !a || !ws || !status) return fail(RC_ERR_INVALID_ARG, "rc_render_batched_status: NULL");
    if (!batch_dims_ok(a->n_env, a->n_desc, a->n_pixels))
        return fail(RC_ERR_INVALID_ARG, "rc_render_batched_status: bad sizes");
    const RenderWs W = render_layout(a->n_env, a->n_pixels, scene->n_links, a->n_desc, a->n_desc);
    uint32_t v[3] = {0, 0, 0};
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(&v[0], (const char*)ws + W.status, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&v[1], (const char*)ws + W.count, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "rc_render_batched_status");
    *status = v[0];
    if (exact_rays) *exact_rays = (int64_t)v[1] + v[2];
    return RC_OK;
}

// ---- schedules and autotuning ----

static RenderCfg to_cfg(const rc_render_config& c) {
    RenderCfg r;
    r.tile_w = c.tile_w; r.tile_h = c.tile_h; r.rays_per_lane = c.rays_per_lane; r.waves = c.waves;
    r.persistent = c.persistent ? 1 : 0;
    r.terrain_packet = c.terrain_packet;
    r.bodies_flat = c.bodies_flat;
    return r;
}

static rc_render_config from_cfg(const RenderCfg& c) {
    rc_render_config r;
    r.tile_w = c.tile_w; r.tile_h = c.tile_h; r.rays_per_lane = c.rays_per_lane; r.waves = c.waves;
    r.persistent = c.persistent;
    r.terrain_packet = c.terrain_packet;
    r.bodies_flat = c.bodies_flat;
    return r;
}

rc_status rc_get_render_config(const rc_scene* scene, int32_t batched, rc_render_config* cfg) {
    if (!scene || !cfg) return fail(RC_ERR_INVALID_ARG, "rc_get_render_config: NULL pointer");
    *cfg = from_cfg(batched ? scene->cfg_batched() : scene->cfg());
    return RC_OK;
}

rc_status rc_set_walk_stack_limit(rc_scene* scene, int32_t entries) {
    if (!scene) return fail(RC_ERR_INVALID_ARG, "rc_set_walk_stack_limit: NULL scene");
    if (entries < 1 || entries > kWalkStack)
        return fail(RC_ERR_INVALID_ARG, "rc_set_walk_stack_limit: entries must be in [1, " +
                                            std::to_string(kWalkStack) + "]");
    scene->wide_stack.store(entries, std::memory_order_release);
    return RC_OK;
}

rc_status rc_set_render_config(rc_scene* scene, int32_t batched, const rc_render_config* cfg) {
    if (!scene || !cfg) return fail(RC_ERR_INVALID_ARG, "rc_set_render_config: NULL pointer");
    RenderCfg c = to_cfg(*cfg);
    if (!render_cfg_ok(c))
        return fail(RC_ERR_INVALID_ARG, "rc_set_render_config: need tile_w * tile_h = 64, "
                                        "rays_per_lane in {1, 2}, waves in {6, 7, 8}, "
                                        "terrain_packet and bodies_flat in {0, 1}");
    scene->set_cfg(batched != 0, c);
    return RC_OK;
}

rc_status rc_autotune(rc_scene* scene, const rc_render_args* plain, const rc_batch_args* batched,
                      void* ws, size_t ws_bytes, int32_t reps, rc_stream stream,
                      rc_render_config* best, float* best_ms) {
    if (!scene || (!plain) == (!batched))
        return fail(RC_ERR_INVALID_ARG, "rc_autotune: give exactly one of plain and batched");
    if (reps < 1 || reps > 1000) return fail(RC_ERR_INVALID_ARG, "rc_autotune: reps in [1, 1000]");
    RenderLaunch L;
    RenderWs W;
    rc_status st = plain ? prep_plain(scene, plain, ws, ws_bytes, L, "rc_autotune")
                         : prep_batched(scene, batched, ws, ws_bytes, L, W, "rc_autotune");
    if (st != RC_OK) return st;
    L.ev_begin = L.ev_end = nullptr;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(RC_ERR_DEVICE, "rc_autotune: hipEventCreate");
    const int tiles[4][2] = {{8, 8}, {16, 4}, {4, 16}, {32, 2}};
    RenderCfg win;
    float win_ms = INFINITY;
    hipError_t e = hipSuccess;
    const int n_modes = plain ? 1 : 2;
    for (int pm = 0; pm < n_modes && e == hipSuccess; ++pm)
    for (int tp = 0; tp < 2 && e == hipSuccess; ++tp)
    for (int bf = 0; bf < 2 && e == hipSuccess; ++bf)
    for (int t = 0; t < 4 && e == hipSuccess; ++t)
        for (int rpl = 1; rpl <= 2 && e == hipSuccess; ++rpl)
            for (int wv = 6; wv <= 8 && e == hipSuccess; ++wv) {
                RenderCfg c;
                c.tile_w = tiles[t][0]; c.tile_h = tiles[t][1]; c.rays_per_lane = rpl; c.waves = wv;
                c.persistent = pm;
                c.terrain_packet = tp;
                c.bodies_flat = bf;
                for (int r = 0; r <= reps && e == hipSuccess; ++r) {
                    if (r == 1) e = hipEventRecord(e0, s);
                    if (e == hipSuccess)
                        e = plain ? run_plain(scene, L, ws, c, s) : run_batched(scene, L, ws, W, c, s);
                }
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                ms /= (float)reps;
                if (e == hipSuccess && ms < win_ms) { win_ms = ms; win = c; }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "rc_autotune");
    scene->set_cfg(plain == nullptr, win);
    if (best) *best = from_cfg(win);
    if (best_ms) *best_ms = win_ms;
    return RC_OK;
}

// ---- graphs ----

rc_status rc_graph_capture_batched(const rc_scene* scene, const rc_batch_args* a, void* ws,
                                   size_t ws_bytes, rc_stream stream, rc_graph** out) {
    if (!out) return fail(RC_ERR_INVALID_ARG, "rc_graph_capture_batched: out is NULL");
    RenderLaunch L;
    RenderWs W;
    rc_status st = prep_batched(scene, a, ws, ws_bytes, L, W, "rc_graph_capture_batched");
    if (st != RC_OK) return st;
    L.ev_begin = L.ev_end = nullptr;
    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cs;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return fail(RC_ERR_STATE, "rc_graph_capture_batched: stream is already capturing");
    rc_graph* g = new (std::nothrow) rc_graph();
    if (!g) return fail(RC_ERR_DEVICE, "rc_graph_capture_batched: out of host memory");
    persistent_blocks(scene->cfg_batched());  // device query outside the capture
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t er = run_batched(scene, L, ws, W, scene->cfg_batched(), s);
        e = hipStreamEndCapture(s, &g->graph);
        if (er != hipSuccess) e = er;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return hip_fail(e, "rc_graph_capture_batched");
    }
    *out = g;
    return RC_OK;
}

rc_status rc_graph_launch(rc_graph* graph, rc_stream stream) {
    if (!graph || !graph->exec) return fail(RC_ERR_INVALID_ARG, "rc_graph_launch: NULL graph");
    hipError_t e = hipGraphLaunch(graph->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rc_graph_launch");
    return RC_OK;
}

rc_status rc_graph_destroy(rc_graph* graph) {
    if (!graph) return RC_OK;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
    return RC_OK;
}

rc_status rc_render_exact_count(const rc_scene* scene, int32_t n_env, int32_t n_cam,
                                int32_t width, int32_t height, const void* ws, int64_t* count,
                                int64_t* recast, rc_stream stream) {
    if (!scene || !ws || !count) return fail(RC_ERR_INVALID_ARG, "rc_render_exact_count: NULL pointer");
    if (!render_dims_ok(n_env, n_cam, width, height))
        return fail(RC_ERR_INVALID_ARG, "rc_render_exact_count: bad sizes");
    const RenderWs W = render_layout(n_env, (int64_t)n_env * n_cam * width * height, scene->n_links, 0,
                                     (int64_t)n_env * n_cam);
    uint32_t c[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(c, (const char*)ws + W.count, 8, hipMemcpyDeviceToHost,
                                  (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rc_render_exact_count");
    *count = (int64_t)c[0] + c[1];
    if (recast) *recast = c[1];
    return RC_OK;
}

static rc_status post_dims(int32_t n_env, int32_t n_cam, int32_t height, int32_t width,
                           int32_t max_latency, const char* who) {
    if (n_env < 1 || n_cam < 1 || height < 1 || width < 1)
        return fail(RC_ERR_INVALID_ARG, std::string(who) + ": sizes must be >= 1");
    if (max_latency < 0 || max_latency > 255)
        return fail(RC_ERR_INVALID_ARG, std::string(who) + ": max_latency must be in [0, 255]");
    const int64_t hw = (int64_t)height * width;
    if (hw > (int64_t)0xFFFFFFFF)
        return fail(RC_ERR_INVALID_ARG, std::string(who) + ": image too large");
    if ((int64_t)n_env * n_cam > (int64_t)0x7FFFFFFF)
        return fail(RC_ERR_INVALID_ARG, std::string(who) + ": more than 2^31 - 1 images");
    return RC_OK;
}

// The ring of max_latency + 1 captures (float) and their dropout masks (byte).
static size_t post_ring_bytes(int64_t n_pix, int32_t max_latency) {
    const size_t L = (size_t)(max_latency + 1);
    return align_up((size_t)n_pix * 4 * L) + align_up((size_t)n_pix * L);
}

rc_status rc_post_size(int32_t n_env, int32_t n_cam, int32_t height, int32_t width,
                       int32_t max_latency, size_t* ws_bytes) {
    if (!ws_bytes) return fail(RC_ERR_INVALID_ARG, "rc_post_size: ws_bytes is NULL");
    rc_status st = post_dims(n_env, n_cam, height, width, max_latency, "rc_post_size");
    if (st != RC_OK) return st;
    const int64_t n_pix = (int64_t)n_env * n_cam * height * width;
    *ws_bytes = post_ring_bytes(n_pix, max_latency);
    return RC_OK;
}

rc_status rc_post_create(int32_t n_env, int32_t n_cam, int32_t height, int32_t width,
                         int32_t max_latency, void* ws, size_t ws_bytes, rc_post** out) {
    if (!out || !ws) return fail(RC_ERR_INVALID_ARG, "rc_post_create: NULL pointer");
    size_t need;
    rc_status st = rc_post_size(n_env, n_cam, height, width, max_latency, &need);
    if (st != RC_OK) return st;
    if (ws_bytes < need || !aligned(ws))
        return fail(RC_ERR_WORKSPACE, "rc_post_create: workspace needs " + std::to_string(need) +
                                          " bytes, 256-byte aligned");
    rc_post* p = new (std::nothrow) rc_post();
    if (!p) return fail(RC_ERR_DEVICE, "rc_post_create: out of host memory");
    p->n_env = n_env; p->n_cam = n_cam; p->height = height; p->width = width;
    p->packed = false;
    p->max_latency = max_latency;
    p->n_pix = (int64_t)n_env * n_cam * height * width;
    p->ring = (float*)ws;
    p->ring_drop = (uint8_t*)ws + align_up((size_t)p->n_pix * 4 * (size_t)(max_latency + 1));
    p->started = false;
    p->s0 = p->last = 0;
    *out = p;
    return RC_OK;
}

rc_status rc_post_reset(rc_post* post) {
    if (!post) return fail(RC_ERR_INVALID_ARG, "rc_post_reset: NULL handle");
    post->started = false;
    return RC_OK;
}

static rc_status post_common(rc_post* post, const float* depth_in, const rc_post_params* pp,
                             uint64_t step, float* depth_out, PostLaunch& L, const char* who) {
    const std::string w(who);
    if (!post || !pp || !depth_in || !depth_out)
        return fail(RC_ERR_INVALID_ARG, w + ": NULL required pointer");
    if (step >= (1ull << 48)) return fail(RC_ERR_INVALID_ARG, w + ": step >= 2^48");
    if (!(pp->p_drop >= 0.0f && pp->p_drop <= 1.0f))
        return fail(RC_ERR_INVALID_ARG, w + ": p_drop must be in [0, 1]");
    if (!(pp->near_plane <= pp->far_plane) || !std::isfinite(pp->near_plane) ||
        !std::isfinite(pp->far_plane))
        return fail(RC_ERR_INVALID_ARG, w + ": need finite near_plane <= far_plane");
    if (!std::isfinite(pp->sigma_abs) || !std::isfinite(pp->sigma_rel) || !std::isfinite(pp->fill))
        return fail(RC_ERR_INVALID_ARG, w + ": non-finite noise or fill parameter");
    if (pp->flags & ~(RC_POST_NOISE | RC_POST_DROPOUT | RC_POST_LATENCY | RC_POST_SIDEMASK))
        return fail(RC_ERR_INVALID_ARG, w + ": unknown flag");
    if (pp->flags & RC_POST_SIDEMASK) {
        for (int m = 0; m < 2; ++m)
            if (!(pp->mask_frac[m] >= 0.0f && pp->mask_frac[m] <= 0.5f))
                return fail(RC_ERR_INVALID_ARG, w + ": mask_frac must be in [0, 0.5]");
        for (int k = 0; k < 4; ++k)
            for (int m = 0; m < 3; ++m)
                if (!(pp->mask_p[k][m] >= 0.0f && pp->mask_p[k][m] <= 1.0f))
                    return fail(RC_ERR_INVALID_ARG, w + ": mask_p entries must be in [0, 1]");
    }
    if (pp->flags & RC_POST_LATENCY) {
        if (pp->lat_min < 0 || pp->lat_max < pp->lat_min)
            return fail(RC_ERR_INVALID_ARG, w + ": need 0 <= lat_min <= lat_max");
        if (pp->lat_max > post->max_latency)
            return fail(RC_ERR_INVALID_ARG, w + ": lat_max exceeds the ring's max_latency");
    }
    if (post->started && step != post->last + 1)
        return fail(RC_ERR_STATE, w + ": steps must be consecutive (call rc_post_reset)");
    L.depth_in = depth_in;
    L.ring = post->ring;
    L.ring_drop = post->ring_drop;
    L.depth_out = depth_out;
    L.n_pix = post->n_pix;
    L.n_env = post->n_env; L.n_cam = post->n_cam; L.height = post->height; L.width = post->width;
    L.ring_len = post->max_latency + 1;
    L.step = step;
    L.s0 = post->started ? post->s0 : step;
    L.slot = (int)(step % (uint64_t)L.ring_len);
    L.seed = pp->seed;
    double t = std::floor((double)pp->p_drop * 4294967296.0);
    L.drop_thr = t > 0.0 ? (uint64_t)t : 0ull;
    L.sigma_abs = pp->sigma_abs; L.sigma_rel = pp->sigma_rel;
    L.near_plane = pp->near_plane; L.far_plane = pp->far_plane; L.fill = pp->fill;
    L.lat_min = pp->lat_min; L.lat_max = pp->lat_max;
    L.flags = pp->flags;
    for (int m = 0; m < 2; ++m) L.mask_frac[m] = pp->mask_frac[m];
    for (int k = 0; k < 4; ++k)
        for (int m = 0; m < 3; ++m) L.mask_p[k][m] = pp->mask_p[k][m];
    L.mask_epoch = pp->mask_epoch;
    L.mask_type = pp->mask_type;
    return RC_OK;
}

static void post_advance(rc_post* post, uint64_t step) {
    if (!post->started) { post->started = true; post->s0 = step; }
    post->last = step;
}

rc_status rc_postprocess(rc_post* post, const float* depth_in, const int32_t* inst_in,
                         const rc_post_params* pp, uint64_t step, const uint32_t* cam_uid,
                         float* depth_out, uint8_t* drop_out, uint8_t* lat_out, rc_stream stream) {
    PostLaunch L;
    rc_status st = post_common(post, depth_in, pp, step, depth_out, L, "rc_postprocess");
    if (st != RC_OK) return st;
    if (post->packed)
        return fail(RC_ERR_STATE, "rc_postprocess: state was created packed; use rc_postprocess_batched");
    L.inst_in = inst_in;
    L.cam_uid = cam_uid;
    L.drop_out = drop_out;
    L.lat_out = lat_out;
    hipError_t e = launch_post(L, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rc_postprocess: launch");
    post_advance(post, step);
    return RC_OK;
}

rc_status rc_postprocess_words(rc_post* post, const float* depth_in, const int32_t* inst_in,
                               const rc_post_params* pp, uint64_t step, const uint32_t* cam_uid,
                               float* depth_out, uint8_t* drop_out, uint8_t* lat_out,
                               uint32_t* words_out, rc_stream stream) {
    if (!words_out || ((uintptr_t)words_out % 16) != 0)
        return fail(RC_ERR_INVALID_ARG, "rc_postprocess_words: words_out must be a 16-byte aligned "
                                        "device pointer");
    PostLaunch L;
    rc_status st = post_common(post, depth_in, pp, step, depth_out, L, "rc_postprocess_words");
    if (st != RC_OK) return st;
    if (post->packed)
        return fail(RC_ERR_STATE, "rc_postprocess_words: state was created packed");
    L.inst_in = inst_in;
    L.cam_uid = cam_uid;
    L.drop_out = drop_out;
    L.lat_out = lat_out;
    L.words_out = reinterpret_cast<uint4*>(words_out);
    hipError_t e = launch_post(L, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rc_postprocess_words: launch");
    post_advance(post, step);
    return RC_OK;
}

rc_status rc_post_size_packed(int64_t n_pixels, int32_t max_latency, size_t* ws_bytes) {
    if (!ws_bytes) return fail(RC_ERR_INVALID_ARG, "rc_post_size_packed: ws_bytes is NULL");
    if (n_pixels < 1 || n_pixels > (int64_t)0xFFFFFFFF || max_latency < 0 || max_latency > 255)
        return fail(RC_ERR_INVALID_ARG, "rc_post_size_packed: need 1 <= n_pixels <= 2^32 - 1, "
                                        "0 <= max_latency <= 255");
    *ws_bytes = post_ring_bytes(n_pixels, max_latency);
    return RC_OK;
}

rc_status rc_post_create_packed(int64_t n_pixels, int32_t max_latency, void* ws, size_t ws_bytes,
                                rc_post** out) {
    if (!out || !ws) return fail(RC_ERR_INVALID_ARG, "rc_post_create_packed: NULL pointer");
    size_t need;
    rc_status st = rc_post_size_packed(n_pixels, max_latency, &need);
    if (st != RC_OK) return st;
    if (ws_bytes < need || !aligned(ws))
        return fail(RC_ERR_WORKSPACE, "rc_post_create_packed: workspace needs " + std::to_string(need) +
                                          " bytes, 256-byte aligned");
    rc_post* p = new (std::nothrow) rc_post();
    if (!p) return fail(RC_ERR_DEVICE, "rc_post_create_packed: out of host memory");
    p->n_env = p->n_cam = p->height = p->width = 0;
    p->packed = true;
    p->max_latency = max_latency;
    p->n_pix = n_pixels;
    p->ring = (float*)ws;
    p->ring_drop = (uint8_t*)ws + align_up((size_t)n_pixels * 4 * (size_t)(max_latency + 1));
    p->started = false;
    p->s0 = p->last = 0;
    *out = p;
    return RC_OK;
}

rc_status rc_postprocess_batched(rc_post* post, const float* depth_in, const int32_t* inst_in,
                                 const rc_post_params* pp, uint64_t step, const rc_cam_desc* desc,
                                 int32_t n_desc, float* depth_out, uint8_t* drop_out,
                                 uint8_t* lat_out, rc_stream stream) {
    PostLaunch L;
    rc_status st = post_common(post, depth_in, pp, step, depth_out, L, "rc_postprocess_batched");
    if (st != RC_OK) return st;
    if (!post->packed)
        return fail(RC_ERR_STATE, "rc_postprocess_batched: state was not created packed");
    if (!desc || n_desc < 1 || n_desc > (1 << 24))
        return fail(RC_ERR_INVALID_ARG, "rc_postprocess_batched: need desc and 1 <= n_desc <= 2^24");
    L.inst_in = inst_in;
    L.cam_uid = nullptr;
    L.drop_out = drop_out;
    L.lat_out = lat_out;
    hipError_t e = launch_post_batched(L, desc, n_desc, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rc_postprocess_batched: launch");
    post_advance(post, step);
    return RC_OK;
}

rc_status rc_heightmap(const rc_scene* scene, const rc_heightmap_args* a, rc_stream stream) {
    if (!scene || !a || !a->base_pos || !a->base_yaw || !a->heights)
        return fail(RC_ERR_INVALID_ARG, "rc_heightmap: NULL pointer");
    if (!scene->ws) return fail(RC_ERR_STATE, "rc_heightmap: scene has no terrain");
    if (a->n_env < 1 || a->nx < 1 || a->ny < 1 || a->nx > 4096 || a->ny > 4096)
        return fail(RC_ERR_INVALID_ARG, "rc_heightmap: need n_env >= 1 and 1 <= nx, ny <= 4096");
    if (!(a->dx > 0.0f) || !(a->dy > 0.0f) || !std::isfinite(a->dx) || !std::isfinite(a->dy) ||
        !(a->depth > 0.0f) || !std::isfinite(a->depth) || !std::isfinite(a->top))
        return fail(RC_ERR_INVALID_ARG, "rc_heightmap: dx, dy, depth must be finite and > 0, top finite");
    HeightLaunch hl;
    hl.nodes = (const Node*)(scene->ws + scene->terrain.nodes);
    hl.wide = (const float4*)(scene->ws + scene->terrain.wide);
    hl.wide_stack = scene->wide_stack.load(std::memory_order_acquire);
    hl.tris = (const float*)(scene->ws + scene->terrain.tris);
    hl.n_prim = (int)scene->terrain.n_prim;
    hl.base_pos = a->base_pos;
    hl.base_yaw = a->base_yaw;
    hl.n_env = a->n_env; hl.nx = a->nx; hl.ny = a->ny;
    hl.dx = a->dx; hl.dy = a->dy; hl.top = a->top; hl.depth = a->depth; hl.miss = a->miss;
    hl.heights = a->heights;
    hipError_t e = launch_heightmap(hl, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rc_heightmap: launch");
    return RC_OK;
}

rc_status rc_downsample(const float* depth_in, const int32_t* inst_in, int64_t n_img, int32_t height,
                        int32_t width, int32_t factor, float far_plane, float* depth_out,
                        rc_stream stream) {
    if (!depth_in || !depth_out) return fail(RC_ERR_INVALID_ARG, "rc_downsample: NULL depth pointer");
    if (n_img < 1 || height < 1 || width < 1 || factor < 1 || factor > height || factor > width)
        return fail(RC_ERR_INVALID_ARG, "rc_downsample: need n_img, height, width >= 1 and "
                                        "1 <= factor <= min(height, width)");
    if ((int64_t)height * width > (int64_t)0x7FFFFFFF)
        return fail(RC_ERR_INVALID_ARG, "rc_downsample: image too large");
    if (!std::isfinite(far_plane)) return fail(RC_ERR_INVALID_ARG, "rc_downsample: far_plane not finite");
    hipError_t e = launch_downsample(depth_in, inst_in, n_img, height, width, factor, far_plane,
                                     depth_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rc_downsample: launch");
    return RC_OK;
}

rc_status rc_post_destroy(rc_post* post) {
    delete post;
    return RC_OK;
}

rc_status rc_bvh_layout_of(const rc_scene* scene, int32_t which, rc_bvh_layout* out) {
    if (!scene || !out) return fail(RC_ERR_INVALID_ARG, "rc_bvh_layout_of: NULL pointer");
    const BvhLayout* L;
    int32_t depth;
    if (which == -1) {
        L = &scene->terrain;
        depth = scene->terrain_depth;
    } else if (which >= 0 && which < scene->n_links) {
        L = &scene->links[which];
        depth = scene->link_depth[which];
    } else {
        return fail(RC_ERR_INVALID_ARG, "rc_bvh_layout_of: no such hierarchy");
    }
    out->n_prim = L->n_prim;
    out->n_nodes = L->n_nodes;
    out->node_offset = (int64_t)L->nodes;
    out->tri_offset = (int64_t)L->tris;
    out->tri_id_offset = (int64_t)L->tri_id;
    out->key_offset = (int64_t)L->keys;
    out->max_depth = depth;
    out->reserved = 0;
    out->wide_offset = (int64_t)L->wide;
    return RC_OK;
}

}  // extern "C"

// Helpers for the serving loop (C++ linkage, used by server.hip).

namespace rc {

size_t batched_ws_bytes(const rc_scene* scene, int64_t n_env, int64_t n_desc, int64_t cap_rays) {
    return render_layout(n_env, 1, scene->n_links, n_desc, n_desc, cap_rays).end;
}

rc_status enqueue_batched(const rc_scene* scene, const rc_batch_args* a, int64_t cap_rays, void* ws,
                          size_t ws_bytes, hipStream_t s) {
    RenderLaunch L;
    RenderWs W;
    rc_status st = prep_batched(scene, a, ws, ws_bytes, L, W, "serving batch", cap_rays);
    if (st != RC_OK) return st;
    L.ev_begin = L.ev_end = nullptr;
    hipError_t e = run_batched(scene, L, ws, W, scene->cfg_batched(), s);
    if (e != hipSuccess) return hip_fail(e, "serving batch: launch");
    return RC_OK;
}

int scene_links(const rc_scene* scene) { return scene->n_links; }
bool scene_ready(const rc_scene* scene) { return scene && scene->ws; }

}  // namespace rc

