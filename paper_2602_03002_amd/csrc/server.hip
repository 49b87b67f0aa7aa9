// Serving loop: a FIFO request queue over a device-resident scene, admission
// by memory (output planes and a scratch heap carved from the caller's arena),
// continuous batching of waiting requests into batched launches on several
// streams, and latency statistics.  The scheduler is plain host code; the
// simulated mode replaces the device by a timing model so the scheduling
// logic can be tested without a GPU.
#include "rc_internal.h"

#include <algorithm>
#include <cmath>
#include <deque>
#include <map>
#include <new>
#include <unordered_map>
#include <vector>

namespace rc {
namespace {

// First-fit allocator over [0, cap) with coalescing of freed ranges.
class RangeAlloc {
  public:
    explicit RangeAlloc(uint64_t cap = 0) {
        if (cap) free_[0] = cap;
    }
    bool alloc(uint64_t n, uint64_t align, uint64_t* off) {
        if (n == 0) n = 1;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            const uint64_t b = it->first, e = it->first + it->second;
            const uint64_t a = (b + align - 1) / align * align;
            if (a + n > e) continue;
            free_.erase(it);
            if (a > b) free_[b] = a - b;
            if (a + n < e) free_[a + n] = e - (a + n);
            *off = a;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t n) {
        if (n == 0) n = 1;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<uint64_t, uint64_t> free_;
};

struct Req {
    int64_t id;
    rc_request r;
    double arrival;
    int64_t pixels;
    uint64_t out_off = 0;
};

struct Batch {
    bool active = false;
    std::vector<Req> reqs;
    int64_t rays = 0;
    uint64_t scr_off = 0, scr_len = 0;
    double launch_s = 0, sim_done = 0;
    rc_status err = RC_OK;
};

struct Taken {
    uint64_t out_off;
    int64_t pixels;
};

// Descriptors of one request: camera (e, c) -> batch env env_base + e, image
// packed at out_off + (e * n_cam + c) * W * H, camera uid e * n_cam + c.
__global__ void k_request_desc(rc_request r, int env_base, uint32_t out_off, rc_cam_desc* desc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= r.n_env * r.n_cam) return;
    const int e = i / r.n_cam;
    rc_cam_desc D;
    D.env = env_base + e;
    D.width = r.width;
    D.height = r.height;
    D.out_offset = out_off + (uint32_t)i * (uint32_t)(r.width * r.height);
    D.cam_uid = (uint32_t)i;
    for (int k = 0; k < 3; ++k) D.pos[k] = r.cam_pos[3 * i + k];
    for (int k = 0; k < 4; ++k) D.quat[k] = r.cam_quat[4 * i + k];
    for (int k = 0; k < 4; ++k) D.intr[k] = r.intr[4 * i + k];
    desc[i] = D;
}

size_t pose_bytes(int64_t n_env, int n_links) {
    return align_up((size_t)n_env * (size_t)n_links * 3 * 4) + align_up((size_t)n_env * n_links * 4 * 4);
}

}  // namespace
}  // namespace rc

using namespace rc;

struct rc_server {
    rc_server_config cfg;
    bool sim = false;
    double sim_launch = 0, sim_per_ray = 0;
    const rc_scene* scene = nullptr;
    int n_links = 0;
    float* depth = nullptr;
    int32_t* inst = nullptr;
    int32_t* tri = nullptr;
    char* scratch = nullptr;
    size_t scratch_bytes = 0;
    RangeAlloc pix, scr;
    std::deque<Req> queue;
    std::vector<Batch> slots;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::deque<rc_result> ready;
    std::unordered_map<int64_t, Taken> out_of;  // finished results -> their output range
    int64_t next_id = 1;
    int32_t fail_next = 0;  // batches still to report an injected failure
    std::vector<double> lat;
    rc_server_stats st{};

    // scratch a batch of these requests needs (poses, camera table, render workspace)
    size_t batch_scratch(int64_t n_env, int64_t n_desc, int64_t rays) const {
        size_t b = pose_bytes(n_env, n_links) + align_up((size_t)n_desc * sizeof(rc_cam_desc));
        b += sim ? align_up((size_t)rays / 16 * 16 + 65536) : batched_ws_bytes(scene, n_env, n_desc, rays);
        return b;
    }
};

namespace {

rc_status fail_s(rc_status st, const std::string& m) {
    set_error(m);
    return st;
}

bool cfg_ok(const rc_server_config* c) {
    return c && c->n_streams >= 1 && c->n_streams <= 16 && c->max_batch_rays >= 1 &&
           c->out_pixels >= 1 && c->out_pixels <= (int64_t)0xFFFFFFFF && c->far_plane > 0.0f &&
           std::isfinite(c->far_plane) &&
           (c->depth_mode == RC_DEPTH_PLANAR || c->depth_mode == RC_DEPTH_RANGE);
}

size_t planes_bytes(const rc_server_config* c) { return 3 * align_up((size_t)c->out_pixels * 4); }

void finish_batch(rc_server* s, Batch& b, double now, rc_status err) {
    for (Req& q : b.reqs) {
        rc_result r{};
        r.id = q.id;
        r.status = err;
        r.n_pixels = q.pixels;
        r.depth = s->depth ? s->depth + q.out_off : nullptr;
        r.inst = s->inst ? s->inst + q.out_off : nullptr;
        r.tri = s->tri ? s->tri + q.out_off : nullptr;
        r.arrival_s = q.arrival;
        r.launch_s = b.launch_s;
        r.done_s = now;
        s->ready.push_back(r);
        s->out_of[q.id] = Taken{q.out_off, q.pixels};
        s->lat.push_back(now - q.arrival);
        s->st.completed += 1;
        s->st.rays_completed += q.pixels;
        s->st.in_flight -= 1;
        if (now > s->st.last_done_s) s->st.last_done_s = now;
    }
    s->scr.release(b.scr_off, b.scr_len);
    b = Batch();
}

// Start one batch on slot k from the queue head; false if nothing could start.
bool start_batch(rc_server* s, int k, double now) {
    Batch& b = s->slots[k];
    std::vector<Req> take;
    int64_t rays = 0, n_env = 0, n_desc = 0;
    int max_w = 1, max_h = 1;
    uint64_t scr_off = 0, scr_len = 0;
    while (!s->queue.empty()) {
        Req q = s->queue.front();
        if (!take.empty() && rays + q.pixels > s->cfg.max_batch_rays) break;
        uint64_t off;
        if (!s->pix.alloc((uint64_t)q.pixels, 1, &off)) break;  // outputs must wait for memory
        q.out_off = off;
        const int64_t ne = n_env + q.r.n_env, nd = n_desc + (int64_t)q.r.n_env * q.r.n_cam;
        const size_t need = s->batch_scratch(ne, nd, rays + q.pixels);
        if (scr_len) s->scr.release(scr_off, scr_len);
        if (!s->scr.alloc(need, 256, &scr_off)) {
            s->pix.release(off, (uint64_t)q.pixels);
            scr_len = 0;
            if (!take.empty()) {  // re-take the scratch of the requests already in
                const size_t need0 = s->batch_scratch(n_env, n_desc, rays);
                if (s->scr.alloc(need0, 256, &scr_off)) scr_len = need0;
            }
            break;
        }
        scr_len = need;
        s->queue.pop_front();
        take.push_back(q);
        rays += q.pixels;
        n_env = ne;
        n_desc = nd;
        max_w = std::max(max_w, (int)q.r.width);
        max_h = std::max(max_h, (int)q.r.height);
    }
    if (take.empty()) return false;
    if (scr_len == 0) {  // could not re-take scratch: give everything back and wait
        for (auto it = take.rbegin(); it != take.rend(); ++it) {
            s->pix.release(it->out_off, (uint64_t)it->pixels);
            s->queue.push_front(*it);
        }
        return false;
    }
    b.active = true;
    b.reqs = take;
    b.rays = rays;
    b.scr_off = scr_off;
    b.scr_len = scr_len;
    b.launch_s = now;
    b.err = RC_OK;
    s->st.batches += 1;
    s->st.queued -= (int64_t)take.size();
    s->st.in_flight += (int64_t)take.size();
    if (s->sim) {
        b.sim_done = now + s->sim_launch + (double)rays * s->sim_per_ray;
        return true;
    }
    // device work on this slot's stream: gather poses, build the camera table, render
    hipStream_t st = s->streams[k];
    char* base = s->scratch + scr_off;
    const int B = s->n_links;
    float* lp = (float*)base;
    float* lq = (float*)(base + align_up((size_t)n_env * B * 3 * 4));
    rc_cam_desc* desc = (rc_cam_desc*)(base + pose_bytes(n_env, B));
    char* ws = (char*)desc + align_up((size_t)n_desc * sizeof(rc_cam_desc));
    const size_t ws_bytes = scr_len - (size_t)(ws - base);
    hipError_t e = hipSuccess;
    int env_base = 0;
    int64_t d0 = 0;
    for (const Req& q : take) {
        if (B > 0 && e == hipSuccess)
            e = hipMemcpyAsync(lp + (size_t)env_base * B * 3, q.r.link_pos, (size_t)q.r.n_env * B * 12,
                               hipMemcpyDeviceToDevice, st);
        if (B > 0 && e == hipSuccess)
            e = hipMemcpyAsync(lq + (size_t)env_base * B * 4, q.r.link_quat, (size_t)q.r.n_env * B * 16,
                               hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) {
            const int nd = q.r.n_env * q.r.n_cam;
            hipLaunchKernelGGL(k_request_desc, dim3((nd + 255) / 256), dim3(256), 0, st, q.r, env_base,
                               (uint32_t)q.out_off, desc + d0);
            e = hipGetLastError();
            d0 += nd;
        }
        env_base += q.r.n_env;
    }
    rc_status rs = RC_OK;
    if (e == hipSuccess) {
        rc_batch_args a{};
        a.n_env = (int32_t)n_env;
        a.n_desc = (int32_t)n_desc;
        a.link_pos = B > 0 ? lp : nullptr;
        a.link_quat = B > 0 ? lq : nullptr;
        a.desc = desc;
        a.n_pixels = s->cfg.out_pixels;
        a.max_width = max_w;
        a.max_height = max_h;
        a.far_plane = s->cfg.far_plane;
        a.depth_mode = s->cfg.depth_mode;
        a.depth = s->depth;
        a.inst = s->inst;
        a.tri = s->tri;
        a.timing = nullptr;
        rs = enqueue_batched(s->scene, &a, rays, ws, ws_bytes, st);
    } else {
        rs = RC_ERR_DEVICE;
        set_error(std::string("serving batch: ") + hipGetErrorString(e));
    }
    if (rs == RC_OK) {
        e = hipEventRecord(s->events[k], st);
        if (e != hipSuccess) rs = RC_ERR_DEVICE;
    }
    b.err = rs;
    if (rs != RC_OK) finish_batch(s, b, now, rs);  // report the failure on its requests
    return true;
}

}  // namespace

extern "C" {

rc_status rc_server_arena_size(const rc_server_config* cfg, size_t scratch_bytes, size_t* bytes) {
    if (!cfg_ok(cfg) || !bytes) return fail_s(RC_ERR_INVALID_ARG, "rc_server_arena_size: bad config");
    *bytes = planes_bytes(cfg) + align_up(scratch_bytes);
    return RC_OK;
}

static rc_server* make_server(const rc_server_config* cfg, size_t arena_bytes) {
    rc_server* s = new (std::nothrow) rc_server();
    if (!s) return nullptr;
    s->cfg = *cfg;
    s->pix = RangeAlloc((uint64_t)cfg->out_pixels);
    s->scratch_bytes = arena_bytes - planes_bytes(cfg);
    s->scr = RangeAlloc((uint64_t)s->scratch_bytes);
    s->slots.resize((size_t)cfg->n_streams);
    return s;
}

rc_status rc_server_create(const rc_scene* scene, const rc_server_config* cfg, void* arena,
                           size_t arena_bytes, rc_server** out) {
    if (!out || !arena || !scene_ready(scene)) return fail_s(RC_ERR_INVALID_ARG, "rc_server_create: NULL");
    if (!cfg_ok(cfg)) return fail_s(RC_ERR_INVALID_ARG, "rc_server_create: bad config");
    if (((uintptr_t)arena % 256) != 0 || arena_bytes <= planes_bytes(cfg))
        return fail_s(RC_ERR_WORKSPACE, "rc_server_create: arena too small or misaligned");
    rc_server* s = make_server(cfg, arena_bytes);
    if (!s) return fail_s(RC_ERR_DEVICE, "rc_server_create: out of host memory");
    s->scene = scene;
    s->n_links = scene_links(scene);
    char* a = (char*)arena;
    const size_t plane = align_up((size_t)cfg->out_pixels * 4);
    s->depth = (float*)a;
    s->inst = (int32_t*)(a + plane);
    s->tri = (int32_t*)(a + 2 * plane);
    s->scratch = a + 3 * plane;
    for (int k = 0; k < cfg->n_streams; ++k) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        const bool st_ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        const bool ev_ok = st_ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
        if (!ev_ok) {  // release what was made (cleanup is best effort)
            if (st_ok) (void)hipStreamDestroy(st);
            for (size_t j = 0; j < s->streams.size(); ++j) {
                (void)hipStreamDestroy(s->streams[j]);
                (void)hipEventDestroy(s->events[j]);
            }
            delete s;
            return fail_s(RC_ERR_DEVICE, "rc_server_create: stream or event creation failed");
        }
        s->streams.push_back(st);
        s->events.push_back(ev);
    }
    *out = s;
    return RC_OK;
}

rc_status rc_server_create_simulated(const rc_server_config* cfg, size_t arena_bytes,
                                     double launch_s, double s_per_ray, rc_server** out) {
    if (!out || !cfg_ok(cfg)) return fail_s(RC_ERR_INVALID_ARG, "rc_server_create_simulated: bad args");
    if (arena_bytes <= planes_bytes(cfg) || !(launch_s >= 0) || !(s_per_ray >= 0))
        return fail_s(RC_ERR_INVALID_ARG, "rc_server_create_simulated: bad arena or model");
    rc_server* s = make_server(cfg, arena_bytes);
    if (!s) return fail_s(RC_ERR_DEVICE, "rc_server_create_simulated: out of host memory");
    s->sim = true;
    s->sim_launch = launch_s;
    s->sim_per_ray = s_per_ray;
    s->n_links = 30;
    *out = s;
    return RC_OK;
}

rc_status rc_server_submit(rc_server* s, const rc_request* r, double now_s, int64_t* id) {
    if (!s || !r) return fail_s(RC_ERR_INVALID_ARG, "rc_server_submit: NULL");
    if (r->n_env < 1 || r->n_cam < 1 || r->width < 1 || r->height < 1 || r->width > 65535 ||
        r->height > 65535)
        return fail_s(RC_ERR_INVALID_ARG, "rc_server_submit: sizes must be >= 1");
    if (!s->sim && (!r->cam_pos || !r->cam_quat || !r->intr ||
                    (s->n_links > 0 && (!r->link_pos || !r->link_quat))))
        return fail_s(RC_ERR_INVALID_ARG, "rc_server_submit: NULL device array");
    const int64_t px = (int64_t)r->n_env * r->n_cam * r->width * r->height;
    if (px > s->cfg.out_pixels || s->batch_scratch(r->n_env, (int64_t)r->n_env * r->n_cam, px) >
                                      s->scratch_bytes) {
        s->st.rejected += 1;
        return fail_s(RC_ERR_WORKSPACE, "rc_server_submit: request can never fit the arena");
    }
    Req q;
    q.id = s->next_id++;
    q.r = *r;
    q.arrival = now_s;
    q.pixels = px;
    s->queue.push_back(q);
    s->st.submitted += 1;
    s->st.queued += 1;
    if (s->st.submitted == 1 || now_s < s->st.first_arrival_s) s->st.first_arrival_s = now_s;
    if (id) *id = q.id;
    return RC_OK;
}

// A batch that finished on the device, or failed on purpose when a failure
// was injected (rc_server_fail_next).
static void finish_ok(rc_server* s, Batch& b, double now_s) {
    if (s->fail_next > 0) {
        s->fail_next -= 1;
        set_error("serving batch: injected failure (rc_server_fail_next)");
        finish_batch(s, b, now_s, RC_ERR_DEVICE);
        return;
    }
    finish_batch(s, b, now_s, RC_OK);
}

rc_status rc_server_fail_next(rc_server* s, int32_t n_batches) {
    if (!s || n_batches < 0) return fail_s(RC_ERR_INVALID_ARG, "rc_server_fail_next: bad args");
    s->fail_next = n_batches;
    return RC_OK;
}

rc_status rc_server_poll(rc_server* s, double now_s, int32_t* n_done) {
    if (!s) return fail_s(RC_ERR_INVALID_ARG, "rc_server_poll: NULL");
    for (size_t k = 0; k < s->slots.size(); ++k) {
        Batch& b = s->slots[k];
        if (!b.active) continue;
        if (s->sim) {
            if (now_s >= b.sim_done) finish_ok(s, b, now_s);
            continue;
        }
        const hipError_t q = hipEventQuery(s->events[k]);
        if (q == hipSuccess) finish_ok(s, b, now_s);
        else if (q != hipErrorNotReady) {
            set_error(std::string("serving batch: ") + hipGetErrorString(q));
            finish_batch(s, b, now_s, RC_ERR_DEVICE);
        }
    }
    for (size_t k = 0; k < s->slots.size() && !s->queue.empty(); ++k)
        if (!s->slots[k].active && !start_batch(s, (int)k, now_s)) break;
    if (n_done) *n_done = (int32_t)s->ready.size();
    return RC_OK;
}

rc_status rc_server_next_result(rc_server* s, rc_result* out) {
    if (!s || !out) return fail_s(RC_ERR_INVALID_ARG, "rc_server_next_result: NULL");
    if (s->ready.empty()) return fail_s(RC_ERR_STATE, "rc_server_next_result: nothing finished");
    *out = s->ready.front();
    s->ready.pop_front();
    return RC_OK;
}

rc_status rc_server_release(rc_server* s, int64_t id) {
    if (!s) return fail_s(RC_ERR_INVALID_ARG, "rc_server_release: NULL");
    auto it = s->out_of.find(id);
    if (it == s->out_of.end()) return fail_s(RC_ERR_STATE, "rc_server_release: unknown or live id");
    for (const rc_result& r : s->ready)
        if (r.id == id) return fail_s(RC_ERR_STATE, "rc_server_release: result not taken yet");
    s->pix.release(it->second.out_off, (uint64_t)it->second.pixels);
    s->out_of.erase(it);
    return RC_OK;
}

rc_status rc_server_stats_get(const rc_server* s, rc_server_stats* out) {
    if (!s || !out) return fail_s(RC_ERR_INVALID_ARG, "rc_server_stats_get: NULL");
    *out = s->st;
    if (!s->lat.empty()) {
        std::vector<double> v = s->lat;
        std::sort(v.begin(), v.end());
        auto rank = [&](double q) {  // nearest-rank percentile
            size_t i = (size_t)std::ceil(q * (double)v.size());
            return v[i == 0 ? 0 : i - 1];
        };
        out->p50_s = rank(0.50);
        out->p99_s = rank(0.99);
        double sum = 0;
        for (double x : v) sum += x;
        out->mean_s = sum / (double)v.size();
        out->max_s = v.back();
    }
    return RC_OK;
}

rc_status rc_server_destroy(rc_server* s) {
    if (!s) return RC_OK;
    hipError_t first = hipSuccess;  // everything is released even after a device error
    for (size_t k = 0; k < s->streams.size(); ++k) {
        const hipError_t e = hipStreamSynchronize(s->streams[k]);
        if (first == hipSuccess) first = e;
        (void)hipStreamDestroy(s->streams[k]);
        (void)hipEventDestroy(s->events[k]);
    }
    delete s;
    if (first != hipSuccess) return fail_s(RC_ERR_DEVICE, std::string("rc_server_destroy: ") +
                                                              hipGetErrorString(first));
    return RC_OK;
}

}  // extern "C"
