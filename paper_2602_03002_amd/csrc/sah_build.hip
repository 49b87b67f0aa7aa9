// Top-down binned surface-area-heuristic build of a binary hierarchy over
// triangles, on the host, in the renderer's record layout (one triangle per
// leaf).  The static terrain (Sec. 3.2.2: built once, shared by every
// environment) gets it after its Morton build: the records, the leaf-order
// triangles and their input ids are replaced in place, so every walk reads
// the same layout and finds the same closest hits, with fewer visits.
//
// Method: binned SAH (MacDonald and Booth 1990; binning as in Wald 2007).
// A range of triangles is split along the axis and bin boundary (32 bins of
// its centroid bounds per axis) that minimise area(left) * n_left +
// area(right) * n_right; a range whose centroids coincide on every axis is
// halved.  Child boxes are the unions of their triangles' boxes, padded
// outward like the Morton build's; a zero-area triangle keeps its centroid
// for the split but has an empty box, so a child holding only such
// triangles gets the far point.  Node numbering is pre-order with the root
// at 0: a node over s leaves heads s - 1 internal nodes, so the right child
// of node i over [b, e) split at m is i + (m - b) without any ordering pass,
// and leaves are numbered by their final position.  Deterministic: stable
// partitions, first minimum in (axis, bin) order; below the top levels the
// subtrees are built on up to 16 threads, each in its own index range and
// records, so the result does not depend on the threads.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "rc_internal.h"

namespace rc {

namespace {

constexpr int kBins = 32;
constexpr float kPadRelH = 1.0f / 1048576.0f;  // 2^-20, as the Morton build's padding
constexpr float kPadAbsH = 1e-5f;

struct HBox {
    float lo[3] = {INFINITY, INFINITY, INFINITY};
    float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    void grow(const HBox& o) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], o.lo[a]);
            hi[a] = std::max(hi[a], o.hi[a]);
        }
    }
    bool empty() const { return lo[0] > hi[0] || lo[1] > hi[1] || lo[2] > hi[2]; }
    double area() const {
        if (empty()) return 0.0;
        const double x = (double)hi[0] - lo[0], y = (double)hi[1] - lo[1], z = (double)hi[2] - lo[2];
        return 2.0 * (x * y + y * z + z * x);
    }
};

// Padded child box into a record's six floats (the far point when empty).
void put_box(float* dst, const HBox& b) {
    const bool e = b.empty();
    for (int a = 0; a < 3; ++a) {
        dst[2 * a] = e ? kFarBox : b.lo[a] - (std::fabs(b.lo[a]) * kPadRelH + kPadAbsH);
        dst[2 * a + 1] = e ? kFarBox : b.hi[a] + (std::fabs(b.hi[a]) * kPadRelH + kPadAbsH);
    }
}

// Bin of a centroid coordinate; a non-finite coordinate (NaN, or an infinite
// extent) falls into bin 0 instead of an undefined conversion.
int bin_of(float c, float lo, float scale) {
    const float f = (c - lo) * scale;
    if (!(f >= 0.0f)) return 0;
    return f >= (float)kBins ? kBins - 1 : (int)f;
}

struct Task {
    int64_t b, e;  // range of the index array
    int32_t node;  // its record
    int32_t depth;
};

}  // namespace

int32_t sah_build_host(const float* tri, int64_t n, const int32_t* ids_in, float* rec, float* tris_out,
                       int32_t* ids_out) {
    if (n < 1) return -1;
    std::vector<HBox> pb((size_t)n);
    std::vector<float> cen((size_t)n * 3);
    for (int64_t i = 0; i < n; ++i) {
        const float* v = tri + 9 * i;
        HBox b;
        for (int a = 0; a < 3; ++a) {
            b.lo[a] = std::min(v[a], std::min(v[3 + a], v[6 + a]));
            b.hi[a] = std::max(v[a], std::max(v[3 + a], v[6 + a]));
            cen[3 * i + a] = 0.5f * (b.lo[a] + b.hi[a]);
        }
        // zero-area test: the FP64 cross product of the edges is exactly zero
        const double ux = (double)v[3] - v[0], uy = (double)v[4] - v[1], uz = (double)v[5] - v[2];
        const double wx = (double)v[6] - v[0], wy = (double)v[7] - v[1], wz = (double)v[8] - v[2];
        if (uy * wz - uz * wy == 0.0 && uz * wx - ux * wz == 0.0 && ux * wy - uy * wx == 0.0) b = HBox();
        pb[(size_t)i] = b;
    }
    std::vector<int32_t> idx((size_t)n);
    for (int64_t i = 0; i < n; ++i) idx[(size_t)i] = (int32_t)i;
    int32_t* ri = reinterpret_cast<int32_t*>(rec);
    int32_t max_depth = 0;

    if (n == 1) {  // one leaf: its box and the far point
        put_box(rec, pb[0]);
        for (int k = 0; k < 6; ++k) rec[6 + k] = kFarBox;
        ri[12] = ~0;
        ri[13] = ~0;
        ri[14] = -1;
        ri[15] = -1;
    } else {
        ri[14] = -1;
        ri[15] = -1;
        // One task: split its range, write its record, hand its internal
        // children on.  Tasks touch disjoint ranges and records, so subtrees
        // can be built on separate threads with the same result.
        auto split = [&](const Task& t, std::vector<Task>& out) {
            const int64_t s = t.e - t.b;
            HBox cb;
            for (int64_t k = t.b; k < t.e; ++k) {
                const float* c = &cen[3 * (size_t)idx[(size_t)k]];
                for (int a = 0; a < 3; ++a) {
                    cb.lo[a] = std::min(cb.lo[a], c[a]);
                    cb.hi[a] = std::max(cb.hi[a], c[a]);
                }
            }
            int best_axis = -1, best_bin = -1;
            double best_cost = INFINITY;
            HBox best_l, best_r;
            for (int a = 0; a < 3; ++a) {
                const float ext = cb.hi[a] - cb.lo[a];
                if (!(ext > 0.0f)) continue;
                const float scale = (float)kBins / ext;
                HBox bin[kBins];
                int64_t cnt[kBins] = {};
                for (int64_t k = t.b; k < t.e; ++k) {
                    const int32_t p = idx[(size_t)k];
                    const int j = bin_of(cen[3 * (size_t)p + a], cb.lo[a], scale);
                    bin[j].grow(pb[(size_t)p]);
                    ++cnt[j];
                }
                HBox racc[kBins];
                int64_t rcnt[kBins];
                HBox acc;
                int64_t c = 0;
                for (int j = kBins - 1; j > 0; --j) {
                    acc.grow(bin[j]);
                    c += cnt[j];
                    racc[j] = acc;
                    rcnt[j] = c;
                }
                HBox lacc;
                int64_t lc = 0;
                for (int j = 0; j < kBins - 1; ++j) {
                    lacc.grow(bin[j]);
                    lc += cnt[j];
                    if (lc == 0 || rcnt[j + 1] == 0) continue;
                    const double cost = lacc.area() * (double)lc + racc[j + 1].area() * (double)rcnt[j + 1];
                    if (cost < best_cost) {
                        best_cost = cost;
                        best_axis = a;
                        best_bin = j;
                        best_l = lacc;
                        best_r = racc[j + 1];
                    }
                }
            }
            int64_t m;
            if (best_axis >= 0) {
                const int a = best_axis;
                const float scale = (float)kBins / (cb.hi[a] - cb.lo[a]);
                auto left = [&](int32_t p) { return bin_of(cen[3 * (size_t)p + a], cb.lo[a], scale) <= best_bin; };
                m = std::stable_partition(idx.begin() + t.b, idx.begin() + t.e, left) - idx.begin();
            } else {  // every centroid coincides: halve the range
                m = t.b + s / 2;
                best_l = HBox();
                best_r = HBox();
                for (int64_t k = t.b; k < m; ++k) best_l.grow(pb[(size_t)idx[(size_t)k]]);
                for (int64_t k = m; k < t.e; ++k) best_r.grow(pb[(size_t)idx[(size_t)k]]);
            }
            const int32_t i = t.node;
            float* r = rec + 16 * (int64_t)i;
            put_box(r, best_l);
            put_box(r + 6, best_r);
            const int32_t c0 = (m - t.b == 1) ? ~(int32_t)t.b : i + 1;
            const int32_t c1 = (t.e - m == 1) ? ~(int32_t)m : i + (int32_t)(m - t.b);
            ri[16 * (int64_t)i + 12] = c0;
            ri[16 * (int64_t)i + 13] = c1;
            if (c0 >= 0) {
                ri[16 * (int64_t)c0 + 14] = i;
                ri[16 * (int64_t)c0 + 15] = c1;
            }
            if (c1 >= 0) {
                ri[16 * (int64_t)c1 + 14] = i;
                ri[16 * (int64_t)c1 + 15] = c0;
            }
            // right first, so the left subtree is finished first (any order works)
            if (c1 >= 0) out.push_back({m, t.e, c1, t.depth + 1});
            if (c0 >= 0) out.push_back({t.b, m, c0, t.depth + 1});
        };
        auto run = [&](std::vector<Task> stack, int32_t* depth) {
            while (!stack.empty()) {
                const Task t = stack.back();
                stack.pop_back();
                *depth = std::max(*depth, t.depth);
                split(t, stack);
            }
        };
        // the top of the hierarchy on this thread, until the pending
        // subtrees are small enough to share out
        const int64_t grain = std::max<int64_t>(n / 64, 4096);
        std::vector<Task> pending{{0, n, 0, 0}}, big;
        for (;;) {
            std::vector<Task> next;
            bool any = false;
            for (const Task& t : pending) {
                if (t.e - t.b > grain) {
                    max_depth = std::max(max_depth, t.depth);
                    split(t, next);
                    any = true;
                } else {
                    next.push_back(t);
                }
            }
            pending.swap(next);
            if (!any) break;
        }
        const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        const unsigned nt = (unsigned)std::min<size_t>(hw, pending.size());
        std::vector<std::vector<Task>> share(nt);
        for (size_t k = 0; k < pending.size(); ++k) share[k % nt].push_back(pending[k]);
        std::vector<int32_t> depth(nt, 0);
        std::vector<std::thread> pool;
        try {
            for (unsigned k = 1; k < nt; ++k) pool.emplace_back(run, share[k], &depth[k]);
        } catch (...) {  // no threads to be had: the rest on this one
            for (unsigned k = (unsigned)pool.size() + 1; k < nt; ++k) run(share[k], &depth[k]);
        }
        if (nt > 0) run(share[0], &depth[0]);
        for (std::thread& th : pool) th.join();
        for (int32_t d : depth) max_depth = std::max(max_depth, d);
    }
    for (int64_t k = 0; k < n; ++k) {
        const int32_t p = idx[(size_t)k];
        std::memcpy(tris_out + 9 * k, tri + 9 * (int64_t)p, 36);
        ids_out[k] = ids_in ? ids_in[p] : p;
    }
    return max_depth;
}

}  // namespace rc
