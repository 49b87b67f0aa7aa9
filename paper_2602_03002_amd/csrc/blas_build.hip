// Bottom-level hierarchy build: a linear BVH over 63-bit Morton codes.
//
// Steps (all integer work is bit-exact, boxes are exact FP32 min/max):
//   1. per-triangle box and centroid (box centre), block min/max of centroids
//   2. centroid bounds
//   3. 21-bit quantisation (one scale for all axes) and 63-bit Morton interleave
//   4. stable LSD radix sort of (key, index), 8 passes of 8-bit digits, with
//      per-block LDS histograms and an in-block stable rank from wave ballots
//   5. Karras (2012) hierarchy from the sorted keys (duplicate keys broken by
//      leaf index)
//   6. bottom-up box fit with per-node arrival counters
//   7. outward padding of every child box (conservative FP32 traversal),
//      leaf-order copies of the triangles and their input indices
//
// The paper keeps each body mesh canonical in its local frame and never
// refits it per frame (Sec. 3.2.2); this builder runs once per mesh.
#include "rc_internal.h"

#pragma clang fp contract(off)

namespace rc {

namespace {

constexpr int kThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kThreads * kSortItems;

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1FFFFFu;
    x = (x | (x << 32)) & 0x1F00000000FFFFull;
    x = (x | (x << 16)) & 0x1F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__global__ void k_prim_bounds(const float* __restrict__ tri, int64_t n, float* __restrict__ box,
                              float* __restrict__ partial) {
    __shared__ float red[6][kThreads];
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    float cmin[3] = {INFINITY, INFINITY, INFINITY}, cmax[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (i < n) {
        const float* t = tri + 9 * i;
        for (int a = 0; a < 3; ++a) {
            float lo = fminf(fminf(t[a], t[3 + a]), t[6 + a]);
            float hi = fmaxf(fmaxf(t[a], t[3 + a]), t[6 + a]);
            box[6 * i + 2 * a] = lo;
            box[6 * i + 2 * a + 1] = hi;
            float c = (lo + hi) * 0.5f;
            cmin[a] = c;
            cmax[a] = c;
        }
    }
    for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = cmin[a];
        red[3 + a][threadIdx.x] = cmax[a];
    }
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int a = 0; a < 3; ++a) {
                red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + s]);
                red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[6 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_reduce_bounds(const float* __restrict__ partial, int64_t nb, float* __restrict__ out) {
    __shared__ float red[6][kThreads];
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t b = threadIdx.x; b < nb; b += kThreads) {
        for (int a = 0; a < 3; ++a) {
            v[a] = fminf(v[a], partial[6 * b + a]);
            v[3 + a] = fmaxf(v[3 + a], partial[6 * b + 3 + a]);
        }
    }
    for (int a = 0; a < 6; ++a) red[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int a = 0; a < 3; ++a) {
                red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + s]);
                red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = red[threadIdx.x][0];
}

// key = spread(qx) << 2 | spread(qy) << 1 | spread(qz), q = trunc(clamp((c - cmin) * s)),
// c = (lo + hi) * 0.5, with ONE scale for all axes, s = 2^21 / (largest centroid
// extent) (0 if every centroid coincides).  A common scale keeps the cells
// cubic: a terrain spans ~100 m in x and y but metres in z, and per-axis
// scales would spend Morton bits on thin z slices and split poorly.
__global__ void k_morton(const float* __restrict__ box, int64_t n, const float* __restrict__ cb,
                         uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const float ext = fmaxf(fmaxf(cb[3] - cb[0], cb[4] - cb[1]), cb[5] - cb[2]);
    const float s = ext > 0.0f ? __fdiv_rn(2097152.0f, ext) : 0.0f;
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
        float lo = box[6 * i + 2 * a], hi = box[6 * i + 2 * a + 1];
        float c = (lo + hi) * 0.5f;
        float f = (c - cb[a]) * s;
        f = fminf(fmaxf(f, 0.0f), 2097151.0f);
        q[a] = (uint32_t)f;
    }
    keys[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    vals[i] = (uint32_t)i;
}

__global__ void k_radix_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                             uint32_t* __restrict__ hist, int64_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive prefix sum of `total` counters, one block of 1024 threads.
__global__ void __launch_bounds__(1024) k_exclusive_scan(uint32_t* __restrict__ v, int64_t total) {
    __shared__ uint32_t sums[1024];
    int64_t chunk = (total + 1023) / 1024;
    int64_t b = (int64_t)threadIdx.x * chunk;
    int64_t e = b + chunk < total ? b + chunk : total;
    uint32_t s = 0;
    for (int64_t k = b; k < e; ++k) s += v[k];
    sums[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t add = threadIdx.x >= (unsigned)off ? sums[threadIdx.x - off] : 0u;
        __syncthreads();
        sums[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = sums[threadIdx.x] - s;
    for (int64_t k = b; k < e; ++k) {
        uint32_t x = v[k];
        v[k] = run;
        run += x;
    }
}

// Stable scatter: within a round the 256 elements are ranked by (wave, lane)
// among equal digits (ballot match), rounds are taken in element order.
__global__ void k_radix_scatter(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, int64_t n,
                                int shift, const uint32_t* __restrict__ hist, int64_t nblocks) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[kThreads / 64][256];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    base[tid] = hist[(int64_t)tid * nblocks + blockIdx.x];
    int64_t tile = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        for (int w = 0; w < kThreads / 64; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        int64_t i = tile + (int64_t)r * kThreads + tid;
        bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0ull;
        uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t mask = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t bal = __ballot(bit);
            mask &= bit ? bal : ~bal;
        }
        uint32_t rank = (uint32_t)__popcll(mask & lt);
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(mask);
        __syncthreads();
        if (valid) {
            uint32_t off = base[d] + rank;
            for (int w = 0; w < wave; ++w) off += wcnt[w][d];
            kout[off] = key;
            vout[off] = vin[i];
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kThreads / 64; ++w) add += wcnt[w][tid];
        base[tid] += add;
        __syncthreads();
    }
}

__device__ __forceinline__ int kdelta(const uint64_t* __restrict__ keys, int64_t n, int64_t i,
                                      int64_t j) {
    if (j < 0 || j >= n) return -1;
    uint64_t a = keys[i], b = keys[j];
    if (a != b) return __clzll((long long)(a ^ b));
    return 64 + __clz((int)((uint32_t)i ^ (uint32_t)j));
}

__global__ void k_karras(const uint64_t* __restrict__ keys, int64_t n, Node* __restrict__ nodes,
                         int32_t* __restrict__ leaf_parent) {
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n - 1) return;
    int d = (kdelta(keys, n, i, i + 1) - kdelta(keys, n, i, i - 1)) > 0 ? 1 : -1;
    int dmin = kdelta(keys, n, i, i - d);
    int64_t lmax = 2;
    while (kdelta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int64_t l = 0;
    for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
        if (kdelta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    int64_t j = i + l * d;
    int dnode = kdelta(keys, n, i, j);
    int64_t s = 0;
    for (int64_t div = 2;; div <<= 1) {
        int64_t t = (l + div - 1) / div;
        if (kdelta(keys, n, i, i + (s + t) * d) > dnode) s += t;
        if (t <= 1) break;
    }
    int64_t g = i + s * d + (d < 0 ? -1 : 0);
    int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    int32_t c0 = (lo == g) ? ~(int32_t)g : (int32_t)g;
    int32_t c1 = (hi == g + 1) ? ~(int32_t)(g + 1) : (int32_t)(g + 1);
    nodes[i].c0 = c0;
    nodes[i].c1 = c1;
    if (c0 >= 0) { nodes[c0].parent = (int32_t)i; nodes[c0].sibling = c1; }
    else leaf_parent[~c0] = (int32_t)i;
    if (c1 >= 0) { nodes[c1].parent = (int32_t)i; nodes[c1].sibling = c0; }
    else leaf_parent[~c1] = (int32_t)i;
    if (i == 0) { nodes[0].parent = -1; nodes[0].sibling = -1; }
}

__global__ void k_zero_u32(uint32_t* __restrict__ p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__device__ __forceinline__ float aload(const float* p) {
    uint32_t u = __hip_atomic_load((const uint32_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __uint_as_float(u);
}

// A triangle of zero area (its edge vectors parallel: coincident or
// collinear vertices) is met by no ray; its leaf box becomes empty, which the
// bottom-up union ignores, and the padding step makes it unreachable.  Edges
// and cross product in FP64 (exact for single-precision vertices of similar
// magnitude), zero in all three components.
__global__ void k_drop_degenerate(const float* __restrict__ tri, int64_t n, float* __restrict__ box) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const float* t = tri + 9 * i;
    const double ux = (double)t[3] - (double)t[0], uy = (double)t[4] - (double)t[1],
                 uz = (double)t[5] - (double)t[2];
    const double vx = (double)t[6] - (double)t[0], vy = (double)t[7] - (double)t[1],
                 vz = (double)t[8] - (double)t[2];
    const double cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
    if (cx == 0.0 && cy == 0.0 && cz == 0.0) {
        for (int a = 0; a < 3; ++a) {
            box[6 * i + 2 * a] = INFINITY;
            box[6 * i + 2 * a + 1] = -INFINITY;
        }
    }
}

__global__ void k_fit(const float* __restrict__ box, const uint32_t* __restrict__ vals, int64_t n,
                      Node* nodes, const int32_t* __restrict__ leaf_parent, uint32_t* flags) {
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    float b[6];
    const float* pb = box + 6 * (int64_t)vals[i];
    for (int k = 0; k < 6; ++k) b[k] = pb[k];
    int32_t me = ~(int32_t)i;
    int32_t p = leaf_parent[i];
    // a valid hierarchy is at most 96 levels deep (63 key bits + 32 index bits)
    for (int guard = 0; p >= 0 && p < n - 1 && guard < 128; ++guard) {
        Node* P = nodes + p;
        int slot = (P->c0 == me) ? 0 : 1;
        float* dst = slot == 0 ? P->b0 : P->b1;
        for (int k = 0; k < 6; ++k) dst[k] = b[k];
        __threadfence();
        uint32_t old = atomicAdd(flags + p, 1u);
        if (old == 0u) return;
        __threadfence();
        const float* oth = slot == 0 ? P->b1 : P->b0;
        for (int a = 0; a < 3; ++a) {
            b[2 * a] = fminf(b[2 * a], aload(oth + 2 * a));
            b[2 * a + 1] = fmaxf(b[2 * a + 1], aload(oth + 2 * a + 1));
        }
        me = p;
        p = P->parent;
    }
}

// Deepest internal node (root depth 0), by climbing from every internal node.
__global__ void k_depth(const Node* __restrict__ nodes, int64_t n_int, int32_t* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n_int) return;
    int d = 0;
    int32_t p = nodes[i].parent;
    while (p >= 0 && d <= 1000000) { ++d; p = nodes[p].parent; }
    atomicMax(out, d);
}

__device__ __forceinline__ float pad_lo(float x) { return x - (fabsf(x) * kPadRel + kPadAbs); }
__device__ __forceinline__ float pad_hi(float x) { return x + (fabsf(x) * kPadRel + kPadAbs); }

// Pad a child box outward, or, if it is empty (a subtree of zero-area
// triangles only), replace it by the far point no ray reaches.
__device__ __forceinline__ void pad_box(float* b) {
    const bool empty = (b[0] > b[1]) | (b[2] > b[3]) | (b[4] > b[5]);
    for (int a = 0; a < 3; ++a) {
        b[2 * a] = empty ? kFarBox : pad_lo(b[2 * a]);
        b[2 * a + 1] = empty ? kFarBox : pad_hi(b[2 * a + 1]);
    }
}

__global__ void k_pad_and_gather(Node* __restrict__ nodes, int64_t n_int, const float* __restrict__ tri,
                                 const uint32_t* __restrict__ vals, int64_t n,
                                 float* __restrict__ tris, int32_t* __restrict__ tri_id) {
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n_int) {
        Node* P = nodes + i;
        pad_box(P->b0);
        pad_box(P->b1);
    }
    if (i < n) {
        uint32_t v = vals[i];
        for (int k = 0; k < 9; ++k) tris[9 * i + k] = tri[9 * (int64_t)v + k];
        tri_id[i] = (int32_t)v;
    }
}

// One-leaf hierarchy: a single record whose second box is a point far beyond
// any far plane (an inverted box would not be empty under a min/max slab test).
__global__ void k_single_leaf(const float* __restrict__ box, Node* __restrict__ nodes,
                              const float* __restrict__ tri, float* __restrict__ tris,
                              int32_t* __restrict__ tri_id, uint64_t* __restrict__ keys,
                              int32_t* __restrict__ depth) {
    Node* P = nodes;
    for (int k = 0; k < 6; ++k) {
        P->b0[k] = box[k];
        P->b1[k] = kFarBox;
    }
    pad_box(P->b0);
    P->c0 = ~0;
    P->c1 = ~0;
    P->parent = -1;
    P->sibling = -1;
    for (int k = 0; k < 9; ++k) tris[k] = tri[k];
    tri_id[0] = 0;
    keys[0] = 0ull;
    *depth = 0;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// 4-wide records, one per binary node (the layout is described with
// kWideRec).  Every node gets one, since a walk may enter the hierarchy at any
// node; slots keep the binary children's order (child 0's side first).
__global__ void k_collapse4(const Node* __restrict__ nodes, int64_t n_nodes, float4* __restrict__ out) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    const Node N = nodes[n];
    float b[4][6];
    int c[4];
    int m = 0;
    for (int h = 0; h < 2; ++h) {
        const int ch = h ? N.c1 : N.c0;
        const float* bx = h ? N.b1 : N.b0;
        if (ch < 0 || ch >= n_nodes || bx[0] == kFarBox) {  // leaf, or a child no ray reaches
            for (int k = 0; k < 6; ++k) b[m][k] = bx[k];
            c[m++] = ch;
        } else {
            const Node C = nodes[ch];
            for (int k = 0; k < 6; ++k) b[m][k] = C.b0[k];
            c[m++] = C.c0;
            for (int k = 0; k < 6; ++k) b[m][k] = C.b1[k];
            c[m++] = C.c1;
        }
    }
    for (; m < 4; ++m) {
        for (int k = 0; k < 6; ++k) b[m][k] = kFarBox;
        c[m] = 0;
    }
    float4* o = out + kWideRec * n;
    for (int k = 0; k < 6; ++k) o[k] = make_float4(b[0][k], b[1][k], b[2][k], b[3][k]);
    o[6] = make_float4(__int_as_float(c[0]), __int_as_float(c[1]), __int_as_float(c[2]),
                       __int_as_float(c[3]));
    o[7] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

}  // namespace

hipError_t launch_collapse4(const Node* nodes, int64_t n_nodes, float4* out, hipStream_t s) {
    hipLaunchKernelGGL(k_collapse4, dim3(nblk(n_nodes)), dim3(kThreads), 0, s, nodes, n_nodes, out);
    return hipGetLastError();
}

BvhLayout bvh_layout(int64_t n, size_t base) {
    BvhLayout L;
    L.n_prim = n;
    L.n_nodes = n > 1 ? n - 1 : 1;
    L.n_blocks_sort = (n + kSortTile - 1) / kSortTile;
    L.n_blocks_red = (n + kThreads - 1) / kThreads;
    size_t o = align_up(base);
    L.nodes = o;     o = align_up(o + (size_t)L.n_nodes * sizeof(Node));
    L.wide = o;      o = align_up(o + (size_t)L.n_nodes * kWideRec * sizeof(float4));
    L.tris = o;      o = align_up(o + (size_t)n * 36);
    L.tri_id = o;    o = align_up(o + (size_t)n * 4);
    L.keys = o;      o = align_up(o + (size_t)n * 8);
    L.keys_alt = o;  o = align_up(o + (size_t)n * 8);
    L.vals = o;      o = align_up(o + (size_t)n * 4);
    L.vals_alt = o;  o = align_up(o + (size_t)n * 4);
    L.prim_box = o;  o = align_up(o + (size_t)n * 24);
    L.flags = o;     o = align_up(o + (size_t)L.n_nodes * 4);
    L.leaf_parent = o; o = align_up(o + (size_t)n * 4);
    L.hist = o;      o = align_up(o + (size_t)256 * L.n_blocks_sort * 4);
    L.partial = o;   o = align_up(o + (size_t)L.n_blocks_red * 24);
    L.cbounds = o;   o = align_up(o + 32);
    L.depth = o;     o = align_up(o + 4);
    L.end = o;
    return L;
}

hipError_t launch_blas_build(const float* tri, int64_t n, char* ws, const BvhLayout& L,
                             hipStream_t s) {
    Node* nodes = (Node*)(ws + L.nodes);
    float* tris = (float*)(ws + L.tris);
    int32_t* tri_id = (int32_t*)(ws + L.tri_id);
    uint64_t* keys = (uint64_t*)(ws + L.keys);
    uint64_t* keys_alt = (uint64_t*)(ws + L.keys_alt);
    uint32_t* vals = (uint32_t*)(ws + L.vals);
    uint32_t* vals_alt = (uint32_t*)(ws + L.vals_alt);
    float* box = (float*)(ws + L.prim_box);
    uint32_t* flags = (uint32_t*)(ws + L.flags);
    int32_t* leaf_parent = (int32_t*)(ws + L.leaf_parent);
    uint32_t* hist = (uint32_t*)(ws + L.hist);
    float* partial = (float*)(ws + L.partial);
    float* cb = (float*)(ws + L.cbounds);
    int32_t* depth = (int32_t*)(ws + L.depth);

    hipLaunchKernelGGL(k_prim_bounds, dim3(nblk(n)), dim3(kThreads), 0, s, tri, n, box, partial);
    if (n == 1) {
        hipLaunchKernelGGL(k_drop_degenerate, dim3(1), dim3(kThreads), 0, s, tri, n, box);
        hipLaunchKernelGGL(k_single_leaf, dim3(1), dim3(1), 0, s, box, nodes, tri, tris, tri_id,
                           keys, depth);
        hipLaunchKernelGGL(k_collapse4, dim3(1), dim3(kThreads), 0, s, nodes, (int64_t)1,
                           (float4*)(ws + L.wide));
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_reduce_bounds, dim3(1), dim3(kThreads), 0, s, partial, L.n_blocks_red, cb);
    hipLaunchKernelGGL(k_morton, dim3(nblk(n)), dim3(kThreads), 0, s, box, n, cb, keys, vals);
    // after the codes (box centres): zero-area triangles get empty leaf boxes
    hipLaunchKernelGGL(k_drop_degenerate, dim3(nblk(n)), dim3(kThreads), 0, s, tri, n, box);
    const int64_t nb = L.n_blocks_sort;
    uint64_t* kin = keys;
    uint64_t* kout = keys_alt;
    uint32_t* vin = vals;
    uint32_t* vout = vals_alt;
    for (int pass = 0; pass < 8; ++pass) {
        int shift = 8 * pass;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kThreads), 0, s, kin, n, shift, hist, nb);
        hipLaunchKernelGGL(k_exclusive_scan, dim3(1), dim3(1024), 0, s, hist, (int64_t)256 * nb);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kThreads), 0, s, kin, vin, kout,
                           vout, n, shift, hist, nb);
        uint64_t* tk = kin; kin = kout; kout = tk;
        uint32_t* tv = vin; vin = vout; vout = tv;
    }
    // after 8 passes the sorted data is back in keys / vals
    hipLaunchKernelGGL(k_karras, dim3(nblk(n - 1)), dim3(kThreads), 0, s, keys, n, nodes, leaf_parent);
    hipLaunchKernelGGL(k_zero_u32, dim3(nblk(n - 1)), dim3(kThreads), 0, s, flags, n - 1);
    hipLaunchKernelGGL(k_fit, dim3(nblk(n)), dim3(kThreads), 0, s, box, vals, n, nodes, leaf_parent, flags);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(kThreads), 0, s, (uint32_t*)depth, (int64_t)1);
    hipLaunchKernelGGL(k_depth, dim3(nblk(n - 1)), dim3(kThreads), 0, s, nodes, n - 1, depth);
    hipLaunchKernelGGL(k_pad_and_gather, dim3(nblk(n)), dim3(kThreads), 0, s, nodes, n - 1, tri, vals,
                       n, tris, tri_id);
    hipLaunchKernelGGL(k_collapse4, dim3(nblk(n - 1)), dim3(kThreads), 0, s, nodes, n - 1,
                       (float4*)(ws + L.wide));
    return hipGetLastError();
}

}  // namespace rc
