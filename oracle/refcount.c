/*
 * Reference traversal counts for the bandwidth roofline (MEASUREMENT AID,
 * test/bench infrastructure only; not a parity oracle, shares no code with
 * the GPU renderer).
 *
 * The roofline prices what a bounding-volume-hierarchy ray caster must move
 * per ray: node records, triangles and instance poses.  To keep that figure
 * independent of the GPU's own hierarchy quality, the counts come from a
 * classic reference: binned surface-area-heuristic BVH2 per mesh (32 bins,
 * traversal cost 1, triangle cost 1, leaves of at most 4 triangles), an SAH
 * top level over each environment's link instances, and ordered
 * closest-first traversal with an explicit stack under the same bound as
 * the renderer (links first, then terrain, Algorithm 1 of the paper).
 * Counted per ray: internal-node visits (each reads two child boxes and two
 * child references), triangles tested, link instances entered.  FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NBINS 32
#define MAX_LEAF 4

typedef struct { double lo[3], hi[3]; } box_t;
typedef struct { box_t b[2]; int child[2]; /* >= 0 internal; < 0: leaf ~k */ } rnode_t;
typedef struct { int first, count; } rleaf_t;
typedef struct {
    rnode_t* nodes; int n_nodes, cap_nodes;
    rleaf_t* leaves; int n_leaves, cap_leaves;
    int* prim;  /* leaf ranges index into prim[] */
    box_t root; int root_ref;
} rbvh_t;

static void box_empty(box_t* b) {
    for (int a = 0; a < 3; ++a) { b->lo[a] = INFINITY; b->hi[a] = -INFINITY; }
}
static void box_grow(box_t* b, const box_t* o) {
    for (int a = 0; a < 3; ++a) {
        if (o->lo[a] < b->lo[a]) b->lo[a] = o->lo[a];
        if (o->hi[a] > b->hi[a]) b->hi[a] = o->hi[a];
    }
}
static double box_area(const box_t* b) {
    double d[3];
    for (int a = 0; a < 3; ++a) { d[a] = b->hi[a] - b->lo[a]; if (d[a] < 0) return 0.0; }
    return 2.0 * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0]);
}

static int new_node(rbvh_t* t) {
    if (t->n_nodes == t->cap_nodes) {
        t->cap_nodes = t->cap_nodes ? 2 * t->cap_nodes : 64;
        t->nodes = (rnode_t*)realloc(t->nodes, sizeof(rnode_t) * t->cap_nodes);
    }
    return t->n_nodes++;
}
static int new_leaf(rbvh_t* t, int first, int count) {
    if (t->n_leaves == t->cap_leaves) {
        t->cap_leaves = t->cap_leaves ? 2 * t->cap_leaves : 64;
        t->leaves = (rleaf_t*)realloc(t->leaves, sizeof(rleaf_t) * t->cap_leaves);
    }
    t->leaves[t->n_leaves].first = first;
    t->leaves[t->n_leaves].count = count;
    return ~(t->n_leaves++);
}

/* Build over prim[first, first + n); returns the ref of the subtree. */
static int build_rec(rbvh_t* t, const box_t* pb, const double* cen, int first, int n, box_t* out) {
    box_t bb, cb;
    box_empty(&bb); box_empty(&cb);
    for (int i = first; i < first + n; ++i) {
        box_grow(&bb, &pb[t->prim[i]]);
        box_t c; for (int a = 0; a < 3; ++a) c.lo[a] = c.hi[a] = cen[3 * t->prim[i] + a];
        box_grow(&cb, &c);
    }
    *out = bb;
    if (n == 1) return new_leaf(t, first, n);
    double best = INFINITY; int best_axis = -1, best_split = -1;
    for (int a = 0; a < 3; ++a) {
        double ext = cb.hi[a] - cb.lo[a];
        if (!(ext > 0)) continue;
        box_t bin[NBINS]; int cnt[NBINS];
        for (int k = 0; k < NBINS; ++k) { box_empty(&bin[k]); cnt[k] = 0; }
        for (int i = first; i < first + n; ++i) {
            int k = (int)((cen[3 * t->prim[i] + a] - cb.lo[a]) / ext * NBINS);
            if (k >= NBINS) k = NBINS - 1;
            box_grow(&bin[k], &pb[t->prim[i]]); cnt[k]++;
        }
        double rarea[NBINS]; int rcnt[NBINS]; box_t acc; box_empty(&acc); int c = 0;
        for (int k = NBINS - 1; k > 0; --k) { box_grow(&acc, &bin[k]); c += cnt[k]; rarea[k] = box_area(&acc); rcnt[k] = c; }
        box_empty(&acc); c = 0;
        for (int k = 0; k < NBINS - 1; ++k) {
            box_grow(&acc, &bin[k]); c += cnt[k];
            if (c == 0 || rcnt[k + 1] == 0) continue;
            double cost = box_area(&acc) * c + rarea[k + 1] * rcnt[k + 1];
            if (cost < best) { best = cost; best_axis = a; best_split = k; }
        }
    }
    double leaf_cost = (double)n;  /* C_tri = 1 per triangle */
    double split_cost = best_axis >= 0 ? 1.0 + best / box_area(&bb) : INFINITY;
    if (best_axis < 0 || (n <= MAX_LEAF && leaf_cost <= split_cost)) {
        if (n <= MAX_LEAF || best_axis < 0) {
            if (n <= MAX_LEAF) return new_leaf(t, first, n);
            /* degenerate centroids: split in the middle of the list */
            best_axis = -2;
        }
    }
    int mid;
    if (best_axis >= 0) {
        double ext = cb.hi[best_axis] - cb.lo[best_axis];
        int i = first, j = first + n - 1;
        while (i <= j) {
            int k = (int)((cen[3 * t->prim[i] + best_axis] - cb.lo[best_axis]) / ext * NBINS);
            if (k >= NBINS) k = NBINS - 1;
            if (k <= best_split) ++i;
            else { int s = t->prim[i]; t->prim[i] = t->prim[j]; t->prim[j] = s; --j; }
        }
        mid = i - first;
        if (mid == 0 || mid == n) mid = n / 2;
    } else {
        mid = n / 2;
    }
    int me = new_node(t);
    box_t b0, b1;
    int c0 = build_rec(t, pb, cen, first, mid, &b0);
    int c1 = build_rec(t, pb, cen, first + mid, n - mid, &b1);
    t->nodes[me].b[0] = b0; t->nodes[me].b[1] = b1;
    t->nodes[me].child[0] = c0; t->nodes[me].child[1] = c1;
    return me;
}

static void rbvh_build(rbvh_t* t, const box_t* pb, int n) {
    memset(t, 0, sizeof(*t));
    double* cen = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    t->prim = (int*)malloc(sizeof(int) * (size_t)n);
    for (int i = 0; i < n; ++i) {
        t->prim[i] = i;
        for (int a = 0; a < 3; ++a) cen[3 * i + a] = 0.5 * (pb[i].lo[a] + pb[i].hi[a]);
    }
    t->root_ref = build_rec(t, pb, cen, 0, n, &t->root);
    free(cen);
}

static void rbvh_free(rbvh_t* t) { free(t->nodes); free(t->leaves); free(t->prim); }

static void tri_box(const float* v, box_t* b) {
    box_empty(b);
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 3; ++a) {
            double x = v[3 * k + a];
            if (x < b->lo[a]) b->lo[a] = x;
            if (x > b->hi[a]) b->hi[a] = x;
        }
}

static int slab(const box_t* b, const double o[3], const double inv[3], double tmax, double* tn) {
    double a = 0.0, z = tmax;
    for (int k = 0; k < 3; ++k) {
        double t0 = (b->lo[k] - o[k]) * inv[k], t1 = (b->hi[k] - o[k]) * inv[k];
        if (t0 > t1) { double s = t0; t0 = t1; t1 = s; }
        if (t0 > a) a = t0;
        if (t1 < z) z = t1;
    }
    *tn = a;
    return a <= z;
}

static int tri_hit(const float* v, const double o[3], const double d[3], double* lam) {
    double p0[3] = {v[0], v[1], v[2]}, e1[3], e2[3], P[3], T[3], Q[3];
    for (int a = 0; a < 3; ++a) { e1[a] = v[3 + a] - p0[a]; e2[a] = v[6 + a] - p0[a]; T[a] = o[a] - p0[a]; }
    P[0] = d[1] * e2[2] - d[2] * e2[1]; P[1] = d[2] * e2[0] - d[0] * e2[2]; P[2] = d[0] * e2[1] - d[1] * e2[0];
    double det = e1[0] * P[0] + e1[1] * P[1] + e1[2] * P[2];
    if (det == 0.0) return 0;
    double u = (T[0] * P[0] + T[1] * P[1] + T[2] * P[2]) / det;
    Q[0] = T[1] * e1[2] - T[2] * e1[1]; Q[1] = T[2] * e1[0] - T[0] * e1[2]; Q[2] = T[0] * e1[1] - T[1] * e1[0];
    double w = (d[0] * Q[0] + d[1] * Q[1] + d[2] * Q[2]) / det;
    if (u < 0 || w < 0 || u + w > 1) return 0;
    *lam = (e2[0] * Q[0] + e2[1] * Q[1] + e2[2] * Q[2]) / det;
    return *lam > 0.0;
}

static void quat_mat(const float* q4, double R[9]) {
    double x = q4[0], y = q4[1], z = q4[2], w = q4[3];
    double n = sqrt(x * x + y * y + z * z + w * w);
    x /= n; y /= n; z /= n; w /= n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - z * w); R[2] = 2 * (x * z + y * w);
    R[3] = 2 * (x * y + z * w); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - x * w);
    R[6] = 2 * (x * z - y * w); R[7] = 2 * (y * z + x * w); R[8] = 1 - 2 * (x * x + y * y);
}

typedef struct { double node, tri, inst; } counts_t;

/* Ordered closest-first traversal with a stack; leaf prims handled by `kind`:
 * 0 = triangles of `tris`, 1 = instances (recursing into link hierarchies). */
typedef struct ctx_s {
    const float* const* mesh_tris; const rbvh_t* link_bvh;
    const float* link_pos; const float* link_quat; int env, n_links;
} ctx_t;

static void trace(const rbvh_t* t, int kind, const float* tris, const double o[3], const double d[3],
                  double* tmax, counts_t* c, const ctx_t* cx) {
    double inv[3];
    for (int a = 0; a < 3; ++a) inv[a] = 1.0 / (fabs(d[a]) < 1e-300 ? copysign(1e-300, d[a]) : d[a]);
    int stack[128]; double sdist[128]; int sp = 0;
    double tn;
    if (!slab(&t->root, o, inv, *tmax, &tn)) return;
    stack[sp] = t->root_ref; sdist[sp++] = tn;
    while (sp) {
        --sp;
        int ref = stack[sp];
        if (sdist[sp] > *tmax) continue;
        if (ref < 0) {
            const rleaf_t* L = &t->leaves[~ref];
            for (int k = L->first; k < L->first + L->count; ++k) {
                int p = t->prim[k];
                if (kind == 0) {
                    double lam;
                    c->tri += 1;
                    if (tri_hit(tris + 9 * (int64_t)p, o, d, &lam) && lam <= *tmax) *tmax = lam;
                } else {
                    double R[9]; int64_t eb = (int64_t)cx->env * cx->n_links + p;
                    quat_mat(cx->link_quat + 4 * eb, R);
                    const float* tp = cx->link_pos + 3 * eb;
                    double po[3] = {o[0] - tp[0], o[1] - tp[1], o[2] - tp[2]}, lo[3], ld[3];
                    for (int a = 0; a < 3; ++a) {
                        lo[a] = R[a] * po[0] + R[3 + a] * po[1] + R[6 + a] * po[2];
                        ld[a] = R[a] * d[0] + R[3 + a] * d[1] + R[6 + a] * d[2];
                    }
                    c->inst += 1;
                    trace(&cx->link_bvh[p], 0, cx->mesh_tris[p], lo, ld, tmax, c, cx);
                }
            }
            continue;
        }
        const rnode_t* N = &t->nodes[ref];
        c->node += 1;
        double t0, t1;
        int h0 = slab(&N->b[0], o, inv, *tmax, &t0), h1 = slab(&N->b[1], o, inv, *tmax, &t1);
        if (h0 && h1) {
            int near = t0 <= t1 ? 0 : 1;
            if (sp + 2 > 128) return;
            stack[sp] = N->child[1 - near]; sdist[sp++] = near ? t0 : t1;
            stack[sp] = N->child[near]; sdist[sp++] = near ? t1 : t0;
        } else if (h0 || h1) {
            if (sp + 1 > 128) return;
            stack[sp] = N->child[h0 ? 0 : 1]; sdist[sp++] = h0 ? t0 : t1;
        }
    }
}

/* Surface-area cost of a hierarchy (C_trav = C_tri = 1): sum over internal
 * nodes of area / root area, plus sum over leaves of area x triangles /
 * root area. */
static double sah_rec(const rbvh_t* t, int ref, const box_t* b) {
    if (ref < 0) return box_area(b) * t->leaves[~ref].count;
    const rnode_t* N = &t->nodes[ref];
    return box_area(b) + sah_rec(t, N->child[0], &N->b[0]) + sah_rec(t, N->child[1], &N->b[1]);
}

double ref_sah_cost(const float* tris, int64_t n) {
    box_t* pb = (box_t*)malloc(sizeof(box_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) tri_box(tris + 9 * i, &pb[i]);
    rbvh_t t;
    rbvh_build(&t, pb, (int)n);
    free(pb);
    double c = sah_rec(&t, t.root_ref, &t.root) / box_area(&t.root);
    rbvh_free(&t);
    return c;
}

/*
 * ref_counts: per ray counts, out [n][6] = (robot nodes (top level + links),
 * terrain nodes, link triangles, terrain triangles, instances entered,
 * hit flag).
 * Rays: linear pixel ids into [E][C][H][W].  Returns 0.
 */
int ref_counts(const float* terrain, int64_t n_terrain, const float* link_tri,
               const int64_t* link_off, int n_links, const float* link_pos, const float* link_quat,
               const float* cam_pos, const float* cam_quat, const float* intr, int E, int C, int W,
               int H, double far, const int64_t* rays, int64_t n, double* out) {
    /* terrain and link hierarchies */
    box_t* pb = (box_t*)malloc(sizeof(box_t) * (size_t)n_terrain);
    for (int64_t i = 0; i < n_terrain; ++i) tri_box(terrain + 9 * i, &pb[i]);
    rbvh_t terr;
    rbvh_build(&terr, pb, (int)n_terrain);
    free(pb);
    rbvh_t* lb = (rbvh_t*)calloc((size_t)(n_links > 0 ? n_links : 1), sizeof(rbvh_t));
    const float** mt = (const float**)calloc((size_t)(n_links > 0 ? n_links : 1), sizeof(float*));
    for (int b = 0; b < n_links; ++b) {
        int nb = (int)(link_off[b + 1] - link_off[b]);
        box_t* q = (box_t*)malloc(sizeof(box_t) * (size_t)nb);
        mt[b] = link_tri + 9 * link_off[b];
        for (int i = 0; i < nb; ++i) tri_box(mt[b] + 9 * i, &q[i]);
        rbvh_build(&lb[b], q, nb);
        free(q);
    }
    /* per-environment top levels over world instance boxes, built on demand */
    rbvh_t* top = (rbvh_t*)calloc((size_t)E, sizeof(rbvh_t));
    char* have = (char*)calloc((size_t)E, 1);
    for (int64_t r = 0; r < n; ++r) {
        int64_t p = rays[r];
        int64_t x = p % W, y = (p / W) % H, ec = p / ((int64_t)W * H);
        int e = (int)(ec / C);
        if (n_links > 0 && !have[e]) {
            box_t ib[64];
            for (int b = 0; b < n_links; ++b) {
                double R[9]; int64_t eb = (int64_t)e * n_links + b;
                quat_mat(link_quat + 4 * eb, R);
                box_empty(&ib[b]);
                const box_t* rb = &lb[b].root;
                for (int k = 0; k < 8; ++k) {
                    double v[3] = {(k & 1) ? rb->hi[0] : rb->lo[0], (k & 2) ? rb->hi[1] : rb->lo[1],
                                   (k & 4) ? rb->hi[2] : rb->lo[2]};
                    box_t pt;
                    for (int a = 0; a < 3; ++a)
                        pt.lo[a] = pt.hi[a] = R[3 * a] * v[0] + R[3 * a + 1] * v[1] + R[3 * a + 2] * v[2] +
                                              link_pos[3 * eb + a];
                    box_grow(&ib[b], &pt);
                }
            }
            rbvh_build(&top[e], ib, n_links);
            have[e] = 1;
        }
        const float* K = intr + 4 * ec;
        double rr[3] = {((double)x + 0.5 - K[2]) / K[0], ((double)y + 0.5 - K[3]) / K[1], 1.0}, R[9], d[3];
        quat_mat(cam_quat + 4 * ec, R);
        for (int a = 0; a < 3; ++a) d[a] = R[3 * a] * rr[0] + R[3 * a + 1] * rr[1] + R[3 * a + 2] * rr[2];
        double o[3] = {cam_pos[3 * ec], cam_pos[3 * ec + 1], cam_pos[3 * ec + 2]};
        double tmax = far;
        counts_t cl = {0, 0, 0}, cterr = {0, 0, 0};
        if (n_links > 0) {
            ctx_t cx = {mt, lb, link_pos, link_quat, e, n_links};
            trace(&top[e], 1, NULL, o, d, &tmax, &cl, &cx);
        }
        trace(&terr, 0, terrain, o, d, &tmax, &cterr, NULL);
        out[6 * r + 0] = cl.node;     /* top-level + link nodes */
        out[6 * r + 1] = cterr.node;  /* terrain nodes */
        out[6 * r + 2] = cl.tri;
        out[6 * r + 3] = cterr.tri;
        out[6 * r + 4] = cl.inst;
        out[6 * r + 5] = (double)(tmax < far);
    }
    for (int e = 0; e < E; ++e) if (have[e]) rbvh_free(&top[e]);
    free(top); free(have);
    for (int b = 0; b < n_links; ++b) rbvh_free(&lb[b]);
    free(lb); free(mt);
    rbvh_free(&terr);
    return 0;
}
