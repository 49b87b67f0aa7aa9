/* Drives every entry point of the oracle's C library on small inputs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (host code
 * only).  Compiled together with oracle/oracle.c by tests/test_oracle_sanitized.py. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/oracle.c"

static float frand(unsigned* s) {
    *s = *s * 1664525u + 1013904223u;
    return (float)((*s >> 8) & 0xFFFFFF) / 16777216.0f;
}

int main(void) {
    unsigned seed = 12345u;
    enum { NT = 34, NL = 8, E = 2, C = 2, W = 5, H = 4, K = 4 };
    float terrain[NT * 9];
    /* a ground quad and random triangles */
    const float quad[18] = {-5, -5, 0, 5, -5, 0, 5, 5, 0, -5, -5, 0, 5, 5, 0, -5, 5, 0};
    memcpy(terrain, quad, sizeof quad);
    for (int i = 18; i < NT * 9; ++i) terrain[i] = 2.0f * frand(&seed) - 1.0f + (i % 3 == 0 ? 1.5f : 0.0f);
    float link[NL * 9];  /* an octahedron */
    const float V[6][3] = {{.2f, 0, 0}, {-.2f, 0, 0}, {0, .2f, 0}, {0, -.2f, 0}, {0, 0, .2f}, {0, 0, -.2f}};
    const int F[8][3] = {{0, 2, 4}, {2, 1, 4}, {1, 3, 4}, {3, 0, 4}, {2, 0, 5}, {1, 2, 5}, {3, 1, 5}, {0, 3, 5}};
    for (int f = 0; f < NL; ++f)
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a) link[9 * f + 3 * k + a] = V[F[f][k]][a];
    int64_t link_off[2] = {0, NL};
    float lp[E * 3] = {1.0f, 0.0f, 0.4f, 1.2f, 0.1f, 0.3f};
    float lq[E * 4] = {0, 0, 0, 1, 0.1f, 0.2f, 0.3f, 0.9f};
    float cp[E * C * 3], cq[E * C * 4], intr[E * C * 4];
    for (int i = 0; i < E * C; ++i) {
        cp[3 * i] = 0.0f; cp[3 * i + 1] = 0.1f * i; cp[3 * i + 2] = 1.0f;
        /* optical z along +x, pitched down */
        cq[4 * i] = -0.27f; cq[4 * i + 1] = 0.65f; cq[4 * i + 2] = -0.27f; cq[4 * i + 3] = 0.65f;
        intr[4 * i] = 3.0f; intr[4 * i + 1] = 3.0f; intr[4 * i + 2] = W / 2.0f; intr[4 * i + 3] = H / 2.0f;
    }
    const int64_t N = (int64_t)E * C * H * W;
    double depth[N], cand_d[N * K];
    int32_t inst[N], tri[N], flags[N], cand[N * K * 2];
    for (int mode = 0; mode < 2; ++mode)
        if (oracle_render(terrain, NT, link, link_off, 1, lp, lq, cp, cq, intr, E, C, W, H, 3.0, mode,
                          NULL, 0, depth, inst, tri, flags, cand, cand_d, K, NULL) != 0)
            return 1;
    int hits = 0;
    for (int64_t i = 0; i < N; ++i) hits += inst[i] >= 0;
    const int64_t rays[3] = {0, N / 2, N - 1};
    if (oracle_render(terrain, NT, link, link_off, 1, lp, lq, cp, cq, intr, E, C, W, H, 3.0, 0, rays, 3,
                      depth, inst, tri, flags, cand, cand_d, K, NULL) != 0)
        return 1;
    double cam64[E * C * 16];
    for (int i = 0; i < E * C; ++i) {
        for (int k = 0; k < 16; ++k) cam64[16 * i + k] = 0.0;
        cam64[16 * i + 2] = 1.0; cam64[16 * i + 3] = -1.0; cam64[16 * i + 7] = -1.0;  /* R */
        cam64[16 * i + 11] = 1.0;
        cam64[16 * i + 12] = 3.0; cam64[16 * i + 13] = 3.0; cam64[16 * i + 14] = W / 2.0; cam64[16 * i + 15] = H / 2.0;
    }
    if (oracle_render(terrain, NT, link, link_off, 1, lp, lq, cp, cq, intr, E, C, W, H, 3.0, 0, NULL, 0,
                      depth, inst, tri, flags, cand, cand_d, K, cam64) != 0)
        return 1;
    /* a link with a pose that places it nowhere */
    float bad_q[E * 4] = {0, 0, 0, 0, NAN, 0, 0, 1};
    if (oracle_render(terrain, NT, link, link_off, 1, lp, bad_q, cp, cq, intr, E, C, W, H, 3.0, 0, NULL, 0,
                      depth, inst, tri, flags, cand, cand_d, K, NULL) != 0)
        return 1;
    float base[6] = {0.0f, 0.0f, 0.75f, 0.5f, 0.5f, 0.8f}, yaw[2] = {0.0f, 1.0f};
    double hm[2 * 11 * 17];
    oracle_heightmap(terrain, NT, base, yaw, 2, 17, 11, 0.1, 0.1, 1.0, 3.0, NAN, hm);
    float fd[3 * N];
    int32_t fi[3 * N];
    for (int64_t i = 0; i < 3 * N; ++i) { fd[i] = 0.05f + 2.0f * frand(&seed); fi[i] = (i % 5) ? 0 : -1; }
    post_params_t pp = {0x123456789ABCull, 0.01f, 0.02f, 0.05f, 0.05f, 3.0f, 0.0f, 1, 3,
                        POST_NOISE | POST_DROPOUT | POST_LATENCY};
    double out[3 * N];
    uint8_t drop[3 * N], lat[3 * E * C];
    if (oracle_post(fd, fi, E, C, H, W, 3, 7, NULL, &pp, out, drop, lat) != 0) return 1;
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, w4[4];
    oracle_philox4x32_10(ctr, key, w4);
    printf("ok hits=%d lat0=%d w=%08x\n", hits, (int)lat[0], w4[0]);
    return 0;
}
