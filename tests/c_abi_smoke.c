/* The C ABI used from plain C, without Python or torch: one sample at
 * L = 8, heat-bath + overrelaxation steps, tempering, a measurement, and
 * checks that need nothing but the header -- unit spins, the energy of the
 * returned spins recomputed here from Eq. (1) against pt_get_energy, a
 * permutation of the slots (per replica and all at once), a checkpoint
 * restored into a fresh context.
 * Prints "ok" and exits 0 on success. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "ptsg.h"

#define CHECK(call)                                                        \
    do {                                                                   \
        pt_status st_ = (call);                                            \
        if (st_ != PT_OK) {                                                \
            fprintf(stderr, "%s failed (%d): %s\n", #call, (int)st_,       \
                    pt_last_error());                                      \
            return 1;                                                      \
        }                                                                  \
    } while (0)

static int site(int L, int x, int y, int z)
{
    x = (x + L) % L;
    y = (y + L) % L;
    z = (z + L) % L;
    return x + L * (y + L * z);
}

/* E = -sum over bonds (x, x+e_mu) of s_x^T M_{mu,x} s_{x+e_mu} */
static double energy(int L, const float *M, const float *s)
{
    const int N = L * L * L;
    double e = 0.0;
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                const int i = site(L, x, y, z);
                const int nb[3] = {site(L, x + 1, y, z), site(L, x, y + 1, z), site(L, x, y, z + 1)};
                for (int mu = 0; mu < 3; ++mu) {
                    const float *m = M + ((size_t)mu * N + i) * 9;
                    const float *a = s + 3 * i, *b = s + 3 * nb[mu];
                    for (int p = 0; p < 3; ++p)
                        for (int q = 0; q < 3; ++q) e -= (double)a[p] * m[3 * p + q] * b[q];
                }
            }
    return e;
}

int main(void)
{
    const int L = 8, N = L * L * L, T = 3, R = 2;
    const double temps[3] = {0.8, 1.2, 1.8};
    float *M = malloc(sizeof(float) * 27 * N);
    unsigned v = 12345u;  /* a small deterministic generator for the couplings */
    for (int i = 0; i < 27 * N; ++i) {
        v = v * 1664525u + 1013904223u;
        M[i] = (float)((double)(v >> 8) / 16777216.0 * 2.0 - 1.0);
    }
    pt_ctx *ctx = NULL;
    CHECK(pt_init(&ctx, L, M, temps, T, R, 7));
    for (int step = 0; step < 5; ++step) {
        CHECK(pt_step(ctx, 1, 4));
        CHECK(pt_swap(ctx));
    }
    size_t n = 0;
    CHECK(pt_measure(ctx, PT_M_ALL, NULL, 0, &n));
    if (n != (size_t)(T * R * (R - 1) / 2)) { fprintf(stderr, "record count %zu\n", n); return 1; }
    pt_meas *recs = malloc(sizeof(pt_meas) * n);
    CHECK(pt_measure(ctx, PT_M_ALL, recs, n, &n));
    double E[6];
    CHECK(pt_get_energy(ctx, E));
    float *s = malloc(sizeof(float) * 3 * N);
    int all[6];
    CHECK(pt_get_perms(ctx, all));
    for (int r = 0; r < R; ++r) {
        int perm[3], seen[3] = {0, 0, 0};
        CHECK(pt_get_perm(ctx, 0, r, perm));
        for (int k = 0; k < T; ++k)
            if (all[r * T + k] != perm[k]) { fprintf(stderr, "pt_get_perms differs\n"); return 1; }
        for (int k = 0; k < T; ++k) {
            if (perm[k] < 0 || perm[k] >= T || seen[perm[k]]++) { fprintf(stderr, "bad permutation\n"); return 1; }
            CHECK(pt_get_spins(ctx, 0, r, k, s));
            for (int i = 0; i < N; ++i) {
                const double norm = sqrt((double)s[3 * i] * s[3 * i] + (double)s[3 * i + 1] * s[3 * i + 1] +
                                         (double)s[3 * i + 2] * s[3 * i + 2]);
                if (fabs(norm - 1.0) > 1e-5) { fprintf(stderr, "|s| = %g\n", norm); return 1; }
            }
            const double e = energy(L, M, s);
            if (fabs(e - E[r * T + k]) > 1e-4 * (3.0 * N)) {
                fprintf(stderr, "energy %g vs %g\n", E[r * T + k], e);
                return 1;
            }
        }
    }
    /* checkpoint into a fresh context, one more step on both: same spins */
    size_t bytes = 0;
    CHECK(pt_save(ctx, NULL, 0, &bytes));
    void *blob = malloc(bytes);
    CHECK(pt_save(ctx, blob, bytes, &bytes));
    pt_ctx *copy = NULL;
    CHECK(pt_init(&copy, L, M, temps, T, R, 7));
    CHECK(pt_load(copy, blob, bytes));
    CHECK(pt_step(ctx, 1, 2));
    CHECK(pt_step(copy, 1, 2));
    float *s2 = malloc(sizeof(float) * 3 * N);
    CHECK(pt_get_spins(ctx, 0, 1, 2, s));
    CHECK(pt_get_spins(copy, 0, 1, 2, s2));
    for (int i = 0; i < 3 * N; ++i)
        if (s[i] != s2[i]) { fprintf(stderr, "resumed run differs at %d\n", i); return 1; }
    /* three whole steps through pt_run on one, the separate calls on the
       other: same spins and counters */
    CHECK(pt_run(ctx, 3, 1, 2, 0, 0, NULL, 0));
    for (int t = 0; t < 3; ++t) {
        CHECK(pt_step(copy, 1, 2));
        CHECK(pt_swap(copy));
    }
    CHECK(pt_get_spins(ctx, 0, 1, 2, s));
    CHECK(pt_get_spins(copy, 0, 1, 2, s2));
    for (int i = 0; i < 3 * N; ++i)
        if (s[i] != s2[i]) { fprintf(stderr, "pt_run differs at %d\n", i); return 1; }
    uint64_t hb1, pt1, hb2, pt2;
    CHECK(pt_get_counters(ctx, &hb1, &pt1));
    CHECK(pt_get_counters(copy, &hb2, &pt2));
    if (hb1 != hb2 || pt1 != pt2) { fprintf(stderr, "pt_run counters differ\n"); return 1; }
    /* an invalid call reports through the status and the message */
    if (pt_step(ctx, -1, 0) != PT_EINVAL || pt_last_error()[0] == '\0') { fprintf(stderr, "error path\n"); return 1; }
    pt_free(copy);
    pt_free(ctx);
    free(s2);
    free(blob);
    free(s);
    free(recs);
    free(M);
    printf("ok\n");
    return 0;
}
