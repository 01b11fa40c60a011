/* Exercises every oracle entry point on a small seeded problem; built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_oracle_sanitizers.py. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gcb_oracle.h"

static double unit(uint64_t *s) { return (double)(orc_splitmix64_next(s) >> 11) * (1.0 / 9007199254740992.0); }

int main(void) {
    const int64_t nb = 300;
    double *xyz = malloc(sizeof(double) * 3 * nb), *disp = malloc(sizeof(double) * 3 * nb);
    uint64_t s = 12345;
    for (int64_t j = 0; j < nb; ++j) {
        double u = 2 * M_PI * unit(&s), v = acos(2 * unit(&s) - 1);
        xyz[3 * j] = sin(v) * cos(u);
        xyz[3 * j + 1] = 0.5 * sin(v) * sin(u);
        xyz[3 * j + 2] = 0.2 * cos(v);
        disp[3 * j] = 0.0;
        disp[3 * j + 1] = 0.05 * xyz[3 * j] * xyz[3 * j];
        disp[3 * j + 2] = 0.02 * sin(M_PI * xyz[3 * j]);
    }
    orc_problem p;
    memset(&p, 0, sizeof(p));
    p.nb = nb; p.xyz = xyz; p.disp = disp; p.radius = 1.5; p.m = 7; p.seed = 3; p.tol_abs = 1e-4; p.nc_max = nb;
    int64_t cap = 4096;
    orc_log lg;
    memset(&lg, 0, sizeof(lg));
    lg.cap = cap;
    lg.group = malloc(sizeof(int32_t) * cap);
    lg.node = malloc(sizeof(int64_t) * cap);
    lg.err = malloc(sizeof(double) * cap);
    lg.appended = malloc(cap);
    lg.monitor_every = 7;
    lg.mon_max = malloc(sizeof(double) * cap);
    lg.mon_rms = malloc(sizeof(double) * cap);
    int64_t *S = malloc(sizeof(int64_t) * nb);
    double *W = malloc(sizeof(double) * 3 * nb);
    orc_info info;
    int rc = orc_select(&p, S, W, &lg, &info);
    if (rc < 0 || info.nc < 3) { fprintf(stderr, "select failed %d\n", rc); return 1; }
    int64_t init[3] = {S[0], S[1], S[2]};
    int32_t reason = 0;
    double gap = 0.0;
    int64_t bad = orc_validate(&p, init, info.iterations, lg.group, lg.node, lg.appended, 1e-12, &reason, &gap);
    if (bad != -1) { fprintf(stderr, "replay failed at %ld (%d)\n", (long)bad, reason); return 1; }
    /* warm start with a new field */
    double *disp2 = malloc(sizeof(double) * 3 * nb);
    for (int64_t j = 0; j < 3 * nb; ++j) disp2[j] = 1.3 * disp[(j + 1) % (3 * nb)];
    orc_problem q = p;
    q.disp = disp2; q.warm_S = S; q.warm_n = info.nc;
    int64_t *S2 = malloc(sizeof(int64_t) * nb);
    double *W2 = malloc(sizeof(double) * 3 * nb);
    orc_info info2;
    rc = orc_select(&q, S2, W2, &lg, &info2);
    if (rc < 0) { fprintf(stderr, "warm select failed %d\n", rc); return 1; }
    /* inverse factor and K-RHS solve on the support set */
    int64_t n = info.nc;
    double *M = malloc(sizeof(double) * n * n), *Wk = malloc(sizeof(double) * n * 3);
    if (orc_inverse_factor(nb, xyz, S, n, p.radius, M) != ORC_OK) return 1;
    if (orc_solve_on_support(nb, xyz, S, n, p.radius, 3, disp, Wk) != ORC_OK) return 1;
    double *F = malloc(sizeof(double) * 3 * nb);
    double *sx = malloc(sizeof(double) * 3 * n);
    for (int64_t t = 0; t < n; ++t) for (int c = 0; c < 3; ++c) sx[3 * t + c] = xyz[3 * S[t] + c];
    orc_interpolate(n, sx, W, 3, p.radius, nb, xyz, F, 1);
    double emax = 0.0;
    for (int64_t t = 0; t < n; ++t)   /* Eq. 3 at the supports */
        for (int c = 0; c < 3; ++c) emax = fmax(emax, fabs(F[3 * S[t] + c] - disp[3 * S[t] + c]));
    if (emax > 1e-10) { fprintf(stderr, "interpolation condition violated: %g\n", emax); return 1; }
    /* several nodes per iteration, and its block replay */
    orc_problem b = p;
    b.per_iter = 4;
    int64_t *S3 = malloc(sizeof(int64_t) * nb);
    double *W3 = malloc(sizeof(double) * 3 * nb);
    orc_info info3;
    rc = orc_select(&b, S3, W3, &lg, &info3);
    if (rc < 0) { fprintf(stderr, "block select failed %d\n", rc); return 1; }
    bad = orc_validate_block(&b, S3, info3.nc, info3.iterations, lg.group, lg.appended, 1e-12, &reason, &gap);
    if (bad != -1) { fprintf(stderr, "block replay failed at %ld (%d)\n", (long)bad, reason); return 1; }
    free(S3); free(W3);
    int32_t *g = malloc(sizeof(int32_t) * nb);
    orc_partition(nb, 7, 99, g);
    printf("ok nc=%ld iterations=%ld warm_iterations=%ld\n", (long)info.nc, (long)info.iterations,
           (long)info2.iterations);
    free(xyz); free(disp); free(disp2); free(S); free(W); free(S2); free(W2); free(M); free(Wk); free(F); free(g); free(sx);
    free(lg.group); free(lg.node); free(lg.err); free(lg.appended); free(lg.mon_max); free(lg.mon_rms);
    return 0;
}
