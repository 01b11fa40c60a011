/*
 * CPU FP64 oracle for GCB greedy RBF mesh deformation.
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).
 *
 * Follows the paper step by step:
 *   Eq. (1)  interpolant F(r) = sum_i w_i phi(|r - r_i|)
 *   Eq. (2)  Wendland C2 basis
 *   Eqs. (3)-(5)  interpolation condition Phi W = Delta, Phi SPD -> Cholesky
 *   Eq. (6)  volume displacements
 *   Section 1  recurrence Cholesky (RC): L grows one row per support node
 *   Section 3  stochastic uniform partition into G_0..G_{m-1}
 *   Algorithm 1  GCB greedy: at iteration k only G_{k mod m} is evaluated,
 *                its worst node is appended when its error exceeds E*.
 * Build: plain C11, -O2 -ffp-contract=off, optional OpenMP over targets.
 */
#include "gcb_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* ------------------------------------------------------------------ Eq. (2) */
double orc_phi(double eta) {
    if (eta > 1.0) return 0.0;
    double a = 1.0 - eta;
    return a * a * a * a * (4.0 * eta + 1.0);
}

static double dist3(const double *a, const double *b) {
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

static double sq3(double x, double y, double z) {
    double s = x * x + y * y;
    return s + z * z;
}

/* ------------------------------------------------------------------ splitmix64 */
uint64_t orc_splitmix64_next(uint64_t *state) {
    *state += 0x9E3779B97F4A7C15ull;
    uint64_t z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------------ Section 3 partition */
void orc_partition(int64_t nb, int32_t m, uint64_t seed, int32_t *group_of) {
    int64_t *pi = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb > 0 ? nb : 1));
    for (int64_t i = 0; i < nb; ++i) pi[i] = i;
    uint64_t st = seed;
    for (int64_t i = nb - 1; i >= 1; --i) {
        uint64_t j = orc_splitmix64_next(&st) % (uint64_t)(i + 1);
        int64_t t = pi[i];
        pi[i] = pi[j];
        pi[j] = t;
    }
    for (int64_t t = 0; t < nb; ++t) group_of[pi[t]] = (int32_t)(t % m);
    free(pi);
}

/* ------------------------------------------------------------------ starting nodes */
void orc_initial_nodes(int64_t nb, const double *xyz, const double *disp, int64_t out[3]) {
    int64_t n0 = 0;
    double best = -1.0;
    for (int64_t j = 0; j < nb; ++j) {
        double v = sq3(disp[3 * j], disp[3 * j + 1], disp[3 * j + 2]);
        if (v > best) { best = v; n0 = j; }
    }
    int64_t n1 = 0;
    best = -1.0;
    for (int64_t j = 0; j < nb; ++j) {
        double v = sq3(xyz[3 * j] - xyz[3 * n0], xyz[3 * j + 1] - xyz[3 * n0 + 1], xyz[3 * j + 2] - xyz[3 * n0 + 2]);
        if (v > best) { best = v; n1 = j; }
    }
    int64_t n2 = 0;
    best = -1.0;
    for (int64_t j = 0; j < nb; ++j) {
        double a = sq3(xyz[3 * j] - xyz[3 * n0], xyz[3 * j + 1] - xyz[3 * n0 + 1], xyz[3 * j + 2] - xyz[3 * n0 + 2]);
        double b = sq3(xyz[3 * j] - xyz[3 * n1], xyz[3 * j + 1] - xyz[3 * n1 + 1], xyz[3 * j + 2] - xyz[3 * n1 + 2]);
        double v = a < b ? a : b;
        if (v > best) { best = v; n2 = j; }
    }
    out[0] = n0;
    out[1] = n1;
    out[2] = n2;
}

/* ------------------------------------------------------------------ Eq. (1) / Eq. (6) */
void orc_interpolate(int64_t nc, const double *sup_xyz, const double *w, int32_t K, double radius,
                     int64_t nt, const double *tgt_xyz, double *out, int32_t nthreads) {
#ifdef _OPENMP
    int nth = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nth)
#endif
    for (int64_t t = 0; t < nt; ++t) {
        double *o = out + (size_t)t * (size_t)K;
        for (int32_t c = 0; c < K; ++c) o[c] = 0.0;
        for (int64_t s = 0; s < nc; ++s) {
            double phi = orc_phi(dist3(tgt_xyz + 3 * t, sup_xyz + 3 * s) / radius);
            for (int32_t c = 0; c < K; ++c) o[c] += w[(size_t)s * (size_t)K + (size_t)c] * phi;
        }
    }
    (void)nthreads;
}

/* ------------------------------------------------------------------ RC factor */
struct orc_rc {
    int32_t K;
    int64_t n, cap;
    double *L;   /* packed lower triangle by rows: row i at i*(i+1)/2 */
    double *y;   /* (cap, K): y = L^-1 rhs */
    double *l;   /* scratch row */
};

orc_rc *orc_rc_create(int32_t K) {
    orc_rc *rc = (orc_rc *)calloc(1, sizeof(orc_rc));
    rc->K = K;
    rc->cap = 16;
    rc->L = (double *)malloc(sizeof(double) * (size_t)(rc->cap * (rc->cap + 1) / 2));
    rc->y = (double *)malloc(sizeof(double) * (size_t)(rc->cap * K));
    rc->l = (double *)malloc(sizeof(double) * (size_t)rc->cap);
    return rc;
}

void orc_rc_destroy(orc_rc *rc) {
    if (!rc) return;
    free(rc->L);
    free(rc->y);
    free(rc->l);
    free(rc);
}

int64_t orc_rc_size(const orc_rc *rc) { return rc->n; }

static void rc_grow(orc_rc *rc) {
    int64_t cap = rc->cap * 2;
    rc->L = (double *)realloc(rc->L, sizeof(double) * (size_t)(cap * (cap + 1) / 2));
    rc->y = (double *)realloc(rc->y, sizeof(double) * (size_t)(cap * rc->K));
    rc->l = (double *)realloc(rc->l, sizeof(double) * (size_t)cap);
    rc->cap = cap;
}

int orc_rc_append(orc_rc *rc, const double *b, double phi0, const double *rhs) {
    int64_t n = rc->n;
    if (n + 1 > rc->cap) rc_grow(rc);
    /* forward substitution L l = b */
    double ll = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double *Li = rc->L + (size_t)(i * (i + 1) / 2);
        double acc = b[i];
        for (int64_t j = 0; j < i; ++j) acc -= Li[j] * rc->l[j];
        rc->l[i] = acc / Li[i];
        ll += rc->l[i] * rc->l[i];
    }
    double s = phi0 - ll;
    if (!(s > 64.0 * DBL_EPSILON)) return ORC_E_SINGULAR;
    double d = sqrt(s);
    double *Ln = rc->L + (size_t)(n * (n + 1) / 2);
    for (int64_t j = 0; j < n; ++j) Ln[j] = rc->l[j];
    Ln[n] = d;
    /* y_n = (rhs - l . y) / d, per component */
    for (int32_t c = 0; c < rc->K; ++c) {
        double acc = rhs[c];
        for (int64_t j = 0; j < n; ++j) acc -= rc->l[j] * rc->y[(size_t)j * (size_t)rc->K + (size_t)c];
        rc->y[(size_t)n * (size_t)rc->K + (size_t)c] = acc / d;
    }
    rc->n = n + 1;
    return ORC_OK;
}

void orc_rc_weights(const orc_rc *rc, double *w) {
    int64_t n = rc->n;
    int32_t K = rc->K;
    memcpy(w, rc->y, sizeof(double) * (size_t)(n * K));
    /* L^T w = y, column sweep over the rows of L from the last one up */
    for (int64_t j = n - 1; j >= 0; --j) {
        const double *Lj = rc->L + (size_t)(j * (j + 1) / 2);
        for (int32_t c = 0; c < K; ++c) w[(size_t)j * (size_t)K + (size_t)c] /= Lj[j];
        for (int64_t i = 0; i < j; ++i)
            for (int32_t c = 0; c < K; ++c)
                w[(size_t)i * (size_t)K + (size_t)c] -= Lj[i] * w[(size_t)j * (size_t)K + (size_t)c];
    }
}

void orc_rc_factor(const orc_rc *rc, double *L) {
    int64_t n = rc->n;
    memset(L, 0, sizeof(double) * (size_t)(n * n));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) L[i * n + j] = rc->L[i * (i + 1) / 2 + j];
}

/* ------------------------------------------------------------------ Algorithm 1 */
typedef struct {
    const orc_problem *p;
    int32_t *group_of;
    int64_t *members;     /* nodes grouped: group g at members[goff[g] .. goff[g+1]) */
    int64_t *goff;
    char *in_S;
    int64_t *S;
    double *Sxyz;         /* (cap,3) support coordinates in S order */
    int64_t nS;
    orc_rc *rc;
    double *W;            /* (cap,3) */
    double *F;            /* scratch (group size,3) */
    double *e;            /* scratch errors */
} orc_state;

static int validate_problem(const orc_problem *p) {
    if (!p || !p->xyz || !p->disp) return 0;
    if (p->nb < 3 || p->m < 1 || p->m > p->nb) return 0;
    if (!(p->radius > 0.0) || !isfinite(p->radius)) return 0;
    if (!(p->tol_abs >= 0.0) || !isfinite(p->tol_abs)) return 0;
    if (p->nc_max < 3 || p->nc_max > p->nb) return 0;
    for (int64_t j = 0; j < 3 * p->nb; ++j)
        if (!isfinite(p->xyz[j]) || !isfinite(p->disp[j])) return 0;
    if (p->group_of)
        for (int64_t j = 0; j < p->nb; ++j)
            if (p->group_of[j] < 0 || p->group_of[j] >= p->m) return 0;
    if (p->warm_n != 0) {
        if (!p->warm_S || p->warm_n < 3 || p->warm_n > p->nc_max) return 0;
        char *seen = (char *)calloc((size_t)p->nb, 1);
        int ok = 1;
        for (int64_t t = 0; t < p->warm_n && ok; ++t) {
            int64_t j = p->warm_S[t];
            if (j < 0 || j >= p->nb || seen[j]) ok = 0;
            else seen[j] = 1;
        }
        free(seen);
        if (!ok) return 0;
    }
    if (p->per_iter < 0 || p->per_iter > 64) return 0;
    if (p->init_idx) {
        for (int t = 0; t < 3; ++t)
            if (p->init_idx[t] < 0 || p->init_idx[t] >= p->nb) return 0;
        if (p->init_idx[0] == p->init_idx[1] || p->init_idx[0] == p->init_idx[2] ||
            p->init_idx[1] == p->init_idx[2])
            return 0;
    }
    return 1;
}

static void state_free(orc_state *st) {
    free(st->group_of);
    free(st->members);
    free(st->goff);
    free(st->in_S);
    free(st->S);
    free(st->Sxyz);
    free(st->W);
    free(st->F);
    free(st->e);
    orc_rc_destroy(st->rc);
}

static void state_init(orc_state *st, const orc_problem *p) {
    memset(st, 0, sizeof(*st));
    st->p = p;
    int64_t nb = p->nb;
    st->group_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)nb);
    if (p->group_of) memcpy(st->group_of, p->group_of, sizeof(int32_t) * (size_t)nb);
    else orc_partition(nb, p->m, p->seed, st->group_of);
    st->goff = (int64_t *)calloc((size_t)p->m + 1, sizeof(int64_t));
    for (int64_t j = 0; j < nb; ++j) st->goff[st->group_of[j] + 1]++;
    for (int32_t g = 0; g < p->m; ++g) st->goff[g + 1] += st->goff[g];
    st->members = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)p->m);
    for (int32_t g = 0; g < p->m; ++g) fill[g] = st->goff[g];
    for (int64_t j = 0; j < nb; ++j) st->members[fill[st->group_of[j]]++] = j;
    free(fill);
    int64_t gmax = 0;
    for (int32_t g = 0; g < p->m; ++g)
        if (st->goff[g + 1] - st->goff[g] > gmax) gmax = st->goff[g + 1] - st->goff[g];
    st->in_S = (char *)calloc((size_t)nb, 1);
    st->S = (int64_t *)malloc(sizeof(int64_t) * (size_t)p->nc_max);
    st->Sxyz = (double *)malloc(sizeof(double) * 3 * (size_t)p->nc_max);
    st->W = (double *)malloc(sizeof(double) * 3 * (size_t)p->nc_max);
    st->F = (double *)malloc(sizeof(double) * 3 * (size_t)(gmax > 0 ? gmax : 1));
    st->e = (double *)malloc(sizeof(double) * (size_t)(gmax > 0 ? gmax : 1));
    st->rc = orc_rc_create(3);
}

/* Append node n to S with the RC recurrence; recompute W by back substitution. */
static int state_append(orc_state *st, int64_t n) {
    const orc_problem *p = st->p;
    double *b = (double *)malloc(sizeof(double) * (size_t)(st->nS > 0 ? st->nS : 1));
    for (int64_t s = 0; s < st->nS; ++s)
        b[s] = orc_phi(dist3(st->Sxyz + 3 * s, p->xyz + 3 * n) / p->radius);
    int rc = orc_rc_append(st->rc, b, orc_phi(0.0), p->disp + 3 * n);
    free(b);
    if (rc != ORC_OK) return rc;
    st->S[st->nS] = n;
    st->Sxyz[3 * st->nS + 0] = p->xyz[3 * n + 0];
    st->Sxyz[3 * st->nS + 1] = p->xyz[3 * n + 1];
    st->Sxyz[3 * st->nS + 2] = p->xyz[3 * n + 2];
    st->in_S[n] = 1;
    st->nS++;
    orc_rc_weights(st->rc, st->W);
    return ORC_OK;
}

/* Errors e_j = |F(r_j) - d_j| for j in G_g \ S; returns the count written to
 * st->e (aligned with the member list, -1 marks members already in S). */
static void group_errors(orc_state *st, int32_t g, int32_t nthreads) {
    const orc_problem *p = st->p;
    int64_t lo = st->goff[g], hi = st->goff[g + 1];
#ifdef _OPENMP
    int nth = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nth)
#endif
    for (int64_t t = lo; t < hi; ++t) {
        int64_t j = st->members[t];
        if (st->in_S[j]) { st->e[t - lo] = -1.0; continue; }
        double F[3] = {0.0, 0.0, 0.0};
        for (int64_t s = 0; s < st->nS; ++s) {
            double phi = orc_phi(dist3(p->xyz + 3 * j, st->Sxyz + 3 * s) / p->radius);
            F[0] += st->W[3 * s + 0] * phi;
            F[1] += st->W[3 * s + 1] * phi;
            F[2] += st->W[3 * s + 2] * phi;
        }
        double ex = F[0] - p->disp[3 * j], ey = F[1] - p->disp[3 * j + 1], ez = F[2] - p->disp[3 * j + 2];
        st->e[t - lo] = sqrt(ex * ex + ey * ey + ez * ez);
    }
    (void)nthreads;
}

/* (E, n) = max over the group, lowest node index on ties; E = 0, n = -1 if empty. */
static void group_argmax(const orc_state *st, int32_t g, double *E, int64_t *n) {
    int64_t lo = st->goff[g], hi = st->goff[g + 1];
    double best = -1.0;
    int64_t arg = -1;
    for (int64_t t = lo; t < hi; ++t) {
        double v = st->e[t - lo];
        if (v < 0.0) continue;
        int64_t j = st->members[t];
        if (v > best || (v == best && j < arg)) { best = v; arg = j; }
    }
    *E = arg < 0 ? 0.0 : best;
    *n = arg;
}

/* The several-nodes-per-iteration rule: the nodes of G_g \ S whose error
 * exceeds tol, ranked by (error descending, node index ascending).  Returns
 * a malloc'd array of *count node indices. */
typedef struct {
    double e;
    int64_t j;
} orc_cand;

static int cand_order(const void *a, const void *b) {
    const orc_cand *x = (const orc_cand *)a, *y = (const orc_cand *)b;
    if (x->e > y->e) return -1;
    if (x->e < y->e) return 1;
    return x->j < y->j ? -1 : (x->j > y->j ? 1 : 0);
}

static orc_cand *group_ranking(const orc_state *st, int32_t g, double tol, int64_t *count) {
    int64_t lo = st->goff[g], hi = st->goff[g + 1];
    orc_cand *c = (orc_cand *)malloc(sizeof(orc_cand) * (size_t)(hi > lo ? hi - lo : 1));
    int64_t n = 0;
    for (int64_t t = lo; t < hi; ++t) {
        double v = st->e[t - lo];
        if (v < 0.0 || !(v > tol)) continue;
        c[n].e = v;
        c[n].j = st->members[t];
        n++;
    }
    qsort(c, (size_t)n, sizeof(orc_cand), cand_order);
    *count = n;
    return c;
}

static int start_support(orc_state *st) {
    const orc_problem *p = st->p;
    int64_t init[3];
    if (p->init_idx) { init[0] = p->init_idx[0]; init[1] = p->init_idx[1]; init[2] = p->init_idx[2]; }
    else orc_initial_nodes(p->nb, p->xyz, p->disp, init);
    if (init[0] == init[1] || init[0] == init[2] || init[1] == init[2]) return ORC_E_SINGULAR;
    for (int t = 0; t < 3; ++t) {
        int rc = state_append(st, init[t]);
        if (rc != ORC_OK) return rc;
    }
    return ORC_OK;
}

/* Warm start: the kept support set in its order, factor and W for the current displacements. */
static int warm_support(orc_state *st) {
    const orc_problem *p = st->p;
    for (int64_t t = 0; t < p->warm_n; ++t) {
        int rc = state_append(st, p->warm_S[t]);
        if (rc != ORC_OK) return rc;
    }
    return ORC_OK;
}

static void certificate(orc_state *st, orc_info *info) {
    const orc_problem *p = st->p;
    double *F = (double *)malloc(sizeof(double) * 3 * (size_t)p->nb);
    orc_interpolate(st->nS, st->Sxyz, st->W, 3, p->radius, p->nb, p->xyz, F, p->nthreads);
    double mx = 0.0, ss = 0.0;
    for (int64_t j = 0; j < p->nb; ++j) {
        double ex = F[3 * j] - p->disp[3 * j], ey = F[3 * j + 1] - p->disp[3 * j + 1], ez = F[3 * j + 2] - p->disp[3 * j + 2];
        double e2 = ex * ex + ey * ey + ez * ez;
        double e = sqrt(e2);
        if (e > mx) mx = e;
        ss += e2;
    }
    free(F);
    info->final_max_err = mx;
    info->final_rms_err = sqrt(ss / (double)p->nb);
    info->converged = mx <= p->tol_abs;
    info->pairs_cert = (uint64_t)p->nb * (uint64_t)st->nS;
}

int orc_select(const orc_problem *p, int64_t *S_out, double *W_out, orc_log *log, orc_info *info) {
    orc_info dummy;
    if (!info) info = &dummy;
    memset(info, 0, sizeof(*info));
    info->singular_node = -1;
    if (!validate_problem(p)) { info->status = ORC_E_INVALID; return ORC_E_INVALID; }
    if (log) log->n_monitor = 0;
    orc_state st;
    state_init(&st, p);
    double t0 = now_s();
    int rc = p->warm_n >= 3 ? warm_support(&st) : start_support(&st);
    info->t_solve += now_s() - t0;
    if (rc != ORC_OK) {
        info->status = rc;
        state_free(&st);
        return rc;
    }
    const int64_t k0 = p->warm_n >= 3 ? p->warm_n : 3;
    int64_t k = k0, quiet = 0;
    int status = ORC_OK;
    if (p->warm_n >= 3) {
        /* the kept support set may already meet E* for the new displacements */
        certificate(&st, info);
        if (info->converged) {
            info->nc = st.nS;
            info->status = ORC_OK;
            if (S_out) memcpy(S_out, st.S, sizeof(int64_t) * (size_t)st.nS);
            if (W_out) memcpy(W_out, st.W, sizeof(double) * 3 * (size_t)st.nS);
            state_free(&st);
            return ORC_OK;
        }
    }
    for (;;) {
        int32_t g = (int32_t)(k % p->m);
        int64_t gsize = st.goff[g + 1] - st.goff[g];
        double ta = now_s();
        group_errors(&st, g, p->nthreads);
        double E;
        int64_t n;
        group_argmax(&st, g, &E, &n);
        info->t_error += now_s() - ta;
        int64_t outside = 0;
        for (int64_t t = st.goff[g]; t < st.goff[g + 1]; ++t) outside += !st.in_S[st.members[t]];
        info->pairs_group += (uint64_t)outside * (uint64_t)st.nS;
        (void)gsize;
        int8_t app = 0;
        int stop = 0;
        if (p->per_iter <= 1) {
            if (n >= 0 && E > p->tol_abs) {
                if (st.nS < p->nc_max) {
                    double tb = now_s();
                    info->pairs_append += (uint64_t)st.nS;
                    rc = state_append(&st, n);
                    info->t_solve += now_s() - tb;
                    if (rc != ORC_OK) { status = rc; info->singular_node = n; stop = 1; }
                    else { app = 1; quiet = 0; }
                } else {
                    status = ORC_NOT_CONVERGED;
                    stop = 1;
                }
            } else {
                quiet++;
            }
        } else {
            /* several nodes per iteration: the top per_iter nodes over E*, appended in rank order */
            int64_t over = 0;
            orc_cand *c = group_ranking(&st, g, p->tol_abs, &over);
            if (over > 0) {
                if (st.nS < p->nc_max) {
                    int64_t q = over < p->per_iter ? over : p->per_iter;
                    if (q > p->nc_max - st.nS) q = p->nc_max - st.nS;
                    double tb = now_s();
                    for (int64_t t = 0; t < q && !stop; ++t) {
                        info->pairs_append += (uint64_t)st.nS;
                        rc = state_append(&st, c[t].j);
                        if (rc != ORC_OK) { status = rc; info->singular_node = c[t].j; stop = 1; }
                        else app++;
                    }
                    info->t_solve += now_s() - tb;
                    quiet = 0;
                } else {
                    status = ORC_NOT_CONVERGED;
                    stop = 1;
                }
            } else {
                quiet++;
            }
            free(c);
        }
        int64_t it = k - k0;
        if (log && it < log->cap) {
            if (log->group) log->group[it] = g;
            if (log->node) log->node[it] = n;
            if (log->err) log->err[it] = E;
            if (log->appended) log->appended[it] = app;
        }
        if (log && log->monitor_every > 0 && (it + 1) % log->monitor_every == 0) {
            int64_t s = (it + 1) / log->monitor_every - 1;
            if (s < log->cap) {
                orc_info mi;
                memset(&mi, 0, sizeof(mi));
                certificate(&st, &mi);
                if (log->mon_max) log->mon_max[s] = mi.final_max_err;
                if (log->mon_rms) log->mon_rms[s] = mi.final_rms_err;
                log->n_monitor = s + 1;
            }
        }
        k++;
        if (stop) break;
        if (quiet >= p->m) break;
    }
    info->iterations = k - k0;
    info->nc = st.nS;
    if (status >= 0) certificate(&st, info);
    info->status = status;
    if (S_out) memcpy(S_out, st.S, sizeof(int64_t) * (size_t)st.nS);
    if (W_out) memcpy(W_out, st.W, sizeof(double) * 3 * (size_t)st.nS);
    state_free(&st);
    return status;
}

/* ------------------------------------------------------------------ several right-hand sides */
int orc_solve_on_support(int64_t nb, const double *xyz, const int64_t *S, int64_t n, double radius, int32_t K,
                         const double *D, double *W_out) {
    (void)nb;
    orc_rc *rc = orc_rc_create(K);
    double *b = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int status = ORC_OK;
    for (int64_t t = 0; t < n && status == ORC_OK; ++t) {
        for (int64_t s = 0; s < t; ++s) b[s] = orc_phi(dist3(xyz + 3 * S[s], xyz + 3 * S[t]) / radius);
        status = orc_rc_append(rc, b, orc_phi(0.0), D + (size_t)S[t] * (size_t)K);
    }
    if (status == ORC_OK) orc_rc_weights(rc, W_out);
    free(b);
    orc_rc_destroy(rc);
    return status;
}

int orc_inverse_factor(int64_t nb, const double *xyz, const int64_t *S, int64_t n, double radius, double *M_out) {
    (void)nb;
    orc_rc *rc = orc_rc_create(1);
    double *b = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double zero = 0.0;
    int status = ORC_OK;
    for (int64_t t = 0; t < n && status == ORC_OK; ++t) {
        for (int64_t s = 0; s < t; ++s) b[s] = orc_phi(dist3(xyz + 3 * S[s], xyz + 3 * S[t]) / radius);
        status = orc_rc_append(rc, b, orc_phi(0.0), &zero);
    }
    free(b);
    if (status != ORC_OK) {
        orc_rc_destroy(rc);
        return status;
    }
    double *L = (double *)malloc(sizeof(double) * (size_t)(n * n));
    orc_rc_factor(rc, L);
    orc_rc_destroy(rc);
    memset(M_out, 0, sizeof(double) * (size_t)(n * n));
    /* column c of M solves L x = e_c: x_i = 0 for i < c, then forward substitution */
    for (int64_t col = 0; col < n; ++col) {
        for (int64_t i = col; i < n; ++i) {
            double acc = i == col ? 1.0 : 0.0;
            for (int64_t k = col; k < i; ++k) acc -= L[i * n + k] * M_out[k * n + col];
            M_out[i * n + col] = acc / L[i * n + i];
        }
    }
    free(L);
    return ORC_OK;
}

/* ------------------------------------------------------------------ follow-mode replay */
int64_t orc_validate(const orc_problem *p, const int64_t S_init[3], int64_t n_iter,
                     const int32_t *group, const int64_t *node, const int8_t *appended,
                     double tau, int32_t *reason, double *max_gap) {
    int32_t r = 0;
    double gap_max = 0.0;
    int64_t bad = -1;
    if (!validate_problem(p)) { if (reason) *reason = 1; return 0; }
    orc_state st;
    state_init(&st, p);
    int64_t k0 = 3;
    if (p->warm_n >= 3) {
        /* warm start: the foreign run keeps warm_S; it may skip the loop only when the
         * kept set already meets E* (within tau), and must run it otherwise */
        k0 = p->warm_n;
        if (warm_support(&st) != ORC_OK) { if (reason) *reason = 5; state_free(&st); return 0; }
        orc_info ci;
        memset(&ci, 0, sizeof(ci));
        certificate(&st, &ci);
        if ((n_iter == 0 && !(ci.final_max_err <= p->tol_abs + tau)) ||
            (n_iter > 0 && !(ci.final_max_err > p->tol_abs - tau))) {
            if (reason) *reason = 6;
            state_free(&st);
            return 0;
        }
        if (n_iter == 0) {
            if (reason) *reason = 0;
            if (max_gap) *max_gap = 0.0;
            state_free(&st);
            return -1;
        }
    } else {
        int64_t init[3];
        orc_initial_nodes(p->nb, p->xyz, p->disp, init);
        if (p->init_idx) { init[0] = p->init_idx[0]; init[1] = p->init_idx[1]; init[2] = p->init_idx[2]; }
        if (S_init[0] != init[0] || S_init[1] != init[1] || S_init[2] != init[2]) {
            if (reason) *reason = 2;
            state_free(&st);
            return 0;
        }
        if (start_support(&st) != ORC_OK) { if (reason) *reason = 5; state_free(&st); return 0; }
    }
    int64_t quiet = 0;
    for (int64_t it = 0; it < n_iter; ++it) {
        int64_t k = it + k0;
        int32_t g = (int32_t)(k % p->m);
        if (group[it] != g) { bad = it; r = 1; break; }
        group_errors(&st, g, p->nthreads);
        double E;
        int64_t n;
        group_argmax(&st, g, &E, &n);
        if (appended[it]) {
            int64_t c = node[it];
            if (c < 0 || c >= p->nb || st.group_of[c] != g || st.in_S[c]) { bad = it; r = 2; break; }
            double ec = st.e[0];
            for (int64_t t = st.goff[g]; t < st.goff[g + 1]; ++t)
                if (st.members[t] == c) ec = st.e[t - st.goff[g]];
            double gap = E - ec;
            if (gap > gap_max) gap_max = gap;
            if (gap > tau) { bad = it; r = 3; break; }
            if (!(ec > p->tol_abs - tau) || st.nS >= p->nc_max) { bad = it; r = 4; break; }
            if (state_append(&st, c) != ORC_OK) { bad = it; r = 5; break; }
            quiet = 0;
        } else {
            if (n >= 0 && E > p->tol_abs + tau && st.nS < p->nc_max) { bad = it; r = 4; break; }
            quiet++;
        }
    }
    if (bad < 0) {
        /* the run must end after m quiet iterations or at the cap */
        if (!(quiet == p->m || st.nS == p->nc_max)) { bad = n_iter; r = 6; }
    }
    if (reason) *reason = r;
    if (max_gap) *max_gap = gap_max;
    state_free(&st);
    return bad;
}

/* ------------------------------------------------------------------ follow-mode replay, several nodes per iteration */
int64_t orc_validate_block(const orc_problem *p, const int64_t *S_seq, int64_t n_S, int64_t n_iter,
                           const int32_t *group, const int8_t *appended, double tau, int32_t *reason,
                           double *max_gap) {
    int32_t r = 0;
    double gap_max = 0.0;
    int64_t bad = -1;
    if (!validate_problem(p) || p->warm_n != 0 || n_S < 3) { if (reason) *reason = 1; return 0; }
    const int64_t pm = p->per_iter > 1 ? p->per_iter : 1;
    orc_state st;
    state_init(&st, p);
    int64_t init[3];
    orc_initial_nodes(p->nb, p->xyz, p->disp, init);
    if (p->init_idx) { init[0] = p->init_idx[0]; init[1] = p->init_idx[1]; init[2] = p->init_idx[2]; }
    if (S_seq[0] != init[0] || S_seq[1] != init[1] || S_seq[2] != init[2]) {
        if (reason) *reason = 2;
        state_free(&st);
        return 0;
    }
    if (start_support(&st) != ORC_OK) { if (reason) *reason = 5; state_free(&st); return 0; }
    int64_t used = 3, quiet = 0;
    for (int64_t it = 0; it < n_iter && bad < 0; ++it) {
        int64_t k = it + 3;
        int32_t g = (int32_t)(k % p->m);
        if (group[it] != g) { bad = it; r = 1; break; }
        group_errors(&st, g, p->nthreads);
        /* every candidate ranked (tol = -1 keeps them all), and the counts the rule gives at E* +- tau */
        int64_t nall = 0;
        orc_cand *c = group_ranking(&st, g, -1.0, &nall);
        int64_t hi = 0, lo = 0;
        for (int64_t t = 0; t < nall; ++t) {
            if (c[t].e > p->tol_abs + tau) hi++;
            if (c[t].e > p->tol_abs - tau) lo++;
        }
        const int64_t room = p->nc_max - st.nS;
        int64_t qmin = hi < pm ? hi : pm, qmax = lo < pm ? lo : pm;
        if (qmin > room) qmin = room;
        if (qmax > room) qmax = room;
        if (qmin < 0) qmin = 0;
        if (qmax < 0) qmax = 0;
        int64_t q = appended[it];
        if (q < qmin || q > qmax) { bad = it; r = 4; free(c); break; }
        if (used + q > n_S) { bad = it; r = 7; free(c); break; }
        for (int64_t t = 0; t < q && bad < 0; ++t) {
            int64_t j = S_seq[used + t];
            if (j < 0 || j >= p->nb || st.group_of[j] != g || st.in_S[j]) { bad = it; r = 2; break; }
            double ej = -1.0;
            for (int64_t u = 0; u < nall; ++u)
                if (c[u].j == j) ej = c[u].e;
            /* the t-th appended node against the t-th largest error of the sweep */
            double gap = c[t].e - ej;
            if (gap > gap_max) gap_max = gap;
            if (gap > tau) { bad = it; r = 3; break; }
            if (!(ej > p->tol_abs - tau)) { bad = it; r = 4; break; }
        }
        free(c);
        if (bad >= 0) break;
        for (int64_t t = 0; t < q; ++t)
            if (state_append(&st, S_seq[used + t]) != ORC_OK) { bad = it; r = 5; break; }
        if (bad >= 0) break;
        used += q;
        if (q > 0) quiet = 0;
        else quiet++;
    }
    if (bad < 0) {
        if (used != n_S) { bad = n_iter; r = 7; }
        else if (!(st.nS == p->nc_max || quiet == p->m)) { bad = n_iter; r = 6; }
    }
    if (reason) *reason = r;
    if (max_gap) *max_gap = gap_max;
    state_free(&st);
    return bad;
}
