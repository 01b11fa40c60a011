/*
 * CPU FP64 oracle for grouping-circular-based (GCB) greedy RBF mesh
 * deformation.  TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and
 * the benchmark's CPU-baseline leg load it; the product library never does.
 *
 * Plain, slow, obviously correct double precision.  Each function below is
 * pinned by CPU tests against closed forms, invariants, textbook routines or
 * brute force; none is parity-unpinned.
 */
#ifndef GCB_ORACLE_H
#define GCB_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_E_INVALID = -1, ORC_E_SINGULAR = -4 };

/* Wendland C2 basis, Eq. (2): (1-eta)^4 (4 eta + 1) for eta <= 1, else 0. */
double orc_phi(double eta);

/* splitmix64 (Steele, Lea and Flood 2014; the 64-bit mixer published with
 * xoshiro): advances *state and returns the next output. */
uint64_t orc_splitmix64_next(uint64_t *state);

/* Stochastic uniform partition (Section 3, the conditions on G_0..G_{m-1}):
 * Fisher-Yates permutation pi of 0..nb-1 driven by splitmix64(seed)
 * (for i = nb-1 down to 1: j = next() % (i+1); swap pi[i], pi[j]), then node
 * pi[t] goes to group t mod m.  Writes group_of[nb]. */
void orc_partition(int64_t nb, int32_t m, uint64_t seed, int32_t *group_of);

/* The three starting nodes (Algorithm 1 says "any 3 nodes"; the reading used
 * here): n0 = argmax |d_j|^2, n1 = argmax |r_j - r_n0|^2,
 * n2 = argmax min(|r_j - r_n0|^2, |r_j - r_n1|^2); squared norms summed as
 * (x^2 + y^2) + z^2 without fused multiply-add; ties go to the lowest index. */
void orc_initial_nodes(int64_t nb, const double *xyz, const double *disp, int64_t out[3]);

/* RBF interpolant, Eq. (1) / Eq. (6): out[t][c] = sum_s w[s][c] phi(|x_t - x_s| / R),
 * summed in support order.  sup_xyz (nc,3), w (nc,K), tgt (nt,3), out (nt,K). */
void orc_interpolate(int64_t nc, const double *sup_xyz, const double *w, int32_t K, double radius,
                     int64_t nt, const double *tgt_xyz, double *out, int32_t nthreads);

/* Recurrence-Cholesky (RC) factor of Phi_S, grown one row per appended node
 * (Section 1, the RC scheme; Table 1 row 1). */
typedef struct orc_rc orc_rc;
orc_rc *orc_rc_create(int32_t K);
void orc_rc_destroy(orc_rc *rc);
int64_t orc_rc_size(const orc_rc *rc);
/* Append a node: b[0..n) = phi(|r_s - r_new|/R) over the current supports,
 * phi0 = phi(0) = 1, rhs[K] = its prescribed values.  Forward substitution
 * gives the new row l of L, its diagonal sqrt(phi0 - l.l), and the new entry
 * of y = L^-1 rhs.  Returns ORC_E_SINGULAR (and leaves the factor unchanged)
 * when phi0 - l.l <= 64 * DBL_EPSILON. */
int orc_rc_append(orc_rc *rc, const double *b, double phi0, const double *rhs);
/* Back substitution L^T w = y, w (n,K). */
void orc_rc_weights(const orc_rc *rc, double *w);
/* Copy L out as a dense row-major (n,n) lower-triangular matrix. */
void orc_rc_factor(const orc_rc *rc, double *L);

typedef struct {
    int64_t nb;
    const double *xyz;        /* (nb,3) boundary coordinates */
    const double *disp;       /* (nb,3) prescribed displacements */
    double radius;            /* R */
    int32_t m;                /* number of groups, 1 <= m <= nb */
    uint64_t seed;            /* partition seed */
    double tol_abs;           /* E* (absolute) */
    int64_t nc_max;           /* cap on |S|, 3 <= nc_max <= nb */
    const int32_t *group_of;  /* optional explicit partition (NULL: seeded) */
    const int64_t *init_idx;  /* optional 3 starting nodes (NULL: farthest rule) */
    int32_t nthreads;         /* OpenMP threads for the sweeps (<= 0: runtime default) */
    /* Warm start (an extension of Algorithm 1 for a mesh whose support set is
     * kept while its displacements change): when warm_n >= 3, S starts as
     * warm_S[0..warm_n) (distinct node indices, in that order), the factor and
     * W are built over it for the current displacements, and if the all-node
     * error is already <= E* the selection ends with no iteration; otherwise
     * the loop of Algorithm 1 runs from k = warm_n.  init_idx is ignored. */
    const int64_t *warm_S;
    int64_t warm_n;
    /* Nodes appended per iteration (0 or 1: Algorithm 1).  per_iter = p > 1 is
     * the several-nodes-per-iteration variant, a block form of the peak-
     * selection idea the paper cites in Section 1 (not Algorithm 1): every
     * node of G_i \ S whose error exceeds E* is ranked by (error descending,
     * index ascending) and the first p of them are appended in that order
     * (fewer when |S| reaches nc_max), all ranked on the errors of one sweep.
     * An iteration with no such node is quiet; the stopping rule is unchanged.
     * 1 <= p <= 64. */
    int32_t per_iter;
} orc_problem;

typedef struct {
    int64_t nc;               /* |S| */
    int64_t iterations;       /* loop iterations k = 3, 4, ... (k = warm_n, ... for a warm start) that ran */
    int32_t status;           /* ORC_OK, ORC_NOT_CONVERGED, ORC_E_* */
    int32_t converged;        /* final all-node max error <= E* */
    double final_max_err;     /* certificate: max_j |F(r_j) - d_j| over all nb nodes */
    double final_rms_err;     /* sqrt(mean_j |F(r_j) - d_j|^2) */
    uint64_t pairs_group;     /* sum over iterations of |G_i \ S| * |S| */
    uint64_t pairs_append;    /* sum over appends of |S| (phi vector) */
    uint64_t pairs_cert;      /* nb * nc */
    double t_error;           /* wall seconds in group error sweeps (t1) */
    double t_solve;           /* wall seconds in the RC solve (t2) */
    int64_t singular_node;    /* node whose append was singular, else -1 */
} orc_info;

/* Per-iteration record: arrays of length cap; the first min(iterations, cap)
 * entries are written.  Any pointer may be NULL.  With per_iter = p > 1,
 * appended[it] is the number of nodes the iteration appended (the nodes are
 * the next entries of S), node[it] / err[it] still the group maximum. */
typedef struct {
    int64_t cap;
    int32_t *group;           /* i = k mod m */
    int64_t *node;            /* argmax node in G_i \ S (-1 if empty) */
    double *err;              /* E, its error */
    int8_t *appended;         /* 1 if appended */
    /* Monitor (never alters the selection): after every monitor_every-th loop
     * iteration (iterations it with (it + 1) % monitor_every == 0, counted
     * from 0), the all-node max and RMS of |F(r_j) - d_j| with the current W.
     * Sample s goes to mon_max[s], mon_rms[s] (s < cap).  0: no monitor. */
    int32_t monitor_every;
    double *mon_max;
    double *mon_rms;
    int64_t n_monitor;        /* samples written (output) */
} orc_log;

/* Algorithm 1 (GCB greedy; m = 1 is the traditional greedy).  S_out (nc_max)
 * gets the support nodes in selection order, W_out (nc_max,3) their weights. */
int orc_select(const orc_problem *p, int64_t *S_out, double *W_out, orc_log *log, orc_info *info);

/* Weights of K right-hand sides on a given support set (Eqs. 4-5 restricted
 * to S): the RC factor is grown over S in the given order, then
 * Phi_S W = D_S is solved by forward and back substitution.  D (nb,K) holds
 * the displacements of every boundary node; W_out (n,K).  Returns ORC_OK or
 * ORC_E_SINGULAR. */
int orc_solve_on_support(int64_t nb, const double *xyz, const int64_t *S, int64_t n, double radius, int32_t K,
                         const double *D, double *W_out);

/* Inverse Cholesky factor of the support system: L L^T = Phi_S (Eq. 5
 * restricted to S, in the given order; L from the same row recurrence as the
 * selection), then M = L^-1 by forward substitution, column by column.
 * M_out (n,n) row-major, zero above the diagonal.  Returns ORC_OK or
 * ORC_E_SINGULAR. */
int orc_inverse_factor(int64_t nb, const double *xyz, const int64_t *S, int64_t n, double radius, double *M_out);

/* Replays a foreign selection (per iteration: group, node, appended) and
 * checks each step against FP64 errors computed here, following the foreign
 * choice afterwards: the group is k mod m; an appended node lies in G_i \ S,
 * its error is >= E_max - tau and > E* - tau; a skipped iteration has
 * E_max <= E* + tau (or |S| = nc_max).  The foreign start must equal
 * S_init (with a warm start, S_init is ignored: the run starts from warm_S,
 * and it has no iteration only if the kept set meets E* within tau, or
 * reason 6).  Returns -1 when every step is valid, else the first bad
 * iteration index; *reason gets a code (1 group, 2 node outside group or in
 * S, 3 not within tau of the max, 4 wrong append decision, 5 singular,
 * 6 bad termination).  *max_gap gets the largest E_max - e(chosen). */
int64_t orc_validate(const orc_problem *p, const int64_t S_init[3], int64_t n_iter,
                     const int32_t *group, const int64_t *node, const int8_t *appended,
                     double tau, int32_t *reason, double *max_gap);

/* Follow-mode replay of a foreign run of the several-nodes-per-iteration
 * variant (per_iter = p; p = 1 is Algorithm 1): S_seq[0..n_S) is the foreign
 * support sequence (the three starting nodes, then every appended node in
 * order), appended[it] the count appended at iteration it.  At every
 * iteration: the group is k mod m; the count lies between the counts the
 * rule gives with E* + tau and with E* - tau; the t-th appended node lies in
 * G_i \ S and its error is >= (the t-th largest error) - tau and > E* - tau;
 * then the foreign nodes are appended.  Termination as in orc_validate.
 * Returns -1 or the first bad iteration; reasons as in orc_validate, plus
 * 7 (the appended counts do not add up to n_S). */
int64_t orc_validate_block(const orc_problem *p, const int64_t *S_seq, int64_t n_S, int64_t n_iter,
                           const int32_t *group, const int8_t *appended, double tau, int32_t *reason,
                           double *max_gap);

#ifdef __cplusplus
}
#endif
#endif
