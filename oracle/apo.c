/*
 * apo.c -- FP64 CPU oracle for dense affinity propagation (AP), partition AP
 * and landmark AP.  TEST INFRASTRUCTURE ONLY: the GPU library never links,
 * loads or calls this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header or constant
 * table with the GPU path.
 *
 * Everything is computed in IEEE double precision (compile with
 * -ffp-contract=off so that no multiply-add is fused behind our back).
 * Parallel loops are split so that every floating-point sum is formed in one
 * fixed order (ascending index), independent of the thread count.
 *
 * Paper: Xia, Wu, Zhang, Zhuang, "Local and global approaches of affinity
 * propagation clustering for large scale data", Section 2 (Algorithm 1,
 * Eqs. (1)-(4)), Section 3 (Algorithm 2), Section 4 (Algorithm 3).
 */
#include "apo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define IDX(i, k, n) ((size_t)(i) * (size_t)(n) + (size_t)(k))

int apo_num_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* Similarity, Section 2: s(i,k) = -||x_i - x_k||^2 for i != k.  Written as  */
/* the direct difference form; the diagonal (the preferences) is left 0.     */
/* ------------------------------------------------------------------------ */
void apo_similarity(int64_t n, int64_t d, const float *X, int64_t ldx, double *S)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = 0; k < n; ++k) {
            if (k == i) { S[IDX(i, k, n)] = 0.0; continue; }
            double acc = 0.0;
            for (int64_t j = 0; j < d; ++j) {
                double diff = (double)X[i * ldx + j] - (double)X[k * ldx + j];
                acc += diff * diff;
            }
            S[IDX(i, k, n)] = -acc;
        }
    }
}

/* Squared distance of two points, ascending coordinate order, no fusion. */
double apo_sqdist(int64_t d, const float *x, const float *y)
{
    double acc = 0.0;
    for (int64_t j = 0; j < d; ++j) {
        double diff = (double)x[j] - (double)y[j];
        acc += diff * diff;
    }
    return acc;
}

/* ------------------------------------------------------------------------ */
/* Tie-break noise.  u(seed,i,k) is the SplitMix64 output function (Steele,  */
/* Lea and Flood, 2014) applied to the counter seed + (i*n+k+1)*golden-gamma, */
/* its top 53 bits scaled into [0,1).                                        */
/* ------------------------------------------------------------------------ */
static uint64_t splitmix64_output(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

double apo_noise_u(uint64_t seed, int64_t n, int64_t i, int64_t k)
{
    uint64_t counter = (uint64_t)(i * n + k + 1);
    uint64_t z = splitmix64_output(seed + counter * 0x9E3779B97F4A7C15ULL);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0); /* 2^-53 */
}

void apo_add_noise(int64_t n, double *S, uint64_t seed, double scale)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = 0; k < n; ++k)
            S[IDX(i, k, n)] += scale * apo_noise_u(seed, n, i, k);
}

/* ------------------------------------------------------------------------ */
/* One step of Algorithm 1, Step 2 (Eq. (2)) with damping, for one row.      */
/* The maximum over k' != k of a(i,k')+s(i,k') is the row maximum v1 unless  */
/* k is the (lowest-index) arg-max k1, where it is the runner-up v2.  This   */
/* is an exact rewrite of the max: no rounding is involved.                  */
/* ------------------------------------------------------------------------ */
static void responsibility_row(int64_t n, int64_t i, const double *S, const double *A,
                               double *R, double lam)
{
    const double *s = S + IDX(i, 0, n);
    const double *a = A + IDX(i, 0, n);
    double *r = R + IDX(i, 0, n);
    double v1 = -INFINITY, v2 = -INFINITY;
    int64_t k1 = -1;
    for (int64_t k = 0; k < n; ++k) {
        double v = a[k] + s[k];
        if (v > v1) { v2 = v1; v1 = v; k1 = k; }
        else if (v > v2) { v2 = v; }
    }
    for (int64_t k = 0; k < n; ++k) {
        double maxother = (k == k1) ? v2 : v1;
        double upd = s[k] - maxother;                 /* Eq. (2) */
        r[k] = lam * r[k] + (1.0 - lam) * upd;        /* damping, Section 2 */
    }
}

/* Column sums c_k = sum_{i' != k} max(0, r(i',k)), i' ascending.            */
static void column_sums(int64_t n, const double *R, double *c)
{
    const int64_t CH = 256; /* column chunk per task; each column summed whole */
#pragma omp parallel for schedule(static)
    for (int64_t k0 = 0; k0 < n; k0 += CH) {
        int64_t k1 = k0 + CH < n ? k0 + CH : n;
        for (int64_t k = k0; k < k1; ++k) c[k] = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            const double *r = R + IDX(i, 0, n);
            for (int64_t k = k0; k < k1; ++k)
                if (k != i && r[k] > 0.0) c[k] += r[k];
        }
    }
}

/* Algorithm 1, Step 3 (Eqs. (3) and (4)) with damping, for one row.  The    */
/* sum over i' not in {i,k} is the column sum minus the i-th term.           */
static void availability_row(int64_t n, int64_t i, const double *R, const double *c,
                             double *A, double lam)
{
    const double *r = R + IDX(i, 0, n);
    double *a = A + IDX(i, 0, n);
    for (int64_t k = 0; k < n; ++k) {
        double upd;
        if (k == i) {
            upd = c[k];                                           /* Eq. (4) */
        } else {
            double rik_pos = r[k] > 0.0 ? r[k] : 0.0;
            double rkk = R[IDX(k, k, n)];
            double v = rkk + (c[k] - rik_pos);                    /* Eq. (3) */
            upd = v < 0.0 ? v : 0.0;
        }
        a[k] = lam * a[k] + (1.0 - lam) * upd;                    /* damping */
    }
}

/* Exemplar decision: the k maximising a(i,k)+r(i,k), lowest k on ties.      */
static int32_t decision_row(int64_t n, int64_t i, const double *A, const double *R)
{
    const double *a = A + IDX(i, 0, n);
    const double *r = R + IDX(i, 0, n);
    double best = -INFINITY;
    int32_t bk = 0;
    for (int64_t k = 0; k < n; ++k) {
        double v = a[k] + r[k];
        if (v > best) { best = v; bk = (int32_t)k; }
    }
    return bk;
}

/* Largest |x - y| over n*n entries. */
static double max_abs_diff(int64_t n, const double *x, const double *y)
{
    double m = 0.0;
    for (int64_t q = 0; q < n * n; ++q) {
        const double v = fabs(x[q] - y[q]);
        if (v > m) m = v;
    }
    return m;
}

int apo_ap(int64_t n, const double *S, double lam, int32_t max_iter, int32_t conv_iter,
           double *R, double *A, int32_t *dec, int32_t *iters_out, int32_t *converged_out,
           int32_t *trace_nex)
{
    return apo_ap_tol(n, S, lam, max_iter, conv_iter, -1.0, R, A, dec, iters_out, converged_out, trace_nex);
}

int apo_ap_tol(int64_t n, const double *S, double lam, int32_t max_iter, int32_t conv_iter, double msg_tol,
               double *R, double *A, int32_t *dec, int32_t *iters_out, int32_t *converged_out,
               int32_t *trace_nex)
{
    if (n < 1 || max_iter < 1 || !(lam >= 0.0 && lam < 1.0) || conv_iter < 0) return 1;
    if (n == 1) {
        /* The maximum of Eq. (2) would run over an empty set: a single point
         * is its own exemplar and no message is passed. */
        dec[0] = 0;
        if (iters_out) *iters_out = 0;
        if (converged_out) *converged_out = 1;
        return 0;
    }
    double *c = (double *)malloc(sizeof(double) * (size_t)n);
    uint8_t *e_prev = (uint8_t *)calloc((size_t)n, 1);
    uint8_t *e_cur = (uint8_t *)calloc((size_t)n, 1);
    /* message-change rule: copies of the previous iteration's messages */
    const int msg_on = msg_tol >= 0.0;
    double *Rp = msg_on ? (double *)malloc(sizeof(double) * (size_t)(n * n)) : NULL;
    double *Ap = msg_on ? (double *)malloc(sizeof(double) * (size_t)(n * n)) : NULL;
    if (!c || !e_prev || !e_cur || (msg_on && (!Rp || !Ap))) {
        free(c); free(e_prev); free(e_cur); free(Rp); free(Ap);
        return 2;
    }

    int32_t run = 0, t = 0, converged = 0;
    for (t = 1; t <= max_iter; ++t) {
        if (msg_on) {
            memcpy(Rp, R, sizeof(double) * (size_t)(n * n));
            memcpy(Ap, A, sizeof(double) * (size_t)(n * n));
        }
        /* Step 2: responsibilities from the previous availabilities. */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) responsibility_row(n, i, S, A, R, lam);
        /* Step 3: availabilities from the new responsibilities. */
        column_sums(n, R, c);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) availability_row(n, i, R, c, A, lam);
        /* Decisions and the set of exemplars E_t = { i : d_i = i }. */
        int32_t nex = 0;
#pragma omp parallel for schedule(static) reduction(+ : nex)
        for (int64_t i = 0; i < n; ++i) {
            dec[i] = decision_row(n, i, A, R);
            e_cur[i] = (uint8_t)(dec[i] == i);
            nex += e_cur[i];
        }
        if (trace_nex) trace_nex[t - 1] = nex;
        /* Step 4: stop once the exemplar set has stayed the same for
         * conv_iter consecutive iterations (and is non-empty), or at the
         * iteration cap. */
        int same = (t > 1) && memcmp(e_cur, e_prev, (size_t)n) == 0;
        run = same ? run + 1 : 1;
        uint8_t *tmp = e_prev; e_prev = e_cur; e_cur = tmp;
        if (conv_iter > 0 && run >= conv_iter && nex > 0) { converged = 1; break; }
        /* Step 4, second rule: every message changed by at most msg_tol in
         * this iteration (from the second iteration on). */
        if (msg_on && t >= 2 && max_abs_diff(n, R, Rp) <= msg_tol && max_abs_diff(n, A, Ap) <= msg_tol) {
            converged = 1;
            break;
        }
    }
    if (t > max_iter) t = max_iter;
    if (iters_out) *iters_out = t;
    if (converged_out) *converged_out = converged;
    free(c); free(e_prev); free(e_cur); free(Rp); free(Ap);
    return 0;
}

/* Raw decisions of a given message state (used after a fixed count). */
void apo_decisions(int64_t n, const double *A, const double *R, int32_t *dec)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) dec[i] = decision_row(n, i, A, R);
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 outputs.  Exemplars E = {k : d_k = k} label themselves; every */
/* other point takes the exemplar of largest similarity (lowest index on     */
/* ties), which gives a valid configuration for the energy of Section 2.     */
/* dpsim sums s(i,idx(i)) over non-exemplars, expref sums s(k,k) over E and  */
/* netsim = dpsim + expref.  Returns |E|; with E empty all labels are -1.    */
/* ------------------------------------------------------------------------ */
int64_t apo_finalize(int64_t n, const double *S, const int32_t *dec, int32_t *idx,
                     double *dpsim, double *expref, double *netsim)
{
    int64_t nex = 0;
    for (int64_t k = 0; k < n; ++k) nex += (dec[k] == k);
    if (nex == 0) {
        for (int64_t i = 0; i < n; ++i) idx[i] = -1;
        *dpsim = NAN; *expref = NAN; *netsim = NAN;
        return 0;
    }
    int64_t *ex = (int64_t *)malloc(sizeof(int64_t) * (size_t)nex);
    int64_t m = 0;
    for (int64_t k = 0; k < n; ++k) if (dec[k] == k) ex[m++] = k;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        if (dec[i] == i) { idx[i] = (int32_t)i; continue; }
        double best = -INFINITY; int64_t bk = ex[0];
        for (int64_t j = 0; j < nex; ++j) {
            double v = S[IDX(i, ex[j], n)];
            if (v > best) { best = v; bk = ex[j]; }
        }
        idx[i] = (int32_t)bk;
    }
    double dp = 0.0, ep = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (idx[i] == i) ep += S[IDX(i, i, n)];
        else dp += S[IDX(i, idx[i], n)];
    }
    free(ex);
    *dpsim = dp; *expref = ep; *netsim = dp + ep;
    return nex;
}

/* ------------------------------------------------------------------------ */
/* Landmark AP, Algorithm 3 Step 2 without the distance threshold: each      */
/* point goes to the exemplar at the least squared distance (lowest exemplar */
/* index on ties); exemplars label themselves.  Returns the sum of           */
/* -||x_i - x_idx(i)||^2 over non-exemplars in *dpsim.                       */
/* ------------------------------------------------------------------------ */
/* Nearest of the nex candidate points ex (ascending global indices) for each
 * of the m query points q (global indices), FP64 squared distance, lowest
 * candidate on ties: idx[i] = the candidate's global index, dist[i] its
 * distance (Algorithm 3, Step 2 and the reassignment of Step 4). */
void apo_nearest_of(int64_t d, const float *X, int64_t ldx, int64_t m, const int64_t *q, int64_t nex,
                    const int64_t *ex, int32_t *idx, double *dist)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double best = INFINITY; int64_t bk = nex > 0 ? ex[0] : -1;
        for (int64_t j = 0; j < nex; ++j) {
            double dd = apo_sqdist(d, X + q[i] * ldx, X + ex[j] * ldx);
            if (dd < best) { best = dd; bk = ex[j]; }
        }
        idx[i] = (int32_t)bk; dist[i] = best;
    }
}

/* The medoid of a set of m points (global indices, ascending): the member
 * whose summed FP64 squared distance to all members (summed in member
 * order) is least; the lowest index on ties. */
int64_t apo_medoid(int64_t d, const float *X, int64_t ldx, int64_t m, const int64_t *members)
{
    double *tot = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    if (!tot) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < m; ++q) {
        double t = 0.0;
        for (int64_t i = 0; i < m; ++i) t += apo_sqdist(d, X + members[i] * ldx, X + members[q] * ldx);
        tot[q] = t;
    }
    int64_t best = m > 0 ? members[0] : -1;
    double bt = INFINITY;
    for (int64_t q = 0; q < m; ++q)
        if (tot[q] < bt) { bt = tot[q]; best = members[q]; }
    free(tot);
    return best;
}

/* FP64 squared distances of m point pairs (a[i], b[i]), global indices. */
void apo_pair_dist(int64_t d, const float *X, int64_t ldx, int64_t m, const int64_t *a, const int64_t *b,
                   double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) out[i] = apo_sqdist(d, X + a[i] * ldx, X + b[i] * ldx);
}

void apo_assign_nearest(int64_t n, int64_t d, const float *X, int64_t ldx, int64_t nex,
                        const int64_t *ex /* ascending global indices */, int32_t *idx,
                        double *dpsim)
{
    uint8_t *is_ex = (uint8_t *)calloc((size_t)n, 1);
    for (int64_t j = 0; j < nex; ++j) is_ex[ex[j]] = 1;
    double *best_d = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        if (is_ex[i]) { idx[i] = (int32_t)i; best_d[i] = 0.0; continue; }
        double best = INFINITY; int64_t bk = ex[0];
        for (int64_t j = 0; j < nex; ++j) {
            double dist = apo_sqdist(d, X + i * ldx, X + ex[j] * ldx);
            if (dist < best) { best = dist; bk = ex[j]; }
        }
        idx[i] = (int32_t)bk; best_d[i] = best;
    }
    double dp = 0.0;
    for (int64_t i = 0; i < n; ++i) if (!is_ex[i]) dp -= best_d[i];
    *dpsim = dp;
    free(is_ex); free(best_d);
}

/* ------------------------------------------------------------------------ */
/* Single-row pieces of one iteration, for checking large runs row by row.  */
/* R_next rows: Eq. (2) with damping from (S, A, R) for the listed rows.    */
/* ------------------------------------------------------------------------ */
void apo_resp_rows(int64_t n, const double *S, const double *A, const double *R, double lam,
                   const int64_t *rows, int64_t nrows, double *out /* nrows x n */)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nrows; ++q) {
        const int64_t i = rows[q];
        double *o = out + (size_t)q * (size_t)n;
        for (int64_t k = 0; k < n; ++k) o[k] = R[IDX(i, k, n)];
        /* responsibility_row updates row i of a matrix in place; point it
         * at the output row by offsetting the base so that row i lands on o. */
        responsibility_row(n, 0, S + IDX(i, 0, n), A + IDX(i, 0, n), o, lam);
    }
}

/* Column sums c_k = sum_{i != k} max(0, r(i,k)) of a full R. */
void apo_column_sums(int64_t n, const double *R, double *c) { column_sums(n, R, c); }

/* A_next rows: Eqs. (3), (4) with damping from (R_new, c, A) for the listed rows. */
void apo_avail_rows(int64_t n, const double *Rnew, const double *c, const double *A, double lam,
                    const int64_t *rows, int64_t nrows, double *out /* nrows x n */)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nrows; ++q) {
        const int64_t i = rows[q];
        double *o = out + (size_t)q * (size_t)n;
        const double *r = Rnew + IDX(i, 0, n);
        for (int64_t k = 0; k < n; ++k) {
            double upd;
            if (k == i) {
                upd = c[k];
            } else {
                double rik_pos = r[k] > 0.0 ? r[k] : 0.0;
                double v = Rnew[IDX(k, k, n)] + (c[k] - rik_pos);
                upd = v < 0.0 ? v : 0.0;
            }
            o[k] = lam * A[IDX(i, k, n)] + (1.0 - lam) * upd;
        }
    }
}
