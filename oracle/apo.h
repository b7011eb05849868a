/*
 * apo.h -- declarations of the FP64 CPU oracle (test infrastructure only).
 * All matrices are dense, row-major, leading dimension n, IEEE double.
 * X (point coordinates) is float32, row-major with leading dimension ldx,
 * exactly the values the GPU library receives, promoted to double.
 */
#ifndef APO_H
#define APO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int apo_num_threads(void);

/* s(i,k) = -||x_i - x_k||^2 off the diagonal, 0 on it (Section 2). */
void apo_similarity(int64_t n, int64_t d, const float *X, int64_t ldx, double *S);
double apo_sqdist(int64_t d, const float *x, const float *y);

/* Counter-based uniform in [0,1) from the SplitMix64 output function. */
double apo_noise_u(uint64_t seed, int64_t n, int64_t i, int64_t k);
/* S[i,k] += scale * u(seed,i,k) for all n*n entries. */
void apo_add_noise(int64_t n, double *S, uint64_t seed, double scale);

/* Algorithm 1 (Eqs. (2)-(4), damping, decision, stop rule).  R and A hold
 * R_0 and A_0 on entry and R_T, A_T on exit; dec gets the raw decisions of
 * iteration T.  trace_nex (nullable, max_iter entries) gets |E_t|.
 * Returns 0 on success, 1 on bad arguments, 2 on allocation failure. */
int apo_ap(int64_t n, const double *S, double lam, int32_t max_iter, int32_t conv_iter,
           double *R, double *A, int32_t *dec, int32_t *iters_out, int32_t *converged_out,
           int32_t *trace_nex);
/* apo_ap with the message-change rule of Algorithm 1, Step 4 as well:
 * msg_tol >= 0 also stops (converged) after the first iteration t >= 2 in
 * which every r and every a changed by at most msg_tol; msg_tol < 0 is
 * apo_ap. */
int apo_ap_tol(int64_t n, const double *S, double lam, int32_t max_iter, int32_t conv_iter, double msg_tol,
               double *R, double *A, int32_t *dec, int32_t *iters_out, int32_t *converged_out,
               int32_t *trace_nex);
void apo_decisions(int64_t n, const double *A, const double *R, int32_t *dec);

/* Algorithm 1 outputs idx, dpsim, expref, netsim from the decisions. */
int64_t apo_finalize(int64_t n, const double *S, const int32_t *dec, int32_t *idx,
                     double *dpsim, double *expref, double *netsim);

/* Nearest candidate (FP64 squared distance, lowest index on ties) for m
 * query points; dist receives the distances. */
void apo_nearest_of(int64_t d, const float *X, int64_t ldx, int64_t m, const int64_t *q, int64_t nex,
                    const int64_t *ex, int32_t *idx, double *dist);
/* Medoid of m points (ascending global indices): least summed FP64 squared
 * distance to the members, lowest index on ties. */
int64_t apo_medoid(int64_t d, const float *X, int64_t ldx, int64_t m, const int64_t *members);
/* FP64 squared distances of m point pairs (a[i], b[i]). */
void apo_pair_dist(int64_t d, const float *X, int64_t ldx, int64_t m, const int64_t *a, const int64_t *b,
                   double *out);
/* Nearest-exemplar assignment in FP64 (Algorithm 3, Step 2). */
void apo_assign_nearest(int64_t n, int64_t d, const float *X, int64_t ldx, int64_t nex,
                        const int64_t *ex, int32_t *idx, double *dpsim);

/* Row-wise pieces of one iteration (for sampled checks of large runs). */
void apo_resp_rows(int64_t n, const double *S, const double *A, const double *R, double lam,
                   const int64_t *rows, int64_t nrows, double *out);
void apo_column_sums(int64_t n, const double *R, double *c);
void apo_avail_rows(int64_t n, const double *Rnew, const double *c, const double *A, double lam,
                    const int64_t *rows, int64_t nrows, double *out);

#ifdef __cplusplus
}
#endif
#endif
