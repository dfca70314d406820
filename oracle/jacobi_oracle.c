/*
 * CPU oracle for the mixed-precision Jacobi eigensolver.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the library
 * shares no code with it and never calls it.
 *
 * Source: Z. Zhou, "A Mixed Precision Eigensolver Based on the Jacobi
 * Algorithm" (arXiv 2509.00495).  Each function names the passage it follows.
 * Storage: dense, row-major, leading dimension n, FP64 unless stated.
 * No BLAS, no blocking, no reordering beyond what the cited algorithm states.
 *
 * Pins (tests/test_oracle.py): 2x2 closed forms; the per-rotation off-norm
 * identity of Section 3.1; the small-angle behaviour of Appendix A; diagonal and
 * known-spectrum inputs; trace and Frobenius invariants (orthogonal
 * invariance); brute-force comparison with LAPACK on small inputs; the
 * quadratic-convergence bound of Section 5.2.2; the scalar Newton-Schulz map
 * of the convergence lemma in Section 4.3.4 on matrices of known singular
 * values; the calculus identities
 * and central finite differences for the adjoint.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, n) ((size_t)(i) * (size_t)(n) + (size_t)(j))

/* ------------------------------------------------------------------------ */
/* Algorithm 2 (Jacobi pair, Section 3.1.1), with t from approach 2 of
 * Appendix A:
 *   a_pq = 0            -> c = 1, s = 0
 *   tau = (a_qq - a_pp) / (2 a_pq)
 *   t   = 1/(tau + sqrt(1 + tau^2))  if tau >= 0
 *         1/(tau - sqrt(1 + tau^2))  if tau <  0      (|t| <= 1, |theta| <= pi/4)
 *   c = 1/sqrt(1 + t^2), s = t c.
 * The rotation J = [c s; -s c] zeroes the (p,q) entry of J^T A J (Section 3.1,
 * the 2x2 subproblem). */
void orc_jacobi_pair(double app, double aqq, double apq, double *c, double *s)
{
    if (apq == 0.0) {
        *c = 1.0;
        *s = 0.0;
        return;
    }
    double tau = (aqq - app) / (2.0 * apq);
    double t;
    if (tau >= 0.0)
        t = 1.0 / (tau + sqrt(1.0 + tau * tau));
    else
        t = 1.0 / (tau - sqrt(1.0 + tau * tau));
    *c = 1.0 / sqrt(1.0 + t * t);
    *s = t * (*c);
}

/* off(A) = Frobenius norm of the off-diagonal part (Section 3.1 definition). */
double orc_off(int64_t n, const double *A)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            if (i != j)
                acc += A[IDX(i, j, n)] * A[IDX(i, j, n)];
    return sqrt(acc);
}

double orc_off_f32(int64_t n, const float *A)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            if (i != j)
                acc += (double)A[IDX(i, j, n)] * (double)A[IDX(i, j, n)];
    return sqrt(acc);
}

/* One rotation applied as in the cyclic-by-row code of Section 3.3: with
 * J = [c s; -s c],
 *   rows    A([p q], :) <- J^T A([p q], :)
 *   columns A(:, [p q]) <- A(:, [p q]) J
 *   V(:, [p q]) <- V(:, [p q]) J.
 * Only rows and columns p and q change (Section 2.2.1, the proposition on
 * applying a Givens rotation).  V may be NULL. */
#define DEFINE_ROTATE(NAME, T)                                                 \
    void NAME(int64_t n, T *A, T *V, int64_t p, int64_t q, double cd,          \
              double sd)                                                       \
    {                                                                          \
        const T c = (T)cd, s = (T)sd;                                          \
        for (int64_t j = 0; j < n; ++j) { /* J^T A([p q],:) */                 \
            T ap = A[IDX(p, j, n)], aq = A[IDX(q, j, n)];                      \
            A[IDX(p, j, n)] = c * ap - s * aq;                                 \
            A[IDX(q, j, n)] = s * ap + c * aq;                                 \
        }                                                                      \
        for (int64_t i = 0; i < n; ++i) { /* A(:,[p q]) J */                   \
            T ap = A[IDX(i, p, n)], aq = A[IDX(i, q, n)];                      \
            A[IDX(i, p, n)] = c * ap - s * aq;                                 \
            A[IDX(i, q, n)] = s * ap + c * aq;                                 \
        }                                                                      \
        if (V)                                                                 \
            for (int64_t i = 0; i < n; ++i) { /* V(:,[p q]) J */               \
                T vp = V[IDX(i, p, n)], vq = V[IDX(i, q, n)];                  \
                V[IDX(i, p, n)] = c * vp - s * vq;                             \
                V[IDX(i, q, n)] = s * vp + c * vq;                             \
            }                                                                  \
    }

DEFINE_ROTATE(orc_rotate, double)
DEFINE_ROTATE(orc_rotate_f32, float)

/* Algorithm 4, cyclic-by-row Jacobi (Section 3.3).
 *
 * Sweeps visit (p,q) row by row, p < q.  A pair is rotated when
 *   a_pq != 0  and  |a_pq| > rel_eps * sqrt(|a_pp a_qq|)
 * (the algorithm's per-pair test with tol = rel_eps).  After a sweep that
 * rotated, A <- (A + A^T)/2 and the sweep counter advances.  The iteration
 * stops when a sweep rotates nothing (the paper's rule), when off(A) <= tol_abs
 * (the stopping rule on off), or after max_sweeps sweeps (status 1).
 *
 * The FP32 instantiation serves the low-precision stage: data and rotation
 * updates are in float, the angle (c, s) is computed in double from the float
 * entries and rounded once to float.
 *
 * off_hist (optional, max_sweeps+1 entries) receives off(A) before the first
 * sweep and after each counted sweep.  Returns 0 or 1 (not converged). */
#define DEFINE_CYCLIC(NAME, T, ROT, OFF)                                       \
    int NAME(int64_t n, T *A, T *V, double tol_abs, double rel_eps,            \
             int max_sweeps, int *sweeps_out, double *off_hist,                \
             int64_t *rotations_out)                                           \
    {                                                                          \
        int sweeps = 0, status = 0;                                            \
        int64_t rotations = 0;                                                 \
        if (off_hist)                                                          \
            off_hist[0] = OFF(n, A);                                           \
        for (;;) {                                                             \
            if (sweeps >= max_sweeps) {                                        \
                status = 1;                                                    \
                break;                                                         \
            }                                                                  \
            int rotated = 0;                                                   \
            for (int64_t p = 0; p < n - 1; ++p)                                \
                for (int64_t q = p + 1; q < n; ++q) {                          \
                    double apq = (double)A[IDX(p, q, n)];                      \
                    double app = (double)A[IDX(p, p, n)];                      \
                    double aqq = (double)A[IDX(q, q, n)];                      \
                    if (apq != 0.0 && fabs(apq) > rel_eps * sqrt(fabs(app * aqq))) { \
                        double c, s;                                           \
                        orc_jacobi_pair(app, aqq, apq, &c, &s);                \
                        ROT(n, A, V, p, q, c, s);                              \
                        rotated = 1;                                           \
                        ++rotations;                                           \
                    }                                                          \
                }                                                              \
            if (!rotated)                                                      \
                break;                                                         \
            for (int64_t i = 0; i < n; ++i) /* (A + A^T)/2 */                  \
                for (int64_t j = i + 1; j < n; ++j) {                          \
                    T m = (T)0.5 * (A[IDX(i, j, n)] + A[IDX(j, i, n)]);        \
                    A[IDX(i, j, n)] = m;                                       \
                    A[IDX(j, i, n)] = m;                                       \
                }                                                              \
            ++sweeps;                                                          \
            double off = OFF(n, A);                                            \
            if (off_hist)                                                      \
                off_hist[sweeps] = off;                                        \
            if (off <= tol_abs)                                                \
                break;                                                         \
        }                                                                      \
        if (sweeps_out)                                                        \
            *sweeps_out = sweeps;                                              \
        if (rotations_out)                                                     \
            *rotations_out = rotations;                                        \
        return status;                                                         \
    }

DEFINE_CYCLIC(orc_jacobi_cyclic, double, orc_rotate, orc_off)
DEFINE_CYCLIC(orc_jacobi_cyclic_f32, float, orc_rotate_f32, orc_off_f32)

/* Rounding to IEEE binary16 (half precision: 11 significant bits, exponents
 * -14 .. 15, subnormals down to 2^-24), round to nearest with ties to even,
 * |x| >= 65520 to +-infinity.  Written from the format's definition: the
 * spacing of binary16 numbers around x is 2^(e - 10) for 2^e <= |x| < 2^(e+1)
 * in the normal range and 2^-24 below 2^-14; rint rounds to the nearest
 * integer with ties to even in the default rounding mode. */
double orc_round_half(double x)
{
    if (x != x || x == 0.0)
        return x;
    double a = fabs(x);
    if (a >= 65520.0)
        return x > 0 ? INFINITY : -INFINITY;
    int e;
    frexp(a, &e); /* a = f 2^e, f in [0.5, 1): 2^(e-1) <= a < 2^e */
    int q = (e - 1) - 10;   /* exponent of the spacing */
    if (q < -24)
        q = -24;            /* subnormal spacing */
    double r = ldexp(rint(ldexp(a, -q)), q);
    return x > 0 ? r : -r;
}

/* The half-precision stage of the precision ladder (the lower-precision
 * first stage the paper names as further work, Chapter 6): Algorithm 4 in
 * the cyclic order with the matrix stored in binary16: the angle is computed
 * in double from the stored entries and rounded to float, each rotation's
 * row and column updates are computed in float and every updated entry is
 * rounded to binary16, (A + A^T)/2 at the end of a rotating sweep likewise;
 * V (the accumulated rotations) stays in float.  The iteration stops when off
 * drops to tol_abs, when a sweep rotates nothing, when a sweep lowers off by
 * less than the factor `stall` (the binary16 rounding floor), or after
 * max_sweeps sweeps (status 1).  A holds binary16 values on entry. */
int orc_jacobi_cyclic_h(int64_t n, float *A, float *V, double tol_abs, double rel_eps,
                        double stall, int max_sweeps, int *sweeps_out, double *off_hist)
{
    int sweeps = 0, status = 0;
    double off = orc_off_f32(n, A);
    if (off_hist)
        off_hist[0] = off;
    for (;;) {
        if (off <= tol_abs)
            break;
        if (sweeps >= max_sweeps) {
            status = 1;
            break;
        }
        int rotated = 0;
        for (int64_t p = 0; p < n - 1; ++p)
            for (int64_t q = p + 1; q < n; ++q) {
                double apq = (double)A[IDX(p, q, n)];
                double app = (double)A[IDX(p, p, n)];
                double aqq = (double)A[IDX(q, q, n)];
                if (apq != 0.0 && fabs(apq) > rel_eps * sqrt(fabs(app * aqq))) {
                    double cd, sd;
                    orc_jacobi_pair(app, aqq, apq, &cd, &sd);
                    const float c = (float)cd, s = (float)sd;
                    for (int64_t j = 0; j < n; ++j) { /* J^T A([p q],:) */
                        float ap = A[IDX(p, j, n)], aq = A[IDX(q, j, n)];
                        A[IDX(p, j, n)] = (float)orc_round_half((double)(c * ap - s * aq));
                        A[IDX(q, j, n)] = (float)orc_round_half((double)(s * ap + c * aq));
                    }
                    for (int64_t i = 0; i < n; ++i) { /* A(:,[p q]) J */
                        float ap = A[IDX(i, p, n)], aq = A[IDX(i, q, n)];
                        A[IDX(i, p, n)] = (float)orc_round_half((double)(c * ap - s * aq));
                        A[IDX(i, q, n)] = (float)orc_round_half((double)(s * ap + c * aq));
                    }
                    for (int64_t i = 0; i < n; ++i) { /* V(:,[p q]) J, float */
                        float xp = V[IDX(i, p, n)], xq = V[IDX(i, q, n)];
                        V[IDX(i, p, n)] = c * xp - s * xq;
                        V[IDX(i, q, n)] = s * xp + c * xq;
                    }
                    rotated = 1;
                }
            }
        if (!rotated)
            break;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j) {
                float m = (float)orc_round_half(0.5 * ((double)A[IDX(i, j, n)] +
                                                       (double)A[IDX(j, i, n)]));
                A[IDX(i, j, n)] = m;
                A[IDX(j, i, n)] = m;
            }
        ++sweeps;
        double prev = off;
        off = orc_off_f32(n, A);
        if (off_hist)
            off_hist[sweeps] = off;
        if (off > stall * prev)
            break;
    }
    if (sweeps_out)
        *sweeps_out = sweeps;
    return status;
}

/* Newton-Schulz iterations that the analysis of Section 4.3.4 asks for when
 * the low-precision eigenvectors have unit roundoff u_low: the singular values
 * of X_0 lie in [sqrt(1 - n u_low), sqrt(1 + n u_low)], the error after k
 * iterations is about (sqrt(1 + n u_low) - 1)^(2^k), and k is the smallest
 * count with that <= n u_high.  Returns -1 when n u_low >= 2 (sqrt(1 + n u_low)
 * >= sqrt(3): the iteration is no longer guaranteed to converge). */
int orc_ns_iterations(double n, double u_low, double u_high)
{
    if (n * u_low >= 2.0)
        return -1;
    double e = sqrt(1.0 + n * u_low) - 1.0;
    int k = 0;
    double err = e;
    while (err > n * u_high && k < 64) {
        err = err * err;
        ++k;
    }
    return k;
}

/* A bounded piece of one sweep of Algorithm 4: the cyclic-by-row visits of
 * pivot rows p in [p_begin, p_end) (all q > p), with the same per-pair test
 * and rotation as orc_jacobi_cyclic, no end-of-sweep step.  Used to time the
 * oracle on a sample of a large workload.  Returns the rotations made. */
int64_t orc_jacobi_rows(int64_t n, double *A, double *V, int64_t p_begin,
                        int64_t p_end, double rel_eps)
{
    int64_t rotations = 0;
    for (int64_t p = p_begin; p < p_end && p < n - 1; ++p)
        for (int64_t q = p + 1; q < n; ++q) {
            double apq = A[IDX(p, q, n)], app = A[IDX(p, p, n)], aqq = A[IDX(q, q, n)];
            if (apq != 0.0 && fabs(apq) > rel_eps * sqrt(fabs(app * aqq))) {
                double c, s;
                orc_jacobi_pair(app, aqq, apq, &c, &s);
                orc_rotate(n, A, V, p, q, c, s);
                ++rotations;
            }
        }
    return rotations;
}

/* Output convention (the paper leaves the order free, Section 3.2): W ascending,
 * ties kept in diagonal order; the columns of V are permuted alike and each is
 * scaled by +-1 so that its entry of largest magnitude (lowest row on ties) is
 * positive.  D holds the diagonal of the converged matrix; V is n x n. */
void orc_sort_signfix(int64_t n, const double *D, double *V, double *W)
{
    int64_t *perm = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    double *tmp = (double *)malloc((size_t)(n > 0 ? n * n : 1) * sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        perm[i] = i;
    /* insertion sort: stable */
    for (int64_t i = 1; i < n; ++i) {
        int64_t k = perm[i];
        int64_t j = i - 1;
        while (j >= 0 && D[perm[j]] > D[k]) {
            perm[j + 1] = perm[j];
            --j;
        }
        perm[j + 1] = k;
    }
    memcpy(tmp, V, (size_t)(n * n) * sizeof(double));
    for (int64_t c = 0; c < n; ++c) {
        int64_t src = perm[c];
        W[c] = D[src];
        int64_t imax = 0;
        double amax = -1.0;
        for (int64_t i = 0; i < n; ++i) {
            double a = fabs(tmp[IDX(i, src, n)]);
            if (a > amax) {
                amax = a;
                imax = i;
            }
        }
        double sg = tmp[IDX(imax, src, n)] < 0.0 ? -1.0 : 1.0;
        for (int64_t i = 0; i < n; ++i)
            V[IDX(i, c, n)] = sg * tmp[IDX(i, src, n)];
    }
    free(perm);
    free(tmp);
}

/* Plain FP64 eigendecomposition: Algorithm 4 from V = I, then the output
 * convention above.  A is not modified.  rel_eps = 2^-53 as in the paper's
 * tests (tol = 2^(-53)). */
int orc_eigh(int64_t n, const double *A, double *W, double *V, double tol_abs,
             int max_sweeps, int *sweeps, double *off_hist)
{
    double *B = (double *)malloc((size_t)(n > 0 ? n * n : 1) * sizeof(double));
    double *D = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    memcpy(B, A, (size_t)(n * n) * sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            V[IDX(i, j, n)] = (i == j) ? 1.0 : 0.0;
    int st = orc_jacobi_cyclic(n, B, V, tol_abs, ldexp(1.0, -53), max_sweeps,
                               sweeps, off_hist, NULL);
    for (int64_t i = 0; i < n; ++i)
        D[i] = B[IDX(i, i, n)];
    orc_sort_signfix(n, D, V, W);
    free(B);
    free(D);
    return st;
}

/* Newton-Schulz iteration for the unitary polar factor (Section 4.3.4;
 * Algorithm 8):
 *   X_{k+1} = 1/2 X_k (3 I - X_k^T X_k),   `iters` times, in place. */
void orc_newton_schulz(int64_t n, double *X, int iters)
{
    double *M = (double *)malloc((size_t)(n > 0 ? n * n : 1) * sizeof(double));
    double *Y = (double *)malloc((size_t)(n > 0 ? n * n : 1) * sizeof(double));
    for (int it = 0; it < iters; ++it) {
        for (int64_t i = 0; i < n; ++i) /* M = 3I - X^T X */
            for (int64_t j = 0; j < n; ++j) {
                double acc = 0.0;
                for (int64_t k = 0; k < n; ++k)
                    acc += X[IDX(k, i, n)] * X[IDX(k, j, n)];
                M[IDX(i, j, n)] = (i == j ? 3.0 : 0.0) - acc;
            }
        for (int64_t i = 0; i < n; ++i) /* Y = 1/2 X M */
            for (int64_t j = 0; j < n; ++j) {
                double acc = 0.0;
                for (int64_t k = 0; k < n; ++k)
                    acc += X[IDX(i, k, n)] * M[IDX(k, j, n)];
                Y[IDX(i, j, n)] = 0.5 * acc;
            }
        memcpy(X, Y, (size_t)(n * n) * sizeof(double));
    }
    free(M);
    free(Y);
}

/* Householder vector (Algorithm 1, Section 2.2.2): for x != 0 of length m,
 * v = [v_1, x_2 .. x_m] and beta = 2 / (v^T v) with
 *   sigma = x(2:m)^T x(2:m),  mu = sqrt(x_1^2 + sigma),
 *   v_1 = x_1 + mu if x_1 >= 0, else x_1 - mu,
 * so that (I - beta v v^T) x = -sign(x_1) ||x|| e_1.  A zero x gives beta = 0
 * (P = I).  The algorithm prints the x_1 < 0 branch as -sigma / (x_1 + mu),
 * equal to x_1 - mu in exact arithmetic; with this sign convention x_1 - mu
 * adds two numbers of the same sign, while x_1 + mu cancels (it is 0 when
 * sigma is below the rounding of x_1^2), so the direct form is used. */
void orc_house(int64_t m, const double *x, double *v, double *beta)
{
    double sigma = 0.0;
    for (int64_t i = 1; i < m; ++i)
        sigma += x[i] * x[i];
    for (int64_t i = 1; i < m; ++i)
        v[i] = x[i];
    double mu = sqrt(x[0] * x[0] + sigma);
    if (mu == 0.0) {
        v[0] = 1.0;
        *beta = 0.0;
        return;
    }
    if (x[0] >= 0.0)
        v[0] = x[0] + mu;
    else
        v[0] = x[0] - mu;
    *beta = 2.0 / (v[0] * v[0] + sigma);
}

/* Householder QR factorization (Algorithm 5, Section 4.2): A = Q R with
 * Q = I at the start and, for k = 1 .. n-1,
 *   [v, beta] = house(A(k:n, k))
 *   A(k:n, k:n) <- A(k:n, k:n) - (beta v)(v^T A(k:n, k:n))
 *   Q(:, k:n)   <- Q(:, k:n) - (Q(:, k:n) v)(beta v^T).
 * A (n x n, row-major) is overwritten by the final iterate; R is its upper
 * triangle (written to R, zeros below).  Q is n x n. */
void orc_householder_qr(int64_t n, double *A, double *Q, double *R)
{
    size_t m1 = (size_t)(n > 0 ? n : 1);
    double *x = (double *)malloc(m1 * sizeof(double));
    double *v = (double *)malloc(m1 * sizeof(double));
    double *w = (double *)malloc(m1 * sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            Q[IDX(i, j, n)] = (i == j) ? 1.0 : 0.0;
    for (int64_t k = 0; k < n - 1; ++k) {
        int64_t m = n - k;
        double beta;
        for (int64_t i = 0; i < m; ++i)
            x[i] = A[IDX(k + i, k, n)];
        orc_house(m, x, v, &beta);
        for (int64_t j = 0; j < m; ++j) { /* w = v^T A(k:n, k:n) */
            double acc = 0.0;
            for (int64_t i = 0; i < m; ++i)
                acc += v[i] * A[IDX(k + i, k + j, n)];
            w[j] = acc;
        }
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < m; ++j)
                A[IDX(k + i, k + j, n)] -= (beta * v[i]) * w[j];
        for (int64_t i = 0; i < n; ++i) { /* Q(:, k:n) v, then the rank-1 update */
            double acc = 0.0;
            for (int64_t j = 0; j < m; ++j)
                acc += Q[IDX(i, k + j, n)] * v[j];
            for (int64_t j = 0; j < m; ++j)
                Q[IDX(i, k + j, n)] -= acc * (beta * v[j]);
        }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            R[IDX(i, j, n)] = (j >= i) ? A[IDX(i, j, n)] : 0.0;
    free(x);
    free(v);
    free(w);
}

/* Cholesky factorization of a symmetric positive definite G = R^T R, R upper
 * triangular with positive diagonal (the textbook row-by-row recurrence):
 *   r_ii = sqrt(g_ii - sum_{k<i} r_ki^2),
 *   r_ij = (g_ij - sum_{k<i} r_ki r_kj) / r_ii   (j > i).
 * Returns 0, or i + 1 when the pivot of row i is not positive. */
int orc_cholesky(int64_t n, const double *G, double *R)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            R[IDX(i, j, n)] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = G[IDX(i, i, n)];
        for (int64_t k = 0; k < i; ++k)
            d -= R[IDX(k, i, n)] * R[IDX(k, i, n)];
        if (!(d > 0.0))
            return (int)(i + 1);
        double rii = sqrt(d);
        R[IDX(i, i, n)] = rii;
        for (int64_t j = i + 1; j < n; ++j) {
            double g = G[IDX(i, j, n)];
            for (int64_t k = 0; k < i; ++k)
                g -= R[IDX(k, i, n)] * R[IDX(k, j, n)];
            R[IDX(i, j, n)] = g / rii;
        }
    }
    return 0;
}

/* Cholesky QR of X (the orthogonaliser named as further work in Chapter 6):
 * G = X^T X, R = chol(G), Q = X R^{-1} (Q R = X solved row by row, column by
 * column: q_j = (x_j - sum_{k<j} q_k r_kj) / r_jj).  Returns the Cholesky
 * status. */
int orc_cholesky_qr(int64_t n, const double *X, double *Q, double *R)
{
    size_t nn = (size_t)(n > 0 ? n * n : 1);
    double *G = (double *)malloc(nn * sizeof(double));
    for (int64_t i = 0; i < n; ++i) /* G = X^T X */
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k)
                acc += X[IDX(k, i, n)] * X[IDX(k, j, n)];
            G[IDX(i, j, n)] = acc;
        }
    int st = orc_cholesky(n, G, R);
    if (st == 0)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) {
                double acc = X[IDX(i, j, n)];
                for (int64_t k = 0; k < j; ++k)
                    acc -= Q[IDX(i, k, n)] * R[IDX(k, j, n)];
                Q[IDX(i, j, n)] = acc / R[IDX(j, j, n)];
            }
    free(G);
    return st;
}

/* Preconditioning step of Algorithm 9 (Section 5.1): B = Q^T A Q, then symmetrised. */
void orc_qtaq(int64_t n, const double *Q, const double *A, double *B)
{
    double *T = (double *)malloc((size_t)(n > 0 ? n * n : 1) * sizeof(double));
    for (int64_t i = 0; i < n; ++i) /* T = A Q */
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k)
                acc += A[IDX(i, k, n)] * Q[IDX(k, j, n)];
            T[IDX(i, j, n)] = acc;
        }
    for (int64_t i = 0; i < n; ++i) /* B = Q^T T */
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k)
                acc += Q[IDX(k, i, n)] * T[IDX(k, j, n)];
            B[IDX(i, j, n)] = acc;
        }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            double m = 0.5 * (B[IDX(i, j, n)] + B[IDX(j, i, n)]);
            B[IDX(i, j, n)] = m;
            B[IDX(j, i, n)] = m;
        }
    free(T);
}

/* Algorithm 9 (Section 5.1), mixed-precision (preconditioned) Jacobi, with the
 * low-precision spectral decomposition computed by Algorithm 4 in FP32:
 *   1. fl32(A) -> FP32 cyclic Jacobi until off <= c32 n u_l ||A||_F -> Q_l
 *   2. Q_d = Newton-Schulz(double(Q_l)), ns_iters iterations (Algorithm 8: 2 for
 *      n < 52 000); orth = 1: Q_d = Q of the Householder QR of double(Q_l)
 *      (Algorithm 5), orth = 2: Q of its Cholesky QR (the alternatives the
 *      comparison of Section 4.4 and Chapter 6 name)
 *   3. A_cond = Q_d^T A Q_d (symmetrised); FP64 cyclic Jacobi -> V, Lambda
 *   4. Q = Q_d V, then the output convention.
 * diag (optional, 6 entries) receives: FP32 sweeps, FP64 sweeps,
 * ||Q_l^T Q_l - I||_F, ||Q_d^T Q_d - I||_F, off(A_cond), status of stage 1. */
int orc_eigh_mixed(int64_t n, const double *A, double *W, double *Q,
                   double tol_abs, int max_sweeps, int ns_iters, double c32,
                   int orth, double *diag)
{
    size_t nn = (size_t)(n > 0 ? n * n : 1);
    float *A32 = (float *)malloc(nn * sizeof(float));
    float *V32 = (float *)malloc(nn * sizeof(float));
    double *Qd = (double *)malloc(nn * sizeof(double));
    double *B = (double *)malloc(nn * sizeof(double));
    double *V = (double *)malloc(nn * sizeof(double));
    double *D = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double normF = 0.0;
    for (size_t k = 0; k < (size_t)(n * n); ++k)
        normF += A[k] * A[k];
    normF = sqrt(normF);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            A32[IDX(i, j, n)] = (float)A[IDX(i, j, n)];
            V32[IDX(i, j, n)] = (i == j) ? 1.0f : 0.0f;
        }
    int sw32 = 0, sw64 = 0;
    double ul = ldexp(1.0, -24);
    int st32 = orc_jacobi_cyclic_f32(n, A32, V32, c32 * (double)n * ul * normF,
                                     ul, max_sweeps, &sw32, NULL, NULL);
    for (size_t k = 0; k < (size_t)(n * n); ++k)
        Qd[k] = (double)V32[k];
    double orth_l = 0.0, orth_d = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k)
                acc += Qd[IDX(k, i, n)] * Qd[IDX(k, j, n)];
            acc -= (i == j) ? 1.0 : 0.0;
            orth_l += acc * acc;
        }
    if (orth == 1 || orth == 2) { /* Q_d from a QR factorization of Q_l */
        double *Xl = (double *)malloc(nn * sizeof(double));
        double *Rq = (double *)malloc(nn * sizeof(double));
        memcpy(Xl, Qd, nn * sizeof(double));
        if (orth == 1)
            orc_householder_qr(n, Xl, Qd, Rq);
        else
            orc_cholesky_qr(n, Xl, Qd, Rq);
        free(Xl);
        free(Rq);
    } else {
        orc_newton_schulz(n, Qd, ns_iters);
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k)
                acc += Qd[IDX(k, i, n)] * Qd[IDX(k, j, n)];
            acc -= (i == j) ? 1.0 : 0.0;
            orth_d += acc * acc;
        }
    orc_qtaq(n, Qd, A, B);
    double offc = orc_off(n, B);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            V[IDX(i, j, n)] = (i == j) ? 1.0 : 0.0;
    int st = orc_jacobi_cyclic(n, B, V, tol_abs, ldexp(1.0, -53), max_sweeps,
                               &sw64, NULL, NULL);
    for (int64_t i = 0; i < n; ++i) /* Q = Q_d V */
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k)
                acc += Qd[IDX(i, k, n)] * V[IDX(k, j, n)];
            Q[IDX(i, j, n)] = acc;
        }
    for (int64_t i = 0; i < n; ++i)
        D[i] = B[IDX(i, i, n)];
    orc_sort_signfix(n, D, Q, W);
    if (diag) {
        diag[0] = sw32;
        diag[1] = sw64;
        diag[2] = sqrt(orth_l);
        diag[3] = sqrt(orth_d);
        diag[4] = offc;
        diag[5] = st32;
    }
    free(A32);
    free(V32);
    free(Qd);
    free(B);
    free(V);
    free(D);
    return st;
}

/* Rayleigh quotient and residual of each column of V against A (plain
 * definitions; used to certify the oracle's own eigenpairs at sizes where its
 * diagonal readout carries the rounding of many sweeps):
 *   y = A v_k,  rq_k = (v_k^T y) / (v_k^T v_k),
 *   res_k = ||y - rq_k v_k||_2 / ||v_k||_2.
 * For an exact eigenpair res_k = 0 and rq_k = lambda_k; otherwise some
 * eigenvalue lies within res_k of rq_k, and within res_k^2 / gap_k when every
 * other eigenvalue is at least gap_k away (Kato-Temple).  The sums are
 * accumulated in long double so that the check adds little rounding of its
 * own.  V is n x n, columns are the vectors. */
void orc_rayleigh(int64_t n, const double *A, const double *V, double *rq,
                  double *res)
{
    size_t m = (size_t)(n > 0 ? n : 1);
    long double *y = (long double *)malloc(m * sizeof(long double));
    long double *v = (long double *)malloc(m * sizeof(long double));
    for (int64_t k = 0; k < n; ++k) {
        long double vv = 0.0L, vy = 0.0L;
        for (int64_t i = 0; i < n; ++i) /* column k, contiguous */
            v[i] = (long double)V[IDX(i, k, n)];
        for (int64_t i = 0; i < n; ++i) {
            long double acc = 0.0L;
            for (int64_t j = 0; j < n; ++j)
                acc += (long double)A[IDX(i, j, n)] * v[j];
            y[i] = acc;
            vv += v[i] * v[i];
            vy += v[i] * acc;
        }
        long double q = vv > 0.0L ? vy / vv : 0.0L;
        long double rr = 0.0L;
        for (int64_t i = 0; i < n; ++i) {
            long double d = y[i] - q * v[i];
            rr += d * d;
        }
        rq[k] = (double)q;
        res[k] = vv > 0.0L ? (double)sqrtl(rr / vv) : 0.0;
    }
    free(y);
    free(v);
}

/* Adjoint of A = V diag(W) V^T (the paper does not treat derivatives; this is
 * the standard first-order perturbation result for distinct eigenvalues):
 *   M = V^T dV;  M_ij <- M_ij / (W_j - W_i) for i != j;  M_ii <- dW_i
 *   G = V M V^T;  dA = (G + G^T)/2.
 * A pair with |W_j - W_i| < gap_tol contributes 0 and raises the return value
 * to 4 when its coupling M_ij is nonzero.  dW or dV may be NULL (zero). */
int orc_eigh_backward(int64_t n, const double *W, const double *V,
                      const double *dW, const double *dV, double gap_tol,
                      double *dA)
{
    size_t nn = (size_t)(n > 0 ? n * n : 1);
    double *M = (double *)calloc(nn, sizeof(double));
    double *T = (double *)malloc(nn * sizeof(double));
    int status = 0;
    if (dV)
        for (int64_t i = 0; i < n; ++i) /* M = V^T dV */
            for (int64_t j = 0; j < n; ++j) {
                double acc = 0.0;
                for (int64_t k = 0; k < n; ++k)
                    acc += V[IDX(k, i, n)] * dV[IDX(k, j, n)];
                M[IDX(i, j, n)] = acc;
            }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            if (i == j) {
                M[IDX(i, i, n)] = dW ? dW[i] : 0.0;
                continue;
            }
            double gap = W[j] - W[i];
            if (fabs(gap) < gap_tol) {
                if (M[IDX(i, j, n)] != 0.0)
                    status = 4;
                M[IDX(i, j, n)] = 0.0;
            } else {
                M[IDX(i, j, n)] = M[IDX(i, j, n)] / gap;
            }
        }
    for (int64_t i = 0; i < n; ++i) /* T = V M */
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k)
                acc += V[IDX(i, k, n)] * M[IDX(k, j, n)];
            T[IDX(i, j, n)] = acc;
        }
    for (int64_t i = 0; i < n; ++i) /* G = T V^T -> dA */
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k)
                acc += T[IDX(i, k, n)] * V[IDX(j, k, n)];
            dA[IDX(i, j, n)] = acc;
        }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            double m = 0.5 * (dA[IDX(i, j, n)] + dA[IDX(j, i, n)]);
            dA[IDX(i, j, n)] = m;
            dA[IDX(j, i, n)] = m;
        }
    free(M);
    free(T);
    return status;
}
