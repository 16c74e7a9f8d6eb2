/*
 * CPU oracle for C := alpha*A*B + beta*C in IEEE binary64.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library calls, links or
 * includes this file; only the tests, the smoke check and the CPU baseline of
 * the benchmark use it.  It shares no code with the HIP path.
 *
 * What it computes: the ordinary matrix product of the paper (Sec. 2.1, the
 * footnote defining gamma_ij = sum_p alpha_ip beta_pj; Sec. 2.2.1 for
 * C += A B), with BLAS alpha/beta semantics on top.  Every entry is one plain
 * dot product over p = 0..k-1 in ascending order, evaluated with the
 * compensated "Dot2" scheme of Ogita, Rump and Oishi (SIAM J. Sci. Comput.
 * 26(6), 2005): each product is split exactly into fl(a*b) plus its rounding
 * error via an FMA (TwoProduct), each running sum into fl(s+h) plus its
 * rounding error (TwoSum), and the collected errors are added back once at
 * the end.  The result is as accurate as if computed in twice the working
 * precision and then rounded once.
 *
 * The alpha/beta step is done in the same style: alpha*(p+s) and beta*c are
 * each split by TwoProduct, the two leading parts are added by TwoSum, and the
 * result is rounded once.  With alpha = 1 and beta = 0 the entry is fl(p+s).
 *
 * Row-major storage: A is m x k with leading dimension lda, B is k x n (ldb),
 * C is m x n (ldc).  Build with -O2 -ffp-contract=off -fno-fast-math so that
 * the only fused operation is the explicit fma().
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

/* Error-free transformation of a product: a*b = h + r exactly. */
static inline void two_product(double a, double b, double *h, double *r) {
    *h = a * b;
    *r = fma(a, b, -*h);
}

/* Error-free transformation of a sum (Knuth): a+b = s + q exactly. */
static inline void two_sum(double a, double b, double *s, double *q) {
    double x = a + b;
    double z = x - a;
    *q = (a - (x - z)) + (b - z);
    *s = x;
}

/* One entry: beta*c + alpha * sum_p A[i,p] B[p,j], compensated. */
static double entry(int64_t i, int64_t j, int64_t k, double alpha,
                    const double *A, int64_t lda, const double *B, int64_t ldb,
                    double beta, double c) {
    double p = 0.0, s = 0.0;
    for (int64_t q = 0; q < k; ++q) {
        double h, r, t, e;
        two_product(A[i * lda + q], B[q * ldb + j], &h, &r);
        if (q == 0) {
            p = h;
            s = r;
        } else {
            two_sum(p, h, &t, &e);
            p = t;
            s = s + (e + r);
        }
    }
    /* alpha*(p + s) + beta*c, rounded once. */
    double h1, r1, h2 = 0.0, r2 = 0.0, t, e;
    two_product(alpha, p, &h1, &r1);
    double tail_a = alpha * s;
    if (beta != 0.0) two_product(beta, c, &h2, &r2);
    two_sum(h1, h2, &t, &e);
    return t + (((e + r1) + tail_a) + r2);
}

/*
 * Full product.  beta == 0 means C is not read (so NaNs in C are not
 * propagated), following the BLAS convention.  Rows are split across OpenMP
 * threads; the result does not depend on the thread count.
 */
void oracle_dgemm(int64_t m, int64_t n, int64_t k, double alpha,
                  const double *A, int64_t lda, const double *B, int64_t ldb,
                  double beta, double *C, int64_t ldc) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double c = (beta != 0.0) ? C[i * ldc + j] : 0.0;
            C[i * ldc + j] = entry(i, j, k, alpha, A, lda, B, ldb, beta, c);
        }
    }
}

/*
 * Selected entries only: out[t] = beta*C[rows[t], cols[t]] + alpha*(A B)[rows[t], cols[t]].
 * C is read (when beta != 0) but not written.  Used where the full product
 * would take too long on the CPU.
 */
void oracle_dgemm_entries(int64_t npts, const int64_t *rows, const int64_t *cols,
                          int64_t k, double alpha,
                          const double *A, int64_t lda, const double *B, int64_t ldb,
                          double beta, const double *C, int64_t ldc, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < npts; ++t) {
        int64_t i = rows[t], j = cols[t];
        double c = (beta != 0.0) ? C[i * ldc + j] : 0.0;
        out[t] = entry(i, j, k, alpha, A, lda, B, ldb, beta, c);
    }
}

/* Number of OpenMP threads the oracle runs with. */
int oracle_num_threads(void) {
    int nt = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            nt = omp_get_num_threads();
#endif
        }
    }
    return nt;
}
