/*
 * Reference oracle for batched low-rank products -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, obviously correct CPU definition of what the
 * GPU library computes.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header or table with the GPU library.
 *
 * Paper: Deshmukh, Yokota, Bosilca, "Cache Optimization and Performance
 * Modeling of Batched, Small, and Rectangular Matrix Multiplication on Intel,
 * AMD, and Fujitsu Processors" (arXiv 2311.07602).
 *
 * Conventions (the paper fixes none; readings stated here):
 *   - IEEE binary64 throughout (the paper runs every test in double
 *     precision, Sec. 7).
 *   - Column-major storage, element (i,j) of X at X[i + j*ldx], ldx >= rows.
 *   - Each output entry is one accumulator, started at 0.0 and updated
 *     s = s + a*b with the contraction index ascending; compiled with
 *     -ffp-contract=off so every product is rounded before it is added.
 *   - The output is overwritten (no alpha/beta): the paper's six-loop form
 *     (Alg. 2) accumulates G with "+=" but never states that G starts at
 *     zero, while Alg. 1 defines G as the result of the products.
 *   - Instances are independent; OpenMP splits the instance loop only, so the
 *     arithmetic of each instance is the same for any thread count.
 *
 * Parity pins for every function live in tests/test_oracle_pins.py
 * (identity / permutation / rank-1 closed forms, integer-exact inputs,
 * exact rational brute force, compensated dot products, associativity).
 */
#include <stdint.h>
#include <stddef.h>
#include <math.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(X, i, j, ld) ((X)[(size_t)(i) + (size_t)(j) * (size_t)(ld)])

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Dense x tall-skinny product C = A * U  (A m x k, U k x n, C m x n).
 * In the low-rank setting m = k = b (dense block) and n = r (rank): the dense
 * block times a basis, as in the paper's BLR matrix times multiple right-hand
 * sides (Sec. 7, BLR evaluation) and its batched skinny products (Sec. 3).
 */
static void dense_ts_one(int m, int n, int k, const double *A, int lda,
                         const double *U, int ldu, double *C, int ldc)
{
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int l = 0; l < k; ++l)
                s = s + AT(A, i, l, lda) * AT(U, l, j, ldu);
            AT(C, i, j, ldc) = s;
        }
}

void orc_dense_ts(int64_t count, const int32_t *m, const int32_t *n,
                  const int32_t *k, const double *const *A, const int32_t *lda,
                  const double *const *U, const int32_t *ldu,
                  double *const *C, const int32_t *ldc, int nthreads)
{
    set_threads(nthreads);
    int64_t t;
#pragma omp parallel for schedule(dynamic, 1)
    for (t = 0; t < count; ++t)
        dense_ts_one(m[t], n[t], k[t], A[t], lda[t], U[t], ldu[t], C[t], ldc[t]);
}

/*
 * Rank-sized inner product T = V1^T * U2  (V1 k x m, U2 k x n, T m x n).
 * This is the first step of the paper's low-rank product, C_temp = A_{V^T} B_U
 * (Alg. 1), the loop-4 accumulation C_MN of the six-loop form (Alg. 2).
 * V1 is stored k x m (b x r), so its transpose is implied by the indexing.
 */
static void inner_one(int m, int n, int k, const double *V1, int ldv,
                      const double *U2, int ldu, double *T, int ldt)
{
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int l = 0; l < k; ++l)
                s = s + AT(V1, l, i, ldv) * AT(U2, l, j, ldu);
            AT(T, i, j, ldt) = s;
        }
}

void orc_inner(int64_t count, const int32_t *m, const int32_t *n,
               const int32_t *k, const double *const *V1, const int32_t *ldv,
               const double *const *U2, const int32_t *ldu,
               double *const *T, const int32_t *ldt, int nthreads)
{
    set_threads(nthreads);
    int64_t t;
#pragma omp parallel for schedule(dynamic, 1)
    for (t = 0; t < count; ++t)
        inner_one(m[t], n[t], k[t], V1[t], ldv[t], U2[t], ldu[t], T[t], ldt[t]);
}

/*
 * Recompression product W = U1 * (S * V2^T)
 *   U1 m x k, S k x k, V2 n x k, W m x n  (k = r, m = n = b in the chain).
 * Evaluated in the stated association: first the small core times the skinny
 * basis, P = S * V2^T (k x n), which is the role of the paper's E/G small-by-
 * skinny products (Alg. 1 steps 2-3), then W = U1 * P.  This is the product
 * that rebuilds a block from the r x r core of a low-rank product (Sec. 2:
 * the low-rank multiply is the first step of rounded addition).
 */
static int recomp_one(int m, int n, int k, const double *U1, int ldu,
                      const double *S, int lds, const double *V2, int ldv,
                      double *W, int ldw)
{
    double *P = NULL;
    if (k > 0 && n > 0) {
        P = (double *)malloc(sizeof(double) * (size_t)k * (size_t)n);
        if (!P) return 1;
    }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < k; ++i) {
            double s = 0.0;
            for (int l = 0; l < k; ++l)
                s = s + AT(S, i, l, lds) * AT(V2, j, l, ldv);
            P[(size_t)i + (size_t)j * (size_t)k] = s;
        }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int l = 0; l < k; ++l)
                s = s + AT(U1, i, l, ldu) * P[(size_t)l + (size_t)j * (size_t)k];
            AT(W, i, j, ldw) = s;
        }
    free(P);
    return 0;
}

int orc_recomp(int64_t count, const int32_t *m, const int32_t *n,
               const int32_t *k, const double *const *U1, const int32_t *ldu,
               const double *const *S, const int32_t *lds,
               const double *const *V2, const int32_t *ldv,
               double *const *W, const int32_t *ldw, int nthreads)
{
    set_threads(nthreads);
    int failed = 0;
    int64_t t;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : failed)
    for (t = 0; t < count; ++t)
        failed |= recomp_one(m[t], n[t], k[t], U1[t], ldu[t], S[t], lds[t],
                             V2[t], ldv[t], W[t], ldw[t]);
    return failed;
}

/*
 * The paper's full low-rank product (Alg. 1), in its stated order:
 *   C_temp = A_{V^T} * B_U        (ra x rb;  A_{V^T} is stored kk x ra)
 *   E_temp = A_X * C_temp         (ra x rb;  A_X is ra x ra)
 *   G_XY   = E_temp * B_X         (ra x rb;  B_X is rb x rb)
 * with kk the shared block dimension.  Used to pin the fused form.
 */
static int lr_mult_one(int ra, int rb, int kk, const double *AV, int ldav,
                       const double *BU, int ldbu, const double *AX, int ldax,
                       const double *BX, int ldbx, double *G, int ldg)
{
    size_t sz = sizeof(double) * (size_t)(ra > 0 ? ra : 1) * (size_t)(rb > 0 ? rb : 1);
    double *Ct = (double *)malloc(sz), *Et = (double *)malloc(sz);
    if (!Ct || !Et) { free(Ct); free(Et); return 1; }
    for (int j = 0; j < rb; ++j)
        for (int i = 0; i < ra; ++i) {
            double s = 0.0;
            for (int l = 0; l < kk; ++l)
                s = s + AT(AV, l, i, ldav) * AT(BU, l, j, ldbu);
            Ct[(size_t)i + (size_t)j * ra] = s;
        }
    for (int j = 0; j < rb; ++j)
        for (int i = 0; i < ra; ++i) {
            double s = 0.0;
            for (int l = 0; l < ra; ++l)
                s = s + AT(AX, i, l, ldax) * Ct[(size_t)l + (size_t)j * ra];
            Et[(size_t)i + (size_t)j * ra] = s;
        }
    for (int j = 0; j < rb; ++j)
        for (int i = 0; i < ra; ++i) {
            double s = 0.0;
            for (int l = 0; l < rb; ++l)
                s = s + Et[(size_t)i + (size_t)l * ra] * AT(BX, l, j, ldbx);
            AT(G, i, j, ldg) = s;
        }
    free(Ct);
    free(Et);
    return 0;
}

int orc_lr_mult(int64_t count, const int32_t *ra, const int32_t *rb,
                const int32_t *kk, const double *const *AV, const int32_t *ldav,
                const double *const *BU, const int32_t *ldbu,
                const double *const *AX, const int32_t *ldax,
                const double *const *BX, const int32_t *ldbx,
                double *const *G, const int32_t *ldg, int nthreads)
{
    set_threads(nthreads);
    int failed = 0;
    int64_t t;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : failed)
    for (t = 0; t < count; ++t)
        failed |= lr_mult_one(ra[t], rb[t], kk[t], AV[t], ldav[t], BU[t], ldbu[t],
                              AX[t], ldax[t], BX[t], ldbx[t], G[t], ldg[t]);
    return failed;
}

/*
 * Compensated dot product "Dot2" of Ogita, Rump and Oishi (Accurate sum and
 * dot product, SIAM J. Sci. Comput. 26(6), 2005): the result is as accurate
 * as if computed in twice the working precision and then rounded.  Used only
 * to pin the plain loops above at full size: it is a different evaluation of
 * the same sum, built from error-free transformations.
 *   TwoSum(a,b)     : s = a+b, z = s-a, e = (a-(s-z)) + (b-z)       (Knuth)
 *   TwoProduct(a,b) : p = a*b, e = fma(a,b,-p)                      (exact)
 */
double orc_dot2(int64_t n, const double *x, int64_t incx, const double *y,
                int64_t incy)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double a = x[i * incx], b = y[i * incy];
        double p = a * b;
        double ep = fma(a, b, -p);
        double t = s + p;
        double z = t - s;
        double es = (s - (t - z)) + (p - z);
        s = t;
        c = c + (ep + es);
    }
    return s + c;
}

/*
 * Thin QR factorisation W = Q R by Householder reflections, the first step of
 * the rounded addition of two low-rank blocks (Sec. 2 names the low-rank
 * product as the first step of that algorithm; the addition itself stacks
 * the two blocks' bases, [A_U | B_U] and [A_V | B_V], and orthogonalises
 * them before the small core is decomposed).
 *   W m x n (read only), Q m x p, R p x n, p = min(m, n).
 * Textbook column-by-column Householder QR (Golub and Van Loan, Matrix
 * Computations, the Householder vector of Sec. 5.1.3 and the QR of
 * Sec. 5.2.2), with Q formed by backward accumulation (Sec. 5.1.6):
 *   for j = 0 .. p-1, with x = H(j:m-1, j):
 *     sigma = x(1:)^T x(1:);  v = [1; x(1:) / v0]
 *     sigma = 0:  beta = 0 if x0 >= 0 (H_j = I), else beta = 2, v = e_1
 *                 (H_j flips the sign of row j)
 *     otherwise:  mu = sqrt(x0^2 + sigma),
 *                 v0 = x0 - mu if x0 <= 0, else -sigma / (x0 + mu),
 *                 beta = 2 v0^2 / (sigma + v0^2)
 *     H(j:m-1, j:n-1) <- (I - beta v v^T) H(j:m-1, j:n-1)
 *   so that H_j x = |x| e_1: R has a non-negative diagonal, and Q and R are
 *   unique when W has full column rank.  Q = H_0 H_1 ... H_{p-1} [I_p; 0].
 * Returns non-zero if scratch memory could not be allocated.
 */
static int householder_qr_one(int m, int n, const double *W, int ldw,
                              double *Q, int ldq, double *R, int ldr)
{
    const int p = m < n ? m : n;
    double *H = NULL, *v = NULL, *beta = NULL, *V = NULL;
    if (m > 0 && n > 0) {
        H = (double *)malloc(sizeof(double) * (size_t)m * (size_t)n);
        v = (double *)malloc(sizeof(double) * (size_t)m);
        V = (double *)malloc(sizeof(double) * (size_t)m * (size_t)(p > 0 ? p : 1));
        beta = (double *)malloc(sizeof(double) * (size_t)(p > 0 ? p : 1));
        if (!H || !v || !V || !beta) { free(H); free(v); free(V); free(beta); return 1; }
    }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i)
            H[(size_t)i + (size_t)j * m] = AT(W, i, j, ldw);
    for (int j = 0; j < p; ++j) {
        const double x0 = H[(size_t)j + (size_t)j * m];
        double sigma = 0.0;
        for (int i = j + 1; i < m; ++i)
            sigma = sigma + H[(size_t)i + (size_t)j * m] * H[(size_t)i + (size_t)j * m];
        double b;
        v[j] = 1.0;
        if (sigma == 0.0) {
            b = x0 >= 0.0 ? 0.0 : 2.0;
            for (int i = j + 1; i < m; ++i) v[i] = 0.0;
        } else {
            const double mu = sqrt(x0 * x0 + sigma);
            const double v0 = x0 <= 0.0 ? x0 - mu : -sigma / (x0 + mu);
            b = 2.0 * v0 * v0 / (sigma + v0 * v0);
            for (int i = j + 1; i < m; ++i) v[i] = H[(size_t)i + (size_t)j * m] / v0;
        }
        beta[j] = b;
        for (int c = j; c < n; ++c) {
            double w = 0.0;
            for (int i = j; i < m; ++i)
                w = w + v[i] * H[(size_t)i + (size_t)c * m];
            for (int i = j; i < m; ++i)
                H[(size_t)i + (size_t)c * m] = H[(size_t)i + (size_t)c * m] - b * w * v[i];
        }
        for (int i = 0; i < m; ++i)
            V[(size_t)i + (size_t)j * m] = i < j ? 0.0 : v[i];
    }
    /* R: the upper trapezoid of the reduced matrix */
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < p; ++i)
            AT(R, i, j, ldr) = i <= j ? H[(size_t)i + (size_t)j * m] : 0.0;
    /* Q = H_0 ... H_{p-1} [I_p; 0], applied from the last reflector back */
    for (int j = 0; j < p; ++j)
        for (int i = 0; i < m; ++i)
            AT(Q, i, j, ldq) = i == j ? 1.0 : 0.0;
    for (int j = p - 1; j >= 0; --j)
        for (int c = j; c < p; ++c) {
            double w = 0.0;
            for (int i = j; i < m; ++i)
                w = w + V[(size_t)i + (size_t)j * m] * AT(Q, i, c, ldq);
            for (int i = j; i < m; ++i)
                AT(Q, i, c, ldq) = AT(Q, i, c, ldq) - beta[j] * w * V[(size_t)i + (size_t)j * m];
        }
    free(H);
    free(v);
    free(V);
    free(beta);
    return 0;
}

int orc_householder_qr(int64_t count, const int32_t *m, const int32_t *n,
                       const double *const *W, const int32_t *ldw,
                       double *const *Q, const int32_t *ldq,
                       double *const *R, const int32_t *ldr, int nthreads)
{
    set_threads(nthreads);
    int failed = 0;
    int64_t t;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : failed)
    for (t = 0; t < count; ++t)
        failed |= householder_qr_one(m[t], n[t], W[t], ldw[t], Q[t], ldq[t], R[t], ldr[t]);
    return failed;
}
