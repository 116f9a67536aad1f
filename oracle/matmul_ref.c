/*
 * Oracle O1: the plain value of a matrix product over Z/pZ.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
 * leg of the benchmark may load this code.  It shares nothing with the GPU
 * library and must never be reached from the product path.
 *
 * What it computes (Section 3.2, the operation C <- alpha*A*B + beta*C, taken
 * over the prime field Z/pZ; Section 2 fixes the shapes m x k times k x n):
 *
 *     C[i][j] <- ( alpha * sum_l A[i][l] * B[l][j]  +  beta * C[i][j] ) mod p
 *
 * written as the textbook triple loop in 64-bit integers.  Winograd's
 * identity reproduces this value exactly in any ring, so every schedule of
 * the paper must return it bit for bit.
 *
 * Exactness: entries are canonical residues in [0, p).  A partial sum of t
 * products is at most t*(p-1)^2; the loop folds the running sum with % p
 * every `chunk` terms, where chunk is the largest t with
 * t*(p-1)^2 + (p-1) <= INT64_MAX, so no intermediate ever overflows.
 * For the moduli used here (p < 2^24) chunk exceeds 2^15, so most products
 * take the single final % p.
 *
 * Loop order i-l-j (row of C accumulated in a private int64 buffer), OpenMP
 * over rows.  Nothing else: no blocking, no vectorised tricks.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static int64_t canon(int64_t x, int64_t p)
{
    int64_t r = x % p;
    return r < 0 ? r + p : r;
}

static int64_t fold_chunk(int64_t p)
{
    const uint64_t q = (uint64_t)(p - 1) * (uint64_t)(p - 1);
    if (q == 0)
        return INT64_MAX;
    return (int64_t)(((uint64_t)INT64_MAX - (uint64_t)(p - 1)) / q);
}

/* Returns 0 on success; -1 on bad arguments; -2 if an entry of A, B (or C
 * when beta != 0) is outside [0, p). */
int oracle_matmul_mod_p(int64_t m, int64_t k, int64_t n, int64_t p,
                        const int64_t *A, int64_t lda,
                        const int64_t *B, int64_t ldb,
                        int64_t *C, int64_t ldc,
                        int64_t alpha, int64_t beta, int nthreads)
{
    if (m < 0 || k < 0 || n < 0 || p < 2 || p > (INT64_C(1) << 31))
        return -1;
    if ((m > 0 && k > 0 && lda < k) || (k > 0 && n > 0 && ldb < n) ||
        (m > 0 && n > 0 && ldc < n))
        return -1;
    const int64_t a = canon(alpha, p);
    const int64_t b = canon(beta, p);
    const int64_t chunk = fold_chunk(p);

    for (int64_t i = 0; i < m; ++i) {
        for (int64_t l = 0; l < k; ++l)
            if (A[i * lda + l] < 0 || A[i * lda + l] >= p)
                return -2;
        if (b != 0)
            for (int64_t j = 0; j < n; ++j)
                if (C[i * ldc + j] < 0 || C[i * ldc + j] >= p)
                    return -2;
    }
    for (int64_t l = 0; l < k; ++l)
        for (int64_t j = 0; j < n; ++j)
            if (B[l * ldb + j] < 0 || B[l * ldb + j] >= p)
                return -2;

    if (nthreads <= 0)
        nthreads = omp_get_max_threads();

#pragma omp parallel num_threads(nthreads)
    {
        int64_t *s = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            memset(s, 0, (size_t)(n > 0 ? n : 1) * sizeof(int64_t));
            int64_t since_fold = 0;
            for (int64_t l = 0; l < k; ++l) {
                const int64_t x = A[i * lda + l];
                const int64_t *brow = B + l * ldb;
                for (int64_t j = 0; j < n; ++j)
                    s[j] += x * brow[j];
                if (++since_fold == chunk) {
                    for (int64_t j = 0; j < n; ++j)
                        s[j] %= p;
                    since_fold = 0;
                }
            }
            for (int64_t j = 0; j < n; ++j) {
                int64_t r = (a * (s[j] % p)) % p;
                if (b != 0)
                    r = (r + b * C[i * ldc + j]) % p;
                C[i * ldc + j] = r;
            }
        }
        free(s);
    }
    return 0;
}

/* The same value at `count` chosen positions only, for products too large to
 * form whole on the host: out[t] = C_new[rows[t]][cols[t]].  Cin is read only
 * when beta != 0.  Returns 0, or -1 on bad arguments / out-of-range index. */
int oracle_matmul_entries(int64_t m, int64_t k, int64_t n, int64_t p,
                          const int64_t *A, int64_t lda,
                          const int64_t *B, int64_t ldb,
                          const int64_t *Cin, int64_t ldc,
                          int64_t alpha, int64_t beta,
                          int64_t count, const int64_t *rows,
                          const int64_t *cols, int64_t *out, int nthreads)
{
    if (m < 0 || k < 0 || n < 0 || p < 2 || p > (INT64_C(1) << 31) || count < 0)
        return -1;
    for (int64_t t = 0; t < count; ++t)
        if (rows[t] < 0 || rows[t] >= m || cols[t] < 0 || cols[t] >= n)
            return -1;
    const int64_t a = canon(alpha, p);
    const int64_t b = canon(beta, p);
    const int64_t chunk = fold_chunk(p);
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();

#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t t = 0; t < count; ++t) {
        const int64_t i = rows[t], j = cols[t];
        int64_t s = 0, since_fold = 0;
        for (int64_t l = 0; l < k; ++l) {
            s += A[i * lda + l] * B[l * ldb + j];
            if (++since_fold == chunk) {
                s %= p;
                since_fold = 0;
            }
        }
        int64_t r = (a * (s % p)) % p;
        if (b != 0)
            r = (r + b * Cin[i * ldc + j]) % p;
        out[t] = r;
    }
    return 0;
}
