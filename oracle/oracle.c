/*
 * Oracle for the truncated block-sparse algebra of linear-scaling density-matrix
 * RT-TDDFT (O'Rourke & Bowler, arXiv:1404.5776).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct FP64 C that the
 * test-suite, the smoke check and the CPU baseline of the benchmark call to
 * check the GPU library.  It shares no code, header or table with the GPU path.
 *
 * Two primitives live here because numpy cannot express them at useful sizes:
 *
 *   oracle_pattern_*  the spatial cut-off of Sec. II.A: the block (i,j) of a
 *                     matrix is kept iff i == j or |r_i - r_j| < R, tested as
 *                     dx*dx + dy*dy + dz*dz < R*R in double precision;
 *                     brute force over all pairs.
 *
 *   oracle_spgemm     C = P_C(alpha * op(A) op(B)), the product of two
 *                     atom-pair-blocked matrices with every element outside
 *                     C's cut-off pattern dropped (Sec. II.A cut-off applied to
 *                     each product, Sec. V.A truncation of S^-1 and S^-1 H).
 *                     Row-by-row Gustavson: for each output row i, each k with
 *                     op(A)_ik stored, each j with op(B)_kj stored and (i,j)
 *                     kept in C, accumulate op(A)_ik op(B)_kj.  op is the
 *                     identity or the conjugate transpose (for U^dagger).
 *
 * Storage (oracle's own): a matrix of n atoms with b functions each is
 * row_ptr[n+1] (int64), col[nnzb] (int32, ascending inside each row) and
 * val[nnzb][b][b][2] (interleaved real/imaginary doubles, row-major blocks).
 * Cut-off patterns are symmetric ((i,j) kept iff (j,i) kept), which the
 * conjugate-transpose lookups below rely on; the Python side asserts it.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- pattern */

static int in_range(const double *xyz, int64_t i, int64_t j, double R)
{
    if (i == j) return 1;
    double dx = xyz[3 * i + 0] - xyz[3 * j + 0];
    double dy = xyz[3 * i + 1] - xyz[3 * j + 1];
    double dz = xyz[3 * i + 2] - xyz[3 * j + 2];
    return dx * dx + dy * dy + dz * dz < R * R;
}

/* row_count[i] = number of atoms j kept in row i. */
void oracle_pattern_count(int64_t n, const double *xyz, double R, int64_t *row_count)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j) c += in_range(xyz, i, j, R);
        row_count[i] = c;
    }
}

/* col[row_ptr[i] ...] = kept atoms j of row i, ascending. */
void oracle_pattern_fill(int64_t n, const double *xyz, double R,
                         const int64_t *row_ptr, int32_t *col)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        int64_t p = row_ptr[i];
        for (int64_t j = 0; j < n; ++j)
            if (in_range(xyz, i, j, R)) col[p++] = (int32_t)j;
    }
}

/* ---------------------------------------------------------------- product */

/* Position of column j in row i, or -1. */
static int64_t find_block(const int64_t *row_ptr, const int32_t *col, int64_t i, int64_t j)
{
    int64_t lo = row_ptr[i], hi = row_ptr[i + 1] - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] == j) return mid;
        if (col[mid] < j) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Element (r, c) of op(M) for one stored block; op = 0 identity, 1 conjugate transpose. */
static void block_elem(const double *blk, int b, int op, int r, int c, double *re, double *im)
{
    if (op == 0) {
        *re = blk[2 * (r * b + c)];
        *im = blk[2 * (r * b + c) + 1];
    } else {
        *re = blk[2 * (c * b + r)];
        *im = -blk[2 * (c * b + r) + 1];
    }
}

/*
 * C = P_C(alpha * op(A) * op(B)) for output rows [row_lo, row_hi).
 * Blocks of C in those rows are overwritten.  Returns the number of
 * (i, k, j) block triples that contributed (the algorithmic unit of work).
 */
int64_t oracle_spgemm(int64_t n, int b,
                      const int64_t *a_ptr, const int32_t *a_col, const double *a_val, int op_a,
                      const int64_t *b_ptr, const int32_t *b_col, const double *b_val, int op_b,
                      const int64_t *c_ptr, const int32_t *c_col, double *c_val,
                      double alpha_re, double alpha_im, int64_t row_lo, int64_t row_hi)
{
    const int64_t bb2 = 2 * (int64_t)b * b;
    int64_t triples = 0;
#pragma omp parallel reduction(+ : triples)
    {
        int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        double *acc = NULL;
        int64_t acc_cap = 0;
        for (int64_t j = 0; j < n; ++j) slot[j] = -1;
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = row_lo; i < row_hi; ++i) {
            int64_t c0 = c_ptr[i], c1 = c_ptr[i + 1];
            if (c1 - c0 > acc_cap) {
                acc_cap = c1 - c0;
                acc = (double *)realloc(acc, sizeof(double) * (size_t)(acc_cap * bb2));
            }
            memset(acc, 0, sizeof(double) * (size_t)((c1 - c0) * bb2));
            for (int64_t p = c0; p < c1; ++p) slot[c_col[p]] = p - c0;

            /* k runs over the stored blocks of op(A) in row i. */
            for (int64_t pa = a_ptr[i]; pa < a_ptr[i + 1]; ++pa) {
                int64_t k = a_col[pa];
                int64_t ablk = (op_a == 0) ? pa : find_block(a_ptr, a_col, k, i);
                if (ablk < 0) continue;
                const double *A = a_val + ablk * bb2;
                /* j runs over the stored blocks of op(B) in row k. */
                for (int64_t pb = b_ptr[k]; pb < b_ptr[k + 1]; ++pb) {
                    int64_t j = b_col[pb];
                    int64_t s = slot[j];
                    if (s < 0) continue;                   /* outside C's cut-off */
                    int64_t bblk = (op_b == 0) ? pb : find_block(b_ptr, b_col, j, k);
                    if (bblk < 0) continue;
                    const double *B = b_val + bblk * bb2;
                    double *C = acc + s * bb2;
                    ++triples;
                    for (int r = 0; r < b; ++r)
                        for (int c = 0; c < b; ++c) {
                            double sr = 0.0, si = 0.0;
                            for (int m = 0; m < b; ++m) {
                                double ar, ai, br, bi;
                                block_elem(A, b, op_a, r, m, &ar, &ai);
                                block_elem(B, b, op_b, m, c, &br, &bi);
                                sr += ar * br - ai * bi;
                                si += ar * bi + ai * br;
                            }
                            C[2 * (r * b + c)] += sr;
                            C[2 * (r * b + c) + 1] += si;
                        }
                }
            }
            for (int64_t p = c0; p < c1; ++p) {
                double *dst = c_val + p * bb2;
                const double *src = acc + (p - c0) * bb2;
                for (int64_t e = 0; e < bb2; e += 2) {
                    double xr = src[e], xi = src[e + 1];
                    dst[e] = alpha_re * xr - alpha_im * xi;
                    dst[e + 1] = alpha_re * xi + alpha_im * xr;
                }
                slot[c_col[p]] = -1;
            }
        }
        free(acc);
        free(slot);
    }
    return triples;
}

/* Threads of the OpenMP regions above (timing of the oracle at a fixed
 * thread count); returns the count in force afterwards. */
int oracle_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}
