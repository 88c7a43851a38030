/*
 * FP64 CPU oracle for the tile-wise LISI / augLISI image-similarity path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this code.  The product path (the
 * HIP library) never calls it and shares no code, header or table with it.
 *
 * What it computes (Li, Adamek & Armour, "GPU Accelerated Image Quality
 * Assessment-Based Software for Transient Detection"):
 *
 *   pre-processing (Sec. 2): every negative input pixel is set to zero.
 *   Eq. (1)  LISI(x,y)    = D * sum |x+y| / (|x-y| + C1)  /  (max(sum x, sum y) + C2)
 *   Eq. (2)  augLISI(x,y) = 1 - sum |x+y| * |x-y|  /  (sum x + sum y + C)
 *   tiling (Sec. 2, Sec. 3): the N x N images are cut into (N/N_T)^2 tiles of
 *   N_T x N_T pixels; each tile gets one LISI and one augLISI value, giving the
 *   (N/N_T) x (N/N_T) IQA matrix.
 *   Eq. (3), Eq. (4) (Sec. 3): the per-tile values merge exactly into the value
 *   of the whole image or of any larger tile built from whole tiles.
 *
 * Readings where the paper is silent, and the choice made here:
 *   - NaN inputs count as negative (blank pixel -> 0); -0 becomes +0.
 *   - images are row-major (column index fastest); tile t = ty*(N/N_T) + tx.
 *   - N must be a multiple of N_T (no partial edge tiles).
 *   - D, C1, C2, C are caller parameters; callers that want LISI(x,x) ~ 1
 *     pass D = C1/2 (the only choice for which identical inputs give ~1).
 *
 * Parity status: both functions are pinned by tests/test_oracle.py (worked
 * examples derived by hand, exact-rational brute force, closed forms,
 * invariants and the Eq. 3/4 identities), and tests/test_oracle_mutants.py
 * shows those pins catch planted slips.
 *
 * Every sum is accumulated in double, pixel by pixel, in row-major order
 * within the tile; no blocking or reordering beyond the definition.  Tile rows
 * may run on several threads (OpenMP) because tiles are independent; the
 * per-tile order, and so every result bit, does not depend on the thread count.
 */

#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_ERR_SHAPE 1
#define ORACLE_ERR_NULL 2

/* Sec. 2 pre-processing: negative pixels become zero.  "v > 0" is false for
 * NaN and for -0, so both map to +0. */
static double clamp_negative(float v)
{
    return (v > 0.0f) ? (double)v : 0.0;
}

/* Eq. (1) and Eq. (2) on every N_T x N_T tile of two N x N images.
 *
 * lisi, auglisi: n_side*n_side doubles each (may be NULL).
 * sums: 4 doubles per tile, (A, P, Sx, Sy) with A = sum |x+y|/(|x-y|+C1),
 *       P = sum |x+y|*|x-y|, Sx = sum x, Sy = sum y (may be NULL).
 * Returns ORACLE_ERR_SHAPE when N or N_T is not positive or N % N_T != 0. */
int oracle_iqa_tiles(const float *x, const float *y, int64_t N, int64_t NT,
                     double D, double C1, double C2, double C,
                     double *lisi, double *auglisi, double *sums)
{
    if (x == NULL || y == NULL) return ORACLE_ERR_NULL;
    if (N <= 0 || NT <= 0 || N % NT != 0) return ORACLE_ERR_SHAPE;
    const int64_t ns = N / NT;

#pragma omp parallel for schedule(static)
    for (int64_t ty = 0; ty < ns; ++ty) {
        for (int64_t tx = 0; tx < ns; ++tx) {
            double A = 0.0, P = 0.0, Sx = 0.0, Sy = 0.0;
            for (int64_t r = 0; r < NT; ++r) {
                for (int64_t c = 0; c < NT; ++c) {
                    const int64_t i = (ty * NT + r) * N + tx * NT + c;
                    const double xi = clamp_negative(x[i]);
                    const double yi = clamp_negative(y[i]);
                    const double sum_abs = fabs(xi + yi);   /* |x_i + y_i| */
                    const double dif_abs = fabs(xi - yi);   /* |x_i - y_i| */
                    A += sum_abs / (dif_abs + C1);          /* Eq. (1) numerator term */
                    P += sum_abs * dif_abs;                 /* Eq. (2) numerator term */
                    Sx += xi;
                    Sy += yi;
                }
            }
            const int64_t t = ty * ns + tx;
            if (lisi) lisi[t] = D * A / (fmax(Sx, Sy) + C2);          /* Eq. (1) */
            if (auglisi) auglisi[t] = 1.0 - P / (Sx + Sy + C);        /* Eq. (2) */
            if (sums) {
                sums[4 * t + 0] = A;
                sums[4 * t + 1] = P;
                sums[4 * t + 2] = Sx;
                sums[4 * t + 3] = Sy;
            }
        }
    }
    return ORACLE_OK;
}

/* Eq. (3) and Eq. (4): merge f x f blocks of child tiles into parent tiles.
 *
 * Inputs are a child IQA level with ns x ns tiles: lisi_c, aug_c (row-major)
 * and sums_c (4 doubles per tile; only Sx = [2] and Sy = [3] are read, as the
 * per-tile pixel sums the equations multiply by).  The parent level has
 * (ns/f) x (ns/f) tiles; n = f*f children per parent.
 *
 *   parent LISI    = sum_t lisi_t * (max(Sx_t, Sy_t) + C2) / (max(Sx, Sy) + C2)
 *   parent augLISI = (sum_t auglisi_t * (Sx_t + Sy_t + C) - (n - 1) C) / (Sx + Sy + C)
 *
 * where Sx, Sy are the parent's pixel sums, i.e. the sums over its children.
 * Outputs: lisi_p, aug_p (may be NULL) and sums_p (4 doubles per parent: the
 * children's A, P, Sx, Sy added up; may be NULL).  f == ns gives the whole
 * image.  Returns ORACLE_ERR_SHAPE unless f >= 1 and ns % f == 0. */
int oracle_merge_tiles(const double *lisi_c, const double *aug_c, const double *sums_c,
                       int64_t ns, int64_t f, double C2, double C,
                       double *lisi_p, double *aug_p, double *sums_p)
{
    if (lisi_c == NULL || aug_c == NULL || sums_c == NULL) return ORACLE_ERR_NULL;
    if (ns <= 0 || f <= 0 || ns % f != 0) return ORACLE_ERR_SHAPE;
    const int64_t np = ns / f;
    const double n = (double)(f * f);
    for (int64_t py = 0; py < np; ++py) {
        for (int64_t px = 0; px < np; ++px) {
            double Sx = 0.0, Sy = 0.0, A = 0.0, P = 0.0;
            for (int64_t cy = 0; cy < f; ++cy)
                for (int64_t cx = 0; cx < f; ++cx) {
                    const int64_t t = (py * f + cy) * ns + (px * f + cx);
                    A += sums_c[4 * t + 0];
                    P += sums_c[4 * t + 1];
                    Sx += sums_c[4 * t + 2];
                    Sy += sums_c[4 * t + 3];
                }
            double num_l = 0.0, num_a = 0.0;
            for (int64_t cy = 0; cy < f; ++cy)
                for (int64_t cx = 0; cx < f; ++cx) {
                    const int64_t t = (py * f + cy) * ns + (px * f + cx);
                    const double sx = sums_c[4 * t + 2], sy = sums_c[4 * t + 3];
                    num_l += lisi_c[t] * (fmax(sx, sy) + C2);
                    num_a += aug_c[t] * (sx + sy + C);
                }
            const int64_t p = py * np + px;
            if (lisi_p) lisi_p[p] = num_l / (fmax(Sx, Sy) + C2);            /* Eq. (3) */
            if (aug_p) aug_p[p] = (num_a - (n - 1.0) * C) / (Sx + Sy + C);  /* Eq. (4) */
            if (sums_p) {
                sums_p[4 * p + 0] = A;
                sums_p[4 * p + 1] = P;
                sums_p[4 * p + 2] = Sx;
                sums_p[4 * p + 3] = Sy;
            }
        }
    }
    return ORACLE_OK;
}

/* Threads for later calls (n >= 1); tiles are independent, so the count
 * changes the wall time only, never a result bit.  No effect without OpenMP. */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Number of OpenMP threads a parallel region of this library will use
 * (1 when built without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
