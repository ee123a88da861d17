/*
 * CPU oracle for the correlation hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 reference of what the GPU library
 * computes. Only the test-suite, the smoke check and the benchmark's CPU
 * baseline leg may load it; the product never calls it. It shares no code,
 * header, table or constant generator with the GPU library.
 *
 * Passages followed (arXiv 2309.03308):
 *   - Sec. 3 (problem statement): ensemble of E members on an X x Y x Z grid;
 *     the indicator of a brick pair is the maximum point-to-point correlation.
 *   - Sec. 3.2: Pearson (PPMCC) needs only means and variances; the Kraskov
 *     estimator (KSG, "KMI") with Chebyshev k-th-neighbour distance eps_i,
 *     strict marginal counts n_x,i and n_y,i, and the digamma sum; the digamma
 *     function is the logarithmic derivative of Gamma (Eq. 2).
 *
 * Readings where the paper is silent or garbled:
 *   - the KSG sum is (1/n) * sum_i [psi(n_x,i) + psi(n_y,i)] (brackets missing
 *     in the printed formula);
 *   - marginal counts exclude the sample itself and enter as psi(n + 1), which
 *     equals the printed form whenever eps_i > 0 and stays defined at eps_i = 0;
 *   - eps_i is the k-th smallest value of the multiset {d_ij : j != i};
 *   - distances use FP32 subtraction, abs and max, so integer counts are
 *     reproducible bit for bit; everything else is FP64;
 *   - KSG works on z-scored samples z = fl32(fl32(x - mu32) * inv32) with
 *     mu32 = fl32(mu), inv32 = fl32(1/sigma_pop), mu and sigma from two-pass
 *     FP64 sums in member order;
 *   - a point with zero variance gives r = 0 and MI = 0;
 *   - region maxima take |r| (or MI), skip pA == pB when both regions come
 *     from the same field, and break ties towards the smallest (local pA,
 *     local pB) in x-fastest local order.
 *
 * digamma at integer arguments: psi(n) = -gamma + sum_{j=1}^{n-1} 1/j, which
 * is exact (no approximation) for the integer arguments KSG needs.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EULER_GAMMA 0.57721566490153286060651209008240243

/* digamma at a positive integer n (Eq. 2 evaluated through the recurrence
 * psi(n+1) = psi(n) + 1/n, psi(1) = -gamma). */
double orc_digamma_int(int n)
{
    double s = -EULER_GAMMA;
    for (int j = 1; j < n; ++j) s += 1.0 / (double)j;
    return s;
}

/* Two-pass FP64 mean and sum of squared deviations of one point, in member
 * order. value(m) = x[m * stride + p]. */
static void point_stats(const float* x, int64_t stride, int M, int64_t p, double* mu, double* s2)
{
    double s = 0.0;
    for (int m = 0; m < M; ++m) s += (double)x[(int64_t)m * stride + p];
    double mean = s / (double)M;
    double q = 0.0;
    for (int m = 0; m < M; ++m) {
        double d = (double)x[(int64_t)m * stride + p] - mean;
        q += d * d;
    }
    *mu = mean;
    *s2 = q;
}

/* Per-point statistics for the listed points. Outputs FP64 mean, FP64 sum of
 * squared deviations, and the FP32 KSG standardisation constants. */
void orc_stats(const float* x, int64_t stride, int M, const int32_t* pts, int64_t npts,
               double* mu, double* s2, float* mu32, float* inv32)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npts; ++i) {
        double a, b;
        point_stats(x, stride, M, pts[i], &a, &b);
        if (mu) mu[i] = a;
        if (s2) s2[i] = b;
        if (mu32) mu32[i] = (float)a;
        if (inv32) {
            double sig = sqrt(b / (double)M);
            inv32[i] = (b > 0.0) ? (float)(1.0 / sig) : 0.0f;
        }
    }
}

/* KSG input rows: z[i][m] = fl32(fl32(x - mu32) * inv32) for the listed points. */
void orc_ksg_inputs(const float* x, int64_t stride, int M, const int32_t* pts, int64_t npts, float* z)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npts; ++i) {
        double a, b;
        point_stats(x, stride, M, pts[i], &a, &b);
        float mu32 = (float)a;
        float inv32 = (b > 0.0) ? (float)(1.0 / sqrt(b / (double)M)) : 0.0f;
        for (int m = 0; m < M; ++m) {
            float d = x[(int64_t)m * stride + pts[i]] - mu32;
            z[i * (int64_t)M + m] = d * inv32;
        }
    }
}

/* Pearson coefficient of two points, straight from the definition (Sec. 3.2). */
static double pearson_one(const float* xa, int64_t sa, int64_t pa, const float* xb, int64_t sb, int64_t pb, int M)
{
    double ma, qa, mb, qb;
    point_stats(xa, sa, M, pa, &ma, &qa);
    point_stats(xb, sb, M, pb, &mb, &qb);
    if (qa <= 0.0 || qb <= 0.0) return 0.0;
    double c = 0.0;
    for (int m = 0; m < M; ++m)
        c += ((double)xa[(int64_t)m * sa + pa] - ma) * ((double)xb[(int64_t)m * sb + pb] - mb);
    return c / sqrt(qa * qb);
}

void orc_pearson_pairs(const float* xa, int64_t sa, const float* xb, int64_t sb, int M,
                       const int32_t* pairs, int64_t n, double* r)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i)
        r[i] = pearson_one(xa, sa, pairs[2 * i], xb, sb, pairs[2 * i + 1], M);
}

static int cmp_float(const void* a, const void* b)
{
    float x = *(const float*)a, y = *(const float*)b;
    return (x < y) ? -1 : (x > y) ? 1 : 0;
}

/* KSG mutual information of one pair of sample rows (Sec. 3.2), brute force.
 * counts (optional) receives n_x,i and n_y,i for each sample i. */
static double ksg_one(const float* x, const float* y, int M, int k, const double* psi, int32_t* counts, float* work)
{
    double acc = 0.0;
    for (int i = 0; i < M; ++i) {
        int c = 0;
        for (int j = 0; j < M; ++j) {
            if (j == i) continue;
            float dx = fabsf(x[i] - x[j]);
            float dy = fabsf(y[i] - y[j]);
            work[c++] = dx > dy ? dx : dy;
        }
        qsort(work, (size_t)c, sizeof(float), cmp_float);
        float eps = work[k - 1];
        int nx = 0, ny = 0;
        for (int j = 0; j < M; ++j) {
            if (j == i) continue;
            if (fabsf(x[i] - x[j]) < eps) ++nx;
            if (fabsf(y[i] - y[j]) < eps) ++ny;
        }
        if (counts) {
            counts[2 * i] = nx;
            counts[2 * i + 1] = ny;
        }
        acc += psi[nx + 1] + psi[ny + 1];
    }
    return psi[M] + psi[k] - acc / (double)M;
}

/* KSG over a pair list. za (rows of point A's samples) and zb are point-major:
 * sample m of point p is z[p * ldz + m]. zero_a / zero_b flag zero-variance
 * points (NULL = none); such pairs give MI = 0 with all counts 0. */
void orc_ksg_pairs(const float* za, const float* zb, int64_t ldz, int M, int k,
                   const int32_t* pairs, int64_t n, const uint8_t* zero_a, const uint8_t* zero_b,
                   double* mi, int32_t* counts)
{
    double* psi = (double*)malloc(sizeof(double) * (size_t)(M + 2));
    for (int v = 1; v <= M + 1; ++v) psi[v] = orc_digamma_int(v);
    psi[0] = 0.0;
#pragma omp parallel
    {
        float* work = (float*)malloc(sizeof(float) * (size_t)M);
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < n; ++t) {
            int64_t a = pairs[2 * t], b = pairs[2 * t + 1];
            int32_t* cnt = counts ? counts + t * 2 * (int64_t)M : NULL;
            if ((zero_a && zero_a[a]) || (zero_b && zero_b[b])) {
                mi[t] = 0.0;
                if (cnt) memset(cnt, 0, sizeof(int32_t) * 2 * (size_t)M);
                continue;
            }
            mi[t] = ksg_one(za + a * ldz, zb + b * ldz, M, k, psi, cnt, work);
        }
        free(work);
    }
    free(psi);
}

/* Region maximum over an explicit value list: values[t] for pair t with local
 * coordinates (la[t], lb[t]). Objective |v| if use_abs. Ties go to the smallest
 * (la, lb). Returns the winning index t. */
int64_t orc_argmax_pairs(const double* values, const int32_t* la, const int32_t* lb, int64_t n, int use_abs)
{
    int64_t best = -1;
    double bv = -INFINITY;
    for (int64_t t = 0; t < n; ++t) {
        double v = use_abs ? fabs(values[t]) : values[t];
        if (best < 0 || v > bv || (v == bv && (la[t] < la[best] || (la[t] == la[best] && lb[t] < lb[best])))) {
            best = t;
            bv = v;
        }
    }
    return best;
}

/* Exhaustive Pearson region maximum: every (pA, pB) in A x B, pA and pB global
 * indices listed in local x-fastest order. same_field skips pA == pB.
 * Outputs max |r|, the signed r there, and the local argmax. */
void orc_pearson_region_max(const float* xa, int64_t sa, const int32_t* pa, int64_t na,
                            const float* xb, int64_t sb, const int32_t* pb, int64_t nb, int M,
                            int same_field, double* value, double* signed_value, int64_t* la, int64_t* lb,
                            int64_t* n_evaluated)
{
    double* ma = (double*)malloc(sizeof(double) * (size_t)na);
    double* qa = (double*)malloc(sizeof(double) * (size_t)na);
    double* mb = (double*)malloc(sizeof(double) * (size_t)nb);
    double* qb = (double*)malloc(sizeof(double) * (size_t)nb);
    for (int64_t i = 0; i < na; ++i) point_stats(xa, sa, M, pa[i], &ma[i], &qa[i]);
    for (int64_t j = 0; j < nb; ++j) point_stats(xb, sb, M, pb[j], &mb[j], &qb[j]);
    double* rowv = (double*)malloc(sizeof(double) * (size_t)na);
    double* rows = (double*)malloc(sizeof(double) * (size_t)na);
    int64_t* rowj = (int64_t*)malloc(sizeof(int64_t) * (size_t)na);
    int64_t* rown = (int64_t*)malloc(sizeof(int64_t) * (size_t)na);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < na; ++i) {
        double bv = -1.0, bs = 0.0;
        int64_t bj = -1, cnt = 0;
        for (int64_t j = 0; j < nb; ++j) {
            if (same_field && pa[i] == pb[j]) continue;
            double r = 0.0;
            if (qa[i] > 0.0 && qb[j] > 0.0) {
                double c = 0.0;
                for (int m = 0; m < M; ++m)
                    c += ((double)xa[(int64_t)m * sa + pa[i]] - ma[i]) * ((double)xb[(int64_t)m * sb + pb[j]] - mb[j]);
                r = c / sqrt(qa[i] * qb[j]);
            }
            ++cnt;
            if (fabs(r) > bv) {
                bv = fabs(r);
                bs = r;
                bj = j;
            }
        }
        rowv[i] = bv;
        rows[i] = bs;
        rowj[i] = bj;
        rown[i] = cnt;
    }
    double bv = -1.0, bs = 0.0;
    int64_t bi = -1, bj = -1, tot = 0;
    for (int64_t i = 0; i < na; ++i) {
        tot += rown[i];
        if (rowj[i] >= 0 && rowv[i] > bv) {
            bv = rowv[i];
            bs = rows[i];
            bi = i;
            bj = rowj[i];
        }
    }
    *value = bv;
    *signed_value = bs;
    *la = bi;
    *lb = bj;
    *n_evaluated = tot;
    free(ma); free(qa); free(mb); free(qb);
    free(rowv); free(rows); free(rowj); free(rown);
}

/* Threads an OpenMP parallel region of the oracle uses. */
#include <omp.h>
int orc_num_threads(void) { return omp_get_max_threads(); }
void orc_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
