/* Drives every function of the C oracle on a small field (one constant
 * point, ragged sizes) so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer can check its memory accesses and arithmetic.
 * Also checks a few invariants; prints "ok" when all hold. Test
 * infrastructure only. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

double orc_digamma_int(int n);
void orc_stats(const float* x, int64_t stride, int M, const int32_t* pts, int64_t npts, double* mu, double* s2,
               float* mu32, float* inv32);
void orc_ksg_inputs(const float* x, int64_t stride, int M, const int32_t* pts, int64_t npts, float* z);
void orc_pearson_pairs(const float* xa, int64_t sa, const float* xb, int64_t sb, int M, const int32_t* pairs,
                       int64_t n, double* r);
void orc_ksg_pairs(const float* za, const float* zb, int64_t ldz, int M, int k, const int32_t* pairs, int64_t n,
                   const uint8_t* zero_a, const uint8_t* zero_b, double* mi, int32_t* counts);
int64_t orc_argmax_pairs(const double* values, const int32_t* la, const int32_t* lb, int64_t n, int use_abs);
void orc_pearson_region_max(const float* xa, int64_t sa, const int32_t* pa, int64_t na, const float* xb,
                            int64_t sb, const int32_t* pb, int64_t nb, int M, int same_field, double* value,
                            double* signed_value, int64_t* la, int64_t* lb, int64_t* n_evaluated);

#define M 23
#define P 37

static uint64_t st = 0x9e3779b97f4a7c15ull;
static float urand(void)
{
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    return (float)((st >> 40) & 0xffffff) / 16777216.0f - 0.5f;
}

int main(void)
{
    float* x = malloc(sizeof(float) * M * P);
    for (int m = 0; m < M; ++m)
        for (int p = 0; p < P; ++p) x[m * P + p] = (p == 5) ? 2.0f : urand() + 0.3f * (float)m / M;
    int32_t pts[P];
    for (int p = 0; p < P; ++p) pts[p] = p;
    double mu[P], s2[P];
    float mu32[P], inv32[P];
    orc_stats(x, P, M, pts, P, mu, s2, mu32, inv32);
    if (inv32[5] != 0.0f) { printf("constant point has nonzero inv32\n"); return 1; }
    float* z = malloc(sizeof(float) * M * P);
    orc_ksg_inputs(x, P, M, pts, P, z);
    int32_t pairs[2 * 60];
    for (int t = 0; t < 60; ++t) { pairs[2 * t] = t % P; pairs[2 * t + 1] = (7 * t + 3) % P; }
    pairs[0] = 4; pairs[1] = 4;   /* a point with itself */
    pairs[2] = 5; pairs[3] = 9;   /* the constant point */
    double r[60];
    orc_pearson_pairs(x, P, x, P, M, pairs, 60, r);
    for (int t = 0; t < 60; ++t)
        if (!(fabs(r[t]) <= 1.0 + 1e-12)) { printf("|r| > 1 at %d\n", t); return 1; }
    if (fabs(r[0] - 1.0) > 1e-12 || r[1] != 0.0) { printf("r(a,a) or constant point wrong\n"); return 1; }
    uint8_t zero[P] = {0};
    zero[5] = 1;
    double mi[60];
    int32_t* cnt = malloc(sizeof(int32_t) * 60 * 2 * M);
    orc_ksg_pairs(z, z, M, M, 4, pairs, 60, zero, zero, mi, cnt);
    if (mi[1] != 0.0) { printf("constant point MI not 0\n"); return 1; }
    for (int i = 0; i < 60 * 2 * M; ++i)
        if (cnt[i] < 0 || cnt[i] > M - 1) { printf("count out of range\n"); return 1; }
    int32_t la[60], lb[60];
    for (int t = 0; t < 60; ++t) { la[t] = pairs[2 * t]; lb[t] = pairs[2 * t + 1]; }
    int64_t b = orc_argmax_pairs(mi, la, lb, 60, 0);
    if (b < 0 || b >= 60) { printf("argmax out of range\n"); return 1; }
    double v, sv;
    int64_t ia, ib, ne;
    orc_pearson_region_max(x, P, pts, 17, x, P, pts + 10, 27, M, 1, &v, &sv, &ia, &ib, &ne);
    if (ne != 17 * 27 - 7 || !(v >= 0.0 && v <= 1.0 + 1e-12)) { printf("region max wrong\n"); return 1; }
    if (fabs(orc_digamma_int(1) + 0.5772156649015329) > 1e-15) { printf("psi(1) wrong\n"); return 1; }
    free(x); free(z); free(cnt);
    printf("ok\n");
    return 0;
}
