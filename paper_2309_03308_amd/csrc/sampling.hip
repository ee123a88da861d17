// Random and quasi-random sampling of brick-pair maxima (Sec. 3.1) and the
// choice between BOS, random sampling and exhaustive computation (Sec. 5,
// sampling strategy).
//
// A sample of a brick pair is a cell of its 6-D box (x, y, z in brick A, then
// in brick B): u in [0, 1)^6 maps to c_j = min(floor(u_j d_j), d_j - 1).
//   uniform: u_j = the 53-bit uniform of Philox4x64-10 word 0 at counter
//            (pair, 5, s, j), key (seed, 0x636F7272);
//   Halton:  u_j = frac(h_{b_j}(s + 1) + c_j), bases 2, 3, 5, 7, 11, 13;
//            h_b(n) = (base-b digits of n mirrored) / b^digits, one FP64
//            division of exact integers;
//   plastic: u_j = frac(c_j + (s + 1) alpha_j), alpha_1 = 1 / phi,
//            alpha_{j+1} = alpha_j / phi, phi the real root above 1 of
//            x^7 = x + 1 (the six-dimensional plastic constant);
//   c_j = the uniform of counter (pair, 6, 0, j): one Cranley-Patterson shift
//   per pair and seed.
// Every step is a correctly rounded FP64 operation (the unit is compiled
// without contraction), so a cell is reproducible on any IEEE machine.
//
// corr_sampled_max evaluates all samples of all pairs with the pair-list
// kernels and reduces each pair's samples with one wave (earliest maximum;
// within one field a sample of a point with itself is skipped, as in the
// exhaustive maxima).
#include "common.h"

namespace corr {

namespace {

constexpr double PHI6 = 1.1127756842787055;  // correctly rounded
constexpr uint64_t S_SAMPLE = 5, S_SHIFT = 6;

struct PairBoxes {
    Box a, b;
};

__device__ __forceinline__ double frac01(double x) { return x - floor(x); }

__device__ double radical_inverse(uint32_t n, uint32_t b) {
    uint64_t num = 0, den = 1;
    while (n > 0) {
        const uint32_t q = n / b;
        num = num * b + (n - q * b);
        den *= b;
        n = q;
    }
    return (double)num / (double)den;
}

__global__ __launch_bounds__(256) void sample_pairs_kernel(const PairBoxes* __restrict__ boxes, int32_t n_pairs,
                                                           int32_t n, int sampler, uint64_t seed,
                                                           int32_t* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_pairs * n) return;
    const int32_t p = (int32_t)(t / n), s = (int32_t)(t - (int64_t)p * n);
    const PairBoxes pb = boxes[p];
    const int dims[6] = {pb.a.dx, pb.a.dy, pb.a.dz, pb.b.dx, pb.b.dy, pb.b.dz};
    const uint32_t bases[6] = {2, 3, 5, 7, 11, 13};
    int c[6];
    double alpha = 1.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double u;
        if (sampler == CORR_SAMPLE_UNIFORM) {
            u = ph_uniform(seed, (uint64_t)p, S_SAMPLE, (uint64_t)s, (uint64_t)j);
        } else {
            const double shift = ph_uniform(seed, (uint64_t)p, S_SHIFT, 0, (uint64_t)j);
            if (sampler == CORR_SAMPLE_HALTON) {
                u = frac01(radical_inverse((uint32_t)s + 1u, bases[j]) + shift);
            } else {
                alpha = alpha / PHI6;
                u = frac01(shift + (double)(s + 1) * alpha);
            }
        }
        const int v = (int)floor(u * (double)dims[j]);
        c[j] = v < dims[j] - 1 ? v : dims[j] - 1;
    }
    const int32_t pa = (pb.a.x0 + c[0]) + pb.a.nx * ((pb.a.y0 + c[1]) + pb.a.ny * (pb.a.z0 + c[2]));
    const int32_t pbb = (pb.b.x0 + c[3]) + pb.b.nx * ((pb.b.y0 + c[4]) + pb.b.ny * (pb.b.z0 + c[5]));
    out[2 * t] = pa;
    out[2 * t + 1] = pbb;
}

// One wave per region pair: the earliest maximum of its n samples.
__global__ __launch_bounds__(256) void segment_max_kernel(const float* __restrict__ values,
                                                          const int32_t* __restrict__ pairs, int32_t n_pairs,
                                                          int32_t n, int use_abs, int same_field,
                                                          corr_max* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (p >= n_pairs) return;
    const float* v = values + p * n;
    const int32_t* pp = pairs + 2 * p * n;
    unsigned long long best = 0;
    int counted = 0;
    for (int s = lane; s < n; s += 64) {
        if (same_field && pp[2 * s] == pp[2 * s + 1]) continue;  // a point with itself is no sample
        const float x = v[s];
        const float o = use_abs ? fabsf(x) : x;
        const unsigned long long key = ((unsigned long long)order_bits(o) << 32) | (0xffffffffu - (uint32_t)s);
        best = key > best ? key : best;
        ++counted;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(best, off, 64);
        best = o > best ? o : best;
        counted += __shfl_xor(counted, off, 64);
    }
    if (lane == 0) {
        corr_max r;
        if (counted == 0) {
            r.value = r.signed_value = 0.0f;
            r.pa = r.pb = -1;
        } else {
            const int32_t s = (int32_t)(0xffffffffu - (uint32_t)(best & 0xffffffffu));
            r.value = from_order_bits((uint32_t)(best >> 32));
            r.signed_value = v[s];
            r.pa = pp[2 * s];
            r.pb = pp[2 * s + 1];
        }
        r.n_evaluated = counted;
        out[p] = r;
    }
}

}  // namespace

int launch_sample_pairs(const void* boxes, int32_t n_pairs, int32_t n, int sampler, uint64_t seed, int32_t* out,
                        hipStream_t s) {
    const int64_t total = (int64_t)n_pairs * n;
    if (total == 0) return CORR_OK;
    sample_pairs_kernel<<<dim3((unsigned)((total + 255) / 256)), 256, 0, s>>>((const PairBoxes*)boxes, n_pairs, n,
                                                                              sampler, seed, out);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

int launch_segment_max(const float* values, const int32_t* pairs, int32_t n_pairs, int32_t n, int use_abs,
                       int same_field, corr_max* out, hipStream_t s) {
    if (n_pairs == 0) return CORR_OK;
    segment_max_kernel<<<dim3((unsigned)((n_pairs + 3) / 4)), 256, 0, s>>>(values, pairs, n_pairs, n, use_abs,
                                                                          same_field, out);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

size_t sample_boxes_bytes(int32_t n_pairs) { return sizeof(PairBoxes) * (size_t)n_pairs; }

void fill_sample_boxes(void* host, const corr_region* regions, const int32_t* region_pairs, int32_t n_pairs,
                       const corr_field& A, const corr_field& B) {
    PairBoxes* pb = (PairBoxes*)host;
    for (int32_t p = 0; p < n_pairs; ++p) {
        const corr_region& ra = regions[region_pairs[2 * p]];
        const corr_region& rb = regions[region_pairs[2 * p + 1]];
        pb[p].a = Box{ra.x0, ra.y0, ra.z0, ra.dx, ra.dy, ra.dz, A.nx, A.ny};
        pb[p].b = Box{rb.x0, rb.y0, rb.z0, rb.dx, rb.dy, rb.dz, B.nx, B.ny};
    }
}

}  // namespace corr
