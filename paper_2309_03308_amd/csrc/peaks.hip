// On-device peak probes (measurement helpers; declared in corr_peaks.h).
//
// Each kernel does a fixed amount of one kind of work per thread with no
// data-dependent addressing, and writes one word per thread so that the
// compiler keeps the work. The host side validates the arguments and
// launches; the caller times the launch.
#include "common.h"

#include "../../include/corr_peaks.h"

namespace corr {
namespace {

constexpr int PT = 256;            // threads per workgroup
constexpr int LDS_WORDS = 4096;    // 16-byte words: 64 KiB per workgroup
constexpr int LDS_UNROLL = 8;

__global__ __launch_bounds__(PT) void peak_lds_kernel(int iters, unsigned int* out) {
    __shared__ uint4 buf[LDS_WORDS];
    const int t = threadIdx.x;
    for (int i = t; i < LDS_WORDS; i += PT) buf[i] = make_uint4(i, 3u * i + 1u, 5u * i + 2u, 7u * i + 3u);
    __syncthreads();
    unsigned int a0 = 0, a1 = 0;
    for (int it = 0; it < iters; ++it) {
        // the offset moves every iteration, so no read is loop-invariant;
        // a wave's 64 lanes read 64 consecutive words
        const int base = t + (it & 1) * (LDS_WORDS / 2);
#pragma unroll
        for (int u = 0; u < LDS_UNROLL; ++u) {
            // three-input adds keep the VALU work at two instructions per
            // 16-byte read, well below what the LDS can deliver
            const uint4 v = buf[(base + u * PT) & (LDS_WORDS - 1)];
            a0 = a0 + v.x + v.y;
            a1 = a1 + v.z + v.w;
        }
    }
    out[(size_t)blockIdx.x * PT + t] = a0 ^ a1;
}

typedef _Float16 pk_h8 __attribute__((ext_vector_type(8)));
typedef float pk_f16 __attribute__((ext_vector_type(16)));

// A 32-bit mixing hash (multiply / xor-shift rounds) for the probe's operands.
__device__ __forceinline__ unsigned int pk_mix(unsigned int h) {
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    return h;
}

__global__ __launch_bounds__(PT) void peak_mfma_f16_kernel(int iters, int random_operands, float* out) {
    const int t = threadIdx.x;
    pk_h8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        if (random_operands) {
            const unsigned int h = pk_mix((blockIdx.x * PT + t) * 16u + 2u * e);
            const unsigned int k = pk_mix((blockIdx.x * PT + t) * 16u + 2u * e + 1u);
            a[e] = (_Float16)((float)(h & 0xffffu) * (1.0f / 32768.0f) - 1.0f);
            b[e] = (_Float16)((float)(k & 0xffffu) * (1.0f / 32768.0f) - 1.0f);
        } else {
            a[e] = (_Float16)(0.001f * (float)((t + e) & 7));
            b[e] = (_Float16)(0.002f * (float)((t * 3 + e) & 7));
        }
    }
    pk_f16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
    for (int it = 0; it < iters; ++it) {
        c0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c3, 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) s += c0[r] + c1[r] + c2[r] + c3[r];
    out[(size_t)blockIdx.x * PT + t] = s;
}

constexpr int F32_CHAINS = 16;
constexpr int F64_CHAINS = 8;

__global__ __launch_bounds__(PT) void peak_valu_f32_kernel(int iters, float* out) {
    float x[F32_CHAINS];
#pragma unroll
    for (int i = 0; i < F32_CHAINS; ++i) x[i] = 1e-3f * (float)threadIdx.x + (float)i;
    const float a = 0.999f, b = 1e-3f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < F32_CHAINS; ++i) x[i] = fmaf(x[i], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < F32_CHAINS; ++i) s += x[i];
    out[(size_t)blockIdx.x * PT + threadIdx.x] = s;
}

__global__ __launch_bounds__(PT) void peak_valu_med3_kernel(int iters, float* out) {
    float x[F32_CHAINS];
#pragma unroll
    for (int i = 0; i < F32_CHAINS; ++i) x[i] = (float)(i + (int)threadIdx.x);
    const float hi = 1e6f + (float)threadIdx.x;
    for (int it = 0; it < iters; ++it) {
        const float lo = (float)it;  // moves, so no chain settles into a constant
#pragma unroll
        for (int i = 0; i < F32_CHAINS; ++i) x[i] = __builtin_amdgcn_fmed3f(x[i], lo, hi);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < F32_CHAINS; ++i) s += x[i];
    out[(size_t)blockIdx.x * PT + threadIdx.x] = s;
}

__global__ __launch_bounds__(PT) void peak_valu_f64_kernel(int iters, double* out) {
    double x[F64_CHAINS];
#pragma unroll
    for (int i = 0; i < F64_CHAINS; ++i) x[i] = 1e-3 * (double)threadIdx.x + (double)i;
    const double a = 0.999, b = 1e-3;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < F64_CHAINS; ++i) x[i] = fma(x[i], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < F64_CHAINS; ++i) s += x[i];
    out[(size_t)blockIdx.x * PT + threadIdx.x] = s;
}

constexpr int HBM_INFLIGHT = 8;
typedef unsigned int hb_u4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(PT) void peak_hbm_read_kernel(const uint4* p, size_t n, unsigned int* out) {
    unsigned int a0 = 0, a1 = 0;
    const size_t stride = (size_t)gridDim.x * PT;
    size_t i = (size_t)blockIdx.x * PT + threadIdx.x;
    // HBM_INFLIGHT words in flight per thread (non-temporal: read once), then
    // the remainder; every index is below n
    for (; i + (HBM_INFLIGHT - 1) * stride < n; i += HBM_INFLIGHT * stride) {
        hb_u4 v[HBM_INFLIGHT];
#pragma unroll
        for (int u = 0; u < HBM_INFLIGHT; ++u)
            v[u] = __builtin_nontemporal_load(reinterpret_cast<const hb_u4*>(p) + i + u * stride);
#pragma unroll
        for (int u = 0; u < HBM_INFLIGHT; ++u) {
            a0 = a0 + v[u].x + v[u].y;
            a1 = a1 + v[u].z + v[u].w;
        }
    }
    for (; i < n; i += stride) {
        const uint4 v = p[i];
        a0 = a0 + v.x + v.y;
        a1 = a1 + v.z + v.w;
    }
    out[(size_t)blockIdx.x * PT + threadIdx.x] = a0 ^ a1;
}

int check_args(int n_blocks, int iters, const void* out) {
    if (n_blocks < 1 || iters < 1 || out == nullptr) return fail(CORR_EINVAL, "peak probe: n_blocks and iters must be >= 1, out non-null");
    return CORR_OK;
}

}  // namespace
}  // namespace corr

using namespace corr;

extern "C" {

int corr_peak_lds(int n_blocks, int iters, unsigned int* out, void* stream) {
    if (int rc = check_args(n_blocks, iters, out)) return rc;
    peak_lds_kernel<<<n_blocks, PT, 0, (hipStream_t)stream>>>(iters, out);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

int corr_peak_mfma_f16(int n_blocks, int iters, int random_operands, float* out, void* stream) {
    if (int rc = check_args(n_blocks, iters, out)) return rc;
    peak_mfma_f16_kernel<<<n_blocks, PT, 0, (hipStream_t)stream>>>(iters, random_operands ? 1 : 0, out);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

int corr_peak_valu_f32(int n_blocks, int iters, float* out, void* stream) {
    if (int rc = check_args(n_blocks, iters, out)) return rc;
    peak_valu_f32_kernel<<<n_blocks, PT, 0, (hipStream_t)stream>>>(iters, out);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

int corr_peak_valu_med3(int n_blocks, int iters, float* out, void* stream) {
    if (int rc = check_args(n_blocks, iters, out)) return rc;
    peak_valu_med3_kernel<<<n_blocks, PT, 0, (hipStream_t)stream>>>(iters, out);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

int corr_peak_valu_f64(int n_blocks, int iters, double* out, void* stream) {
    if (int rc = check_args(n_blocks, iters, out)) return rc;
    peak_valu_f64_kernel<<<n_blocks, PT, 0, (hipStream_t)stream>>>(iters, out);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

int corr_peak_hbm_read(const void* buf, size_t bytes, int n_blocks, unsigned int* out, void* stream) {
    if (int rc = check_args(n_blocks, 1, out)) return rc;
    if (buf == nullptr || ((uintptr_t)buf & 15) || (bytes & 15))
        return fail(CORR_EINVAL, "peak probe: buffer must be non-null, 16-byte aligned, a multiple of 16 bytes");
    peak_hbm_read_kernel<<<n_blocks, PT, 0, (hipStream_t)stream>>>((const uint4*)buf, bytes / 16, out);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

}  // extern "C"
