// Per-point standardisation (Sec. 3.2: Pearson needs only the means and
// variances of the two points; KSG operates on the joint samples, here taken
// z-scored).
//
// stats_kernel: one thread per point, two passes over the members in member
//   order (mean, then sum of squared deviations). Reads the member-major field
//   with consecutive threads on consecutive points, so every member row is a
//   coalesced load; loads are unrolled eight deep for memory parallelism.
// stats_tile_kernel: the same two sums for long member rows (M >= 256, up to
//   64 KiB of members per 16 points) over few points (up to 32768, a focus
//   brick). A 256-thread workgroup stages all M members of 16 points in LDS
//   with one read of the field (every thread keeps 32 loads in flight), then
//   16 threads add them up in member order with the same expressions, so the
//   results equal the one-thread-per-point kernel's bit for bit.
// transpose_kernel: 64-point x 64-member LDS tile; loads member-major rows
//   coalesced, normalises, and stores point-major rows (members contiguous),
//   which is the layout both the pair kernels and the MFMA contraction read.
#include "common.h"

namespace corr {

template <typename T>
__device__ __forceinline__ float ld_val(const T* p, int64_t i);
template <>
__device__ __forceinline__ float ld_val<float>(const float* p, int64_t i) { return p[i]; }
template <>
__device__ __forceinline__ float ld_val<__half>(const __half* p, int64_t i) { return __half2float(p[i]); }

template <typename T, typename ACC>
__global__ __launch_bounds__(64) void stats_kernel(const T* __restrict__ x, int64_t stride, int M, Box box,
                                                   Stats st) {
    int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (i >= box.count()) return;
    int64_t p = box.global(i);
    // member order is kept in both sums (the unrolled loads are independent,
    // the additions stay sequential)
    ACC s = 0;
#pragma unroll 8
    for (int m = 0; m < M; ++m) s += (ACC)ld_val(x, (int64_t)m * stride + p);
    ACC mean = s / (ACC)M;
    ACC q = 0;
#pragma unroll 8
    for (int m = 0; m < M; ++m) {
        ACC d = (ACC)ld_val(x, (int64_t)m * stride + p) - mean;
        q += d * d;
    }
    bool pos = q > (ACC)0;
    st.mu32[i] = (float)mean;
    st.inv32[i] = pos ? (float)((ACC)1 / sqrt(q / (ACC)M)) : 0.0f;
    st.rs32[i] = pos ? (float)((ACC)1 / sqrt(q)) : 0.0f;
    st.sigma[i] = (float)sqrt(q / (ACC)M);
}

template <typename T>
__device__ __forceinline__ float to_f32(T v);
template <>
__device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f32<__half>(__half v) { return __half2float(v); }

// Points per workgroup of stats_tile_kernel, and the largest LDS stage it uses.
constexpr int kTilePts = 16;
constexpr int kTileLdsMax = 65536;

template <typename T, typename ACC>
__global__ __launch_bounds__(256) void stats_tile_kernel(const T* __restrict__ x, int64_t stride, int M, Box box,
                                                         Stats st) {
    extern __shared__ __attribute__((aligned(16))) unsigned char stats_lds[];
    T* tile = reinterpret_cast<T*>(stats_lds);  // [M][kTilePts]
    constexpr int RW = 256 / kTilePts;          // member rows per sweep
    constexpr int U = 32;                       // loads in flight per thread
    const int tid = threadIdx.x, tx = tid % kTilePts, ty = tid / kTilePts;
    const int64_t i = (int64_t)blockIdx.x * kTilePts + tx;
    const bool valid = i < box.count();
    const int64_t p = valid ? box.global(i) : 0;
    // stage every member of the workgroup's points (one read of the field)
    for (int m0 = ty; m0 < M; m0 += RW * U) {
        T w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int m = m0 + RW * u;
            w[u] = (valid && m < M) ? x[(int64_t)m * stride + p] : T(0.0f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int m = m0 + RW * u;
            if (m < M) tile[m * kTilePts + tx] = w[u];
        }
    }
    __syncthreads();
    if (tid >= kTilePts || !valid) return;
    // the two sums in member order; LDS reads batched ahead of the additions
    constexpr int B = 16;
    ACC s = 0;
    int m = 0;
    for (; m + B <= M; m += B) {
        float v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) v[u] = to_f32(tile[(m + u) * kTilePts + tx]);
#pragma unroll
        for (int u = 0; u < B; ++u) s += (ACC)v[u];
    }
    for (; m < M; ++m) s += (ACC)to_f32(tile[m * kTilePts + tx]);
    const ACC mean = s / (ACC)M;
    ACC q = 0;
    for (m = 0; m + B <= M; m += B) {
        float v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) v[u] = to_f32(tile[(m + u) * kTilePts + tx]);
#pragma unroll
        for (int u = 0; u < B; ++u) {
            ACC d = (ACC)v[u] - mean;
            q += d * d;
        }
    }
    for (; m < M; ++m) {
        ACC d = (ACC)to_f32(tile[m * kTilePts + tx]) - mean;
        q += d * d;
    }
    bool pos = q > (ACC)0;
    st.mu32[i] = (float)mean;
    st.inv32[i] = pos ? (float)((ACC)1 / sqrt(q / (ACC)M)) : 0.0f;
    st.rs32[i] = pos ? (float)((ACC)1 / sqrt(q)) : 0.0f;
    st.sigma[i] = (float)sqrt(q / (ACC)M);
}

template <typename T, typename ACC>
static void launch_stats_t(const T* x, int64_t stride, int M, const Box& box, Stats st, hipStream_t s) {
    const int64_t n = box.count();
    const size_t lds = (size_t)M * kTilePts * sizeof(T);
    if (M >= 256 && n <= 32768 && lds <= (size_t)kTileLdsMax) {
        // long rows over a few thousand points (a focus brick): 16 points
        // per workgroup, so every CU takes part and all loads of a point's
        // members are in flight together instead of one chain per thread
        stats_tile_kernel<T, ACC><<<dim3((unsigned)((n + kTilePts - 1) / kTilePts)), 256, lds, s>>>(x, stride, M, box,
                                                                                                    st);
    } else {
        // one thread per point in 64-thread workgroups: enough points to keep
        // every CU busy (or short rows)
        stats_kernel<T, ACC><<<dim3((unsigned)((n + 63) / 64)), 64, 0, s>>>(x, stride, M, box, st);
    }
}

template <int FMT>
struct OutT { using type = float; };
template <> struct OutT<ZF_F16> { using type = __half; };
template <> struct OutT<ZF_F16X2> { using type = __half; };
template <> struct OutT<ZF_BF16> { using type = __hip_bfloat16; };
template <> struct OutT<ZF_BF16X2> { using type = __hip_bfloat16; };

template <int FMT>
__device__ __forceinline__ void store_z(void* hi, void* lo, int64_t off, float z) {
    if constexpr (FMT == ZF_KSG || FMT == ZF_RAW || FMT == ZF_F32) {
        ((float*)hi)[off] = z;
    } else if constexpr (FMT == ZF_F16 || FMT == ZF_F16X2) {
        __half h = __float2half_rn(z);
        ((__half*)hi)[off] = h;
        if constexpr (FMT == ZF_F16X2) ((__half*)lo)[off] = __float2half_rn(z - __half2float(h));
    } else {
        __hip_bfloat16 h = __float2bfloat16(z);
        ((__hip_bfloat16*)hi)[off] = h;
        if constexpr (FMT == ZF_BF16X2) ((__hip_bfloat16*)lo)[off] = __float2bfloat16(z - __bfloat162float(h));
    }
}

template <typename T, int FMT>
__global__ __launch_bounds__(256) void transpose_kernel(const T* __restrict__ x, int64_t stride, int M, Box box,
                                                        Stats st, void* __restrict__ hi, void* __restrict__ lo,
                                                        int64_t rows_pad, int64_t ld) {
    __shared__ float tile[64][65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int m0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t cnt = box.count();
    const int64_t i = i0 + tx;
    const bool valid = i < cnt;
    int64_t p = 0;
    float mu = 0.0f, sc = 0.0f;
    if (valid) {
        p = box.global(i);
        if constexpr (FMT == ZF_RAW) {
            sc = 1.0f;
        } else {
            mu = st.mu32[i];
            sc = (FMT == ZF_KSG) ? st.inv32[i] : st.rs32[i];
        }
    }
#pragma unroll 4
    for (int r = 0; r < 16; ++r) {
        int m = m0 + ty + 4 * r;
        float v = 0.0f;
        if (valid && m < M) {
            float d = ld_val(x, (int64_t)m * stride + p) - mu;
            v = d * sc;
        }
        tile[ty + 4 * r][tx] = v;
    }
    __syncthreads();
    const int m = m0 + tx;
    if (m >= ld) return;
#pragma unroll 4
    for (int r = 0; r < 16; ++r) {
        int64_t row = i0 + ty + 4 * r;
        if (row < rows_pad) store_z<FMT>(hi, lo, row * ld + m, tile[tx][ty + 4 * r]);
    }
}

int launch_stats(const corr_field& f, const Box& box, bool acc64, Stats st, hipStream_t s) {
    int64_t n = box.count();
    if (n == 0) return CORR_OK;
    int64_t stride = f.member_stride ? f.member_stride : (int64_t)f.nx * f.ny * f.nz;
    if (f.dtype == CORR_F32) {
        if (acc64)
            launch_stats_t<float, double>((const float*)f.data, stride, f.M, box, st, s);
        else
            launch_stats_t<float, float>((const float*)f.data, stride, f.M, box, st, s);
    } else {
        if (acc64)
            launch_stats_t<__half, double>((const __half*)f.data, stride, f.M, box, st, s);
        else
            launch_stats_t<__half, float>((const __half*)f.data, stride, f.M, box, st, s);
    }
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

template <typename T>
static void launch_transpose_t(const T* x, int64_t stride, int M, const Box& box, Stats st, int fmt, void* hi,
                               void* lo, int64_t rows_pad, int64_t ld, hipStream_t s) {
    dim3 grid((unsigned)((rows_pad + 63) / 64), (unsigned)((ld + 63) / 64));
    switch (fmt) {
        case ZF_KSG: transpose_kernel<T, ZF_KSG><<<grid, 256, 0, s>>>(x, stride, M, box, st, hi, lo, rows_pad, ld); break;
        case ZF_RAW: transpose_kernel<T, ZF_RAW><<<grid, 256, 0, s>>>(x, stride, M, box, st, hi, lo, rows_pad, ld); break;
        case ZF_F32: transpose_kernel<T, ZF_F32><<<grid, 256, 0, s>>>(x, stride, M, box, st, hi, lo, rows_pad, ld); break;
        case ZF_F16: transpose_kernel<T, ZF_F16><<<grid, 256, 0, s>>>(x, stride, M, box, st, hi, lo, rows_pad, ld); break;
        case ZF_BF16: transpose_kernel<T, ZF_BF16><<<grid, 256, 0, s>>>(x, stride, M, box, st, hi, lo, rows_pad, ld); break;
        case ZF_F16X2: transpose_kernel<T, ZF_F16X2><<<grid, 256, 0, s>>>(x, stride, M, box, st, hi, lo, rows_pad, ld); break;
        case ZF_BF16X2: transpose_kernel<T, ZF_BF16X2><<<grid, 256, 0, s>>>(x, stride, M, box, st, hi, lo, rows_pad, ld); break;
    }
}

int launch_transpose(const corr_field& f, const Box& box, Stats st, int fmt, void* hi, void* lo, int64_t rows_pad,
                     int64_t ld, hipStream_t s) {
    if (rows_pad == 0 || ld == 0) return CORR_OK;
    int64_t stride = f.member_stride ? f.member_stride : (int64_t)f.nx * f.ny * f.nz;
    if (f.dtype == CORR_F32)
        launch_transpose_t((const float*)f.data, stride, f.M, box, st, fmt, hi, lo, rows_pad, ld, s);
    else
        launch_transpose_t((const __half*)f.data, stride, f.M, box, st, fmt, hi, lo, rows_pad, ld, s);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

int zfmt_for_prec(int prec) {
    switch (prec) {
        case CORR_PREC_F32: return ZF_F32;
        case CORR_PREC_F16: return ZF_F16;
        case CORR_PREC_BF16: return ZF_BF16;
        case CORR_PREC_F16X3: return ZF_F16X2;
        case CORR_PREC_BF16X3: return ZF_BF16X2;
    }
    return -1;
}

bool prec_split(int prec) { return prec == CORR_PREC_F16X3 || prec == CORR_PREC_BF16X3; }

size_t prec_elem_bytes(int prec) { return prec == CORR_PREC_F32 ? 4 : 2; }

}  // namespace corr
