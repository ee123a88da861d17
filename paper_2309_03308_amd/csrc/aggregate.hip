// Mean-tree levels (Sec. 3.3, sampling from spatial aggregates): per member,
// the mean of the field over every f x f x f block of grid points.
//
// HBM-bound streaming reduction. One wavefront owns 64 consecutive x of one
// block row (fixed block Y, Z) for a group of members: lane l reads column
// x = 64 s + l of the f rows y in [fY, fY+f) of the f planes z in [fZ, fZ+f)
// -- every load instruction is one contiguous 256-byte (FP32) run -- and sums
// them in FP64; the f lanes of one block then combine their partial sums
// with cross-lane shuffles and the first of them writes the block's mean.
// 64 is a multiple of f (f a power of two <= 64), so no block straddles two
// wavefronts. Loads go out 16 at a time before any of them is summed.
// A vector variant (below) serves f = 2 and 4 when rows are aligned.
#include "common.h"

namespace corr {

namespace {

template <typename T>
__device__ __forceinline__ double load_as_double(const T* p);
template <>
__device__ __forceinline__ double load_as_double<float>(const float* p) {
    return (double)__builtin_nontemporal_load(p);
}
template <>
__device__ __forceinline__ double load_as_double<_Float16>(const _Float16* p) {
    return (double)(float)__builtin_nontemporal_load(p);
}

template <typename T>
__device__ __forceinline__ void store_from_double(T* p, double v);
// Streaming (non-temporal) stores: the level is not read back by this kernel.
template <>
__device__ __forceinline__ void store_from_double<float>(float* p, double v) {
    __builtin_nontemporal_store((float)v, p);
}
template <>
__device__ __forceinline__ void store_from_double<_Float16>(_Float16* p, double v) {
    __builtin_nontemporal_store((_Float16)v, p);  // one rounding, FP64 -> FP16
}

// Members handled by one wavefront item: enough independent loads in flight
// for small f, one member when f^2 rows already give that.
template <int F>
constexpr int members_per_item() {
    return F * F >= 16 ? 1 : 16 / (F * F);
}

struct AggArgs {
    const void* in;
    void* out;
    int64_t in_stride, out_stride;  // elements between members
    int M, nx, ny, nz;
    int NX, NY, NZ;                 // level extent
    int nseg;                       // 64-column segments per row
    int64_t items;                  // nseg * NY * NZ * member groups
};

template <typename Tin, typename Tout, int F>
__global__ __launch_bounds__(256) void block_means_kernel(AggArgs a) {
    constexpr int MB = members_per_item<F>();
    constexpr int L = MB * F * F;  // loads per lane per item: 16 for f <= 4, f^2 beyond
    constexpr int C = 16;          // loads issued back to back before their sums
    const int lane = threadIdx.x & 63;
    const int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (item >= a.items) return;
    int64_t r = item;
    const int seg = (int)(r % a.nseg);
    r /= a.nseg;
    const int Y = (int)(r % a.NY);
    r /= a.NY;
    const int Z = (int)(r % a.NZ);
    const int m0 = (int)(r / a.NZ) * MB;

    const int x = seg * 64 + lane;
    const bool xin = x < a.nx;
    const int ylim = min(F, a.ny - F * Y);
    const int zlim = min(F, a.nz - F * Z);
    // Addresses are clamped into the grid so every lane issues every load;
    // the terms outside the block (rows, planes, members, columns past the
    // edge) are then dropped from the sums.
    const Tin* col = (const Tin*)a.in + min(x, a.nx - 1);
    const int64_t plane = (int64_t)a.nx * a.ny;

    double acc[MB];
#pragma unroll
    for (int j = 0; j < MB; ++j) acc[j] = 0.0;

    for (int c = 0; c < L; c += C) {
        float v[C];
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int t = c + i;
            const int j = MB == 1 ? 0 : t / (F * F);
            const int dz = (t % (F * F)) / F, dy = t % F;
            const int m = min(m0 + j, a.M - 1);
            const int y = min(F * Y + dy, a.ny - 1), z = min(F * Z + dz, a.nz - 1);
            v[i] = (float)load_as_double(col + (int64_t)m * a.in_stride + plane * z + (int64_t)a.nx * y);
        }
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int t = c + i;
            const int j = MB == 1 ? 0 : t / (F * F);
            const int dz = (t % (F * F)) / F, dy = t % F;
            if (dz < zlim && dy < ylim) acc[j] += (double)v[i];
        }
    }
#pragma unroll
    for (int j = 0; j < MB; ++j) acc[j] = xin ? acc[j] : 0.0;

    // combine the F lanes of each block (lanes 0..F-1 of an aligned group)
#pragma unroll
    for (int j = 0; j < MB; ++j) {
#pragma unroll
        for (int o = 1; o < F; o <<= 1) acc[j] += __shfl_xor(acc[j], o, 64);
    }

    if ((lane & (F - 1)) == 0 && xin) {
        const int X = x / F;
        const double cnt = (double)(min(F, a.nx - x) * ylim * zlim);
        Tout* out = (Tout*)a.out;
        const int64_t q = X + (int64_t)a.NX * (Y + (int64_t)a.NY * Z);
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            const int m = m0 + j;
            if (m < a.M) store_from_double(out + (int64_t)m * a.out_stride + q, acc[j] / cnt);
        }
    }
}

// f = 2 or 4 with whole blocks along x and F-element-aligned rows: lane l
// owns block X = 64 s + l and reads its f columns as one f-wide vector from
// each of the block's f x f rows, sums them in FP64 and writes the mean: no
// cross-lane step, and each wavefront's stores form one contiguous run.
template <typename Tin, typename Tout, int F>
__global__ __launch_bounds__(256) void block_means_vec_kernel(AggArgs a) {
    using V = Tin __attribute__((ext_vector_type(F)));
    constexpr int MB = F == 2 ? 2 : 1;
    constexpr int L = MB * F * F;  // vector loads per lane per item
    const int lane = threadIdx.x & 63;
    const int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (item >= a.items) return;
    int64_t r = item;
    const int seg = (int)(r % a.nseg);
    r /= a.nseg;
    const int Y = (int)(r % a.NY);
    r /= a.NY;
    const int Z = (int)(r % a.NZ);
    const int m0 = (int)(r / a.NZ) * MB;

    const int X = seg * 64 + lane;
    const bool xin = X < a.NX;
    const int ylim = min(F, a.ny - F * Y);
    const int zlim = min(F, a.nz - F * Z);
    const Tin* col = (const Tin*)a.in + (int64_t)F * min(X, a.NX - 1);
    const int64_t plane = (int64_t)a.nx * a.ny;

    V v[L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
        const int j = t / (F * F), dz = (t % (F * F)) / F, dy = t % F;
        const int m = min(m0 + j, a.M - 1);
        const int y = min(F * Y + dy, a.ny - 1), z = min(F * Z + dz, a.nz - 1);
        v[t] = __builtin_nontemporal_load((const V*)(col + (int64_t)m * a.in_stride + plane * z + (int64_t)a.nx * y));
    }
    if (!xin) return;
    const double cnt = (double)(F * ylim * zlim);
    Tout* out = (Tout*)a.out;
    const int64_t q = X + (int64_t)a.NX * (Y + (int64_t)a.NY * Z);
#pragma unroll
    for (int j = 0; j < MB; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int t = j * F * F; t < (j + 1) * F * F; ++t) {
            const int dz = (t % (F * F)) / F, dy = t % F;
            if (dz < zlim && dy < ylim) {
#pragma unroll
                for (int e = 0; e < F; ++e) acc += (double)(float)v[t][e];
            }
        }
        if (m0 + j < a.M) store_from_double(out + (int64_t)(m0 + j) * a.out_stride + q, acc / cnt);
    }
}

template <typename Tin, typename Tout, int F>
bool vec_ok(const AggArgs& a) {
    if constexpr (F != 2 && F != 4) {
        return false;
    } else {
        return a.nx % F == 0 && a.in_stride % F == 0 && ((uintptr_t)a.in % (F * sizeof(Tin))) == 0;
    }
}

template <typename Tin, typename Tout, int F>
int launch_f(AggArgs a, hipStream_t s) {
    if constexpr (F == 2 || F == 4) {
        if (vec_ok<Tin, Tout, F>(a)) {
            constexpr int MB = F == 2 ? 2 : 1;
            a.nseg = (a.NX + 63) / 64;
            a.items = (int64_t)a.nseg * a.NY * a.NZ * ((a.M + MB - 1) / MB);
            const int64_t wgs = (a.items + 3) / 4;
            if (wgs > 0x7fffffffLL) return fail(CORR_EUNSUPPORTED, "block means: grid too large");
            block_means_vec_kernel<Tin, Tout, F><<<dim3((unsigned)wgs), 256, 0, s>>>(a);
            CORR_LAUNCH_CHECK();
            return CORR_OK;
        }
    }
    constexpr int MB = members_per_item<F>();
    a.items = (int64_t)a.nseg * a.NY * a.NZ * ((a.M + MB - 1) / MB);
    const int64_t wgs = (a.items + 3) / 4;
    if (wgs > 0x7fffffffLL) return fail(CORR_EUNSUPPORTED, "block means: grid too large");
    block_means_kernel<Tin, Tout, F><<<dim3((unsigned)wgs), 256, 0, s>>>(a);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

template <typename Tin, typename Tout>
int launch_io(AggArgs a, int f, hipStream_t s) {
    switch (f) {
        case 1: return launch_f<Tin, Tout, 1>(a, s);
        case 2: return launch_f<Tin, Tout, 2>(a, s);
        case 4: return launch_f<Tin, Tout, 4>(a, s);
        case 8: return launch_f<Tin, Tout, 8>(a, s);
        case 16: return launch_f<Tin, Tout, 16>(a, s);
        case 32: return launch_f<Tin, Tout, 32>(a, s);
        case 64: return launch_f<Tin, Tout, 64>(a, s);
        default: return fail(CORR_EINVAL, "f must be a power of two in [1, 64]");
    }
}

}  // namespace

int launch_block_means(const corr_field& A, int f, int out_dtype, void* out, int64_t out_stride, hipStream_t s) {
    AggArgs a{};
    a.in = A.data;
    a.out = out;
    a.M = A.M;
    a.nx = A.nx;
    a.ny = A.ny;
    a.nz = A.nz;
    a.in_stride = A.member_stride ? A.member_stride : (int64_t)A.nx * A.ny * A.nz;
    a.NX = (A.nx + f - 1) / f;
    a.NY = (A.ny + f - 1) / f;
    a.NZ = (A.nz + f - 1) / f;
    a.out_stride = out_stride ? out_stride : (int64_t)a.NX * a.NY * a.NZ;
    a.nseg = (A.nx + 63) / 64;  // the vector kernel recomputes it over blocks
    const bool in16 = A.dtype == CORR_F16, out16 = out_dtype == CORR_F16;
    if (!in16 && !out16) return launch_io<float, float>(a, f, s);
    if (!in16 && out16) return launch_io<float, _Float16>(a, f, s);
    if (in16 && !out16) return launch_io<_Float16, float>(a, f, s);
    return launch_io<_Float16, _Float16>(a, f, s);
}

}  // namespace corr
