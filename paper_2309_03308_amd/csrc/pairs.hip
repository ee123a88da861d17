// Pearson r for an explicit list of point pairs (Sec. 3.2).
//
// With the standardised rows Zhat[p][m] = (x_pm - mean_p) / sqrt(sum_m (x_pm -
// mean_p)^2) (point-major, members contiguous), r = sum_m Zhat[a][m] Zhat[b][m].
// A pair has no operand reuse, so this is a gather: G lanes per pair stream
// the two rows with 16-byte loads and reduce with cross-lane shuffles.
#include <algorithm>

#include "common.h"

namespace corr {

template <int PREC>
__device__ __forceinline__ float dot16(uint4 a, uint4 b) {
    // 16 bytes = 8 x 16-bit (F16/BF16) or 4 x F32
    float s = 0.0f;
    if constexpr (PREC == CORR_PREC_F32) {
        float4 x = *reinterpret_cast<float4*>(&a), y = *reinterpret_cast<float4*>(&b);
        s = x.x * y.x;
        s = fmaf(x.y, y.y, s);
        s = fmaf(x.z, y.z, s);
        s = fmaf(x.w, y.w, s);
    } else {
        const uint32_t* pa = reinterpret_cast<const uint32_t*>(&a);
        const uint32_t* pb = reinterpret_cast<const uint32_t*>(&b);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            float a0, a1, b0, b1;
            if constexpr (PREC == CORR_PREC_F16 || PREC == CORR_PREC_F16X3) {
                __half2 ha = *reinterpret_cast<const __half2*>(&pa[w]);
                __half2 hb = *reinterpret_cast<const __half2*>(&pb[w]);
                float2 fa = __half22float2(ha), fb = __half22float2(hb);
                a0 = fa.x; a1 = fa.y; b0 = fb.x; b1 = fb.y;
            } else {
                a0 = __uint_as_float(pa[w] << 16);
                a1 = __uint_as_float(pa[w] & 0xffff0000u);
                b0 = __uint_as_float(pb[w] << 16);
                b1 = __uint_as_float(pb[w] & 0xffff0000u);
            }
            s = fmaf(a0, b0, s);
            s = fmaf(a1, b1, s);
        }
    }
    return s;
}

// G lanes per pair; each lane handles 16-byte chunks c = lane_in_group, +G, ...
template <int PREC, int G>
__global__ __launch_bounds__(256) void pearson_pairs_kernel(const uint4* __restrict__ ah, const uint4* __restrict__ al,
                                                            const uint4* __restrict__ bh, const uint4* __restrict__ bl,
                                                            int64_t ld_vec, const int32_t* __restrict__ pairs, int64_t n,
                                                            float* __restrict__ r_out, Box ba, Box bb, int same_field,
                                                            unsigned long long* key) {
    constexpr bool SPLIT = (PREC == CORR_PREC_F16X3 || PREC == CORR_PREC_BF16X3);
    constexpr int PER_WAVE = 64 / G;
    const int lane = threadIdx.x & 63;
    const int g = lane / G, gl = lane % G;
    const int64_t nb = bb.count();
    unsigned long long best = 0;
    uint32_t cnt = 0;
    const int64_t waves_total = (int64_t)gridDim.x * 4;
    const int64_t wave_id = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    for (int64_t base = wave_id * PER_WAVE; base < n; base += waves_total * PER_WAVE) {
        const int64_t t = base + g;
        const bool act = t < n;
        int32_t ga = 0, gb = 0;
        int64_t la = -1, lb = -1;
        if (act) {
            ga = pairs[2 * t];
            gb = pairs[2 * t + 1];
            la = ba.local(ga);
            lb = bb.local(gb);
        }
        // rows of the standardised buffers are the boxes' local indices;
        // a pair outside its box is not evaluated (r = 0, not in the max)
        const bool ok = act && la >= 0 && lb >= 0;
        float s = 0.0f;
        if (ok) {
            const uint4* pa = ah + la * ld_vec;
            const uint4* pb = bh + lb * ld_vec;
            for (int64_t c = gl; c < ld_vec; c += G) {
                uint4 x = pa[c], y = pb[c];
                s += dot16<PREC>(x, y);
                if constexpr (SPLIT) {
                    uint4 xl = (al + la * ld_vec)[c], yl = (bl + lb * ld_vec)[c];
                    s += dot16<PREC>(x, yl) + dot16<PREC>(xl, y);
                }
            }
        }
#pragma unroll
        for (int off = G / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
        s = fminf(1.0f, fmaxf(-1.0f, s));
        if (act && gl == 0) {
            if (r_out) r_out[t] = s;
            if (key && ok && !(same_field && ga == gb)) {
                unsigned long long k = make_key(fabsf(s), (uint32_t)(la * nb + lb), s < 0.0f ? 1u : 0u);
                best = k > best ? k : best;
                ++cnt;
            }
        }
    }
    if (key) {
        // wave reduction of the best key and the count, then one atomic per wave
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            unsigned long long o = __shfl_xor(best, off, 64);
            best = o > best ? o : best;
            cnt += __shfl_xor(cnt, off, 64);
        }
        if (lane == 0 && cnt) {
            atomicMax(key, best);
            atomicAdd(key + 1, (unsigned long long)cnt);
        }
    }
}

template <int PREC>
static void launch_pp(int G, dim3 grid, const uint4* ah, const uint4* al, const uint4* bh, const uint4* bl,
                      int64_t ld_vec, const int32_t* pairs, int64_t n, float* r, Box ba, Box bb, int sf,
                      unsigned long long* key, hipStream_t s) {
    if (G == 16)
        pearson_pairs_kernel<PREC, 16><<<grid, 256, 0, s>>>(ah, al, bh, bl, ld_vec, pairs, n, r, ba, bb, sf, key);
    else
        pearson_pairs_kernel<PREC, 64><<<grid, 256, 0, s>>>(ah, al, bh, bl, ld_vec, pairs, n, r, ba, bb, sf, key);
}

int launch_pearson_pairs(int prec, const void* za_hi, const void* za_lo, const void* zb_hi, const void* zb_lo,
                         int64_t ld, const int32_t* pairs, int64_t n, float* r_out, const Box& ba, const Box& bb,
                         int same_field, unsigned long long* key, hipStream_t s) {
    if (n == 0) return CORR_OK;
    const int64_t ld_vec = ld * (int64_t)prec_elem_bytes(prec) / 16;
    const int G = ld_vec <= 32 ? 16 : 64;
    const int64_t per_block = 4 * (64 / G);
    int64_t blocks = (n + per_block - 1) / per_block;
    if (blocks > 65536) blocks = 65536;
    dim3 grid((unsigned)blocks);
    const uint4 *ah = (const uint4*)za_hi, *al = (const uint4*)za_lo, *bh = (const uint4*)zb_hi,
                *bl = (const uint4*)zb_lo;
    switch (prec) {
        case CORR_PREC_F32: launch_pp<CORR_PREC_F32>(G, grid, ah, al, bh, bl, ld_vec, pairs, n, r_out, ba, bb, same_field, key, s); break;
        case CORR_PREC_F16: launch_pp<CORR_PREC_F16>(G, grid, ah, al, bh, bl, ld_vec, pairs, n, r_out, ba, bb, same_field, key, s); break;
        case CORR_PREC_BF16: launch_pp<CORR_PREC_BF16>(G, grid, ah, al, bh, bl, ld_vec, pairs, n, r_out, ba, bb, same_field, key, s); break;
        case CORR_PREC_F16X3: launch_pp<CORR_PREC_F16X3>(G, grid, ah, al, bh, bl, ld_vec, pairs, n, r_out, ba, bb, same_field, key, s); break;
        case CORR_PREC_BF16X3: launch_pp<CORR_PREC_BF16X3>(G, grid, ah, al, bh, bl, ld_vec, pairs, n, r_out, ba, bb, same_field, key, s); break;
    }
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

}  // namespace corr

namespace corr {

// Exhaustive maxima of many small box pairs (Sec. 3, the brick-pair
// indicator): one workgroup per box pair. The A box's FP32 standardised rows
// are staged in LDS (in chunks of rows when they do not all fit); each
// thread takes (i, j) items with a stride of 256, reads B row j from global
// memory (the B box's rows stay in L1/L2 for the workgroup's lifetime) and
// keeps the largest key (|r|, smallest local index, sign). The workgroup's
// keys meet in one LDS reduction; no atomics.
__global__ __launch_bounds__(256) void box_pairs_max_kernel(const float* __restrict__ za, const float* __restrict__ zb,
                                                            int64_t ld, const Box* __restrict__ boxes, int n,
                                                            int same_field, int rows_lds,
                                                            unsigned long long* __restrict__ keys) {
    extern __shared__ __attribute__((aligned(16))) float sa[];
    __shared__ unsigned long long red[256];
    const int tid = threadIdx.x;
    const int nv = (int)(ld / 4);
    for (int t = blockIdx.x; t < n; t += gridDim.x) {
        const Box A = boxes[t], B = boxes[n + t];
        // bounds of the loops that hold barriers: wave-uniform by construction
        const int na = __builtin_amdgcn_readfirstlane((int)A.count());
        const int nb = __builtin_amdgcn_readfirstlane((int)B.count());
        unsigned long long best = 0;
        for (int a0 = 0; a0 < na; a0 += rows_lds) {
            const int rows = __builtin_amdgcn_readfirstlane(min(rows_lds, na - a0));
            __syncthreads();  // the previous chunk's readers are done
            for (int v = tid; v < rows * nv; v += 256) {
                const int i = v / nv, c = v - i * nv;
                reinterpret_cast<float4*>(sa)[v] =
                    reinterpret_cast<const float4*>(za + (int64_t)A.global(a0 + i) * ld)[c];
            }
            __syncthreads();
            for (int q = tid; q < rows * nb; q += 256) {
                const int i = q / nb, j = q - i * nb;
                const int32_t pa = A.global(a0 + i), pb = B.global(j);
                if (same_field && pa == pb) continue;
                const float4* ra = reinterpret_cast<const float4*>(sa) + (int64_t)i * nv;
                const float4* rb = reinterpret_cast<const float4*>(zb + (int64_t)pb * ld);
                float s = 0.0f;
                for (int c = 0; c < nv; ++c) {
                    const float4 x = ra[c], y = rb[c];
                    s = fmaf(x.x, y.x, s);
                    s = fmaf(x.y, y.y, s);
                    s = fmaf(x.z, y.z, s);
                    s = fmaf(x.w, y.w, s);
                }
                s = fminf(1.0f, fmaxf(-1.0f, s));
                const unsigned long long key =
                    make_key(fabsf(s), (uint32_t)(a0 + i) * (uint32_t)nb + (uint32_t)j, s < 0.0f ? 1u : 0u);
                best = key > best ? key : best;
            }
        }
        red[tid] = best;
        __syncthreads();
        for (int w = 128; w >= 1; w >>= 1) {
            if (tid < w) red[tid] = red[tid + w] > red[tid] ? red[tid + w] : red[tid];
            __syncthreads();
        }
        if (tid == 0) keys[t] = red[0];
        __syncthreads();  // red is rewritten by the next box pair
    }
}

int launch_box_pairs_max(const float* za, const float* zb, int64_t ld, const Box* boxes, int n, int same_field,
                         int max_points, unsigned long long* keys, int num_cus, hipStream_t s) {
    if (n <= 0) return CORR_OK;
    if (ld % 4) return fail(CORR_EINVAL, "box maxima: row stride must be a multiple of 4");
    // LDS budget 48 KiB for A rows
    int rows_lds = (int)std::min<int64_t>(max_points, (48 * 1024) / (ld * 4));
    if (rows_lds < 1) return fail(CORR_EUNSUPPORTED, "box maxima: member rows too long for the LDS stage");
    const size_t lds = (size_t)rows_lds * ld * 4;
    int rc = kernel_setup((const void*)box_pairs_max_kernel, lds, 256, nullptr);
    if (rc) return rc;
    const int grid = (int)std::min<int64_t>(n, (int64_t)num_cus * 8);
    box_pairs_max_kernel<<<dim3((unsigned)grid), 256, lds, s>>>(za, zb, ld, boxes, n, same_field, rows_lds, keys);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

}  // namespace corr
