// Learned BOS proposal: a small MLP (forward, backward, AdamW) and the
// region-pair inputs it reads (self-similarity hot spots and their cross
// correlations). Weights are BF16-rounded copies of FP32 master weights;
// every product of the forward and backward passes runs on the matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation), one wave per 32 x 32 output
// block. FP32 operands (activations, gradients) enter as a BF16 hi part and
// a BF16 lo part (x = hi + lo to about 2^-16 relative), and the products
// hi.hi + hi.lo + lo.hi are accumulated, so the results carry FP32-level
// accuracy; the BF16 weights are exact and need no lo part. No sum uses
// floating-point atomics, so two runs are bitwise identical.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mlp.h"
#include "common.h"

namespace corr {

__device__ __forceinline__ float bf(const __hip_bfloat16 v) { return __bfloat162float(v); }
__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

__global__ void to_bf16_kernel(const float* __restrict__ p, __hip_bfloat16* __restrict__ q, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) q[i] = __float2bfloat16(p[i]);
}

typedef __bf16 mlp_b8 __attribute__((ext_vector_type(8)));
typedef float mlp_f16 __attribute__((ext_vector_type(16)));

// A matrix operand: element (i, j) at p[i * s0 + j * s1], FP32 or BF16.
struct MatRef {
    const void* p;
    int bf16;
    int64_t s0, s1;
};

__device__ __forceinline__ float mat_get(const MatRef& m, int64_t i, int64_t j) {
    const int64_t o = i * m.s0 + j * m.s1;
    return m.bf16 ? __bfloat162float(reinterpret_cast<const __hip_bfloat16*>(m.p)[o])
                  : reinterpret_cast<const float*>(m.p)[o];
}

enum MlpEpilogue { EP_BIAS = 0, EP_DSILU = 1, EP_PLAIN = 2 };

// C[i][j] = sum_k A(i, k) B(k, j) for i < R, j < N, one wave per 32 x 32
// block (four per workgroup). Per K-step of 16, lane (l, h) (l = lane % 32,
// h = lane / 32) holds A(row l, k = 8h .. 8h+7) and B(k = 8h .. 8h+7, col l);
// accumulator register r of lane (l, h) is C(8 (r / 4) + 4 h + r % 4, l).
// Epilogues: EP_BIAS: Z = C + bias[j] (BF16, may be NULL), Aout = silu(Z)
// when Aout != NULL; EP_DSILU: C * silu'(Zp[i][j]); EP_PLAIN: C.
__global__ __launch_bounds__(256) void mlp_mfma_gemm_kernel(MatRef A, MatRef B, int R, int N, int K, int ep,
                                                            const __hip_bfloat16* __restrict__ bias,
                                                            const float* __restrict__ Zp, float* __restrict__ C,
                                                            float* __restrict__ Aout) {
    const int lane = threadIdx.x & 63, l = lane & 31, h = lane >> 5;
    const int nbn = (N + 31) / 32, nbm = (R + 31) / 32;
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= nbm * nbn) return;  // wave-uniform; the kernel has no barriers
    const int i0 = (w / nbn) * 32, j0 = (w % nbn) * 32;
    const int row = i0 + l, col = j0 + l;
    mlp_f16 acc = {};
    for (int k0 = 0; k0 < K; k0 += 16) {
        mlp_b8 ah, al, bh, bl;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + 8 * h + e;
            const float av = (row < R && k < K) ? mat_get(A, row, k) : 0.0f;
            const float bv = (col < N && k < K) ? mat_get(B, k, col) : 0.0f;
            ah[e] = (__bf16)av;
            al[e] = (__bf16)(av - (float)ah[e]);
            bh[e] = (__bf16)bv;
            bl[e] = (__bf16)(bv - (float)bh[e]);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
        if (!A.bf16) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
        if (!B.bf16) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = i0 + 8 * (r >> 2) + 4 * h + (r & 3);
        if (i >= R || col >= N) continue;
        const int64_t o = (int64_t)i * N + col;
        float v = acc[r];
        if (ep == EP_BIAS) {
            if (bias) v += bf(bias[col]);
            C[o] = v;
            if (Aout) Aout[o] = silu_f(v);
        } else if (ep == EP_DSILU) {
            C[o] = v * dsilu_f(Zp[o]);
        } else {
            C[o] = v;
        }
    }
}

// gb[n] = sum_b dZ[b][n], in batch order
__global__ void col_sum_kernel(const float* __restrict__ dZ, int B, int N, float* __restrict__ gb) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float g = 0.0f;
    for (int b = 0; b < B; ++b) g += dZ[(int64_t)b * N + n];
    gb[n] = g;
}

static int mlp_gemm(MatRef A, MatRef B, int R, int N, int K, int ep, const __hip_bfloat16* bias, const float* Zp,
                    float* C, float* Aout, hipStream_t s) {
    const int blocks = ((R + 31) / 32) * ((N + 31) / 32);
    mlp_mfma_gemm_kernel<<<dim3((unsigned)((blocks + 3) / 4)), 256, 0, s>>>(A, B, R, N, K, ep, bias, Zp, C, Aout);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

// dY = 2 w (Y - T) / (B n_out); per-row loss partial in a fixed order.
__global__ void out_grad_kernel(const float* __restrict__ Y, const float* __restrict__ T, const float* __restrict__ w,
                                int B, int n_out, float* __restrict__ dY, float* __restrict__ part) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const float scale = 2.0f / ((float)B * (float)n_out);
    float l = 0.0f;
    for (int o = 0; o < n_out; ++o) {
        const float d = Y[(int64_t)b * n_out + o] - T[(int64_t)b * n_out + o];
        const float wo = w ? w[o] : 1.0f;
        dY[(int64_t)b * n_out + o] = scale * wo * d;
        l = fmaf(wo * d, d, l);
    }
    part[b] = l;
}

// loss = sum(part) / (B n_out), fixed tree order (one block)
__global__ void loss_reduce_kernel(const float* __restrict__ part, int B, int n_out, float* __restrict__ loss) {
    __shared__ float s[256];
    float v = 0.0f;
    for (int b = threadIdx.x; b < B; b += 256) v += part[b];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int st = 128; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = s[0] / ((float)B * (float)n_out);
}

__global__ void adamw_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                             float* __restrict__ v, int64_t n, float lr, float wd, float bc1, float bc2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / bc1, vh = vi / bc2;
    p[i] = p[i] - lr * (mh / (sqrtf(vh) + 1e-8f) + wd * p[i]);
}

// ---------------------------------------------------------------- proposal inputs
template <typename T>
__device__ __forceinline__ float ldv(const T* p, int64_t i);
template <>
__device__ __forceinline__ float ldv<float>(const float* p, int64_t i) { return p[i]; }
template <>
__device__ __forceinline__ float ldv<__half>(const __half* p, int64_t i) { return __half2float(p[i]); }

// s(p): one thread per grid point; member rows of the member-major field are
// read coalesced (neighbours at +-D along x share cache lines).
template <typename T>
__global__ __launch_bounds__(256) void self_sim_kernel(const T* __restrict__ x, int64_t stride, int M, int nx, int ny,
                                                       int nz, int D, const float* __restrict__ mu,
                                                       const float* __restrict__ rs, float* __restrict__ sim) {
    const int64_t P = (int64_t)nx * ny * nz;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const int px = (int)(p % nx), py = (int)((p / nx) % ny), pz = (int)(p / ((int64_t)nx * ny));
    int64_t q[6];
    bool ok[6];
    ok[0] = px + D < nx;  q[0] = p + D;
    ok[1] = px - D >= 0;  q[1] = p - D;
    ok[2] = py + D < ny;  q[2] = p + (int64_t)D * nx;
    ok[3] = py - D >= 0;  q[3] = p - (int64_t)D * nx;
    ok[4] = pz + D < nz;  q[4] = p + (int64_t)D * nx * ny;
    ok[5] = pz - D >= 0;  q[5] = p - (int64_t)D * nx * ny;
    float mq[6], acc[6];
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        if (!ok[t]) q[t] = p;
        mq[t] = mu[q[t]];
        acc[t] = 0.0f;
    }
    const float mp = mu[p];
    for (int m = 0; m < M; ++m) {
        const T* row = x + (int64_t)m * stride;
        const float dp = ldv(row, p) - mp;
#pragma unroll
        for (int t = 0; t < 6; ++t) acc[t] = fmaf(dp, ldv(row, q[t]) - mq[t], acc[t]);
    }
    float sum = 0.0f;
    int cnt = 0;
    const float rp = rs[p];
#pragma unroll
    for (int t = 0; t < 6; ++t)
        if (ok[t]) {
            sum += acc[t] * rp * rs[q[t]];
            ++cnt;
        }
    sim[p] = cnt ? sum / (float)cnt : 0.0f;
}

// One block per region: n_hot suppressed argmax rounds over s, then the
// region's row (picks, mean of mu, mean of sigma, centre).
__global__ __launch_bounds__(256) void hot_spot_kernel(const float* __restrict__ sim, const Box* __restrict__ boxes,
                                                       int n_hot, int r_nms, int nz, const float* __restrict__ mu,
                                                       const float* __restrict__ sigma, int32_t* __restrict__ hot,
                                                       float* __restrict__ rows) {
    __shared__ float bv[256];
    __shared__ int bi[256];
    __shared__ int picks[8][3];
    __shared__ float red[512];
    const int r = blockIdx.x;
    const Box bx = boxes[r];
    const int cnt = (int)bx.count();
    const int F = 4 * n_hot + 5;
    float* row = rows + (int64_t)r * F;
    int prev = 0;
    for (int h = 0; h < n_hot; ++h) {
        float best = -INFINITY;
        int besti = 0x7fffffff;
        for (int i = threadIdx.x; i < cnt; i += 256) {
            const int lx = i % bx.dx, ly = (i / bx.dx) % bx.dy, lz = i / (bx.dx * bx.dy);
            bool ok = true;
            for (int g = 0; g < h; ++g) {
                const int dx = abs(lx - picks[g][0]), dy = abs(ly - picks[g][1]), dz = abs(lz - picks[g][2]);
                if (max(dx, max(dy, dz)) <= r_nms) ok = false;
            }
            if (ok) {
                const float v = sim[bx.global(i)];
                if (v > best) {  // ascending i: this thread's first maximum
                    best = v;
                    besti = i;
                }
            }
        }
        bv[threadIdx.x] = best;
        bi[threadIdx.x] = besti;
        __syncthreads();
        for (int st = 128; st >= 1; st >>= 1) {
            if ((int)threadIdx.x < st) {
                const float o = bv[threadIdx.x + st];
                const int oi = bi[threadIdx.x + st];
                if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                    bv[threadIdx.x] = o;
                    bi[threadIdx.x] = oi;
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const int i = bi[0] == 0x7fffffff ? prev : bi[0];  // nothing eligible: repeat
            prev = i;
            const int lx = i % bx.dx, ly = (i / bx.dx) % bx.dy, lz = i / (bx.dx * bx.dy);
            picks[h][0] = lx;
            picks[h][1] = ly;
            picks[h][2] = lz;
            const int g = bx.global(i);
            hot[(int64_t)r * n_hot + h] = g;
            row[4 * h + 0] = sim[g];
            row[4 * h + 1] = bx.dx > 1 ? (float)lx / (float)(bx.dx - 1) : 0.0f;
            row[4 * h + 2] = bx.dy > 1 ? (float)ly / (float)(bx.dy - 1) : 0.0f;
            row[4 * h + 3] = bx.dz > 1 ? (float)lz / (float)(bx.dz - 1) : 0.0f;
        }
        __syncthreads();
    }
    float smu = 0.0f, ssg = 0.0f;
    for (int i = threadIdx.x; i < cnt; i += 256) {
        const int g = bx.global(i);
        smu += mu[g];
        ssg += sigma[g];
    }
    red[threadIdx.x] = smu;
    red[256 + threadIdx.x] = ssg;
    __syncthreads();
    for (int st = 128; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st) {
            red[threadIdx.x] += red[threadIdx.x + st];
            red[256 + threadIdx.x] += red[256 + threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float* o = row + 4 * n_hot;
        o[0] = red[0] / (float)cnt;
        o[1] = red[256] / (float)cnt;
        o[2] = (float)((bx.x0 + (bx.dx - 1) * 0.5) / bx.nx);
        o[3] = (float)((bx.y0 + (bx.dy - 1) * 0.5) / bx.ny);
        o[4] = (float)((bx.z0 + (bx.dz - 1) * 0.5) / nz);
    }
}

// One wave per region pair: the two region rows, then |zhat_a_i . zhat_b_j|
// with members over lanes and a fixed xor-tree reduction.
template <typename T>
__global__ __launch_bounds__(256) void pair_row_kernel(const T* __restrict__ x, int64_t stride, int M,
                                                       const float* __restrict__ mu, const float* __restrict__ rs,
                                                       const int32_t* __restrict__ hot, const float* __restrict__ rows,
                                                       const int32_t* __restrict__ rpairs, int n_pairs, int n_hot,
                                                       float* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int pr = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pr >= n_pairs) return;
    const int ra = rpairs[2 * pr], rb = rpairs[2 * pr + 1];
    const int F = 4 * n_hot + 5;
    const int W = 2 * F + n_hot * n_hot;
    float* o = out + (int64_t)pr * W;
    for (int t = lane; t < F; t += 64) {
        o[t] = rows[(int64_t)ra * F + t];
        o[F + t] = rows[(int64_t)rb * F + t];
    }
    int ha[8], hb[8];
    float mua[8], mub[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        ha[i] = i < n_hot ? hot[(int64_t)ra * n_hot + i] : 0;
        hb[i] = i < n_hot ? hot[(int64_t)rb * n_hot + i] : 0;
        mua[i] = mu[ha[i]];
        mub[i] = mu[hb[i]];
    }
    float acc[64];
#pragma unroll
    for (int e = 0; e < 64; ++e) acc[e] = 0.0f;
    for (int m = lane; m < M; m += 64) {
        const T* row = x + (int64_t)m * stride;
        float va[8], vb[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            va[i] = i < n_hot ? ldv(row, ha[i]) - mua[i] : 0.0f;
            vb[i] = i < n_hot ? ldv(row, hb[i]) - mub[i] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[8 * i + j] = fmaf(va[i], vb[j], acc[8 * i + j]);
    }
#pragma unroll
    for (int e = 0; e < 64; ++e) {
        float v = acc[e];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
        acc[e] = v;
    }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (i < n_hot && j < n_hot) o[2 * F + i * n_hot + j] = fabsf(acc[8 * i + j] * rs[ha[i]] * rs[hb[j]]);
    }
}

}  // namespace corr

using namespace corr;

struct prop_mlp {
    corr_ctx* ctx = nullptr;
    int n_in = 0, H = 0, n_out = 0;
    int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0, n = 0;
    float* p = nullptr;   // master parameters
    float* g = nullptr;   // gradients
    float* m = nullptr;   // AdamW moments
    float* v = nullptr;
    __hip_bfloat16* pb = nullptr;  // BF16 roundings
    float* act = nullptr;          // activations workspace
    int64_t act_cap = 0;
    float* lw = nullptr;           // loss weights [n_out]
    float* loss = nullptr;         // device scalar
    int step = 0;
};

static int mlp_ws(prop_mlp* mm, int B, hipStream_t s) {
    // z1 a1 z2 a2 y dY dz2 dz1 [B x (4H + 2 n_out + 2H)] + loss parts [B]
    const int64_t need = (int64_t)B * (6 * mm->H + 2 * mm->n_out) + B;
    if (need <= mm->act_cap) return CORR_OK;
    if (mm->act) {
        CORR_HIP(hipStreamSynchronize(s));
        CORR_HIP(hipFree(mm->act));
        mm->act = nullptr;
    }
    if (hipMalloc(&mm->act, sizeof(float) * need) != hipSuccess) {
        (void)hipGetLastError();
        mm->act_cap = 0;
        return fail(CORR_ENOMEM, "prop_mlp: activation workspace");
    }
    mm->act_cap = need;
    return CORR_OK;
}

static int mlp_forward_ws(prop_mlp* mm, const float* x, int B, hipStream_t s, float** z1, float** a1, float** z2,
                          float** a2, float** y) {
    int rc = mlp_ws(mm, B, s);
    if (rc) return rc;
    const int H = mm->H;
    *z1 = mm->act;
    *a1 = *z1 + (int64_t)B * H;
    *z2 = *a1 + (int64_t)B * H;
    *a2 = *z2 + (int64_t)B * H;
    *y = *a2 + (int64_t)B * H;
    to_bf16_kernel<<<dim3((unsigned)((mm->n + 255) / 256)), 256, 0, s>>>(mm->p, mm->pb, mm->n);
    CORR_LAUNCH_CHECK();
    const int n_in = mm->n_in, no = mm->n_out;
    // Z = X W + b with W stored [in][out]
    const MatRef x_r{x, 0, n_in, 1}, a1_r{*a1, 0, H, 1}, a2_r{*a2, 0, H, 1};
    const MatRef w1{mm->pb + mm->oW1, 1, H, 1}, w2{mm->pb + mm->oW2, 1, H, 1}, w3{mm->pb + mm->oW3, 1, no, 1};
    if ((rc = mlp_gemm(x_r, w1, B, H, n_in, EP_BIAS, mm->pb + mm->ob1, nullptr, *z1, *a1, s))) return rc;
    if ((rc = mlp_gemm(a1_r, w2, B, H, H, EP_BIAS, mm->pb + mm->ob2, nullptr, *z2, *a2, s))) return rc;
    return mlp_gemm(a2_r, w3, B, no, H, EP_BIAS, mm->pb + mm->ob3, nullptr, *y, nullptr, s);
}

extern "C" {

void prop_mlp_destroy(prop_mlp* mm) {
    if (!mm) return;
    (void)hipDeviceSynchronize();
    for (void* q : {(void*)mm->p, (void*)mm->g, (void*)mm->m, (void*)mm->v, (void*)mm->pb, (void*)mm->act,
                    (void*)mm->lw, (void*)mm->loss})
        if (q) (void)hipFree(q);
    delete mm;
}

int prop_mlp_create(corr_ctx* ctx, int32_t n_in, int32_t n_hidden, int32_t n_out, uint64_t seed, prop_mlp** out) {
    if (!out) return fail(CORR_EINVAL, "prop_mlp_create: null out");
    *out = nullptr;
    if (!ctx) return fail(CORR_EINVAL, "prop_mlp_create: null context");
    if (n_in < 1 || n_in > 4096 || n_hidden < 1 || n_hidden > 1024 || n_out < 1 || n_out > 64)
        return fail(CORR_EINVAL, "prop_mlp_create: layer sizes");
    prop_mlp* mm = new (std::nothrow) prop_mlp();
    if (!mm) return fail(CORR_ENOMEM, "prop_mlp_create: host allocation");
    mm->ctx = ctx;
    mm->n_in = n_in;
    mm->H = n_hidden;
    mm->n_out = n_out;
    mm->oW1 = 0;
    mm->ob1 = mm->oW1 + (int64_t)n_in * n_hidden;
    mm->oW2 = mm->ob1 + n_hidden;
    mm->ob2 = mm->oW2 + (int64_t)n_hidden * n_hidden;
    mm->oW3 = mm->ob2 + n_hidden;
    mm->ob3 = mm->oW3 + (int64_t)n_hidden * n_out;
    mm->n = mm->ob3 + n_out;
    // Glorot-uniform weights from Philox (stream = layer), zero biases
    std::vector<float> h(mm->n, 0.0f);
    auto fill = [&](int64_t off, int fan_in, int fan_out, int layer) {
        const double a = std::sqrt(6.0 / (fan_in + fan_out));
        for (int64_t i = 0; i < (int64_t)fan_in * fan_out; ++i)
            h[off + i] = (float)((2.0 * ph_uniform(seed, 0, 100 + layer, (uint64_t)i, 0) - 1.0) * a);
    };
    fill(mm->oW1, n_in, n_hidden, 0);
    fill(mm->oW2, n_hidden, n_hidden, 1);
    fill(mm->oW3, n_hidden, n_out, 2);
    hipError_t e = hipMalloc(&mm->p, sizeof(float) * mm->n);
    if (e == hipSuccess) e = hipMalloc(&mm->g, sizeof(float) * mm->n);
    if (e == hipSuccess) e = hipMalloc(&mm->m, sizeof(float) * mm->n);
    if (e == hipSuccess) e = hipMalloc(&mm->v, sizeof(float) * mm->n);
    if (e == hipSuccess) e = hipMalloc(&mm->pb, sizeof(__hip_bfloat16) * mm->n);
    if (e == hipSuccess) e = hipMalloc(&mm->lw, sizeof(float) * 64);
    if (e == hipSuccess) e = hipMalloc(&mm->loss, sizeof(float) * 4);
    if (e == hipSuccess) e = hipMemcpy(mm->p, h.data(), sizeof(float) * mm->n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(mm->g, 0, sizeof(float) * mm->n);
    if (e == hipSuccess) e = hipMemset(mm->m, 0, sizeof(float) * mm->n);
    if (e == hipSuccess) e = hipMemset(mm->v, 0, sizeof(float) * mm->n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        prop_mlp_destroy(mm);
        return fail(CORR_ENOMEM, "prop_mlp_create: device allocation");
    }
    *out = mm;
    return CORR_OK;
}

int prop_mlp_num_params(prop_mlp* mm, int64_t* n) {
    if (!mm || !n) return fail(CORR_EINVAL, "prop_mlp_num_params: null argument");
    *n = mm->n;
    return CORR_OK;
}

int prop_mlp_get_params(prop_mlp* mm, float* params) {
    if (!mm || !params) return fail(CORR_EINVAL, "prop_mlp_get_params: null argument");
    CORR_HIP(hipDeviceSynchronize());
    CORR_HIP(hipMemcpy(params, mm->p, sizeof(float) * mm->n, hipMemcpyDeviceToHost));
    return CORR_OK;
}

int prop_mlp_set_params(prop_mlp* mm, const float* params) {
    if (!mm || !params) return fail(CORR_EINVAL, "prop_mlp_set_params: null argument");
    CORR_HIP(hipDeviceSynchronize());
    CORR_HIP(hipMemcpy(mm->p, params, sizeof(float) * mm->n, hipMemcpyHostToDevice));
    return CORR_OK;
}

int prop_mlp_get_grads(prop_mlp* mm, float* grads) {
    if (!mm || !grads) return fail(CORR_EINVAL, "prop_mlp_get_grads: null argument");
    CORR_HIP(hipDeviceSynchronize());
    CORR_HIP(hipMemcpy(grads, mm->g, sizeof(float) * mm->n, hipMemcpyDeviceToHost));
    return CORR_OK;
}

int prop_mlp_forward(prop_mlp* mm, const float* x, int32_t B, float* y, corr_stream_t stream) {
    if (!mm || (B > 0 && (!x || !y))) return fail(CORR_EINVAL, "prop_mlp_forward: null argument");
    if (B < 0 || B > 4096) return fail(CORR_EINVAL, "prop_mlp_forward: batch size");
    if (B == 0) return CORR_OK;
    hipStream_t s = (hipStream_t)stream;
    float *z1, *a1, *z2, *a2, *yy;
    int rc = mlp_forward_ws(mm, x, B, s, &z1, &a1, &z2, &a2, &yy);
    if (rc) return rc;
    CORR_HIP(hipMemcpyAsync(y, yy, sizeof(float) * (size_t)B * mm->n_out, hipMemcpyDeviceToDevice, s));
    return CORR_OK;
}

int prop_mlp_train_step(prop_mlp* mm, const float* x, const float* target, const float* loss_w, int32_t B, float lr,
                        float wd, float* loss_out, corr_stream_t stream) {
    if (!mm || !x || !target) return fail(CORR_EINVAL, "prop_mlp_train_step: null argument");
    if (B < 1 || B > 4096) return fail(CORR_EINVAL, "prop_mlp_train_step: batch size");
    if (!(lr >= 0.0f) || !(wd >= 0.0f)) return fail(CORR_EINVAL, "prop_mlp_train_step: lr / wd");
    hipStream_t s = (hipStream_t)stream;
    float *z1, *a1, *z2, *a2, *y;
    int rc = mlp_forward_ws(mm, x, B, s, &z1, &a1, &z2, &a2, &y);
    if (rc) return rc;
    const int H = mm->H, no = mm->n_out;
    float* dY = y + (int64_t)B * no;
    float* dz2 = dY + (int64_t)B * no;
    float* dz1 = dz2 + (int64_t)B * H;
    float* part = dz1 + (int64_t)B * H;
    const float* wdev = nullptr;
    if (loss_w) {
        CORR_HIP(hipMemcpyAsync(mm->lw, loss_w, sizeof(float) * no, hipMemcpyHostToDevice, s));
        wdev = mm->lw;
    }
    out_grad_kernel<<<dim3((B + 255) / 256), 256, 0, s>>>(y, target, wdev, B, no, dY, part);
    loss_reduce_kernel<<<1, 256, 0, s>>>(part, B, no, mm->loss);
    // per layer: gW = X^T dZ ([in][out], X as its transpose), gb = column sums
    // of dZ, and dX = (dZ W^T) * silu'(Z_prev) (W [in][out] read transposed)
    const int n_in = mm->n_in;
    const MatRef dY_r{dY, 0, no, 1}, dz2_r{dz2, 0, H, 1}, dz1_r{dz1, 0, H, 1};
    const MatRef a2_t{a2, 0, 1, H}, a1_t{a1, 0, 1, H}, x_t{x, 0, 1, n_in};
    const MatRef w3_t{mm->pb + mm->oW3, 1, 1, no}, w2_t{mm->pb + mm->oW2, 1, 1, H};
    // layer 3
    if ((rc = mlp_gemm(a2_t, dY_r, H, no, B, EP_PLAIN, nullptr, nullptr, mm->g + mm->oW3, nullptr, s))) return rc;
    col_sum_kernel<<<dim3((no + 255) / 256), 256, 0, s>>>(dY, B, no, mm->g + mm->ob3);
    if ((rc = mlp_gemm(dY_r, w3_t, B, H, no, EP_DSILU, nullptr, z2, dz2, nullptr, s))) return rc;
    // layer 2
    if ((rc = mlp_gemm(a1_t, dz2_r, H, H, B, EP_PLAIN, nullptr, nullptr, mm->g + mm->oW2, nullptr, s))) return rc;
    col_sum_kernel<<<dim3((H + 255) / 256), 256, 0, s>>>(dz2, B, H, mm->g + mm->ob2);
    if ((rc = mlp_gemm(dz2_r, w2_t, B, H, H, EP_DSILU, nullptr, z1, dz1, nullptr, s))) return rc;
    // layer 1
    if ((rc = mlp_gemm(x_t, dz1_r, n_in, H, B, EP_PLAIN, nullptr, nullptr, mm->g + mm->oW1, nullptr, s))) return rc;
    col_sum_kernel<<<dim3((H + 255) / 256), 256, 0, s>>>(dz1, B, H, mm->g + mm->ob1);
    mm->step += 1;
    const float bc1 = 1.0f - powf(0.9f, (float)mm->step), bc2 = 1.0f - powf(0.999f, (float)mm->step);
    adamw_kernel<<<dim3((unsigned)((mm->n + 255) / 256)), 256, 0, s>>>(mm->p, mm->g, mm->m, mm->v, mm->n, lr, wd, bc1,
                                                                      bc2);
    CORR_LAUNCH_CHECK();
    if (loss_out) {
        CORR_HIP(hipMemcpyAsync(loss_out, mm->loss, sizeof(float), hipMemcpyDeviceToHost, s));
        CORR_HIP(hipStreamSynchronize(s));
    }
    return CORR_OK;
}

int corr_proposal_inputs(corr_ctx* ctx, const corr_field* A, const corr_region* regions, int32_t n_regions,
                         const int32_t* region_pairs, int32_t n_pairs, int32_t n_hot, int32_t D, int32_t r_nms,
                         float* x_out, int32_t* hot_out, corr_stream_t stream) {
    if (!ctx || !A || !regions || !region_pairs || !x_out)
        return fail(CORR_EINVAL, "corr_proposal_inputs: null argument");
    if (!A->data || (A->dtype != CORR_F32 && A->dtype != CORR_F16) || A->nx < 1 || A->ny < 1 || A->nz < 1)
        return fail(CORR_EINVAL, "corr_proposal_inputs: field");
    if (A->M < 2) return fail(CORR_EINVAL, "corr_proposal_inputs: M must be at least 2");
    if (n_hot < 1 || n_hot > 8 || D < 1 || r_nms < 0) return fail(CORR_EINVAL, "corr_proposal_inputs: n_hot / D / r_nms");
    if (n_regions < 1 || n_pairs < 0) return fail(CORR_EINVAL, "corr_proposal_inputs: region / pair counts");
    const int64_t P = (int64_t)A->nx * A->ny * A->nz;
    if (P > INT32_MAX) return fail(CORR_EUNSUPPORTED, "corr_proposal_inputs: grid too large");
    for (int r = 0; r < n_regions; ++r) {
        const corr_region& g = regions[r];
        if (g.dx < 1 || g.dy < 1 || g.dz < 1 || g.x0 < 0 || g.y0 < 0 || g.z0 < 0 || g.x0 + g.dx > A->nx ||
            g.y0 + g.dy > A->ny || g.z0 + g.dz > A->nz)
            return fail(CORR_EINVAL, "corr_proposal_inputs: region outside the grid");
    }
    for (int64_t i = 0; i < 2 * (int64_t)n_pairs; ++i)
        if (region_pairs[i] < 0 || region_pairs[i] >= n_regions)
            return fail(CORR_EINVAL, "corr_proposal_inputs: region pair index out of range");
    hipStream_t s = (hipStream_t)stream;
    const Box whole{0, 0, 0, A->nx, A->ny, A->nz, A->nx, A->ny};
    const int F = 4 * n_hot + 5;
    void *sb, *simb, *mb;
    int rc = ctx_use_stream(ctx, s);
    if (rc) return rc;
    rc = ws_get(ctx, WS_STATS_A, sizeof(float) * 4 * (size_t)P, s, &sb);
    if (rc) return rc;
    Stats st = stats_view((float*)sb, P);
    if ((rc = launch_stats(*A, whole, true, st, s))) return rc;
    if ((rc = ws_get(ctx, WS_MISC, sizeof(float) * (size_t)P, s, &simb))) return rc;
    const size_t hot_bytes = sizeof(int32_t) * (size_t)n_regions * n_hot;
    const size_t row_bytes = sizeof(float) * (size_t)n_regions * F;
    const size_t box_bytes = sizeof(Box) * (size_t)n_regions;
    const size_t pr_bytes = sizeof(int32_t) * 2 * (size_t)n_pairs;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    if ((rc = ws_get(ctx, WS_PAIRS, al(hot_bytes) + al(row_bytes) + al(box_bytes) + al(pr_bytes), s, &mb))) return rc;
    int32_t* hot = (int32_t*)mb;
    float* rows = (float*)((char*)mb + al(hot_bytes));
    Box* boxes = (Box*)((char*)rows + al(row_bytes));
    int32_t* rp = (int32_t*)((char*)boxes + al(box_bytes));
    std::vector<Box> hb(n_regions);
    for (int r = 0; r < n_regions; ++r) {
        const corr_region& g = regions[r];
        hb[r] = Box{g.x0, g.y0, g.z0, g.dx, g.dy, g.dz, A->nx, A->ny};
    }
    CORR_HIP(hipMemcpyAsync(boxes, hb.data(), box_bytes, hipMemcpyHostToDevice, s));
    if (n_pairs) CORR_HIP(hipMemcpyAsync(rp, region_pairs, pr_bytes, hipMemcpyHostToDevice, s));
    const int64_t stride = A->member_stride ? A->member_stride : P;
    const dim3 g1((unsigned)((P + 255) / 256));
    if (A->dtype == CORR_F32)
        self_sim_kernel<float><<<g1, 256, 0, s>>>((const float*)A->data, stride, A->M, A->nx, A->ny, A->nz, D, st.mu32,
                                                  st.rs32, (float*)simb);
    else
        self_sim_kernel<__half><<<g1, 256, 0, s>>>((const __half*)A->data, stride, A->M, A->nx, A->ny, A->nz, D,
                                                   st.mu32, st.rs32, (float*)simb);
    hot_spot_kernel<<<dim3(n_regions), 256, 0, s>>>((const float*)simb, boxes, n_hot, r_nms, A->nz, st.mu32, st.sigma,
                                                    hot, rows);
    if (n_pairs) {
        const dim3 g2((unsigned)((n_pairs + 3) / 4));
        if (A->dtype == CORR_F32)
            pair_row_kernel<float><<<g2, 256, 0, s>>>((const float*)A->data, stride, A->M, st.mu32, st.rs32, hot, rows,
                                                      rp, n_pairs, n_hot, x_out);
        else
            pair_row_kernel<__half><<<g2, 256, 0, s>>>((const __half*)A->data, stride, A->M, st.mu32, st.rs32, hot,
                                                       rows, rp, n_pairs, n_hot, x_out);
    }
    CORR_LAUNCH_CHECK();
    if (hot_out) CORR_HIP(hipMemcpyAsync(hot_out, hot, hot_bytes, hipMemcpyDeviceToDevice, s));
    CORR_HIP(hipStreamSynchronize(s));
    return CORR_OK;
}

}  // extern "C"
