// Learned BOS proposal: a small MLP (forward, backward, AdamW) and the region
// summaries it reads. FP32 arithmetic on BF16-rounded weights; every sum runs
// in a fixed order (no floating-point atomics), so runs are reproducible.
//
// The network is tiny (about 8e4 parameters); its layers are plain row-major
// products, one thread per output with the input row staged in LDS, and the
// weight gradient one thread per weight summing over the batch in order.
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

// Z[b][n] = bias[n] + sum_k X[b][k] W[k][n]; A = silu(Z) when A != NULL.
__global__ __launch_bounds__(256) void linear_fwd_kernel(const float* __restrict__ X, int K,
                                                         const __hip_bfloat16* __restrict__ W,
                                                         const __hip_bfloat16* __restrict__ bias, int N,
                                                         float* __restrict__ Z, float* __restrict__ A) {
    extern __shared__ float xs[];
    const int b = blockIdx.x;
    for (int k = threadIdx.x; k < K; k += blockDim.x) xs[k] = X[(int64_t)b * K + k];
    __syncthreads();
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        float z = bf(bias[n]);
        for (int k = 0; k < K; ++k) z = fmaf(xs[k], bf(W[(int64_t)k * N + n]), z);
        Z[(int64_t)b * N + n] = z;
        if (A) A[(int64_t)b * N + n] = silu_f(z);
    }
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

// dZprev[b][k] = (sum_n dZ[b][n] W[k][n]) * silu'(Zprev[b][k])
__global__ __launch_bounds__(256) void linear_bwd_data_kernel(const float* __restrict__ dZ, int N,
                                                              const __hip_bfloat16* __restrict__ W, int K,
                                                              const float* __restrict__ Zprev,
                                                              float* __restrict__ dZprev) {
    extern __shared__ float ds[];
    const int b = blockIdx.x;
    for (int n = threadIdx.x; n < N; n += blockDim.x) ds[n] = dZ[(int64_t)b * N + n];
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        float a = 0.0f;
        const __hip_bfloat16* wk = W + (int64_t)k * N;
        for (int n = 0; n < N; ++n) a = fmaf(ds[n], bf(wk[n]), a);
        dZprev[(int64_t)b * K + k] = a * dsilu_f(Zprev[(int64_t)b * K + k]);
    }
}

// gW[k][n] = sum_b X[b][k] dZ[b][n] (blockIdx.y = k < K), gb[n] = sum_b dZ[b][n] (blockIdx.y = K)
__global__ __launch_bounds__(256) void linear_bwd_weight_kernel(const float* __restrict__ X, const float* __restrict__ dZ,
                                                                int B, int K, int N, float* __restrict__ gW,
                                                                float* __restrict__ gb) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (n >= N) return;
    float g = 0.0f;
    if (k < K) {
        for (int b = 0; b < B; ++b) g = fmaf(X[(int64_t)b * K + k], dZ[(int64_t)b * N + n], g);
        gW[(int64_t)k * N + n] = g;
    } else {
        for (int b = 0; b < B; ++b) g += dZ[(int64_t)b * N + n];
        gb[n] = g;
    }
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

// ---------------------------------------------------------------- features
// Partial member-space Gram matrices over chunks of points. Block (c, t)
// accumulates entries e = 4096 t + threadIdx.x + 256 q (q < 16) of the M x M
// matrix over chunk c of the points, in point order.
constexpr int GRAM_E = 16;
__global__ __launch_bounds__(256) void gram_partial_kernel(const float* __restrict__ Z, int64_t ld, int64_t P, int M,
                                                           int64_t chunk, float* __restrict__ partial) {
    __shared__ float zs[16 * 128];
    const int MM = M * M;
    const int ebase = blockIdx.y * (256 * GRAM_E) + threadIdx.x;
    float acc[GRAM_E];
    int ri[GRAM_E], ci[GRAM_E];
#pragma unroll
    for (int q = 0; q < GRAM_E; ++q) {
        acc[q] = 0.0f;
        const int e = min(ebase + 256 * q, MM - 1);
        ri[q] = e / M;
        ci[q] = e - ri[q] * M;
    }
    const int64_t p0 = (int64_t)blockIdx.x * chunk;
    const int64_t p1 = min(P, p0 + chunk);
    for (int64_t pb = p0; pb < p1; pb += 16) {
        const int np = (int)min((int64_t)16, p1 - pb);
        for (int e = threadIdx.x; e < 16 * M; e += 256) {
            const int r = e / M, c = e - r * M;
            zs[e] = r < np ? Z[(pb + r) * ld + c] : 0.0f;
        }
        __syncthreads();
        for (int r = 0; r < np; ++r) {
            const float* z = zs + r * M;
#pragma unroll
            for (int q = 0; q < GRAM_E; ++q) acc[q] = fmaf(z[ri[q]], z[ci[q]], acc[q]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < GRAM_E; ++q) {
        const int e = ebase + 256 * q;
        if (e < MM) partial[(int64_t)blockIdx.x * MM + e] = acc[q];
    }
}

__global__ void gram_reduce_kernel(const float* __restrict__ partial, int nchunks, int MM, double* __restrict__ G,
                                   double scale) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= MM) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += (double)partial[(int64_t)c * MM + e];
    G[e] = s * scale;
}

// One block per region: max |u_j . zhat_p|, mean of mu, mean of sigma
__global__ __launch_bounds__(256) void region_feat_kernel(const float* __restrict__ Z, int64_t ld, int M,
                                                          const float* __restrict__ U, int n_pc,
                                                          const Box* __restrict__ boxes,
                                                          const float* __restrict__ mu32,
                                                          const float* __restrict__ sigma, int nz,
                                                          float* __restrict__ feats) {
    __shared__ float us[128 * 32];
    __shared__ float red[256 * 2];
    __shared__ float mx[256];
    const int r = blockIdx.x;
    const Box bx = boxes[r];
    for (int e = threadIdx.x; e < n_pc * M; e += 256) us[e] = U[e];
    __syncthreads();
    float cmax[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) cmax[j] = 0.0f;
    float smu = 0.0f, ssg = 0.0f;
    const int64_t cnt = bx.count();
    for (int64_t i = threadIdx.x; i < cnt; i += 256) {
        const int64_t p = bx.global(i);
        const float* z = Z + p * ld;
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            if (j < n_pc) {
                float s = 0.0f;
                for (int m = 0; m < M; ++m) s = fmaf(us[j * M + m], z[m], s);
                cmax[j] = fmaxf(cmax[j], fabsf(s));
            }
        }
        smu += mu32[p];
        ssg += sigma[p];
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
    const int F = n_pc + 5;
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        if (j < n_pc) {  // uniform over the block
            mx[threadIdx.x] = cmax[j];
            __syncthreads();
            for (int st = 128; st >= 1; st >>= 1) {
                if ((int)threadIdx.x < st) mx[threadIdx.x] = fmaxf(mx[threadIdx.x], mx[threadIdx.x + st]);
                __syncthreads();
            }
            if (threadIdx.x == 0) feats[(int64_t)r * F + j] = mx[0];
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        feats[(int64_t)r * F + n_pc] = red[0] / (float)cnt;
        feats[(int64_t)r * F + n_pc + 1] = red[256] / (float)cnt;
        feats[(int64_t)r * F + n_pc + 2] = (float)((bx.x0 + (bx.dx - 1) * 0.5) / bx.nx);
        feats[(int64_t)r * F + n_pc + 3] = (float)((bx.y0 + (bx.dy - 1) * 0.5) / bx.ny);
        feats[(int64_t)r * F + n_pc + 4] = (float)((bx.z0 + (bx.dz - 1) * 0.5) / nz);
    }
}

// Cyclic Jacobi eigendecomposition of a symmetric n x n matrix (row-major,
// overwritten); V receives the eigenvectors as columns.
static void jacobi_eigen(std::vector<double>& A, int n, std::vector<double>& V, std::vector<double>& w) {
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
    double scale = 0.0;
    for (int i = 0; i < n; ++i) scale += a(i, i) * a(i, i);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += a(p, q) * a(p, q);
        if (off <= 1e-30 * (scale + 1e-300)) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a(p, q);
                if (std::fabs(apq) < 1e-300) continue;
                const double theta = (a(q, q) - a(p, p)) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, q
                    const double akp = a(k, p), akq = a(k, q);
                    a(k, p) = c * akp - s * akq;
                    a(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q
                    const double apk = a(p, k), aqk = a(q, k);
                    a(p, k) = c * apk - s * aqk;
                    a(q, k) = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = a(i, i);
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
    const int th = 256;
    linear_fwd_kernel<<<dim3(B), th, sizeof(float) * mm->n_in, s>>>(x, mm->n_in, mm->pb + mm->oW1, mm->pb + mm->ob1, H,
                                                                     *z1, *a1);
    linear_fwd_kernel<<<dim3(B), th, sizeof(float) * H, s>>>(*a1, H, mm->pb + mm->oW2, mm->pb + mm->ob2, H, *z2, *a2);
    linear_fwd_kernel<<<dim3(B), th, sizeof(float) * H, s>>>(*a2, H, mm->pb + mm->oW3, mm->pb + mm->ob3, mm->n_out, *y,
                                                             nullptr);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
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
    // layer 3
    linear_bwd_weight_kernel<<<dim3((no + 255) / 256, H + 1), 256, 0, s>>>(a2, dY, B, H, no, mm->g + mm->oW3,
                                                                          mm->g + mm->ob3);
    linear_bwd_data_kernel<<<dim3(B), 256, sizeof(float) * no, s>>>(dY, no, mm->pb + mm->oW3, H, z2, dz2);
    // layer 2
    linear_bwd_weight_kernel<<<dim3((H + 255) / 256, H + 1), 256, 0, s>>>(a1, dz2, B, H, H, mm->g + mm->oW2,
                                                                         mm->g + mm->ob2);
    linear_bwd_data_kernel<<<dim3(B), 256, sizeof(float) * H, s>>>(dz2, H, mm->pb + mm->oW2, H, z1, dz1);
    // layer 1
    linear_bwd_weight_kernel<<<dim3((H + 255) / 256, mm->n_in + 1), 256, 0, s>>>(x, dz1, B, mm->n_in, H,
                                                                                mm->g + mm->oW1, mm->g + mm->ob1);
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

int corr_region_features(corr_ctx* ctx, const corr_field* A, const corr_region* regions, int32_t n_regions,
                         int32_t n_pc, float* feats, float* evals, corr_stream_t stream) {
    if (!ctx || !A || !regions || !feats) return fail(CORR_EINVAL, "corr_region_features: null argument");
    if (!A->data || (A->dtype != CORR_F32 && A->dtype != CORR_F16)) return fail(CORR_EINVAL, "corr_region_features: field");
    if (A->M < 2 || A->M > 128) return fail(CORR_EUNSUPPORTED, "corr_region_features: M must be in [2, 128]");
    if (n_pc < 1 || n_pc > A->M || n_pc > 32) return fail(CORR_EINVAL, "corr_region_features: n_pc");
    if (n_regions < 1) return fail(CORR_EINVAL, "corr_region_features: no regions");
    for (int r = 0; r < n_regions; ++r) {
        const corr_region& g = regions[r];
        if (g.dx < 1 || g.dy < 1 || g.dz < 1 || g.x0 < 0 || g.y0 < 0 || g.z0 < 0 || g.x0 + g.dx > A->nx ||
            g.y0 + g.dy > A->ny || g.z0 + g.dz > A->nz)
            return fail(CORR_EINVAL, "corr_region_features: region outside the grid");
    }
    hipStream_t s = (hipStream_t)stream;
    const int M = A->M;
    const Box whole{0, 0, 0, A->nx, A->ny, A->nz, A->nx, A->ny};
    const int64_t P = whole.count();
    const int64_t ld = (M + 3) / 4 * 4;
    void *sb, *zb, *pb, *gb, *ub, *bb;
    int rc = ws_get(ctx, WS_STATS_A, sizeof(float) * 4 * (size_t)P, s, &sb);
    if (rc) return rc;
    Stats st = stats_view((float*)sb, P);
    if ((rc = launch_stats(*A, whole, true, st, s))) return rc;
    if ((rc = ws_get(ctx, WS_ZH_A, sizeof(float) * (size_t)(P * ld), s, &zb))) return rc;
    if ((rc = launch_transpose(*A, whole, st, ZF_F32, zb, nullptr, P, ld, s))) return rc;
    const int64_t chunk = 2048;
    const int nchunks = (int)((P + chunk - 1) / chunk);
    const int MM = M * M;
    if ((rc = ws_get(ctx, WS_MISC, sizeof(float) * (size_t)nchunks * MM, s, &pb))) return rc;
    if ((rc = ws_get(ctx, WS_PAIRS, sizeof(double) * (size_t)MM + sizeof(float) * 32 * 128 +
                                         sizeof(Box) * (size_t)n_regions + 1024,
                     s, &gb)))
        return rc;
    gram_partial_kernel<<<dim3(nchunks, (MM + 256 * GRAM_E - 1) / (256 * GRAM_E)), 256, 0, s>>>((const float*)zb, ld, P, M, chunk, (float*)pb);
    gram_reduce_kernel<<<dim3((MM + 255) / 256), 256, 0, s>>>((const float*)pb, nchunks, MM, (double*)gb,
                                                              1.0 / (double)P);
    CORR_LAUNCH_CHECK();
    std::vector<double> G(MM);
    CORR_HIP(hipMemcpyAsync(G.data(), gb, sizeof(double) * MM, hipMemcpyDeviceToHost, s));
    CORR_HIP(hipStreamSynchronize(s));
    std::vector<double> V, w;
    jacobi_eigen(G, M, V, w);
    std::vector<int> order(M);
    for (int i = 0; i < M; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return w[a] > w[b]; });
    std::vector<float> U((size_t)n_pc * M);
    for (int j = 0; j < n_pc; ++j)
        for (int m = 0; m < M; ++m) U[(size_t)j * M + m] = (float)V[(size_t)m * M + order[j]];
    if (evals)
        for (int j = 0; j < n_pc; ++j) evals[j] = (float)w[order[j]];
    ub = (char*)gb + sizeof(double) * MM;
    bb = (char*)ub + sizeof(float) * 32 * 128;
    std::vector<Box> boxes(n_regions);
    for (int r = 0; r < n_regions; ++r) {
        const corr_region& g = regions[r];
        boxes[r] = Box{g.x0, g.y0, g.z0, g.dx, g.dy, g.dz, A->nx, A->ny};
    }
    CORR_HIP(hipMemcpyAsync(ub, U.data(), sizeof(float) * U.size(), hipMemcpyHostToDevice, s));
    CORR_HIP(hipMemcpyAsync(bb, boxes.data(), sizeof(Box) * boxes.size(), hipMemcpyHostToDevice, s));
    region_feat_kernel<<<dim3(n_regions), 256, 0, s>>>((const float*)zb, ld, M, (const float*)ub, n_pc,
                                                       (const Box*)bb, st.mu32, st.sigma, A->nz, feats);
    CORR_LAUNCH_CHECK();
    CORR_HIP(hipStreamSynchronize(s));
    return CORR_OK;
}

}  // extern "C"
