// Kraskov (KSG) mutual information per point pair (Sec. 3.2).
//
// For pair (a, b) the M joint samples (x_i, y_i) are the z-scored member
// values of a and b. For each i: eps_i is the k-th smallest Chebyshev
// distance max(|x_i - x_j|, |y_i - y_j|) over j != i; n_x,i and n_y,i count
// the j != i with marginal distance strictly below eps_i; the estimate is
// psi(M) + psi(k) - mean_i[psi(n_x,i + 1) + psi(n_y,i + 1)].
//
// Design (gfx950, wave64, VALU-bound):
//  - a wave owns a chunk of PW consecutive pairs and stages, per pair, the
//    joint samples as (x_j, y_j), twice in a row (j = 0..M-1, then again),
//    and both marginals sorted ascending (sorted once per point, not per
//    pair, by sort_rows_kernel);
//  - the chunk's PW*M (pair, sample) items are laid densely over the lanes,
//    so no lane idles when M is not a multiple of 64;
//  - eps_i: item i reads the M-1 samples that follow it in the doubled row
//    (i+1 .. i+M-1), so its own zero distance never enters the selection;
//    the KP >= k smallest distances are kept in registers; inserting d is
//    one v_min_f32 and KP-1 mutually independent v_med3_f32:
//    t[p] <- med3(t[p-1], d, t[p]). eps_i = t[k-1] is exactly the k-th
//    smallest over j != i, ties kept as a multiset;
//  - n_x,i: since s -> fl32(x_i - s) is monotone, the j with
//    |fl32(x_i - x_j)| < eps_i form one run of the sorted marginal; two
//    branch-free binary searches find it (the run includes j = i exactly when
//    eps_i > 0, which is subtracted). This replaces M distance tests with
//    2 log2(M) probes and gives the same integer bit for bit;
//  - each item's (n_x, n_y) is kept in LDS; one lane per pair then sums the
//    FP64 digamma terms (integer-argument table) in sample order, so MI is
//    deterministic.
// Distances are plain FP32 subtract/abs/max (no contraction). The unit is
// compiled with IEEE mode off: every operand is finite or +inf, for which
// min/max/med3 give the same results, and no NaN quieting is needed.
#include "common.h"

namespace corr {

constexpr int KSG_WAVES = 4;

template <int KP>
__device__ __forceinline__ void topk_insert(float (&t)[KP], float d) {
#pragma unroll
    for (int p = KP - 1; p >= 1; --p) t[p] = __builtin_amdgcn_fmed3f(t[p - 1], d, t[p]);
    t[0] = fminf(t[0], d);
}

// Marginal counts by binary search on the sorted marginals (p2 a power of
// two > M, rows padded with +inf). For each marginal two runs are located at
// once: lo = number of leading s with fl32(x - s) >= eps, hi = number of
// leading s with fl32(x - s) > -eps; the j with |fl32(x - x_j)| < eps are
// exactly the hi - lo entries in between. The four searches are interleaved
// so their LDS reads overlap.
__device__ __forceinline__ void run_counts(const float* sx, const float* sy, int p2, float x, float y, float eps,
                                           int& cx, int& cy) {
    int lx = 0, ux = 0, ly = 0, uy = 0;
    for (int step = p2 >> 1; step >= 1; step >>= 1) {
        const float a0 = sx[lx + step - 1], a1 = sx[ux + step - 1];
        const float b0 = sy[ly + step - 1], b1 = sy[uy + step - 1];
        lx += (x - a0 < eps) ? 0 : step;
        ux += (x - a1 > -eps) ? step : 0;
        ly += (y - b0 < eps) ? 0 : step;
        uy += (y - b1 > -eps) ? step : 0;
    }
    cx = ux - lx;
    cy = uy - ly;
}

struct KsgLayout {
    int mdup;       // float2 entries of the doubled sample row (2 M)
    int p2;         // power of two > M (sorted marginals)
    int pw;         // pairs per wave chunk (divides 64)
    int slot_f;     // floats per pair slot
    int wave_f;     // floats per wave (slots, packed counts, pair info)
    int psi_f;      // floats of the block-shared digamma table
};

template <int KP>
__global__ __launch_bounds__(256) void ksg_kernel(KsgArgs a, int64_t n_total, KsgLayout L) {
    extern __shared__ __attribute__((aligned(16))) float lds_f[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // block-shared: digamma table psi[0..M] (FP64), then per wave: pair slots,
    // packed counts, per-pair (la, lb, flags)
    double* psi = reinterpret_cast<double*>(lds_f);
    float* wbase = lds_f + L.psi_f + wave * L.wave_f;
    uint32_t* cnt = reinterpret_cast<uint32_t*>(wbase + L.pw * L.slot_f);  // packed n_x | n_y << 16
    int* pinfo = reinterpret_cast<int*>(cnt + L.pw * a.M);                 // [pw][4]: la, lb, state, in_max
    for (int v = threadIdx.x; v <= a.M; v += 256) psi[v] = a.psi[v];
    const int M = a.M;
    const int k = a.k;
    const int64_t nb = a.bb.count();
    const float inf = __builtin_inff();
    unsigned long long best = 0;
    uint32_t n_in_max = 0;
    const int64_t chunk_pairs = (int64_t)KSG_WAVES * L.pw;

    for (int64_t base = (int64_t)blockIdx.x * chunk_pairs; base < n_total; base += (int64_t)gridDim.x * chunk_pairs) {
        const int64_t wbase_pair = base + (int64_t)wave * L.pw;
        // ---- per-pair index math, one lane per pair
        // state: 0 = nothing to evaluate, 1 = evaluate, 2 = constant point (MI 0)
        if (lane < L.pw) {
            const int64_t t = wbase_pair + lane;
            int la = -1, lb = -1, state = 0, in_max = 0;
            if (t < n_total) {
                bool same = false;
                if (a.pairs) {
                    const int32_t ga = a.pairs[2 * t], gb = a.pairs[2 * t + 1];
                    la = a.whole_a ? ga : (int)a.ba.local(ga);
                    lb = a.whole_b ? gb : (int)a.bb.local(gb);
                    same = ga == gb;
                } else {
                    const int32_t tt = (int32_t)t, nb32 = (int32_t)nb;
                    la = tt / nb32;
                    lb = tt - la * nb32;
                    same = a.ba.global(la) == a.bb.global(lb);
                }
                if (la >= 0 && lb >= 0) {
                    state = 1;
                    if (a.inv_a && (a.inv_a[la] == 0.0f || a.inv_b[lb] == 0.0f)) state = 2;
                    in_max = (a.key != nullptr) && !(a.same_field && same);
                }
            }
            int* pi = pinfo + 4 * lane;
            pi[0] = la;
            pi[1] = lb;
            pi[2] = state;
            pi[3] = in_max;
        }
        __syncthreads();
        // ---- stage the wave's pairs (all waves reach every barrier)
        for (int q = 0; q < L.pw; ++q) {
            const int* pi = pinfo + 4 * q;
            if (pi[2] != 1) continue;
            float* slot = wbase + q * L.slot_f;
            float2* xy = reinterpret_cast<float2*>(slot);
            float* sx = slot + 2 * L.mdup;
            float* sy = sx + L.p2;
            const int64_t la = pi[0], lb = pi[1];
            const float* xa = a.za + la * a.ld;
            const float* yb = a.zb + lb * a.ld;
            const float* sxa = a.sa + la * L.p2;
            const float* syb = a.sb + lb * L.p2;
            for (int j = lane; j < M; j += 64) {
                const float2 v = make_float2(xa[j], yb[j]);
                xy[j] = v;
                xy[j + M] = v;
            }
            for (int j = lane; j < L.p2; j += 64) {
                sx[j] = sxa[j];
                sy[j] = syb[j];
            }
        }
        __syncthreads();
        // ---- items: u = q * M + i over the wave's pairs
        const int n_items = L.pw * M;
        for (int u0 = 0; u0 < n_items; u0 += 64) {
            const int u = u0 + lane;
            const int uc = u < n_items ? u : n_items - 1;
            const int q = uc / M, i = uc - q * M;
            const float* slot = wbase + q * L.slot_f;
            const float2* row = reinterpret_cast<const float2*>(slot);
            const float2 me = row[i];
            const float2* nbr = row + i + 1;  // the M-1 other samples, in cyclic order
            float tk[KP];
#pragma unroll
            for (int p = 0; p < KP; ++p) tk[p] = inf;
            int t = 0;
            for (; t + 4 <= M - 1; t += 4) {  // four reads per trip: immediate LDS offsets
                const float2 v0 = nbr[t], v1 = nbr[t + 1], v2 = nbr[t + 2], v3 = nbr[t + 3];
                topk_insert<KP>(tk, fmaxf(fabsf(me.x - v0.x), fabsf(me.y - v0.y)));
                topk_insert<KP>(tk, fmaxf(fabsf(me.x - v1.x), fabsf(me.y - v1.y)));
                topk_insert<KP>(tk, fmaxf(fabsf(me.x - v2.x), fabsf(me.y - v2.y)));
                topk_insert<KP>(tk, fmaxf(fabsf(me.x - v3.x), fabsf(me.y - v3.y)));
            }
            for (; t < M - 1; ++t) {
                const float2 v = nbr[t];
                topk_insert<KP>(tk, fmaxf(fabsf(me.x - v.x), fabsf(me.y - v.y)));
            }
            float eps = tk[0];
#pragma unroll
            for (int p = 1; p < KP; ++p) eps = (p == k - 1) ? tk[p] : eps;
            const float* sx = slot + 2 * L.mdup;
            const float* sy = sx + L.p2;
            const int self = eps > 0.0f ? 1 : 0;
            int nx, ny;
            run_counts(sx, sy, L.p2, me.x, me.y, eps, nx, ny);
            nx -= self;
            ny -= self;
            nx = nx < 0 ? 0 : nx;
            ny = ny < 0 ? 0 : ny;
            if (u < n_items) {
                cnt[u] = (uint32_t)nx | ((uint32_t)ny << 16);
                const int64_t t = wbase_pair + q;
                if (a.counts_out && pinfo[4 * q + 2] == 1)
                    reinterpret_cast<int2*>(a.counts_out)[t * M + i] = make_int2(nx, ny);
            }
        }
        __syncthreads();
        // ---- per pair: G = 64 / pw lanes sum the digamma terms; lane r of a
        // group takes samples r, r + G, ... in order, then a fixed xor tree
        // combines the group -- the same order on every run
        {
            const int G = 64 / L.pw;
            const int q = lane / G, r = lane - q * G;
            const int* pi = pinfo + 4 * q;
            double acc = 0.0;
            if (pi[2] == 1) {
                const uint32_t* cq = cnt + q * M;
                for (int i = r; i < M; i += G) {
                    const uint32_t c = cq[i];
                    acc += psi[(c & 0xffffu) + 1] + psi[(c >> 16) + 1];
                }
            }
            for (int off = G >> 1; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
            const int64_t t = wbase_pair + q;
            if (r == 0 && t < n_total) {
                const int state = pi[2];
                float mi = 0.0f;
                if (state == 1) mi = (float)(psi[M] + psi[k] - acc / (double)M);
                if (a.mi_out) a.mi_out[t] = mi;
                if (pi[3] && state != 0) {
                    const unsigned long long key = make_key(mi, (uint32_t)((int64_t)pi[0] * nb + pi[1]), 0u);
                    best = key > best ? key : best;
                    ++n_in_max;
                }
            }
            if (a.counts_out && t < n_total && pi[2] != 1) {
                int2* c = reinterpret_cast<int2*>(a.counts_out) + t * M;
                for (int i = r; i < M; i += G) c[i] = make_int2(0, 0);
            }
        }
        __syncthreads();  // slots and terms are rewritten by the next chunk
    }
    if (a.key) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            unsigned long long o = __shfl_xor(best, off, 64);
            best = o > best ? o : best;
            n_in_max += __shfl_xor(n_in_max, off, 64);
        }
        if (lane == 0 && n_in_max) {
            atomicMax(a.key, best);
            atomicAdd(a.key + 1, (unsigned long long)n_in_max);
        }
    }
}

// One wave per row: bitonic sort of the row's M values (padded to p2 with
// +inf) in LDS, written to out[row * p2 ...].
__global__ __launch_bounds__(256) void sort_rows_kernel(const float* __restrict__ z, int64_t ld, int64_t nrows, int M,
                                                        int p2, float* __restrict__ out) {
    extern __shared__ float srt[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float* s = srt + wave * p2;
    for (int64_t r0 = (int64_t)blockIdx.x * 4; r0 < nrows; r0 += (int64_t)gridDim.x * 4) {
        const int64_t r = r0 + wave;
        const bool act = r < nrows;
        for (int j = lane; j < p2; j += 64) s[j] = (act && j < M) ? z[r * ld + j] : __builtin_inff();
        __syncthreads();
        for (int size = 2; size <= p2; size <<= 1) {
            for (int stride = size >> 1; stride >= 1; stride >>= 1) {
                for (int e = lane; e < p2 / 2; e += 64) {
                    int lo = 2 * e - (e & (stride - 1));
                    int hi = lo + stride;
                    bool asc = (lo & size) == 0;
                    float x = s[lo], y = s[hi];
                    if ((x > y) == asc) {
                        s[lo] = y;
                        s[hi] = x;
                    }
                }
                __syncthreads();
            }
        }
        if (act)
            for (int j = lane; j < p2; j += 64) out[r * p2 + j] = s[j];
        __syncthreads();
    }
}

// Sorted-row length: a power of two with at least one +inf sentinel after
// the M values, so a run can reach the end of the row (the branch-free
// searches return at most p2 - 1).
int ksg_p2(int M) {
    int p = 64;
    while (p < M + 1) p <<= 1;
    return p;
}

int launch_sort_rows(const float* z, int64_t ld, int64_t nrows, int M, float* out, int num_cus, hipStream_t s) {
    if (nrows == 0) return CORR_OK;
    const int p2 = ksg_p2(M);
    int64_t blocks = (nrows + 3) / 4;
    int64_t cap = (int64_t)num_cus * 8;
    if (blocks > cap) blocks = cap;
    sort_rows_kernel<<<dim3((unsigned)blocks), 256, 4 * p2 * sizeof(float), s>>>(z, ld, nrows, M, p2, out);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

// Pairs per wave chunk: dense items (pw * M close to a multiple of 64) traded
// against LDS per wave (occupancy). pw <= 0 picks the default.
int ksg_default_pw(int M) { return M >= 512 ? 1 : (M >= 192 ? 2 : (M >= 48 ? 4 : 16)); }

static KsgLayout ksg_layout(int M, int pw) {
    KsgLayout L;
    L.mdup = 2 * M;
    L.p2 = ksg_p2(M);
    L.pw = pw > 0 ? pw : ksg_default_pw(M);
    L.slot_f = 2 * L.mdup + 2 * L.p2;
    L.slot_f = (L.slot_f + 3) & ~3;
    L.wave_f = L.pw * L.slot_f + L.pw * M + 4 * L.pw;  // + packed counts, pair info
    L.wave_f = (L.wave_f + 3) & ~3;
    L.psi_f = (2 * (M + 1) + 3) & ~3;
    return L;
}

size_t ksg_lds_bytes(int M, int pw) {
    const KsgLayout L = ksg_layout(M, pw);
    return ((size_t)KSG_WAVES * L.wave_f + L.psi_f) * sizeof(float);
}

template <int KP>
static int launch_kp(const KsgArgs& a, int64_t n_total, const KsgLayout& L, dim3 grid, size_t lds, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        CORR_HIP(hipFuncSetAttribute((const void*)ksg_kernel<KP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     160 * 1024));
        attr = true;
    }
    ksg_kernel<KP><<<grid, 256, lds, s>>>(a, n_total, L);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

int launch_ksg(const KsgArgs& a, int num_cus, hipStream_t s) {
    int64_t n_total = a.pairs ? a.n : a.ba.count() * a.bb.count();
    if (n_total == 0) return CORR_OK;
    const KsgLayout L = ksg_layout(a.M, a.pw);
    if (64 % L.pw) return fail(CORR_EINVAL, "KSG: pairs per wave must divide 64");
    const size_t lds = ksg_lds_bytes(a.M, a.pw);
    if (lds > 160 * 1024) return fail(CORR_EUNSUPPORTED, "KSG: member count too large for the LDS layout");
    const int64_t chunk_pairs = (int64_t)KSG_WAVES * L.pw;
    int64_t blocks = (n_total + chunk_pairs - 1) / chunk_pairs;
    int64_t cap = (int64_t)num_cus * 8;
    dim3 grid((unsigned)(blocks < cap ? blocks : cap));
    // selection width: the smallest instantiated KP >= k
    const int k = a.k;
    if (k == 10) return launch_kp<10>(a, n_total, L, grid, lds, s);
    if (k <= 4) return launch_kp<4>(a, n_total, L, grid, lds, s);
    if (k <= 8) return launch_kp<8>(a, n_total, L, grid, lds, s);
    if (k <= 12) return launch_kp<12>(a, n_total, L, grid, lds, s);
    if (k <= 16) return launch_kp<16>(a, n_total, L, grid, lds, s);
    if (k <= 24) return launch_kp<24>(a, n_total, L, grid, lds, s);
    return launch_kp<32>(a, n_total, L, grid, lds, s);
}

}  // namespace corr
