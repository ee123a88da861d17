// Batched Bayesian optimal sampling of region-pair maxima (Sec. 3.1).
//
// One persistent kernel per iteration. The host knows every pair's batch
// schedule (it is drawn from the seed) and lists, per iteration, the pairs
// that still sample there, costliest first; workgroups (512 threads) walk
// that list with a static stride, so the loop over pairs, like every loop
// that contains a barrier, runs on wave-uniform (scalar) values. For a pair
// the workgroup
//   - rebuilds the Gaussian process of the pair's observations in LDS (FP64
//     Matern-5/2 covariance, packed lower Cholesky factor, solves by one
//     wave with shuffles),
//   - draws the candidate set (Philox4x64-10) and computes for every
//     candidate its posterior mean and the solve vector q = L^-1 k, which it
//     keeps in a per-workgroup global scratch (row-major, one column per
//     candidate, coalesced),
//   - picks the batch by Kriging believer: each pick extends the factor by
//     one row, u_c = (k(theta_c, theta*) - q_c . q*) / d for every candidate,
//     sigma_c^2 -= u_c^2 -- an O(n) update per candidate instead of a new
//     solve; the means do not change,
//   - rounds the picks to cells (Bernoulli of the fractional part), drops
//     cells already observed, and evaluates the new cells itself (Pearson:
//     FP32 dot products of standardised rows; KSG: one wave per cell, the
//     same exact max-norm selection and sorted-marginal counts as the pair
//     kernel), then appends them to the pair's observations.
// An iteration is the kernel followed by a one-thread kernel that advances
// the device-side iteration counter, so the same two launches are replayed
// unchanged: captured once into a HIP graph (default) or launched directly.
//
// Why the pair loop takes no work from an atomic counter: with the fetch
// (thread 0 only) at the head of the loop and the active-pair count (thread 0
// only) at its tail, the compiler merged the two thread-0 branches across the
// back edge into a nested loop in which only thread 0's lane left to fetch
// the next pair while all other lanes went back to the head barrier with the
// old pair -- a livelock on the first pair. Uniform loop control rules that
// shape out; a CPU test checks the compiled kernels for it.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "../../include/bos.h"
#include "common.h"

namespace corr {

// Threads per workgroup (one pair at a time): one candidate per thread at the
// default 512 candidates, two waves per SIMD.
constexpr int BT = 512;
constexpr int NW = BT / 64;
// Rows of the triangular solve handled per pass over the stored solve vectors.
constexpr int SOLVE_R = 8;
// values of a q column kept in flight by the Kriging-believer update
constexpr int BELIEF_R = 16;

__device__ inline double ph_gauss(uint64_t seed, uint64_t pair, uint64_t stream, uint64_t index, uint64_t axis) {
    uint64_t o[4];
    philox4x64(pair, stream, index, axis, seed, KEY_HI, o);
    const double u1 = ph_u01(o[0]), u2 = ph_u01(o[1]);
    return sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * 3.14159265358979323846 * u2);
}

// ------------------------------------------------------------------ kernel arguments
struct BosDev {
    // configuration
    int measure, k, n_init, n_total, n_unif, n_local, C;
    double kappa, ls, local_sd, jitter;
    uint64_t seed;
    int n_pairs, M;
    // geometry
    const Box* ba;
    const Box* bb;
    // standardised data (rows = global point index)
    const float* za;
    const float* zb;
    int64_t ld;
    const float* sa;  // KSG sorted rows
    const float* sb;
    int p2;
    const float* inv_a;  // KSG: 0 marks a constant point
    const float* inv_b;
    const double* psi;
    // per-pair state
    int16_t* cells;  // [n_pairs][n_total][6]
    double* yv;      // [n_pairs][n_total] objective
    float* sv;       // [n_pairs][n_total] signed value (r or MI)
    int* n_obs;
    int* slot;
    const int* sched;    // [n_pairs][16] batch sizes (host-drawn)
    const int* n_sched;  // batches per pair
    int* best;
    const float* prior;  // [n_pairs][6] or NULL
    // control
    int* iter;                // device iteration counter (0: initial design)
    const int* list;          // pairs of every iteration, concatenated
    const int* list_start;    // [n_iter] offset of iteration t's pairs in list
    const int* list_count;    // [n_iter] number of pairs sampling in iteration t
    int n_iter;               // iterations listed (initial design included)
    int* err;                 // bit 0: inconsistent pair state, bit 1: stopped by the host
    const int* stop;          // host-mapped: nonzero asks every workgroup to stop at its next pair
    double* qbuf;  // per workgroup [n_total][C]
    // LDS layout (in doubles)
    int off_L, off_X, off_y, off_a, off_th, off_mu, off_s2, off_qs, off_pk, off_red, off_misc, lds_doubles;
};

__device__ inline double matern52(const double* a, const double* b, double inv_ls) {
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const double d = (a[t] - b[t]) * inv_ls;
        s += d * d;
    }
    const double rho = sqrt(s);
    const double s5 = 2.23606797749978969641 * rho;
    return (1.0 + s5 + 5.0 * s * (1.0 / 3.0)) * exp(-s5);
}

__device__ inline int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// The value of the first active lane: every loop or branch that encloses a
// barrier takes its bounds through this, so the compiler keeps its control
// in scalar registers (all lanes hold the same value there anyway).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <int KP1>
__device__ __forceinline__ void bos_topk_insert(float (&t)[KP1], float d) {
#pragma unroll
    for (int p = KP1 - 1; p >= 1; --p) t[p] = __builtin_amdgcn_fmed3f(t[p - 1], d, t[p]);
    t[0] = fminf(t[0], d);
}

// Objective of one point pair, computed by one wave (all lanes return it).
// Pearson: |r| of standardised FP32 rows. KSG: MI with exact max-norm
// selection and sorted-marginal counts; `slot` is the wave's LDS staging area.
template <int KP1>
__device__ float wave_objective(const BosDev& d, int32_t pa, int32_t pb, float* slot, float* signed_out) {
    const int lane = threadIdx.x & 63;
    if constexpr (KP1 == 0) {
        const float4* ra = reinterpret_cast<const float4*>(d.za + (int64_t)pa * d.ld);
        const float4* rb = reinterpret_cast<const float4*>(d.zb + (int64_t)pb * d.ld);
        float s = 0.0f;
        for (int c = lane; c < d.ld / 4; c += 64) {
            const float4 x = ra[c], y = rb[c];
            s = fmaf(x.x, y.x, s);
            s = fmaf(x.y, y.y, s);
            s = fmaf(x.z, y.z, s);
            s = fmaf(x.w, y.w, s);
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
        s = fminf(1.0f, fmaxf(-1.0f, s));
        *signed_out = s;
        return fabsf(s);
    } else {
        const int M = d.M;
        if (d.inv_a[pa] == 0.0f || d.inv_b[pb] == 0.0f) {
            *signed_out = 0.0f;
            return 0.0f;
        }
        const int mpad2 = (M + 1) & ~1;
        float2* xy = reinterpret_cast<float2*>(slot);
        float* sx = slot + 2 * mpad2;
        float* sy = sx + d.p2;
        const float* xa = d.za + (int64_t)pa * d.ld;
        const float* yb = d.zb + (int64_t)pb * d.ld;
        const float inf = __builtin_inff();
        for (int j = lane; j < mpad2; j += 64) xy[j] = (j < M) ? make_float2(xa[j], yb[j]) : make_float2(inf, inf);
        for (int j = lane; j < d.p2; j += 64) {
            sx[j] = d.sa[(int64_t)pa * d.p2 + j];
            sy[j] = d.sb[(int64_t)pb * d.p2 + j];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double acc = 0.0;
        const float4* xy4 = reinterpret_cast<const float4*>(slot);
        for (int i0 = 0; i0 < M; i0 += 64) {
            const int i = min(i0 + lane, M - 1);
            const float2 me = xy[i];
            float tk[KP1];
#pragma unroll
            for (int p = 0; p < KP1; ++p) tk[p] = inf;
            for (int j2 = 0; j2 < mpad2 / 2; ++j2) {
                const float4 v = xy4[j2];
                bos_topk_insert<KP1>(tk, fmaxf(fabsf(me.x - v.x), fabsf(me.y - v.y)));
                bos_topk_insert<KP1>(tk, fmaxf(fabsf(me.x - v.z), fabsf(me.y - v.w)));
            }
            float eps = tk[0];
#pragma unroll
            for (int p = 1; p < KP1; ++p) eps = (p == d.k) ? tk[p] : eps;
            int lx = 0, ux = 0, ly = 0, uy = 0;
            for (int step = d.p2 >> 1; step >= 1; step >>= 1) {
                const float a0 = sx[lx + step - 1], a1 = sx[ux + step - 1];
                const float b0 = sy[ly + step - 1], b1 = sy[uy + step - 1];
                lx += (me.x - a0 < eps) ? 0 : step;
                ux += (me.x - a1 > -eps) ? step : 0;
                ly += (me.y - b0 < eps) ? 0 : step;
                uy += (me.y - b1 > -eps) ? step : 0;
            }
            const int self = eps > 0.0f ? 1 : 0;
            int nx = ux - lx - self, ny = uy - ly - self;
            nx = nx < 0 ? 0 : nx;
            ny = ny < 0 ? 0 : ny;
            if (i0 + lane < M) acc += d.psi[nx + 1] + d.psi[ny + 1];
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();  // the slot is rewritten by the next cell
        const float mi = (float)(d.psi[M] + d.psi[d.k] - acc / (double)M);
        *signed_out = mi;
        return mi;
    }
}

__device__ inline int32_t cell_point_a(const Box& b, const int* c) {
    return (b.x0 + c[0]) + b.nx * ((b.y0 + c[1]) + b.ny * (b.z0 + c[2]));
}
__device__ inline int32_t cell_point_b(const Box& b, const int* c) {
    return (b.x0 + c[3]) + b.nx * ((b.y0 + c[4]) + b.ny * (b.z0 + c[5]));
}

// Evaluate ncell cells (LDS int[ncell][6]) of `pair`; values to vals/svals.
template <int KP1>
__device__ void eval_cells(const BosDev& d, int pair, const int* cells6, int ncell, double* vals, float* svals,
                           float* stage) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const Box A = d.ba[pair], B = d.bb[pair];
    const int slot_f = 2 * ((d.M + 1) & ~1) + 2 * d.p2;
    for (int m = wave; m < ncell; m += NW) {
        const int* c = cells6 + 6 * m;
        float sgn;
        const float v = wave_objective<KP1>(d, cell_point_a(A, c), cell_point_b(B, c), stage + wave * slot_f, &sgn);
        if (lane == 0) {
            vals[m] = v;
            svals[m] = sgn;
        }
    }
}

// Box dimension of axis a of a pair.
__device__ inline int axis_dim(const Box& A, const Box& B, int a) {
    switch (a) {
        case 0: return A.dx;
        case 1: return A.dy;
        case 2: return A.dz;
        case 3: return B.dx;
        case 4: return B.dy;
        default: return B.dz;
    }
}

// Block-wide argmax of (value, -index) over LDS scratch; returns the index.
__device__ int block_argmax(double v, int idx, double* red_v, int* red_i) {
    // (value, index) pairs are ordered by value, then by smaller index: the
    // winner is unique, so the reduction order does not change it. A wave
    // butterfly leaves every lane with its wave's winner, one lane per wave
    // publishes it and, after one barrier, every thread reduces the NW
    // entries itself. Two calls must be separated by a barrier (the slots
    // are rewritten by the next call).
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int oi = __shfl_xor(idx, off, 64);
        if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
        }
    }
    if (lane == 0) {
        red_v[wave] = v;
        red_i[wave] = idx;
    }
    __syncthreads();
    double bv = red_v[0];
    int bi = red_i[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
        const double ov = red_v[w];
        const int oi = red_i[w];
        if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    return uni(bi);
}

template <int KP1>
__device__ void bos_init_pair(const BosDev& d, int pair, double* sm) {
    const int tid = threadIdx.x;
    int* ic = reinterpret_cast<int*>(sm + d.off_misc);  // [n_init][6] cells
    int* dup = ic + 6 * d.n_init;                         // [n_init]
    int* uniq = dup + d.n_init;                           // [n_init][6] unique cells
    int* nuniq = uniq + 6 * d.n_init;
    double* vals = sm + d.off_y;
    float* svals = reinterpret_cast<float*>(sm + d.off_a);
    const Box A = d.ba[pair], B = d.bb[pair];
    for (int s = tid; s < d.n_init; s += BT) {
        for (int a = 0; a < 6; ++a) {
            const int dim = axis_dim(A, B, a);
            int c = (int)(ph_uniform(d.seed, pair, ST_INIT, s, a) * dim);
            ic[6 * s + a] = c < dim - 1 ? c : dim - 1;
        }
        if (s == 0 && d.prior && d.prior[6 * pair] >= 0.0f) {
            for (int a = 0; a < 6; ++a) {
                const int dim = axis_dim(A, B, a);
                int c = (int)rintf(d.prior[6 * pair + a]);
                ic[a] = c < 0 ? 0 : (c > dim - 1 ? dim - 1 : c);
            }
        }
    }
    __syncthreads();
    for (int s = tid; s < d.n_init; s += BT) {
        int is_dup = 0;
        for (int t = 0; t < s && !is_dup; ++t) {
            bool same = true;
            for (int a = 0; a < 6; ++a) same = same && ic[6 * s + a] == ic[6 * t + a];
            is_dup = same;
        }
        dup[s] = is_dup;
    }
    __syncthreads();
    if (tid == 0) {
        int n = 0;
        for (int s = 0; s < d.n_init; ++s)
            if (!dup[s]) {
                for (int a = 0; a < 6; ++a) uniq[6 * n + a] = ic[6 * s + a];
                ++n;
            }
        *nuniq = n;
    }
    __syncthreads();
    const int n = uni(*nuniq);
    eval_cells<KP1>(d, pair, uniq, n, vals, svals, reinterpret_cast<float*>(sm + d.off_th));
    __syncthreads();
    const int base = pair * d.n_total;
    for (int m = tid; m < n; m += BT) {
        for (int a = 0; a < 6; ++a) d.cells[(int64_t)(base + m) * 6 + a] = (int16_t)uniq[6 * m + a];
        d.yv[base + m] = vals[m];
        d.sv[base + m] = svals[m];
    }
    if (tid == 0) {
        int b = 0;
        for (int m = 1; m < n; ++m)
            if (vals[m] > vals[b]) b = m;
        d.best[pair] = b;
        d.n_obs[pair] = n;
        d.slot[pair] = d.n_init;
    }
}

template <int KP1>
__device__ void bos_batch_pair(const BosDev& d, int pair, int t, double* sm) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = uni(d.n_obs[pair]);
    const int b = uni(d.sched[pair * 16 + t]);
    // every loop below is bounded by n, b and C; state that could not have
    // been written by this sampler is flagged rather than followed
    if (n < 1 || b < 1 || b > 64 || n + b > d.n_total) {
        if (tid == 0) atomicOr(d.err, 1);
        return;
    }
    const int C = d.C;
    const int base = pair * d.n_total;
    double* L = sm + d.off_L;
    double* X = sm + d.off_X;
    double* yt = sm + d.off_y;
    double* alpha = sm + d.off_a;
    double* th = sm + d.off_th;
    double* mu = sm + d.off_mu;
    double* s2 = sm + d.off_s2;
    double* qs = sm + d.off_qs;
    double* pk = sm + d.off_pk;                                   // picks theta [b][6]
    double* red_v = sm + d.off_red;
    int* red_i = reinterpret_cast<int*>(red_v + BT);
    int* misc = reinterpret_cast<int*>(sm + d.off_misc);
    int* taken = misc;                                            // [C]
    int* rc = taken + C;                                          // [b][6] rounded cells
    int* keep = rc + 6 * 64;                                      // [b]
    int* newc = keep + 64;                                        // [b][6]
    int* nnew = newc + 6 * 64;
    double* qcol = d.qbuf + (int64_t)blockIdx.x * d.n_total * C;  // [n_total][C]
    const Box A = d.ba[pair], B = d.bb[pair];
    const double inv_ls = 1.0 / d.ls;

    // ---- observations, standardised values
    for (int i = tid; i < n; i += BT) {
        for (int a = 0; a < 6; ++a) X[6 * i + a] = (double)d.cells[(int64_t)(base + i) * 6 + a];
        yt[i] = d.yv[base + i];
    }
    __syncthreads();
    if (tid == 0) {
        double m = 0.0;
        for (int i = 0; i < n; ++i) m += yt[i];
        m /= (double)n;
        double v = 0.0;
        for (int i = 0; i < n; ++i) v += (yt[i] - m) * (yt[i] - m);
        double sd = sqrt(v / (double)n);
        sd = sd > 1e-6 ? sd : 1e-6;
        red_v[0] = m;
        red_v[1] = sd;
    }
    __syncthreads();
    const double ym = red_v[0], ysd = red_v[1];
    __syncthreads();
    for (int i = tid; i < n; i += BT) yt[i] = (yt[i] - ym) / ysd;
    // ---- covariance (packed lower) and Cholesky, right-looking: once column
    // p is final every trailing element (i, j), p < j <= i, subtracts
    // L_ip L_jp in parallel. Each element subtracts its terms in ascending p
    // and is then divided by (or, on the diagonal, square-rooted from) the
    // same values as in a column-by-column factorisation, so the factor is
    // the same bit for bit; the dependent chain is n steps instead of ~n^2.
    for (int e = tid; e < n * (n + 1) / 2; e += BT) {
        int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (tri(i + 1, 0) <= e) ++i;
        while (tri(i, 0) > e) --i;
        const int j = e - tri(i, 0);
        L[e] = matern52(X + 6 * i, X + 6 * j, inv_ls) + (i == j ? d.jitter : 0.0);
    }
    __syncthreads();
    for (int p = 0; p < n; ++p) {
        const double app = L[tri(p, p)];
        const double dpp = sqrt(app > 1e-300 ? app : 1e-300);
        for (int i = p + 1 + tid; i < n; i += BT) L[tri(i, p)] = L[tri(i, p)] / dpp;
        __syncthreads();
        // trailing triangle over an m x m square (e -> row e / m, column
        // e % m; exact in FP32 for m <= 127, as n_total <= 128)
        const int m = n - p - 1;
        const float inv_m = 1.0f / (float)(m > 0 ? m : 1);
        for (int e = tid; e < m * m; e += BT) {
            const int ii = (int)(((float)e + 0.5f) * inv_m);
            const int jj = e - ii * m;
            if (jj <= ii) {
                const int i = p + 1 + ii, j = p + 1 + jj;
                L[tri(i, j)] -= L[tri(i, p)] * L[tri(j, p)];
            }
        }
        if (tid == 0) L[tri(p, p)] = dpp;
        __syncthreads();
    }
    // ---- alpha = K^-1 yt: two triangular solves by wave 0 (lane owns rows l, l+64)
    if (wave == 0) {
        double r[2];
        for (int q = 0; q < 2; ++q) {
            const int i = lane + 64 * q;
            r[q] = i < n ? yt[i] : 0.0;
        }
        for (int j = 0; j < n; ++j) {  // forward: L z = yt
            const int own = j & 63, q = j >> 6;
            double zj = __shfl(q ? r[1] : r[0], own, 64) / L[tri(j, j)];
            if (lane == own) r[q] = zj;
            for (int qq = 0; qq < 2; ++qq) {
                const int i = lane + 64 * qq;
                if (i > j && i < n) r[qq] -= L[tri(i, j)] * zj;
            }
        }
        for (int j = n - 1; j >= 0; --j) {  // backward: L^T alpha = z
            const int own = j & 63, q = j >> 6;
            double aj = __shfl(q ? r[1] : r[0], own, 64) / L[tri(j, j)];
            if (lane == own) r[q] = aj;
            for (int qq = 0; qq < 2; ++qq) {
                const int i = lane + 64 * qq;
                if (i < j) r[qq] -= L[tri(j, i)] * aj;
            }
        }
        for (int q = 0; q < 2; ++q) {
            const int i = lane + 64 * q;
            if (i < n) alpha[i] = r[q];
        }
    }
    // ---- candidates
    const int bi = uni(d.best[pair]);
    for (int c = tid; c < C; c += BT) {
        taken[c] = 0;
        for (int a = 0; a < 6; ++a) {
            const double up = (double)(axis_dim(A, B, a) - 1);
            double v;
            if (c < d.n_unif) {
                v = ph_uniform(d.seed, pair, ST_UNIF, (uint64_t)t * d.n_unif + c, a) * up;
            } else {
                const int l = c - d.n_unif;
                v = (double)d.cells[(int64_t)(base + bi) * 6 + a] +
                    d.local_sd * ph_gauss(d.seed, pair, ST_LOCAL, (uint64_t)t * d.n_local + l, a);
                v = v < 0.0 ? 0.0 : (v > up ? up : v);
            }
            th[6 * c + a] = v;
        }
    }
    __syncthreads();
    // ---- posterior mean and q = L^-1 k per candidate (q kept in the scratch)
    // Rows are solved SOLVE_R at a time: each stored q_p is read once per block
    // and applied to the block's rows; every row still subtracts its terms in
    // ascending p, so the values are those of a plain row-by-row solve.
    for (int c = tid; c < C; c += BT) {
        const double* x = th + 6 * c;
        double m = 0.0, ss = 0.0;
        for (int i0 = 0; i0 < n; i0 += SOLVE_R) {
            const int nr = min(SOLVE_R, n - i0);
            double sv[SOLVE_R], qb[SOLVE_R], qv[SOLVE_R], qn[SOLVE_R];
            // the first chunk of stored values is in flight during the
            // covariances below (row 0.. of q; re-read, unused, when i0 == 0)
#pragma unroll
            for (int u = 0; u < SOLVE_R; ++u) qv[u] = qcol[(int64_t)min(u, max(i0 - 1, 0)) * C + c];
#pragma unroll
            for (int r = 0; r < SOLVE_R; ++r) {
                sv[r] = 0.0;
                qb[r] = 0.0;
                if (r < nr) {
                    const double ki = matern52(x, X + 6 * (i0 + r), inv_ls);
                    m += ki * alpha[i0 + r];
                    sv[r] = ki;
                }
            }
            // i0 is a multiple of SOLVE_R: the stored values are read
            // SOLVE_R at a time, the next chunk's loads in flight while the
            // current one is applied (the last chunk is re-read past the end
            // so that every load is unconditional)
            if (i0 > 0) {
                for (int p0 = 0; p0 < i0; p0 += SOLVE_R) {
                    const int pn = min(p0 + SOLVE_R, i0 - SOLVE_R);
#pragma unroll
                    for (int u = 0; u < SOLVE_R; ++u) qn[u] = qcol[(int64_t)(pn + u) * C + c];
                    if (nr == SOLVE_R) {  // every block but the last: no row tests
#pragma unroll
                        for (int u = 0; u < SOLVE_R; ++u)
#pragma unroll
                            for (int r = 0; r < SOLVE_R; ++r) sv[r] -= L[tri(i0 + r, p0 + u)] * qv[u];
                    } else {
#pragma unroll
                        for (int u = 0; u < SOLVE_R; ++u)
#pragma unroll
                            for (int r = 0; r < SOLVE_R; ++r)
                                if (r < nr) sv[r] -= L[tri(i0 + r, p0 + u)] * qv[u];
                    }
#pragma unroll
                    for (int u = 0; u < SOLVE_R; ++u) qv[u] = qn[u];
                }
            }
#pragma unroll
            for (int r = 0; r < SOLVE_R; ++r) {
                if (r < nr) {
                    const double* Li = L + tri(i0 + r, 0);
                    double v = sv[r];
#pragma unroll
                    for (int t = 0; t < r; ++t) v -= Li[i0 + t] * qb[t];
                    const double qi = v / Li[i0 + r];
                    qb[r] = qi;
                    qcol[(int64_t)(i0 + r) * C + c] = qi;
                    ss += qi * qi;
                }
            }
        }
        mu[c] = m;
        const double v = 1.0 - ss;
        s2[c] = v > 0.0 ? v : 0.0;
    }
    __syncthreads();
    // ---- Kriging-believer batch
    for (int m = 0; m < b; ++m) {
        double bv = -1e300;
        int bidx = 0x7fffffff;
        for (int c = tid; c < C; c += BT) {
            if (taken[c]) continue;
            const double u = mu[c] + d.kappa * sqrt(s2[c]);
            if (u > bv || (u == bv && c < bidx)) {
                bv = u;
                bidx = c;
            }
        }
        const int cs = block_argmax(bv, bidx, red_v, red_i);
        const int rows = n + m;  // rows of q so far
        // s2[cs] is read before the barrier: after it, thread cs updates it
        const double dm = sqrt(s2[cs] + d.jitter > 1e-300 ? s2[cs] + d.jitter : 1e-300);
        const double* xs = th + 6 * cs;
        for (int r = tid; r < rows; r += BT) qs[r] = qcol[(int64_t)r * C + cs];
        if (tid == 0) {
            taken[cs] = 1;
            for (int a = 0; a < 6; ++a) pk[6 * m + a] = th[6 * cs + a];
        }
        __syncthreads();
        for (int c = tid; c < C; c += BT) {
            // The column of q is streamed BELIEF_R values at a time: the first
            // chunk is in flight during the covariance, each next chunk during
            // the current one's terms (loads past `rows` re-read row rows - 1
            // and are not used). Terms are subtracted in ascending r, as in a
            // plain loop.
            const double* qc = qcol + c;
            double qv[BELIEF_R], qn[BELIEF_R];
#pragma unroll
            for (int u = 0; u < BELIEF_R; ++u) qv[u] = qc[(int64_t)min(u, rows - 1) * C];
            double s = matern52(th + 6 * c, xs, inv_ls);
            for (int r = 0; r < rows; r += BELIEF_R) {
#pragma unroll
                for (int u = 0; u < BELIEF_R; ++u) qn[u] = qc[(int64_t)min(r + BELIEF_R + u, rows - 1) * C];
                if (r + BELIEF_R <= rows) {
#pragma unroll
                    for (int u = 0; u < BELIEF_R; ++u) s -= qv[u] * qs[r + u];
                } else {
#pragma unroll
                    for (int u = 0; u < BELIEF_R; ++u)
                        if (r + u < rows) s -= qv[u] * qs[r + u];
                }
#pragma unroll
                for (int u = 0; u < BELIEF_R; ++u) qv[u] = qn[u];
            }
            const double u = s / dm;
            qcol[(int64_t)rows * C + c] = u;
            const double v = s2[c] - u * u;
            s2[c] = v > 0.0 ? v : 0.0;
        }
        __syncthreads();
    }
    // ---- rounding (Bernoulli of the fractional part) and dedupe
    const int slot0 = uni(d.slot[pair]);
    for (int m = tid; m < b; m += BT) {
        for (int a = 0; a < 6; ++a) {
            const double v = pk[6 * m + a];
            const double f = floor(v);
            const double u = ph_uniform(d.seed, pair, ST_ROUND, (uint64_t)(slot0 + m), a);
            int c = (int)f + ((u < v - f) ? 1 : 0);
            const int dim = axis_dim(A, B, a);
            rc[6 * m + a] = c < 0 ? 0 : (c > dim - 1 ? dim - 1 : c);
        }
    }
    __syncthreads();
    for (int m = tid; m < b; m += BT) {
        bool dupl = false;
        for (int i = 0; i < n && !dupl; ++i) {
            bool same = true;
            for (int a = 0; a < 6; ++a) same = same && rc[6 * m + a] == (int)X[6 * i + a];
            dupl = same;
        }
        for (int j = 0; j < m && !dupl; ++j) {
            bool same = true;
            for (int a = 0; a < 6; ++a) same = same && rc[6 * m + a] == rc[6 * j + a];
            dupl = same;
        }
        keep[m] = dupl ? 0 : 1;
    }
    __syncthreads();
    if (tid == 0) {
        int q = 0;
        for (int m = 0; m < b; ++m)
            if (keep[m]) {
                for (int a = 0; a < 6; ++a) newc[6 * q + a] = rc[6 * m + a];
                ++q;
            }
        *nnew = q;
    }
    __syncthreads();
    const int nn = uni(*nnew);
    // ---- evaluate and append (th / mu / s2 space is free now)
    double* vals = mu;
    float* svals = reinterpret_cast<float*>(s2);
    eval_cells<KP1>(d, pair, newc, nn, vals, svals, reinterpret_cast<float*>(th));
    __syncthreads();
    for (int m = tid; m < nn; m += BT) {
        for (int a = 0; a < 6; ++a) d.cells[(int64_t)(base + n + m) * 6 + a] = (int16_t)newc[6 * m + a];
        d.yv[base + n + m] = vals[m];
        d.sv[base + n + m] = svals[m];
    }
    if (tid == 0) {
        int bb = d.best[pair];
        double bvv = d.yv[base + bb];
        for (int m = 0; m < nn; ++m)
            if (vals[m] > bvv) {
                bvv = vals[m];
                bb = n + m;
            }
        d.best[pair] = bb;
        d.n_obs[pair] = n + nn;
        d.slot[pair] = slot0 + b;
    }
}

template <int KP1>
__global__ __launch_bounds__(BT) void bos_kernel(BosDev d) {
    extern __shared__ __attribute__((aligned(16))) double sm[];
    const int it = uni(*d.iter);
    if (it >= d.n_iter) return;  // every pair is done
    const int start = uni(d.list_start[it]), count = uni(d.list_count[it]);
    // static stride over the iteration's pairs: at most ceil(count / grid) trips
    for (int q = blockIdx.x; q < count; q += gridDim.x) {
        if (uni(__hip_atomic_load(d.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) != 0) {
            if (threadIdx.x == 0) atomicOr(d.err, 2);
            break;
        }
        const int pair = uni(d.list[start + q]);
        if (pair < 0 || pair >= d.n_pairs) {
            if (threadIdx.x == 0) atomicOr(d.err, 1);
            break;
        }
        if (it == 0)
            bos_init_pair<KP1>(d, pair, sm);
        else
            bos_batch_pair<KP1>(d, pair, it - 1, sm);
        __syncthreads();  // the LDS is reused by the next pair
    }
}

__global__ void bos_advance_kernel(int* iter) {
    if (threadIdx.x == 0) *iter += 1;
}

}  // namespace corr

using namespace corr;

struct bos_state {
    corr_ctx* ctx = nullptr;
    bos_config cfg{};
    int n_pairs = 0, M = 0, kp1 = 0;
    BosDev d{};
    size_t lds_bytes = 0;
    int grid = 0;
    std::vector<void*> allocs;
    // device state arrays (also listed in allocs)
    int16_t* cells = nullptr;
    double* yv = nullptr;
    float* sv = nullptr;
    int* ints = nullptr;  // n_obs, slot, best, n_sched, sched[16], iter
    int* lists = nullptr;  // list_start[n_iter], list_count[n_iter], list[]
    float* prior = nullptr;
    Box* boxes = nullptr;  // [2][n_pairs]
    int* h_stop = nullptr;  // pinned, mapped: the kernels' stop request
    std::vector<Box> hb;   // host copy of the pair boxes
    std::vector<int> h_nsched, h_sched;  // host copy of the schedule
    int n_iter = 0;
    // launch
    int mode = BOS_LAUNCH_GRAPH;
    double timeout_s = 300.0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last = nullptr;  // stream of the latest enqueued work
    bool used = false;
    int steps = 0;
    bool done = false;
    bool stopped = false;  // a wait passed its deadline: no further work is accepted
};


static size_t ints_count(size_t np) { return np * 20 + 8; }

static int bos_alloc(bos_state* st, size_t bytes, void** p) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(CORR_ENOMEM, "bos: allocation of " + std::to_string(bytes) + " bytes failed");
    }
    st->allocs.push_back(*p);
    return CORR_OK;
}

// Wait for the work enqueued on `s` so far, polling an event, and give up with
// CORR_EHIP after `timeout_s` seconds instead of blocking without bound. With
// a stop flag, a wait that passes its deadline asks the BOS kernels to stop at
// their next pair and waits up to another 10 s for them to drain.
static int wait_deadline(hipStream_t s, double timeout_s, const char* what, volatile int* stop = nullptr) {
    hipEvent_t ev = nullptr;
    CORR_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, s);
    if (e != hipSuccess) {
        (void)hipEventDestroy(ev);
        return fail(CORR_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    }
    auto t0 = std::chrono::steady_clock::now();
    bool stopping = false;
    for (;;) {
        e = hipEventQuery(ev);
        if (e == hipSuccess) break;
        if (e != hipErrorNotReady) {
            (void)hipEventDestroy(ev);
            return fail(CORR_EHIP, std::string(what) + ": " + hipGetErrorString(e));
        }
        const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (!stopping && dt > timeout_s && stop) {
            *stop = 1;
            stopping = true;
            t0 = std::chrono::steady_clock::now();
            continue;
        }
        if ((!stopping && dt > timeout_s) || (stopping && dt > 10.0)) {
            (void)hipEventDestroy(ev);
            return fail(CORR_EHIP, std::string(what) + ": the GPU work did not finish within " +
                                       std::to_string(timeout_s) + " s" +
                                       (stopping ? " and did not stop on request" : ""));
        }
        std::this_thread::sleep_for(std::chrono::microseconds(dt < 0.01 ? 20 : 500));
    }
    (void)hipEventDestroy(ev);
    if (stopping)
        return fail(CORR_EHIP, std::string(what) + ": the GPU work did not finish within " +
                                   std::to_string(timeout_s) + " s; it was stopped (the sampler's results are incomplete)");
    return CORR_OK;
}

// Wait with the sampler's deadline; a stop by deadline poisons the sampler.
static int bos_wait(bos_state* st, hipStream_t s, const char* what) {
    const int rc = wait_deadline(s, st->timeout_s, what, st->h_stop);
    if (rc && st->h_stop && *(volatile int*)st->h_stop) st->stopped = true;
    return rc;
}

// Standardise a whole field into state-owned buffers: rows (format fmt,
// stride ld), statistics, and for KSG the sorted rows.
static int bos_standardize(bos_state* st, const corr_field& f, int fmt, int64_t ld, hipStream_t s, float** rows,
                           float** stats, float** sorted) {
    const Box box{0, 0, 0, f.nx, f.ny, f.nz, f.nx, f.ny};
    const int64_t n = box.count();
    int rc = bos_alloc(st, sizeof(float) * 4 * (size_t)n, (void**)stats);
    if (rc) return rc;
    Stats sts = stats_view(*stats, n);
    if ((rc = launch_stats(f, box, true, sts, s))) return rc;
    if ((rc = bos_alloc(st, sizeof(float) * (size_t)(n * ld), (void**)rows))) return rc;
    if ((rc = launch_transpose(f, box, sts, fmt, *rows, nullptr, n, ld, s))) return rc;
    *sorted = nullptr;
    if (fmt == ZF_KSG) {
        if ((rc = bos_alloc(st, sizeof(float) * (size_t)n * ksg_p2(f.M), (void**)sorted))) return rc;
        if ((rc = launch_sort_rows(*rows, ld, n, f.M, *sorted, st->ctx->num_cus, s))) return rc;
    }
    return CORR_OK;
}

template <int KP1>
static const void* bos_kernel_ptr() {
    return (const void*)bos_kernel<KP1>;
}

static const void* bos_kernel_for(int kp1) {
    switch (kp1) {
        case 0: return bos_kernel_ptr<0>();
        case 4: return bos_kernel_ptr<4>();
        case 8: return bos_kernel_ptr<8>();
        case 11: return bos_kernel_ptr<11>();
        case 12: return bos_kernel_ptr<12>();
        case 16: return bos_kernel_ptr<16>();
        case 24: return bos_kernel_ptr<24>();
        default: return bos_kernel_ptr<32>();
    }
}

static void bos_launch_kernel(bos_state* st, hipStream_t s) {
    const dim3 grid((unsigned)st->grid), block(BT);
    switch (st->kp1) {
        case 0: bos_kernel<0><<<grid, block, st->lds_bytes, s>>>(st->d); break;
        case 4: bos_kernel<4><<<grid, block, st->lds_bytes, s>>>(st->d); break;
        case 8: bos_kernel<8><<<grid, block, st->lds_bytes, s>>>(st->d); break;
        case 11: bos_kernel<11><<<grid, block, st->lds_bytes, s>>>(st->d); break;
        case 12: bos_kernel<12><<<grid, block, st->lds_bytes, s>>>(st->d); break;
        case 16: bos_kernel<16><<<grid, block, st->lds_bytes, s>>>(st->d); break;
        case 24: bos_kernel<24><<<grid, block, st->lds_bytes, s>>>(st->d); break;
        default: bos_kernel<32><<<grid, block, st->lds_bytes, s>>>(st->d); break;
    }
}

// The uneven batch schedule of one pair (drawn from the seed): batches of
// 8 * p, p = 1 + floor(u * min(8, units left)), until the n_total - n_init
// acquired samples are placed. Returns the number of batches.
static int pair_schedule(const bos_config& c, int pair, int* sched16) {
    int units = (c.n_total - c.n_init) / 8, i = 0;
    while (units > 0 && i < 16) {
        const int mx = units < 8 ? units : 8;
        const int p = 1 + (int)(ph_uniform(c.seed, (uint64_t)pair, ST_SCHED, (uint64_t)i, 0) * mx);
        sched16[i] = 8 * p;
        units -= p;
        ++i;
    }
    return i;
}

// Per iteration, the pairs that sample in it, costliest first (the estimate
// counts the posterior solves, the believer updates and the factorisation at
// the pair's largest possible observation count).
static void build_lists(const bos_config& c, int np, const std::vector<int>& nsched, const std::vector<int>& sched,
                        int* n_iter, std::vector<int>& out) {
    int T = 0;
    for (int p = 0; p < np; ++p) T = std::max(T, nsched[p]);
    T += 1;  // the initial design
    std::vector<int> start(T), count(T), list;
    list.reserve((size_t)np * T);
    const double C = (double)(c.n_uniform + c.n_local);
    for (int t = 0; t < T; ++t) {
        start[t] = (int)list.size();
        std::vector<std::pair<double, int>> cost;
        for (int p = 0; p < np; ++p) {
            if (t == 0) {
                cost.emplace_back(0.0, p);
            } else if (t - 1 < nsched[p]) {
                double n = c.n_init;
                for (int u = 0; u < t - 1; ++u) n += sched[(size_t)p * 16 + u];
                const double b = sched[(size_t)p * 16 + t - 1];
                cost.emplace_back(C * (0.5 * n * n + 6.0 * n) + b * C * (n + 0.5 * b) + n * n * n / 6.0, p);
            }
        }
        std::stable_sort(cost.begin(), cost.end(),
                         [](const std::pair<double, int>& a, const std::pair<double, int>& b) { return a.first > b.first; });
        for (auto& e : cost) list.push_back(e.second);
        count[t] = (int)list.size() - start[t];
    }
    *n_iter = T;
    out.clear();
    out.insert(out.end(), start.begin(), start.end());
    out.insert(out.end(), count.begin(), count.end());
    out.insert(out.end(), list.begin(), list.end());
}

extern "C" {

void bos_config_default(bos_config* c) {
    if (!c) return;
    c->measure = CORR_PEARSON;
    c->k = 10;
    c->n_init = 20;
    c->n_total = 100;
    c->n_uniform = 384;
    c->n_local = 128;
    c->kappa = 0.5;
    c->lengthscale = 3.0;
    c->local_sd = 1.0;
    c->jitter = 1e-6;
    c->seed = 1;
}

void bos_destroy(bos_state* st) {
    if (!st) return;
    // never free memory that enqueued work may still use: if that work does
    // not finish in time the buffers are left allocated
    if (st->used && bos_wait(st, st->last, "bos_destroy") != CORR_OK && !st->stopped) return;
    if (st->exec) (void)hipGraphExecDestroy(st->exec);
    if (st->graph) (void)hipGraphDestroy(st->graph);
    if (st->cap) (void)hipStreamDestroy(st->cap);
    for (void* p : st->allocs) (void)hipFree(p);
    if (st->h_stop) (void)hipHostFree(st->h_stop);
    delete st;
}

int bos_create(corr_ctx* ctx, const corr_field* A, const corr_field* B, const corr_region* regions,
               int32_t n_regions, const int32_t* region_pairs, int32_t n_pairs, const bos_config* cfg,
               bos_state** out, corr_stream_t stream) {
    if (!out) return fail(CORR_EINVAL, "bos_create: null out");
    *out = nullptr;
    if (!ctx || !A || !B || !regions || !region_pairs || !cfg) return fail(CORR_EINVAL, "bos_create: null argument");
    if (!A->data || !B->data) return fail(CORR_EINVAL, "bos_create: null field data");
    if (A->dtype != CORR_F32 && A->dtype != CORR_F16) return fail(CORR_EUNSUPPORTED, "bos_create: dtype");
    if (B->dtype != CORR_F32 && B->dtype != CORR_F16) return fail(CORR_EUNSUPPORTED, "bos_create: dtype");
    if (A->M != B->M || A->M < 2) return fail(CORR_EINVAL, "bos_create: bad member count");
    if (A->M > 1024) return fail(CORR_EUNSUPPORTED, "bos_create: M > 1024");
    if (n_regions < 1 || n_pairs < 1) return fail(CORR_EINVAL, "bos_create: empty region or pair list");
    const bos_config& c = *cfg;
    if (c.measure != CORR_PEARSON && c.measure != CORR_KSG) return fail(CORR_EINVAL, "bos_create: measure");
    if (c.measure == CORR_KSG && (c.k < 1 || c.k > A->M - 1 || c.k > 31)) return fail(CORR_EINVAL, "bos_create: k");
    if (c.n_init < 2 || c.n_total > 128 || c.n_total - c.n_init < 8 || (c.n_total - c.n_init) % 8)
        return fail(CORR_EINVAL, "bos_create: n_init / n_total");
    // a batch picks up to 64 distinct candidates
    if (c.n_uniform < 0 || c.n_local < 0 || c.n_uniform + c.n_local < 64 || c.n_uniform + c.n_local > 1024)
        return fail(CORR_EINVAL, "bos_create: n_uniform + n_local must be in [64, 1024]");
    if (!(c.kappa >= 0.0) || !(c.lengthscale > 0.0) || !(c.local_sd >= 0.0) || !(c.jitter > 0.0))
        return fail(CORR_EINVAL, "bos_create: kappa / lengthscale / local_sd / jitter");
    for (int r = 0; r < n_regions; ++r) {
        const corr_region& g = regions[r];
        if (g.dx < 1 || g.dy < 1 || g.dz < 1 || g.x0 < 0 || g.y0 < 0 || g.z0 < 0)
            return fail(CORR_EINVAL, "bos_create: empty or negative region");
        if (g.dx > 32767 || g.dy > 32767 || g.dz > 32767) return fail(CORR_EUNSUPPORTED, "bos_create: region too large");
    }
    bos_state* st = new (std::nothrow) bos_state();
    if (!st) return fail(CORR_ENOMEM, "bos_create: host allocation");
    st->ctx = ctx;
    st->cfg = c;
    st->n_pairs = n_pairs;
    st->M = A->M;
    st->kp1 = c.measure == CORR_PEARSON ? 0 : (c.k + 1 == 11 ? 11 : (c.k + 1 <= 4 ? 4 : c.k + 1 <= 8 ? 8 : c.k + 1 <= 12 ? 12 : c.k + 1 <= 16 ? 16 : c.k + 1 <= 24 ? 24 : 32));
    st->hb.resize(2 * (size_t)n_pairs);
    for (int p = 0; p < n_pairs; ++p) {
        const int ia = region_pairs[2 * p], ib = region_pairs[2 * p + 1];
        if (ia < 0 || ia >= n_regions || ib < 0 || ib >= n_regions) {
            delete st;
            return fail(CORR_EINVAL, "bos_create: region index out of range");
        }
        const corr_region& ra = regions[ia];
        const corr_region& rb = regions[ib];
        if (ra.x0 + ra.dx > A->nx || ra.y0 + ra.dy > A->ny || ra.z0 + ra.dz > A->nz || rb.x0 + rb.dx > B->nx ||
            rb.y0 + rb.dy > B->ny || rb.z0 + rb.dz > B->nz) {
            delete st;
            return fail(CORR_EINVAL, "bos_create: region outside the grid");
        }
        st->hb[p] = Box{ra.x0, ra.y0, ra.z0, ra.dx, ra.dy, ra.dz, A->nx, A->ny};
        st->hb[n_pairs + p] = Box{rb.x0, rb.y0, rb.z0, rb.dx, rb.dy, rb.dz, B->nx, B->ny};
    }
    hipStream_t s = (hipStream_t)stream;
    st->last = s;
    int rc = CORR_OK;
    BosDev& d = st->d;
    d.measure = c.measure;
    d.k = c.k;
    d.n_init = c.n_init;
    d.n_total = c.n_total;
    d.n_unif = c.n_uniform;
    d.n_local = c.n_local;
    d.C = c.n_uniform + c.n_local;
    d.kappa = c.kappa;
    d.ls = c.lengthscale;
    d.local_sd = c.local_sd;
    d.jitter = c.jitter;
    d.seed = c.seed;
    d.n_pairs = n_pairs;
    d.M = A->M;
    d.psi = ctx->psi;
    // standardised rows
    const bool ksg = c.measure == CORR_KSG;
    const int fmt = ksg ? ZF_KSG : ZF_F32;
    const int64_t ld = (A->M + 3) / 4 * 4;
    float *ra_rows, *ra_stats, *ra_sorted, *rb_rows, *rb_stats, *rb_sorted;
    st->used = true;
    rc = bos_standardize(st, *A, fmt, ld, s, &ra_rows, &ra_stats, &ra_sorted);
    if (!rc) {
        const bool same = A->data == B->data && A->dtype == B->dtype && A->nx == B->nx && A->ny == B->ny &&
                          A->nz == B->nz && A->member_stride == B->member_stride;
        if (same) {
            rb_rows = ra_rows;
            rb_stats = ra_stats;
            rb_sorted = ra_sorted;
        } else {
            rc = bos_standardize(st, *B, fmt, ld, s, &rb_rows, &rb_stats, &rb_sorted);
        }
    }
    if (rc) {
        bos_destroy(st);
        return rc;
    }
    const int64_t na_pts = (int64_t)A->nx * A->ny * A->nz, nb_pts = (int64_t)B->nx * B->ny * B->nz;
    d.za = ra_rows;
    d.zb = rb_rows;
    d.ld = ld;
    d.sa = ra_sorted;
    d.sb = rb_sorted;
    d.p2 = ksg ? ksg_p2(A->M) : 0;
    d.inv_a = ra_stats + na_pts;  // stats layout: mu32, inv32, rs32, sigma
    d.inv_b = rb_stats + nb_pts;
    // host schedule and per-iteration pair lists
    const size_t np = (size_t)n_pairs;
    std::vector<int> hints(ints_count(np), 0);
    st->h_nsched.assign(np, 0);
    st->h_sched.assign(np * 16, 0);
    for (int p = 0; p < n_pairs; ++p) st->h_nsched[p] = pair_schedule(c, p, &st->h_sched[(size_t)p * 16]);
    for (size_t p = 0; p < np; ++p) {
        hints[3 * np + p] = st->h_nsched[p];
        for (int i = 0; i < 16; ++i) hints[4 * np + 16 * p + i] = st->h_sched[16 * p + i];
    }
    std::vector<int> hl;
    build_lists(c, n_pairs, st->h_nsched, st->h_sched, &st->n_iter, hl);
    // state arrays
    if (!rc) rc = bos_alloc(st, sizeof(int16_t) * np * c.n_total * 6, (void**)&st->cells);
    if (!rc) rc = bos_alloc(st, sizeof(double) * np * c.n_total, (void**)&st->yv);
    if (!rc) rc = bos_alloc(st, sizeof(float) * np * c.n_total, (void**)&st->sv);
    if (!rc) rc = bos_alloc(st, sizeof(int) * ints_count(np), (void**)&st->ints);
    if (!rc) rc = bos_alloc(st, sizeof(int) * hl.size(), (void**)&st->lists);
    if (!rc) rc = bos_alloc(st, sizeof(float) * np * 6, (void**)&st->prior);
    if (!rc) rc = bos_alloc(st, sizeof(Box) * 2 * np, (void**)&st->boxes);
    if (!rc) {
        void* dstop = nullptr;
        hipError_t he = hipHostMalloc((void**)&st->h_stop, sizeof(int), hipHostMallocMapped | hipHostMallocCoherent);
        if (he == hipSuccess) {
            *(volatile int*)st->h_stop = 0;
            he = hipHostGetDevicePointer(&dstop, st->h_stop, 0);
        } else {
            st->h_stop = nullptr;
        }
        if (he != hipSuccess) {
            (void)hipGetLastError();
            rc = fail(CORR_ENOMEM, std::string("bos_create: pinned stop flag: ") + hipGetErrorString(he));
        }
        d.stop = (const int*)dstop;
    }
    if (rc) {
        bos_destroy(st);
        return rc;
    }
    d.cells = st->cells;
    d.yv = st->yv;
    d.sv = st->sv;
    d.n_obs = st->ints;
    d.slot = st->ints + np;
    d.best = st->ints + 2 * np;
    d.n_sched = st->ints + 3 * np;
    d.sched = st->ints + 4 * np;  // [np][16]
    d.iter = st->ints + 20 * np;
    d.err = st->ints + 20 * np + 1;
    d.n_iter = st->n_iter;
    d.list_start = st->lists;
    d.list_count = st->lists + st->n_iter;
    d.list = st->lists + 2 * st->n_iter;
    d.prior = nullptr;
    d.ba = st->boxes;
    d.bb = st->boxes + np;
    // LDS layout (doubles)
    const int NT = c.n_total, C = d.C;
    int off = 0;
    d.off_L = off; off += NT * (NT + 1) / 2;
    d.off_X = off; off += 6 * NT;
    d.off_y = off; off += NT;
    d.off_a = off; off += NT;
    d.off_qs = off; off += NT;
    d.off_pk = off; off += 6 * 64;
    d.off_red = off; off += BT + BT / 2;
    d.off_mu = off; off += C;
    d.off_s2 = off; off += C;
    d.off_th = off;
    {
        // candidates theta, reused afterwards as the per-wave evaluation staging
        const int stage_doubles = ksg ? (NW * (2 * ((A->M + 1) & ~1) + 2 * d.p2) + 1) / 2 : 0;
        off += std::max(6 * C, stage_doubles);
    }
    d.off_misc = off;
    // ints: batch (taken[C], rounded, keep, new cells, count) or initial
    // design (cells, duplicate flags, unique cells, count)
    off += (std::max(C + 6 * 64 + 64 + 6 * 64 + 8, 13 * c.n_init + 8) + 1) / 2 + 4;
    d.lds_doubles = off;
    st->lds_bytes = (size_t)off * sizeof(double);
    if (st->lds_bytes > 160 * 1024) {
        bos_destroy(st);
        return fail(CORR_EUNSUPPORTED, "bos_create: configuration needs more than 160 KiB of LDS");
    }
    int per_cu = 1;
    if ((rc = kernel_setup(bos_kernel_for(st->kp1), st->lds_bytes, BT, &per_cu))) {
        bos_destroy(st);
        return rc;
    }
    st->grid = std::min(n_pairs, ctx->num_cus * std::max(1, std::min(per_cu, 2)));
    if ((rc = bos_alloc(st, sizeof(double) * (size_t)st->grid * NT * C, (void**)&d.qbuf))) {
        bos_destroy(st);
        return rc;
    }
    hipError_t e = hipMemcpyAsync(st->boxes, st->hb.data(), sizeof(Box) * 2 * np, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(st->ints, hints.data(), sizeof(int) * hints.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(st->lists, hl.data(), sizeof(int) * hl.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(st->prior, 0xff, sizeof(float) * np * 6, s);  // -nan: no prior
    if (e != hipSuccess) {
        bos_destroy(st);
        return fail(CORR_EHIP, std::string("bos_create: ") + hipGetErrorString(e));
    }
    // the host buffers above are released on return: wait for the copies
    if ((rc = bos_wait(st, s, "bos_create"))) {
        bos_destroy(st);
        return rc;
    }
    *out = st;
    return CORR_OK;
}

int bos_set_launch(bos_state* st, int32_t mode, double timeout_s) {
    if (!st) return fail(CORR_EINVAL, "bos_set_launch: null state");
    if (mode != BOS_LAUNCH_GRAPH && mode != BOS_LAUNCH_PLAIN) return fail(CORR_EINVAL, "bos_set_launch: mode");
    if (!(timeout_s > 0.0)) return fail(CORR_EINVAL, "bos_set_launch: timeout must be positive");
    st->mode = mode;
    st->timeout_s = timeout_s;
    return CORR_OK;
}

int bos_set_prior(bos_state* st, const float* cells) {
    if (!st || !cells) return fail(CORR_EINVAL, "bos_set_prior: null argument");
    if (st->steps > 0) return fail(CORR_ESTATE, "bos_set_prior: sampling has started");
    CORR_HIP(hipMemcpy(st->prior, cells, sizeof(float) * 6 * (size_t)st->n_pairs, hipMemcpyHostToDevice));
    st->d.prior = st->prior;
    if (st->exec) {  // the kernel arguments changed: capture again
        (void)hipGraphExecDestroy(st->exec);
        (void)hipGraphDestroy(st->graph);
        st->exec = nullptr;
        st->graph = nullptr;
    }
    return CORR_OK;
}

static int bos_capture(bos_state* st) {
    if (!st->cap) CORR_HIP(hipStreamCreateWithFlags(&st->cap, hipStreamNonBlocking));
    CORR_HIP(hipStreamBeginCapture(st->cap, hipStreamCaptureModeThreadLocal));
    bos_launch_kernel(st, st->cap);
    bos_advance_kernel<<<1, 64, 0, st->cap>>>(st->d.iter);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st->cap, &g);
    if (e != hipSuccess) return fail(CORR_EHIP, std::string("bos: graph capture: ") + hipGetErrorString(e));
    st->graph = g;
    CORR_HIP(hipGraphInstantiate(&st->exec, g, nullptr, nullptr, 0));
    return CORR_OK;
}

int bos_sample_step(bos_state* st, corr_stream_t stream, int32_t* n_active_out) {
    if (!st) return fail(CORR_EINVAL, "bos_sample_step: null state");
    if (st->stopped) return fail(CORR_ESTATE, "bos_sample_step: the sampler was stopped after a deadline passed");
    hipStream_t s = (hipStream_t)stream;
    if (st->done) {
        if (n_active_out) *n_active_out = 0;
        return CORR_OK;
    }
    if (st->mode == BOS_LAUNCH_GRAPH) {
        if (!st->exec) {
            int rc = bos_capture(st);
            if (rc) return rc;
        }
        CORR_HIP(hipGraphLaunch(st->exec, s));
    } else {
        bos_launch_kernel(st, s);
        CORR_LAUNCH_CHECK();
        bos_advance_kernel<<<1, 64, 0, s>>>(st->d.iter);
        CORR_LAUNCH_CHECK();
    }
    st->last = s;
    // pairs with batches left after this iteration (known from the schedule)
    const int it = st->steps;
    st->steps += 1;
    int active = 0;
    for (int p = 0; p < st->n_pairs; ++p) active += st->h_nsched[p] > it ? 1 : 0;
    if (active == 0 || st->steps >= st->n_iter) st->done = true;
    if (n_active_out) *n_active_out = st->done ? 0 : active;
    return CORR_OK;
}

int bos_run(bos_state* st, corr_stream_t stream) {
    if (!st) return fail(CORR_EINVAL, "bos_run: null state");
    if (st->stopped) return fail(CORR_ESTATE, "bos_run: the sampler was stopped after a deadline passed");
    while (!st->done) {
        int rc = bos_sample_step(st, stream, nullptr);
        if (rc) return rc;
    }
    return bos_wait(st, (hipStream_t)stream, "bos_run");
}

int bos_results(bos_state* st, corr_max* out, corr_stream_t stream) {
    if (!st || !out) return fail(CORR_EINVAL, "bos_results: null argument");
    if (st->stopped) return fail(CORR_ESTATE, "bos_results: the sampler was stopped after a deadline passed");
    hipStream_t s = (hipStream_t)stream;
    const size_t np = (size_t)st->n_pairs;
    const int NT = st->cfg.n_total;
    std::vector<int> ints(ints_count(np));
    std::vector<int16_t> cells(np * NT * 6);
    std::vector<double> yv(np * NT);
    std::vector<float> sv(np * NT);
    int rc = bos_wait(st, s, "bos_results");
    if (rc) return rc;
    CORR_HIP(hipMemcpyAsync(ints.data(), st->ints, sizeof(int) * ints.size(), hipMemcpyDeviceToHost, s));
    CORR_HIP(hipMemcpyAsync(cells.data(), st->cells, sizeof(int16_t) * cells.size(), hipMemcpyDeviceToHost, s));
    CORR_HIP(hipMemcpyAsync(yv.data(), st->yv, sizeof(double) * yv.size(), hipMemcpyDeviceToHost, s));
    CORR_HIP(hipMemcpyAsync(sv.data(), st->sv, sizeof(float) * sv.size(), hipMemcpyDeviceToHost, s));
    if ((rc = bos_wait(st, s, "bos_results"))) return rc;
    if (ints[20 * np + 1] & 1) return fail(CORR_ESTATE, "bos_results: the kernels found inconsistent pair state");
    if (ints[20 * np + 1] & 2) return fail(CORR_ESTATE, "bos_results: the kernels were stopped; results are incomplete");
    for (size_t p = 0; p < np; ++p) {
        const int n = ints[p], b = ints[2 * np + p];
        corr_max& o = out[p];
        if (n <= 0) {
            o.value = 0.0f;
            o.signed_value = 0.0f;
            o.pa = o.pb = -1;
            o.n_evaluated = 0;
            continue;
        }
        const int16_t* c = &cells[(p * NT + b) * 6];
        const Box& A = st->hb[p];
        const Box& B = st->hb[np + p];
        o.value = (float)yv[p * NT + b];
        o.signed_value = sv[p * NT + b];
        o.pa = (A.x0 + c[0]) + A.nx * ((A.y0 + c[1]) + A.ny * (A.z0 + c[2]));
        o.pb = (B.x0 + c[3]) + B.nx * ((B.y0 + c[4]) + B.ny * (B.z0 + c[5]));
        o.n_evaluated = n;
    }
    return CORR_OK;
}

int bos_history(bos_state* st, int32_t pair, int32_t* cells, float* values, int32_t* n_out, corr_stream_t stream) {
    if (!st || !cells || !values || !n_out) return fail(CORR_EINVAL, "bos_history: null argument");
    if (st->stopped) return fail(CORR_ESTATE, "bos_history: the sampler was stopped after a deadline passed");
    if (pair < 0 || pair >= st->n_pairs) return fail(CORR_EINVAL, "bos_history: pair out of range");
    hipStream_t s = (hipStream_t)stream;
    const int NT = st->cfg.n_total;
    std::vector<int> n(1, 0);
    std::vector<int16_t> c(NT * 6);
    std::vector<double> y(NT);
    int rc = bos_wait(st, s, "bos_history");
    if (rc) return rc;
    CORR_HIP(hipMemcpyAsync(n.data(), st->ints + pair, sizeof(int), hipMemcpyDeviceToHost, s));
    CORR_HIP(hipMemcpyAsync(c.data(), st->cells + (size_t)pair * NT * 6, sizeof(int16_t) * NT * 6,
                            hipMemcpyDeviceToHost, s));
    CORR_HIP(hipMemcpyAsync(y.data(), st->yv + (size_t)pair * NT, sizeof(double) * NT, hipMemcpyDeviceToHost, s));
    if ((rc = bos_wait(st, s, "bos_history"))) return rc;
    for (int i = 0; i < n[0]; ++i) {
        for (int a = 0; a < 6; ++a) cells[6 * i + a] = c[6 * i + a];
        values[i] = (float)y[i];
    }
    *n_out = n[0];
    return CORR_OK;
}

int bos_schedule(bos_state* st, int32_t* sched_out, int32_t* n_batches_out) {
    if (!st || !sched_out || !n_batches_out) return fail(CORR_EINVAL, "bos_schedule: null argument");
    for (int p = 0; p < st->n_pairs; ++p) {
        n_batches_out[p] = st->h_nsched[p];
        for (int i = 0; i < 16; ++i) sched_out[16 * p + i] = st->h_sched[16 * (size_t)p + i];
    }
    return CORR_OK;
}

static const char kBosMagic[8] = {'B', 'O', 'S', 'S', 'T', 'A', 'T', '2'};

int bos_save(bos_state* st, const char* path, corr_stream_t stream) {
    if (!st || !path) return fail(CORR_EINVAL, "bos_save: null argument");
    if (st->stopped) return fail(CORR_ESTATE, "bos_save: the sampler was stopped after a deadline passed");
    hipStream_t s = (hipStream_t)stream;
    const size_t np = (size_t)st->n_pairs, NT = (size_t)st->cfg.n_total;
    std::vector<int> ints(ints_count(np));
    std::vector<int16_t> cells(np * NT * 6);
    std::vector<double> yv(np * NT);
    std::vector<float> sv(np * NT), prior(np * 6);
    int rc = bos_wait(st, s, "bos_save");
    if (rc) return rc;
    CORR_HIP(hipMemcpyAsync(ints.data(), st->ints, sizeof(int) * ints.size(), hipMemcpyDeviceToHost, s));
    CORR_HIP(hipMemcpyAsync(cells.data(), st->cells, sizeof(int16_t) * cells.size(), hipMemcpyDeviceToHost, s));
    CORR_HIP(hipMemcpyAsync(yv.data(), st->yv, sizeof(double) * yv.size(), hipMemcpyDeviceToHost, s));
    CORR_HIP(hipMemcpyAsync(sv.data(), st->sv, sizeof(float) * sv.size(), hipMemcpyDeviceToHost, s));
    CORR_HIP(hipMemcpyAsync(prior.data(), st->prior, sizeof(float) * prior.size(), hipMemcpyDeviceToHost, s));
    if ((rc = bos_wait(st, s, "bos_save"))) return rc;
    FILE* f = fopen(path, "wb");
    if (!f) return fail(CORR_EINVAL, std::string("bos_save: cannot write ") + path);
    bool ok = fwrite(kBosMagic, 1, 8, f) == 8;
    ok = ok && fwrite(&st->cfg, sizeof(bos_config), 1, f) == 1;
    ok = ok && fwrite(&st->n_pairs, sizeof(int), 1, f) == 1;
    ok = ok && fwrite(&st->M, sizeof(int), 1, f) == 1;
    ok = ok && fwrite(&st->steps, sizeof(int), 1, f) == 1;
    int has_prior = st->d.prior ? 1 : 0, done = st->done ? 1 : 0;
    ok = ok && fwrite(&has_prior, sizeof(int), 1, f) == 1 && fwrite(&done, sizeof(int), 1, f) == 1;
    ok = ok && fwrite(st->hb.data(), sizeof(Box), st->hb.size(), f) == st->hb.size();
    ok = ok && fwrite(ints.data(), sizeof(int), ints.size(), f) == ints.size();
    ok = ok && fwrite(cells.data(), sizeof(int16_t), cells.size(), f) == cells.size();
    ok = ok && fwrite(yv.data(), sizeof(double), yv.size(), f) == yv.size();
    ok = ok && fwrite(sv.data(), sizeof(float), sv.size(), f) == sv.size();
    ok = ok && fwrite(prior.data(), sizeof(float), prior.size(), f) == prior.size();
    fclose(f);
    if (!ok) return fail(CORR_EINVAL, std::string("bos_save: write failed for ") + path);
    return CORR_OK;
}

int bos_load(bos_state* st, const char* path, corr_stream_t stream) {
    if (!st || !path) return fail(CORR_EINVAL, "bos_load: null argument");
    if (st->stopped) return fail(CORR_ESTATE, "bos_load: the sampler was stopped after a deadline passed");
    hipStream_t s = (hipStream_t)stream;
    FILE* f = fopen(path, "rb");
    if (!f) return fail(CORR_EINVAL, std::string("bos_load: cannot read ") + path);
    const size_t np = (size_t)st->n_pairs, NT = (size_t)st->cfg.n_total;
    char magic[8];
    bos_config cfg;
    int n_pairs = 0, M = 0, steps = 0, has_prior = 0, done = 0;
    std::vector<Box> hb(st->hb.size());
    std::vector<int> ints(ints_count(np));
    std::vector<int16_t> cells(np * NT * 6);
    std::vector<double> yv(np * NT);
    std::vector<float> sv(np * NT), prior(np * 6);
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kBosMagic, 8) == 0;
    ok = ok && fread(&cfg, sizeof(bos_config), 1, f) == 1;
    ok = ok && fread(&n_pairs, sizeof(int), 1, f) == 1 && fread(&M, sizeof(int), 1, f) == 1;
    ok = ok && fread(&steps, sizeof(int), 1, f) == 1;
    ok = ok && fread(&has_prior, sizeof(int), 1, f) == 1 && fread(&done, sizeof(int), 1, f) == 1;
    ok = ok && n_pairs == st->n_pairs && M == st->M && memcmp(&cfg, &st->cfg, sizeof(bos_config)) == 0;
    ok = ok && fread(hb.data(), sizeof(Box), hb.size(), f) == hb.size() &&
         memcmp(hb.data(), st->hb.data(), sizeof(Box) * hb.size()) == 0;
    ok = ok && fread(ints.data(), sizeof(int), ints.size(), f) == ints.size();
    ok = ok && fread(cells.data(), sizeof(int16_t), cells.size(), f) == cells.size();
    ok = ok && fread(yv.data(), sizeof(double), yv.size(), f) == yv.size();
    ok = ok && fread(sv.data(), sizeof(float), sv.size(), f) == sv.size();
    ok = ok && fread(prior.data(), sizeof(float), prior.size(), f) == prior.size();
    ok = ok && steps >= 0 && steps <= st->n_iter && ints[20 * np] == steps;
    fclose(f);
    if (!ok) return fail(CORR_EINVAL, std::string("bos_load: file does not match this sampler: ") + path);
    int rc = bos_wait(st, s, "bos_load");
    if (rc) return rc;
    CORR_HIP(hipMemcpyAsync(st->ints, ints.data(), sizeof(int) * ints.size(), hipMemcpyHostToDevice, s));
    CORR_HIP(hipMemcpyAsync(st->cells, cells.data(), sizeof(int16_t) * cells.size(), hipMemcpyHostToDevice, s));
    CORR_HIP(hipMemcpyAsync(st->yv, yv.data(), sizeof(double) * yv.size(), hipMemcpyHostToDevice, s));
    CORR_HIP(hipMemcpyAsync(st->sv, sv.data(), sizeof(float) * sv.size(), hipMemcpyHostToDevice, s));
    CORR_HIP(hipMemcpyAsync(st->prior, prior.data(), sizeof(float) * prior.size(), hipMemcpyHostToDevice, s));
    if ((rc = bos_wait(st, s, "bos_load"))) return rc;
    st->last = s;
    st->steps = steps;
    st->done = done != 0;
    st->d.prior = has_prior ? st->prior : nullptr;
    if (st->exec) {
        (void)hipGraphExecDestroy(st->exec);
        (void)hipGraphDestroy(st->graph);
        st->exec = nullptr;
        st->graph = nullptr;
    }
    return CORR_OK;
}

}  // extern "C"
