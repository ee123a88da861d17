// Kraskov (KSG) mutual information per point pair (Sec. 3.2).
//
// For pair (a, b) the M joint samples (x_i, y_i) are the z-scored member
// values of a and b. For each i: eps_i is the k-th smallest Chebyshev
// distance max(|x_i - x_j|, |y_i - y_j|) over j != i; n_x,i and n_y,i count
// the j != i with marginal distance strictly below eps_i; the estimate is
// psi(M) + psi(k) - mean_i[psi(n_x,i + 1) + psi(n_y,i + 1)].
//
// Design (gfx950, wave64; bound by VALU issue, chiefly the insertion
// network's v_med3_f32, which issues once per 4 cycles per SIMD where
// add/sub/min/max/FMA issue about every 2.5):
//  - every wave streams through its own contiguous range of pairs; the
//    range's (pair, sample) items are laid densely over the lanes, 64 per
//    trip, so a trip may cover the tail of one pair and the head of the next
//    and no lane idles except in the range's last trip. Waves never wait for
//    one another (the only workgroup barrier is the digamma table load);
//  - a pair is staged into a small per-wave ring of LDS slots just before the
//    first trip that reaches it: its joint samples (x_j, y_j) twice in a row
//    (j = 0..M-1, then again) and both marginals sorted ascending (sorted once
//    per point, not per pair, by sort_rows_kernel); after the trip holding its
//    last item the wave reduces its digamma terms and the slot is reused;
//  - for large M the items of each pair are padded to a multiple of 64 so a
//    trip never straddles two pairs and one slot per wave suffices; each
//    lane then sums its own samples' digamma terms, so the layout keeps no
//    count array and takes the table from global memory, and the smaller
//    workgroups fit more waves per CU;
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
//  - each item's (n_x, n_y) is kept in LDS; the wave then sums a pair's FP64
//    digamma terms (integer-argument table) in a fixed order (lane l takes
//    samples l, l + 64, ..., then a fixed xor tree), so MI is deterministic.
// Distances are plain FP32 subtract/abs/max (no contraction). The unit is
// compiled with IEEE mode off: every operand is finite or +inf, for which
// min/max/med3 give the same results, and no NaN quieting is needed.
#include "common.h"

namespace corr {

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
// so their LDS reads overlap. P2 > 0 fixes the row length at compile time
// (the probes then use immediate LDS offsets); P2 == 0 reads it from p2.
template <int P2>
__device__ __forceinline__ void run_counts(const float* sx, const float* sy, int p2, float x, float y, float eps,
                                           int& cx, int& cy) {
    int lx = 0, ux = 0, ly = 0, uy = 0;
    if constexpr (P2 > 0) {
#pragma unroll
        for (int step = P2 >> 1; step >= 1; step >>= 1) {
            const float a0 = sx[lx + step - 1], a1 = sx[ux + step - 1];
            const float b0 = sy[ly + step - 1], b1 = sy[uy + step - 1];
            lx += (x - a0 < eps) ? 0 : step;
            ux += (x - a1 > -eps) ? step : 0;
            ly += (y - b0 < eps) ? 0 : step;
            uy += (y - b1 > -eps) ? step : 0;
        }
    } else {
        for (int step = p2 >> 1; step >= 1; step >>= 1) {
            const float a0 = sx[lx + step - 1], a1 = sx[ux + step - 1];
            const float b0 = sy[ly + step - 1], b1 = sy[uy + step - 1];
            lx += (x - a0 < eps) ? 0 : step;
            ux += (x - a1 > -eps) ? step : 0;
            ly += (y - b0 < eps) ? 0 : step;
            uy += (y - b1 > -eps) ? step : 0;
        }
    }
    cx = ux - lx;
    cy = uy - ly;
}

struct KsgLayout {
    int mdup;     // float2 entries of the doubled sample row (2 M)
    int p2;       // power of two > M (sorted marginals)
    int stride;   // items per pair: M (packed) or M rounded up to 64 (padded)
    int pad;      // padded items: one slot, per-lane digamma sums, table in global memory
    int ring;     // LDS pair slots per wave
    int slot_f;   // floats per pair slot
    int wave_f;   // floats per wave (slots, packed counts, pair info)
    int psi_f;    // floats of the block-shared digamma table (0 when padded)
    int waves;    // waves per workgroup
};

// Orders LDS accesses of one wave across lanes (a compiler barrier; the LDS
// executes one wave's operations in issue order).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// PAD: items padded to a multiple of 64 per pair (large M). Each trip then
// belongs to one pair, lane l meets samples l, l + 64, ... in order and sums
// their digamma terms itself (the order of the packed reduction), so no count
// array is kept and the digamma table is read from global memory: the
// smaller LDS footprint lets more waves share a CU.
template <int KP, int P2, bool PAD>
__global__ __launch_bounds__(256) void ksg_kernel(KsgArgs a, int64_t n_total, KsgLayout L, int64_t n_waves) {
    extern __shared__ __attribute__((aligned(16))) float lds_f[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // block-shared: digamma table psi[0..M] (FP64, packed layout only), then
    // per wave: pair slots, packed counts (packed layout only), per-pair
    // (la, lb, state, in_max)
    const double* psi = a.psi;
    if constexpr (!PAD) {
        double* spsi = reinterpret_cast<double*>(lds_f);
        for (int v = threadIdx.x; v <= a.M; v += blockDim.x) spsi[v] = a.psi[v];
        __syncthreads();  // the only workgroup barrier: waves are independent from here
        psi = spsi;
    }

    const int M = a.M, k = a.k, S = L.stride, R = L.ring;
    float* wb = lds_f + L.psi_f + wave * L.wave_f;
    uint32_t* cnt = reinterpret_cast<uint32_t*>(wb + R * L.slot_f);  // [R][M] packed n_x | n_y << 16
    int* info = reinterpret_cast<int*>(cnt + (PAD ? 0 : R * M));     // [R][8]: la, lb, state, in_max, pair
    double lacc = 0.0;                                               // PAD: this lane's digamma sum
    const int64_t nb = a.bb.count();
    const float inf = __builtin_inff();
    unsigned long long best = 0;
    uint32_t n_in_max = 0;

    // The wave's pairs: a sequence of chunks. Padded layout (expensive
    // pairs): chunks taken from a device-wide counter with guided sizes (a
    // share of what is left, down to one pair near the end), so waves that
    // start late or share a CU with more waves only cost a short tail. Packed
    // layout: one contiguous range per wave. Local pair s of the sequence is
    // global pair cbase + (s - cstart) of the chunk being staged; a staged
    // pair keeps its global index in `info`.
    // per lane: local pair q, sample i, ring slot r of item U + lane
    int q = lane / S, i = lane - (lane / S) * S, r = q % R;
    int staged = 0, done = 0, np_end = 0x7fffffff;
    int64_t cbase = 0;
    int cstart = 0, cend = 0;
    for (;;) {
        // ---- stage every pair this trip reaches (uniform loop)
        const int need = __builtin_amdgcn_readlane(q, 63);
        for (; staged <= need && staged < np_end; ++staged) {
            if (staged == cend) {  // the current chunk is used up: take the next one
                if constexpr (PAD) {
                    unsigned long long got = 0;
                    if (lane == 0) {
                        const unsigned long long seen =
                            __hip_atomic_load(a.work, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        const long long left = n_total - (long long)seen;
                        long long want = left / (4 * n_waves);
                        want = want < 1 ? 1 : (want > 64 ? 64 : want);
                        got = atomicAdd(a.work, (unsigned long long)want) | ((unsigned long long)want << 48);
                    }
                    got = __shfl(got, 0, 64);
                    cbase = (int64_t)(got & 0xffffffffffffull);
                    cend = staged + (int)(got >> 48);
                } else {
                    // cheap pairs: one static range per wave (a counter shared by
                    // every wave of the device costs more than the tail it saves)
                    if (staged == 0) {
                        const int64_t gw = (int64_t)blockIdx.x * L.waves + wave;
                        cbase = n_total * gw / n_waves;
                        cend = (int)(n_total * (gw + 1) / n_waves - cbase);
                    }  // a later call leaves cend == staged: the range is done
                }
                cstart = staged;
                if (staged >= cend) {  // an empty chunk: this wave's sequence ends here
                    np_end = staged;
                    break;
                }
            }
            const int64_t t = cbase + (staged - cstart);
            if (t >= n_total) {  // the work has run out: this wave's sequence ends here
                np_end = staged;
                break;
            }
            const int sr = staged % R;
            int la = -1, lb = -1, state = 0, in_max = 0;
            bool same = false;
            if (a.pairs) {
                const int32_t ga = a.pairs[2 * t], gb = a.pairs[2 * t + 1];
                la = a.whole_a ? ga : (ga < 0 ? -1 : (int)box_local_fast(a.ba, a.ax, a.ay, ga));
                lb = a.whole_b ? gb : (gb < 0 ? -1 : (int)box_local_fast(a.bb, a.bx, a.by, gb));
                same = ga == gb;
            } else {
                const int32_t tt = (int32_t)t;
                la = (int32_t)a.nbd.div((uint32_t)tt);
                lb = tt - la * (int32_t)a.nbd.d;
                same = a.ba.global(la) == a.bb.global(lb);
            }
            // state: 0 = nothing to evaluate, 1 = evaluate, 2 = constant point (MI 0)
            if (la >= 0 && lb >= 0) {
                state = 1;
                if (a.inv_a && (a.inv_a[la] == 0.0f || a.inv_b[lb] == 0.0f)) state = 2;
                in_max = (a.key != nullptr) && !(a.same_field && same);
            }
            if (lane == 0) {
                info[8 * sr] = la;
                info[8 * sr + 1] = lb;
                info[8 * sr + 2] = state;
                info[8 * sr + 3] = in_max;
                reinterpret_cast<int64_t*>(info + 8 * sr)[2] = t;
            }
            if (state == 1) {
                float* slot = wb + sr * L.slot_f;
                float2* xy = reinterpret_cast<float2*>(slot);
                float* sx = slot + 2 * L.mdup;
                float* sy = sx + L.p2;
                const float* xa = a.za + (int64_t)la * a.ld;
                const float* yb = a.zb + (int64_t)lb * a.ld;
                const float* sxa = a.sa + (int64_t)la * L.p2;
                const float* syb = a.sb + (int64_t)lb * L.p2;
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
        }
        wave_lds_sync();
        if (__builtin_amdgcn_readlane(q, 0) >= np_end) break;  // every staged pair is retired

        // ---- one item per lane
        const bool act = q < np_end && i < M;
        const int ic = i < M ? i : M - 1;
        const float* slot = wb + r * L.slot_f;
        const float2* row = reinterpret_cast<const float2*>(slot);
        const float2 me = row[ic];
        const float2* nbr = row + ic + 1;  // the M-1 other samples, in cyclic order
        float tk[KP];
#pragma unroll
        for (int p = 0; p < KP; ++p) tk[p] = inf;
        const int t4 = (M - 1) & ~3;
        if (t4 > 0) {  // groups of four samples; the next group's LDS reads are
                       // issued before the current group's selection work
            float2 v0 = nbr[0], v1 = nbr[1], v2 = nbr[2], v3 = nbr[3];
            for (int t = 4; t < t4; t += 4) {
                const float2 w0 = nbr[t], w1 = nbr[t + 1], w2 = nbr[t + 2], w3 = nbr[t + 3];
                topk_insert<KP>(tk, fmaxf(fabsf(me.x - v0.x), fabsf(me.y - v0.y)));
                topk_insert<KP>(tk, fmaxf(fabsf(me.x - v1.x), fabsf(me.y - v1.y)));
                topk_insert<KP>(tk, fmaxf(fabsf(me.x - v2.x), fabsf(me.y - v2.y)));
                topk_insert<KP>(tk, fmaxf(fabsf(me.x - v3.x), fabsf(me.y - v3.y)));
                v0 = w0;
                v1 = w1;
                v2 = w2;
                v3 = w3;
            }
            topk_insert<KP>(tk, fmaxf(fabsf(me.x - v0.x), fabsf(me.y - v0.y)));
            topk_insert<KP>(tk, fmaxf(fabsf(me.x - v1.x), fabsf(me.y - v1.y)));
            topk_insert<KP>(tk, fmaxf(fabsf(me.x - v2.x), fabsf(me.y - v2.y)));
            topk_insert<KP>(tk, fmaxf(fabsf(me.x - v3.x), fabsf(me.y - v3.y)));
        }
        {  // the last (M - 1) % 4 samples, without a loop (wave-uniform tests)
            const int rem = (M - 1) & 3;
            const float2* tail = nbr + t4;
            if (rem >= 1) topk_insert<KP>(tk, fmaxf(fabsf(me.x - tail[0].x), fabsf(me.y - tail[0].y)));
            if (rem >= 2) topk_insert<KP>(tk, fmaxf(fabsf(me.x - tail[1].x), fabsf(me.y - tail[1].y)));
            if (rem >= 3) topk_insert<KP>(tk, fmaxf(fabsf(me.x - tail[2].x), fabsf(me.y - tail[2].y)));
        }
        float eps = tk[KP - 1];
        if (k != KP) {
#pragma unroll
            for (int p = 0; p < KP - 1; ++p) eps = (p == k - 1) ? tk[p] : eps;
        }
        const float* sx = slot + 2 * L.mdup;
        const float* sy = sx + L.p2;
        const int self = eps > 0.0f ? 1 : 0;
        int nx, ny;
        run_counts<P2>(sx, sy, L.p2, me.x, me.y, eps, nx, ny);
        nx -= self;
        ny -= self;
        nx = nx < 0 ? 0 : nx;
        ny = ny < 0 ? 0 : ny;
        if (act) {
            const bool eval = info[8 * r + 2] == 1;
            if constexpr (PAD) {
                if (eval) lacc += psi[nx + 1] + psi[ny + 1];
            } else {
                cnt[r * M + i] = (uint32_t)nx | ((uint32_t)ny << 16);
            }
            if (a.counts_out && eval) {
                const int64_t tq = reinterpret_cast<const int64_t*>(info + 8 * r)[2];
                reinterpret_cast<int2*>(a.counts_out)[tq * M + i] = make_int2(nx, ny);
            }
        }
        wave_lds_sync();

        // ---- advance every lane by 64 items, then retire the pairs now complete
        i += 64;
        while (i >= S) {
            i -= S;
            ++q;
            r = (r + 1 == R) ? 0 : r + 1;
        }
        const int complete = min(__builtin_amdgcn_readlane(q, 0), min(staged, np_end));
        for (; done < complete; ++done) {
            const int dr = done % R;
            const int state = info[8 * dr + 2];
            double acc = 0.0;
            if constexpr (PAD) {
                acc = lacc;
                lacc = 0.0;
            } else if (state == 1) {
                const uint32_t* cq = cnt + dr * M;
                for (int j = lane; j < M; j += 64) {
                    const uint32_t c = cq[j];
                    acc += psi[(c & 0xffffu) + 1] + psi[(c >> 16) + 1];
                }
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
            const int64_t tp = reinterpret_cast<const int64_t*>(info + 8 * dr)[2];
            if (lane == 0) {
                float mi = 0.0f;
                if (state == 1) mi = (float)(psi[M] + psi[k] - acc / (double)M);
                if (a.mi_out) a.mi_out[tp] = mi;
                if (info[8 * dr + 3] && state != 0) {
                    const unsigned long long key =
                        make_key(mi, (uint32_t)((int64_t)info[8 * dr] * nb + info[8 * dr + 1]), 0u);
                    best = key > best ? key : best;
                    ++n_in_max;
                }
            }
            if (a.counts_out && state != 1) {
                int2* c = reinterpret_cast<int2*>(a.counts_out) + tp * M;
                for (int j = lane; j < M; j += 64) c[j] = make_int2(0, 0);
            }
        }
        wave_lds_sync();
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
// +inf) in the wave's LDS row, written to out[row * p2 ...]. Waves sort
// independent rows, so they order their LDS steps among their own lanes only.
__global__ __launch_bounds__(256) void sort_rows_kernel(const float* __restrict__ z, int64_t ld, int64_t nrows, int M,
                                                        int p2, float* __restrict__ out) {
    extern __shared__ float srt[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float* s = srt + wave * p2;
    for (int64_t r0 = (int64_t)blockIdx.x * 4; r0 < nrows; r0 += (int64_t)gridDim.x * 4) {
        const int64_t r = r0 + wave;
        if (r >= nrows) break;  // wave-uniform; no workgroup barrier follows
        for (int j = lane; j < p2; j += 64) s[j] = j < M ? z[r * ld + j] : __builtin_inff();
        wave_lds_sync();
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
                wave_lds_sync();
            }
        }
        for (int j = lane; j < p2; j += 64) out[r * p2 + j] = s[j];
        wave_lds_sync();  // the row is rewritten by the next trip
    }
}

// Register form for rows of at most 2048: lane l holds elements
// l E .. l E + E - 1 (E = P2 / 64); compare-exchange partners closer than E
// sit in the same lane, the others E-blocks away in lane l ^ (stride / E).
template <int P2>
__global__ __launch_bounds__(256) void sort_rows_reg_kernel(const float* __restrict__ z, int64_t ld, int64_t nrows,
                                                            int M, float* __restrict__ out) {
    constexpr int E = P2 / 64;
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (r >= nrows) return;
    float v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int e = lane * E + j;
        v[j] = e < M ? z[r * ld + e] : __builtin_inff();
    }
#pragma unroll
    for (int size = 2; size <= P2; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride >= 1; stride >>= 1) {
            if (stride < E) {
#pragma unroll
                for (int j = 0; j < E; ++j) {
                    const int e = lane * E + j;
                    if ((j & stride) == 0) {
                        const bool asc = (e & size) == 0;
                        const float a = v[j], b = v[j | stride];
                        v[j] = asc ? fminf(a, b) : fmaxf(a, b);
                        v[j | stride] = asc ? fmaxf(a, b) : fminf(a, b);
                    }
                }
            } else {
                const int lx = stride / E;
#pragma unroll
                for (int j = 0; j < E; ++j) {
                    const int e = lane * E + j;
                    const float o = __shfl_xor(v[j], lx, 64);
                    const bool lower = (e & stride) == 0, asc = (e & size) == 0;
                    v[j] = (lower == asc) ? fminf(v[j], o) : fmaxf(v[j], o);
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < E; ++j) out[r * P2 + lane * E + j] = v[j];
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
    if (p2 <= 2048) {  // register form, one wave per row
        const unsigned grid = (unsigned)((nrows + 3) / 4);
        switch (p2) {
            case 64: sort_rows_reg_kernel<64><<<dim3(grid), 256, 0, s>>>(z, ld, nrows, M, out); break;
            case 128: sort_rows_reg_kernel<128><<<dim3(grid), 256, 0, s>>>(z, ld, nrows, M, out); break;
            case 256: sort_rows_reg_kernel<256><<<dim3(grid), 256, 0, s>>>(z, ld, nrows, M, out); break;
            case 512: sort_rows_reg_kernel<512><<<dim3(grid), 256, 0, s>>>(z, ld, nrows, M, out); break;
            case 1024: sort_rows_reg_kernel<1024><<<dim3(grid), 256, 0, s>>>(z, ld, nrows, M, out); break;
            default: sort_rows_reg_kernel<2048><<<dim3(grid), 256, 0, s>>>(z, ld, nrows, M, out); break;
        }
        CORR_LAUNCH_CHECK();
        return CORR_OK;
    }
    int64_t blocks = (nrows + 3) / 4;
    int64_t cap = (int64_t)num_cus * 8;
    if (blocks > cap) blocks = cap;
    sort_rows_kernel<<<dim3((unsigned)blocks), 256, 4 * p2 * sizeof(float), s>>>(z, ld, nrows, M, p2, out);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

// Mapping knob (the autotuner's candidate): workgroups per CU of the
// resident grid, capped by what the kernel's registers and LDS allow.
// <= 0 picks the cap.
int ksg_default_pw(int M) {
    (void)M;
    return 0;
}

static KsgLayout ksg_layout(int M) {
    KsgLayout L;
    L.mdup = 2 * M;
    L.p2 = ksg_p2(M);
    L.slot_f = (2 * L.mdup + 2 * L.p2 + 3) & ~3;
    // packed items (no idle lanes) while four waves of it fit next to each
    // other in LDS with room for two workgroups, else padded items
    const int ring_packed = (63 + M - 1) / M + 1;
    const int psi_packed = (2 * (M + 1) + 3) & ~3;
    const int wave_packed = (ring_packed * L.slot_f + ring_packed * M + 8 * ring_packed + 3) & ~3;
    if ((size_t)(4 * wave_packed + psi_packed) * 4 <= 80 * 1024) {
        L.pad = 0;
        L.stride = M;
        L.ring = ring_packed;
        L.psi_f = psi_packed;
        L.wave_f = wave_packed;
        L.waves = 4;
    } else {
        L.pad = 1;
        L.stride = (M + 63) / 64 * 64;
        L.ring = 1;
        L.psi_f = 0;
        L.wave_f = (L.slot_f + 8 + 3) & ~3;
        // the workgroup size that fits the most waves per CU (waves never
        // synchronise in this layout, so one-wave workgroups lose nothing)
        L.waves = 1;
        int best = 0;
        for (int w = 4; w >= 1; w >>= 1) {
            const size_t bytes = (size_t)w * L.wave_f * 4;
            const int per_cu = bytes <= 160 * 1024 ? (int)(160 * 1024 / bytes) * w : 0;
            if (per_cu > best) {
                best = per_cu;
                L.waves = w;
            }
        }
    }
    while (L.waves > 1 && (size_t)(L.waves * L.wave_f + L.psi_f) * 4 > 160 * 1024) --L.waves;
    return L;
}

size_t ksg_lds_bytes(int M, int pw) {
    (void)pw;
    const KsgLayout L = ksg_layout(M);
    return ((size_t)L.waves * L.wave_f + L.psi_f) * sizeof(float);
}

template <int KP, int P2, bool PAD>
static int launch_kp(const KsgArgs& a, int64_t n_total, const KsgLayout& L, int num_cus, size_t lds, hipStream_t s) {
    const void* fn = (const void*)ksg_kernel<KP, P2, PAD>;
    const int threads = 64 * L.waves;
    int per_cu = 1;
    const int rc = kernel_setup(fn, lds, threads, &per_cu);
    if (rc) return rc;
    if (a.pw > 0 && a.pw < per_cu) per_cu = a.pw;
    // a resident grid: every wave's pair range starts at once
    int64_t blocks = (int64_t)num_cus * per_cu;
    const int64_t min_blocks = (n_total + L.waves - 1) / L.waves;  // at least one pair per wave
    if (blocks > min_blocks) blocks = min_blocks;
    const int64_t n_waves = blocks * L.waves;
    ksg_kernel<KP, P2, PAD><<<dim3((unsigned)blocks), threads, lds, s>>>(a, n_total, L, n_waves);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

template <int KP>
static int launch_p2(const KsgArgs& a, int64_t n_total, const KsgLayout& L, int num_cus, size_t lds, hipStream_t s) {
    if (L.pad) return launch_kp<KP, 0, true>(a, n_total, L, num_cus, lds, s);
    switch (L.p2) {
        case 64: return launch_kp<KP, 64, false>(a, n_total, L, num_cus, lds, s);
        case 128: return launch_kp<KP, 128, false>(a, n_total, L, num_cus, lds, s);
        case 256: return launch_kp<KP, 256, false>(a, n_total, L, num_cus, lds, s);
        default: return launch_kp<KP, 0, false>(a, n_total, L, num_cus, lds, s);
    }
}

int launch_ksg(const KsgArgs& a_in, int num_cus, hipStream_t s) {
    KsgArgs a = a_in;
    int64_t n_total = a.pairs ? a.n : a.ba.count() * a.bb.count();
    if (n_total == 0) return CORR_OK;
    if (!a.pairs && n_total >= (int64_t(1) << 31)) return fail(CORR_EUNSUPPORTED, "KSG: 2^31 or more implicit pairs");
    a.ax = FastDiv((uint32_t)a.ba.nx);
    a.ay = FastDiv((uint32_t)a.ba.ny);
    a.bx = FastDiv((uint32_t)a.bb.nx);
    a.by = FastDiv((uint32_t)a.bb.ny);
    a.nbd = FastDiv((uint32_t)std::max<int64_t>(1, a.bb.count()));
    const KsgLayout L = ksg_layout(a.M);
    const size_t lds = ksg_lds_bytes(a.M, a.pw);
    if (lds > 160 * 1024) return fail(CORR_EUNSUPPORTED, "KSG: member count too large for the LDS layout");
    if (!a.work) return fail(CORR_EINVAL, "KSG: no work counter");
    int rc = launch_fill_u64(a.work, 1, 0ull, s);
    if (rc) return rc;
    // selection width: the smallest instantiated KP >= k
    const int k = a.k;
    if (k == 10) return launch_p2<10>(a, n_total, L, num_cus, lds, s);
    if (k <= 4) return launch_p2<4>(a, n_total, L, num_cus, lds, s);
    if (k <= 8) return launch_p2<8>(a, n_total, L, num_cus, lds, s);
    if (k <= 12) return launch_p2<12>(a, n_total, L, num_cus, lds, s);
    if (k <= 16) return launch_p2<16>(a, n_total, L, num_cus, lds, s);
    if (k <= 24) return launch_p2<24>(a, n_total, L, num_cus, lds, s);
    return launch_p2<32>(a, n_total, L, num_cus, lds, s);
}

}  // namespace corr
