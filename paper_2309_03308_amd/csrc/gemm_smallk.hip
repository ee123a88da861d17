// Exhaustive Pearson region maximum for small ensembles (K = padded member
// count <= 128) as one MFMA contraction with the maximum fused (Sec. 3: the
// brick-pair indicator is the maximum point-to-point correlation).
//
// R = Zhat_A Zhat_B^T is never stored. Design for gfx950 when K is small:
//  - a workgroup (4 waves) keeps one B tile of BN standardised rows x K
//    resident in LDS for its whole life (loaded once, one barrier);
//  - every wave holds the complete A fragment of WM x 32 rows x K in
//    registers (loaded straight from global memory, 16 bytes per lane per
//    K-step), so A never touches LDS and the K loop has no barriers;
//  - the wave sweeps the B tile in groups of WNG 32-column blocks:
//    WM x WNG x K/16 MFMA (32x32x16 f16/bf16, or 32x32x2 f32 with a K
//    permutation that lets one float4 read feed four steps) into FP32
//    accumulators, then folds |r| of the group into its running maximum;
//  - the (B tile, A block) work grid is split into one rectangle per XCD
//    (its A rows fit the XCD's L2) and each rectangle evenly over that XCD's
//    resident workgroups, in tile-major runs; per run the B tile is staged
//    once and the waves take every fourth A block (optionally prefetching
//    the next fragment into a second register buffer), so LDS traffic is B
//    only, L2 traffic is about one pass over A per B tile, and no workgroup
//    waits for a second round.
// Epilogue: each lane keeps its own running max of |r| and the group where
// it first occurred (no cross-lane work in the sweep); at the end of a run
// one wave reduction finds the wave maximum, the first group holding it is
// recomputed from the still-resident B tile, its element with the smallest
// linear index is located, and one 64-bit atomicMax publishes (|r|, index,
// sign).
#include "common.h"

#include <atomic>

namespace corr {

typedef _Float16 sk_h8 __attribute__((ext_vector_type(8)));
typedef __bf16 sk_b8 __attribute__((ext_vector_type(8)));
typedef float sk_f16 __attribute__((ext_vector_type(16)));

template <int PREC>
struct SkT {
    static constexpr bool F32 = PREC == CORR_PREC_F32;
    static constexpr bool SPLIT = PREC == CORR_PREC_F16X3 || PREC == CORR_PREC_BF16X3;
    static constexpr bool BF = PREC == CORR_PREC_BF16 || PREC == CORR_PREC_BF16X3;
    static constexpr int ES = F32 ? 4 : 2;
};

__device__ __forceinline__ float sk_wave_max(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// A fragment of WM row blocks (all parts) straight from global memory:
// lane (l32, half) holds row l32 of each block, 16-byte vector 2s + half.
template <int PARTS, int WM, int KV>
__device__ __forceinline__ void sk_load_a(const GemmArgs& g, int64_t row0, int l32, int half, int64_t rowb_g,
                                          uint4 (&av)[PARTS][WM][KV / 2]) {
#pragma unroll
    for (int q = 0; q < PARTS; ++q)
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            const char* src = (const char*)(q ? g.a_lo : g.a_hi) + (row0 + i * 32 + l32) * rowb_g;
#pragma unroll
            for (int s = 0; s < KV / 2; ++s) av[q][i][s] = *reinterpret_cast<const uint4*>(src + (2 * s + half) * 16);
        }
}

// B fragments of K-step s (all parts, WNG column blocks) from LDS.
template <int PARTS, int WNG, int NS, int BN, int ROWB>
__device__ __forceinline__ void sk_load_b(const char* smem, int jg, int l32, int half, int s,
                                          uint4 (&bv)[PARTS][WNG][NS]) {
#pragma unroll
    for (int j = 0; j < WNG; ++j) {
        const char* lb = smem + ((jg + j) * 32 + l32) * ROWB + (2 * s + half) * 16;
        bv[0][j][s] = *reinterpret_cast<const uint4*>(lb);
        if constexpr (PARTS == 2) bv[1][j][s] = *reinterpret_cast<const uint4*>(lb + BN * ROWB);
    }
}

// One group: WM x WNG blocks of 32x32, the whole K, B blocks jg.. from LDS.
// B fragments are read D K-steps ahead of the MFMAs that use them (scheduling
// fences keep the reads where they are issued), so LDS latency is hidden
// behind D steps of MFMAs instead of being waited for at every fragment.
// Lookahead depth: as many K-steps (at most 4) as fit next to the A
// fragments (doubled when prefetched), the accumulators (two sets when
// double-buffered; none when one workgroup per CU leaves them the
// accumulation registers) and ~96 registers of addressing and bookkeeping
// within 256 VGPRs; 0 when not even one step fits (then each fragment is
// read just before its MFMAs).
constexpr int sk_depth(int parts, int wm, int wng, int ns, int pf, int occ, bool dbuf) {
    const int fixed = parts * wm * ns * 4 * (pf ? 2 : 1) + (occ == 1 ? 0 : (dbuf ? 2 : 1) * wm * wng * 16) + 96;
    int d = (256 - fixed) / (parts * wng * 4) - 1;
    if (d > 4) d = 4;
    if (d > ns) d = ns;
    return d < 1 ? 0 : d;
}
// Interior blocks double-buffer the accumulators (the fold of one group
// overlaps the next group's MFMAs) only where a lookahead still fits beside
// them; otherwise the lookahead is kept and each group is folded after its
// MFMAs, while the SIMD's other wave keeps the matrix pipe busy.
constexpr bool sk_dbuf(int parts, int wm, int wng, int ns, int pf, int occ) {
    return occ == 1 || sk_depth(parts, wm, wng, ns, pf, occ, true) >= 1;
}
constexpr int sk_lookahead(int parts, int wm, int wng, int ns, int pf, int occ) {
    return sk_depth(parts, wm, wng, ns, pf, occ, sk_dbuf(parts, wm, wng, ns, pf, occ));
}
// Largest batch of at most 8 vectors that divides a thread's share (more
// would hold too many registers at a run's start).
constexpr int sk_batch(int per) {
    for (int c = 8; c > 1; --c)
        if (per % c == 0) return c;
    return 1;
}

// The lookahead crosses group boundaries: during a group's last D K-steps
// the first D steps of the next group (the next block's first group after a
// block's last one: the B tile stays in LDS for the whole run) are read into
// the slots of steps already consumed, so a group's first products never
// wait for LDS. Needs 0 < D < NS (a slot must be free before its reload).
constexpr bool sk_xgroup(int parts, int wm, int wng, int ns, int pf, int occ) {
    return sk_lookahead(parts, wm, wng, ns, pf, occ) > 0 && sk_lookahead(parts, wm, wng, ns, pf, occ) < ns;
}

// First D steps of group jg, when the lookahead crosses groups (the start of
// a chain of groups: a run's first block, or a lone recomputed group).
template <int PARTS, int WM, int WNG, int KV, int BN, int ROWB, int PF, int OCC>
__device__ __forceinline__ void sk_prologue(const char* smem, int jg, int l32, int half,
                                            uint4 (&bv)[PARTS][WNG][KV / 2]) {
    constexpr int NS = KV / 2;
    constexpr int D = sk_lookahead(PARTS, WM, WNG, NS, PF, OCC);
    if constexpr (sk_xgroup(PARTS, WM, WNG, NS, PF, OCC)) {
#pragma unroll
        for (int s = 0; s < D; ++s) sk_load_b<PARTS, WNG, NS, BN, ROWB>(smem, jg, l32, half, s, bv);
    }
}

// FOLD: while this group's MFMAs run, fold |r| of the previous group's
// accumulators (prev) into mprev, a slice per K-step from the second one on
// (the previous group's last products are still in the pipe at the first),
// so the VALU work overlaps the matrix pipe instead of following it.
// bv: on entry (cross-group lookahead) it holds steps 0..D-1 of group jg; on
// exit, steps 0..D-1 of group jg_next.
template <int PREC, int PARTS, int WM, int WNG, int KV, int BN, int ROWB, int PF, int OCC, bool FOLD = false>
__device__ __forceinline__ void sk_group(const char* smem, int jg, int jg_next, int l32, int half,
                                         const uint4 (&av)[PARTS][WM][KV / 2], sk_f16 (&acc)[WM][WNG],
                                         const sk_f16 (&prev)[WM][WNG], float& mprev, uint4 (&bv)[PARTS][WNG][KV / 2]) {
    using T = SkT<PREC>;
    constexpr int NS = KV / 2;
    constexpr int NPAIR = WM * WNG * 8;  // element pairs of one group per lane
    constexpr int D = sk_lookahead(PARTS, WM, WNG, NS, PF, OCC);
    constexpr bool XG = sk_xgroup(PARTS, WM, WNG, NS, PF, OCC);
    if constexpr (!XG) {
#pragma unroll
        for (int s = 0; s < D; ++s) sk_load_b<PARTS, WNG, NS, BN, ROWB>(smem, jg, l32, half, s, bv);
    }
    if constexpr (D > 0) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WNG; ++j) acc[i][j] = sk_f16{};
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if (s + D < NS)
            sk_load_b<PARTS, WNG, NS, BN, ROWB>(smem, jg, l32, half, s + D, bv);
        else if constexpr (XG)
            sk_load_b<PARTS, WNG, NS, BN, ROWB>(smem, jg_next, l32, half, s + D - NS, bv);
        if constexpr (D > 0) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < WNG; ++j) {
            const uint4 bh = bv[0][j][s];
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                if constexpr (T::F32) {
                    const float* fa = reinterpret_cast<const float*>(&av[0][i][s]);
                    const float* fb = reinterpret_cast<const float*>(&bh);
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[e], fb[e], acc[i][j], 0, 0, 0);
                } else if constexpr (T::BF) {
                    const sk_b8 a8 = *reinterpret_cast<const sk_b8*>(&av[0][i][s]);
                    const sk_b8 b8 = *reinterpret_cast<const sk_b8*>(&bh);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8, b8, acc[i][j], 0, 0, 0);
                    if constexpr (T::SPLIT) {
                        const sk_b8 a8l = *reinterpret_cast<const sk_b8*>(&av[PARTS - 1][i][s]);
                        const sk_b8 b8l = *reinterpret_cast<const sk_b8*>(&bv[PARTS - 1][j][s]);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8, b8l, acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8l, b8, acc[i][j], 0, 0, 0);
                    }
                } else {
                    const sk_h8 a8 = *reinterpret_cast<const sk_h8*>(&av[0][i][s]);
                    const sk_h8 b8 = *reinterpret_cast<const sk_h8*>(&bh);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a8, b8, acc[i][j], 0, 0, 0);
                    if constexpr (T::SPLIT) {
                        const sk_h8 a8l = *reinterpret_cast<const sk_h8*>(&av[PARTS - 1][i][s]);
                        const sk_h8 b8l = *reinterpret_cast<const sk_h8*>(&bv[PARTS - 1][j][s]);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a8, b8l, acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a8l, b8, acc[i][j], 0, 0, 0);
                    }
                }
            }
        }
        if constexpr (FOLD) {
            // slices over steps 1..NS-1 (all at step 0 when NS == 1)
            constexpr int NSL = NS > 1 ? NS - 1 : 1;
            const int sl = NS > 1 ? s - 1 : 0;
#pragma unroll
            for (int q = sl < 0 ? 0 : sl * NPAIR / NSL; q < (sl < 0 ? 0 : (sl + 1) * NPAIR / NSL); ++q) {
                const int e = 2 * q, i = e / (WNG * 16), j = (e / 16) % WNG, r = e % 16;
                mprev = fmaxf(mprev, fmaxf(fabsf(prev[i][j][r]), fabsf(prev[i][j][r + 1])));
            }
        }
    }
}

// All column groups of the B tile against one A block, folding |r| into the
// lane's running maximum (strict >: the first occurrence in sweep order).
template <int PREC, int PARTS, int WM, int WNG, int KV, int BN, int ROWB, int PF, int OCC>
__device__ __forceinline__ void sk_block(const GemmArgs& g, const char* smem, int64_t ab, int64_t col0, int l32,
                                         int half, bool self, int32_t nb, const uint4 (&av)[PARTS][WM][KV / 2],
                                         sk_f16 (&acc)[WM][WNG], float& lane_best, int& lane_ab, int& lane_jg,
                                         uint4 (&bv)[PARTS][WNG][KV / 2]) {
    const int64_t row0 = ab * 32 * WM;
    const bool edge_rows = row0 + 32 * WM > g.na;
    constexpr bool DBUF = sk_dbuf(PARTS, WM, WNG, KV / 2, PF, OCC);
    if (DBUF && !edge_rows && !self && col0 + BN <= nb) {
        // interior block: accumulators double-buffered, group q-1 folded
        // while group q is multiplied
        constexpr int NG = BN / 32 / WNG;
        sk_f16 acc2[WM][WNG];
        float unused = 0.0f;
        sk_group<PREC, PARTS, WM, WNG, KV, BN, ROWB, PF, OCC, false>(smem, 0, NG > 1 ? WNG : 0, l32, half, av, acc, acc,
                                                                   unused, bv);
#pragma unroll
        for (int q = 1; q < NG; ++q) {
            float m = -1.0f;
            const int nx = (q + 1 < NG) ? (q + 1) * WNG : 0;  // after the last group: the next block's first
            if (q & 1)
                sk_group<PREC, PARTS, WM, WNG, KV, BN, ROWB, PF, OCC, true>(smem, q * WNG, nx, l32, half, av, acc2, acc,
                                                                          m, bv);
            else
                sk_group<PREC, PARTS, WM, WNG, KV, BN, ROWB, PF, OCC, true>(smem, q * WNG, nx, l32, half, av, acc, acc2,
                                                                          m, bv);
            if (m > lane_best) {
                lane_best = m;
                lane_ab = (int)ab;
                lane_jg = (q - 1) * WNG;
            }
        }
        float m = -1.0f;
        const sk_f16(&last)[WM][WNG] = ((NG - 1) & 1) ? acc2 : acc;
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < WNG; ++j)
#pragma unroll
                for (int r = 0; r < 16; r += 2) m = fmaxf(m, fmaxf(fabsf(last[i][j][r]), fabsf(last[i][j][r + 1])));
        if (m > lane_best) {
            lane_best = m;
            lane_ab = (int)ab;
            lane_jg = (NG - 1) * WNG;
        }
        return;
    }
    float unused = 0.0f;
#pragma unroll 1
    for (int jg = 0; jg < BN / 32; jg += WNG) {
        const int nx = (jg + WNG < BN / 32) ? jg + WNG : 0;
        sk_group<PREC, PARTS, WM, WNG, KV, BN, ROWB, PF, OCC, false>(smem, jg, nx, l32, half, av, acc, acc, unused, bv);
        const int32_t c0 = (int32_t)(col0 + jg * 32);
        const bool edge = edge_rows || (c0 + 32 * WNG > nb) || self;
        float m = -1.0f;
        if (!edge) {
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WNG; ++j)
#pragma unroll
                    for (int r = 0; r < 16; r += 2) m = fmaxf(m, fmaxf(fabsf(acc[i][j][r]), fabsf(acc[i][j][r + 1])));
        } else {
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WNG; ++j)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int32_t row = (int32_t)row0 + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                        const int32_t col = c0 + j * 32 + l32;
                        const bool ok = row < g.na && col < nb && !(self && g.self_col[row] == col);
                        if (ok) m = fmaxf(m, fabsf(acc[i][j][r]));
                    }
        }
        if (m > lane_best) {
            lane_best = m;
            lane_ab = (int)ab;
            lane_jg = jg;
        }
    }
}

// Wave-level finish of one tile run: one wave reduction, the first group
// (in sweep order) holding the wave maximum is recomputed from the B tile
// still in LDS to find its element, and one 64-bit atomicMax publishes
// (|r|, index, sign).
template <int PREC, int PARTS, int WM, int WNG, int KV, int BN, int ROWB, int PF, int OCC>
__device__ __forceinline__ void sk_finish(const GemmArgs& g, const char* smem, int64_t col0, int lane, int l32,
                                          int half, bool self, int32_t nb, int64_t rowb_g, float lane_best, int lane_ab,
                                          int lane_jg, uint4 (&av)[PARTS][WM][KV / 2], sk_f16 (&acc)[WM][WNG],
                                          uint4 (&bv)[PARTS][WNG][KV / 2]) {
    const float wb = sk_wave_max(lane_best);
    if (wb < 0.0f) return;
    int code = (lane_best == wb) ? lane_ab * (BN / 32) + lane_jg : 0x7fffffff;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int o = __shfl_xor(code, off, 64);
        code = o < code ? o : code;
    }
    const int ab = code / (BN / 32), jg = code - ab * (BN / 32);
    const int64_t row0 = (int64_t)ab * 32 * WM;
    sk_load_a<PARTS, WM, KV>(g, row0, l32, half, rowb_g, av);
    float unused = 0.0f;
    sk_prologue<PARTS, WM, WNG, KV, BN, ROWB, PF, OCC>(smem, jg, l32, half, bv);
    sk_group<PREC, PARTS, WM, WNG, KV, BN, ROWB, PF, OCC, false>(smem, jg, jg, l32, half, av, acc, acc, unused, bv);
    const int32_t c0 = (int32_t)(col0 + jg * 32);
    uint32_t cand = 0xffffffffu, neg = 0;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WNG; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                // 32x32 accumulator layout: register r of lane l holds
                // row 8*(r/4) + 4*(l/32) + r%4, column l%32
                const int32_t row = (int32_t)row0 + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                const int32_t col = c0 + j * 32 + l32;
                const float v = acc[i][j][r];
                const bool ok = row < g.na && col < nb && !(self && g.self_col[row] == col);
                const uint32_t lin = (uint32_t)row * (uint32_t)nb + (uint32_t)col;
                if (ok && fabsf(v) == wb && lin < cand) {
                    cand = lin;
                    neg = v < 0.0f ? 1u : 0u;
                }
            }
    unsigned long long key = (cand == 0xffffffffu) ? 0ull : make_key(wb, cand, neg);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(key, off, 64);
        key = o > key ? o : key;
    }
    if (lane == 0 && key) atomicMax(g.key, key);
}

// Work decomposition. The (B tile, A block) items form a grid of n_tj x
// n_ablk. Workgroups are dealt round-robin to the 8 XCDs, so workgroup b runs
// on XCD b % 8: each XCD owns one rectangle of tiles x A blocks (tx_parts x
// ax_parts rectangles; the A rows of a rectangle fit the XCD's L2), and the
// workgroups of an XCD split its items evenly in tile-major order. The grid
// is the number of resident workgroups, so the whole chip works until the
// end. A workgroup walks its range in runs of one B tile: the tile is staged
// in LDS once per run and its waves take every fourth A block of the run.
// KV = K / 8 (16-bit) or K / 4 (f32): 16-byte vectors per row.
// OCC = workgroups per CU the register budget is sized for: 2 (two waves
// per SIMD, 256 registers each) or 1 (one wave per SIMD, whose 512 registers
// hold the large accumulator tiles).
template <int PREC, int KV, int WM, int WNG, int BN, int PF, int OCC>
__global__ __launch_bounds__(256, OCC) void gemm_smallk_kernel(GemmArgs g, int n_tj, int tx_parts, int ax_parts) {
    using T = SkT<PREC>;
    constexpr int PARTS = T::SPLIT ? 2 : 1;
    constexpr int ROWB = KV * 16 + 16;  // padded LDS row bytes (conflict-free 16-byte reads)
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    const int64_t rowb_g = (int64_t)KV * 16;
    const int64_t n_ablk = g.na_pad / (32 * WM);
    const bool self = g.self_col != nullptr;
    const int32_t nb = (int32_t)g.nb;

    const int G = gridDim.x, b = blockIdx.x;
    const bool xcd = (G % 8 == 0) && tx_parts * ax_parts == 8;
    const int x = xcd ? (b & 7) : 0;
    const int64_t r = xcd ? (b >> 3) : b, R = xcd ? (G >> 3) : G;
    const int txp = xcd ? tx_parts : 1, axp = xcd ? ax_parts : 1;
    const int tx = x % txp, ax = x / txp;
    const int64_t t0 = (int64_t)n_tj * tx / txp, t1 = (int64_t)n_tj * (tx + 1) / txp;
    const int64_t a0 = n_ablk * ax / axp, a1 = n_ablk * (ax + 1) / axp;
    const int64_t na_x = a1 - a0;
    const int64_t items = (t1 - t0) * na_x;
    int64_t it = items * r / R;
    const int64_t it_end = items * (r + 1) / R;

    uint4 av[PARTS][WM][KV / 2];
    uint4 bv[PARTS][WNG][KV / 2];
    sk_f16 acc[WM][WNG];
    while (it < it_end) {
        const int64_t tj = t0 + it / na_x;
        const int64_t ab0 = a0 + it % na_x;
        int64_t run = na_x - it % na_x;
        if (run > it_end - it) run = it_end - it;
        const int64_t ab1 = ab0 + run;
        const int64_t col0 = tj * BN;

        // ---- stage the B tile (all parts); the barrier before protects the
        // previous run's tile until every wave has finished with it
        __syncthreads();
        {
            // every thread copies NV / 256 vectors per part (BN * KV is a
            // multiple of 256 for every configuration); up to 8 loads are
            // issued before their stores, so a run's staging costs a few
            // memory round trips instead of one per vector
            constexpr int NV = BN * KV;  // 16-byte vectors per part
            constexpr int PER = NV / 256, CH = sk_batch(PER);
            static_assert(NV % 256 == 0, "B tile staging: whole vectors per thread");
            // the tile's global rows are contiguous (row pitch KV * 16 bytes):
            // vector v sits at v * 16; in LDS each row is padded by 16 bytes
#pragma unroll
            for (int q = 0; q < PARTS; ++q) {
                const uint4* src = reinterpret_cast<const uint4*>((const char*)(q ? g.b_lo : g.b_hi) + col0 * rowb_g);
                char* dst = smem + q * BN * ROWB;
#pragma unroll
                for (int u0 = 0; u0 < PER; u0 += CH) {
                    uint4 tmp[CH];
#pragma unroll
                    for (int u = 0; u < CH; ++u) tmp[u] = src[tid + (u0 + u) * 256];
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        const int v = tid + (u0 + u) * 256;
                        *reinterpret_cast<uint4*>(dst + (v + v / KV) * 16) = tmp[u];
                    }
                }
            }
        }
        __syncthreads();

        // the run's first group: its first D steps of B fragments
        sk_prologue<PARTS, WM, WNG, KV, BN, ROWB, PF, OCC>(smem, 0, l32, half, bv);

        // Per-lane running maximum and the (A block, column group) where it
        // first occurred; no cross-lane work inside the sweep.
        float lane_best = -1.0f;
        int lane_ab = -1, lane_jg = -1;
        if constexpr (!PF) {
            for (int64_t ab = ab0 + wave; ab < ab1; ab += 4) {
                sk_load_a<PARTS, WM, KV>(g, ab * 32 * WM, l32, half, rowb_g, av);
                sk_block<PREC, PARTS, WM, WNG, KV, BN, ROWB, PF, OCC>(g, smem, ab, col0, l32, half, self, nb, av, acc,
                                                                 lane_best, lane_ab, lane_jg, bv);
            }
        } else {
            // A fragments double-buffered in registers: the next block's
            // loads are in flight while the current block is multiplied.
            // The prefetch is unconditional (past the run's last block it
            // re-reads that block): a conditional load would make the
            // compiler's wait counting treat the current block's operands as
            // the newest loads and wait for the prefetch before the first
            // product, which serialises the two.
            uint4 av2[PARTS][WM][KV / 2];
            int64_t ab = ab0 + wave;
            const int64_t ab_last = ab1 - 1;
            if (ab < ab1) sk_load_a<PARTS, WM, KV>(g, ab * 32 * WM, l32, half, rowb_g, av);
            while (ab < ab1) {
                sk_load_a<PARTS, WM, KV>(g, min(ab + 4, ab_last) * 32 * WM, l32, half, rowb_g, av2);
                sk_block<PREC, PARTS, WM, WNG, KV, BN, ROWB, PF, OCC>(g, smem, ab, col0, l32, half, self, nb, av, acc,
                                                                 lane_best, lane_ab, lane_jg, bv);
                ab += 4;
                if (ab >= ab1) break;
                sk_load_a<PARTS, WM, KV>(g, min(ab + 4, ab_last) * 32 * WM, l32, half, rowb_g, av);
                sk_block<PREC, PARTS, WM, WNG, KV, BN, ROWB, PF, OCC>(g, smem, ab, col0, l32, half, self, nb, av2, acc,
                                                                 lane_best, lane_ab, lane_jg, bv);
                ab += 4;
            }
        }
        sk_finish<PREC, PARTS, WM, WNG, KV, BN, ROWB, PF, OCC>(g, smem, col0, lane, l32, half, self, nb, rowb_g, lane_best,
                                                          lane_ab, lane_jg, av, acc, bv);
        it += run;
    }
}

// ---------------------------------------------------------------- dispatch
struct SkCfg {
    int wm, wng, bn, pf, occ;  // row blocks per wave, column blocks per group, B tile rows, A prefetch,
                               // workgroups per CU
};

// Tile configurations the autotuner chooses from (index = config id).
static const SkCfg kSkCfgs[] = {
    {2, 2, 256, 0, 2}, {1, 4, 256, 0, 2}, {2, 2, 128, 0, 2}, {1, 2, 128, 0, 2}, {1, 2, 128, 1, 2},
    {1, 4, 256, 1, 2}, {1, 2, 256, 1, 2}, {1, 2, 256, 0, 2}, {2, 4, 512, 0, 1}, {4, 2, 512, 0, 1},
    {2, 1, 256, 0, 2}, {2, 1, 128, 0, 2},
};
constexpr int kNumSkCfgs = sizeof(kSkCfgs) / sizeof(kSkCfgs[0]);

// query: report (without launching) whether the instantiation runs without
// scratch -- a configuration whose registers spill is never used.
template <int PREC, int KV, int WM, int WNG, int BN, int PF, int OCC>
static int launch_sk_t(const GemmArgs& g, int num_cus, hipStream_t s, bool query) {
    constexpr int PARTS = SkT<PREC>::SPLIT ? 2 : 1;
    constexpr int ROWB = KV * 16 + 16;
    const size_t lds = (size_t)PARTS * BN * ROWB;
    const void* fn = (const void*)gemm_smallk_kernel<PREC, KV, WM, WNG, BN, PF, OCC>;
    if (query) {
        hipFuncAttributes attr;
        if (hipFuncGetAttributes(&attr, fn) != hipSuccess) {
            (void)hipGetLastError();
            return CORR_EUNSUPPORTED;
        }
        return attr.localSizeBytes == 0 ? CORR_OK : CORR_EUNSUPPORTED;
    }
    int per_cu = 1;
    const int rc = kernel_setup(fn, lds, 256, &per_cu);
    if (rc) return rc;
    const int n_tj = (int)(g.nb_pad / BN);
    const int64_t n_ablk = g.na_pad / (32 * WM);
    // XCD rectangles: split A so that each part's rows (all parts of the
    // split modes) stay within about 2 MiB of the XCD's L2, tiles the rest
    const int64_t a_bytes = g.na_pad * KV * 16 * PARTS;
    int ax = 1;
    while (ax < 8 && a_bytes / ax > (int64_t)2 << 20) ax *= 2;
    const int tx = 8 / ax;
    int64_t grid = (int64_t)num_cus * per_cu;
    grid = (grid + 7) / 8 * 8;
    const int64_t items = (int64_t)n_tj * n_ablk;
    if (grid > (items + 7) / 8 * 8) grid = (items + 7) / 8 * 8;
    if (grid < 8) grid = 8;
    gemm_smallk_kernel<PREC, KV, WM, WNG, BN, PF, OCC><<<dim3((unsigned)grid), 256, lds, s>>>(g, n_tj, tx, ax);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

// Small-K contraction K values: members are zero-padded to 64, 112 or 128.
int smallk_pad_K(int M) { return M <= 64 ? 64 : (M <= 112 ? 112 : 128); }

template <int PREC, int WM, int WNG, int BN, int PF, int OCC = 2>
static int launch_sk_k(const GemmArgs& g, int num_cus, hipStream_t s, bool q) {
    constexpr int ES = SkT<PREC>::ES;
    switch (g.K) {
        case 64: return launch_sk_t<PREC, 64 * ES / 16, WM, WNG, BN, PF, OCC>(g, num_cus, s, q);
        case 112: return launch_sk_t<PREC, 112 * ES / 16, WM, WNG, BN, PF, OCC>(g, num_cus, s, q);
        case 128: return launch_sk_t<PREC, 128 * ES / 16, WM, WNG, BN, PF, OCC>(g, num_cus, s, q);
    }
    return fail(CORR_EUNSUPPORTED, "small-K contraction: K must be 64, 112 or 128");
}

template <int PREC>
static int launch_sk_p(const GemmArgs& g, int cfg, int nc, hipStream_t s, bool q) {
    constexpr bool SPLIT = SkT<PREC>::SPLIT;
    switch (cfg) {
        case 0: if constexpr (!SPLIT) return launch_sk_k<PREC, 2, 2, 256, 0>(g, nc, s, q); break;
        case 1: return launch_sk_k<PREC, 1, 4, 256, 0>(g, nc, s, q);
        case 2: if constexpr (!SPLIT) return launch_sk_k<PREC, 2, 2, 128, 0>(g, nc, s, q); break;
        case 3: return launch_sk_k<PREC, 1, 2, 128, 0>(g, nc, s, q);
        case 4: return launch_sk_k<PREC, 1, 2, 128, 1>(g, nc, s, q);
        case 5: return launch_sk_k<PREC, 1, 4, 256, 1>(g, nc, s, q);
        case 6: return launch_sk_k<PREC, 1, 2, 256, 1>(g, nc, s, q);
        case 7: return launch_sk_k<PREC, 1, 2, 256, 0>(g, nc, s, q);
        case 8: if constexpr (!SPLIT) return launch_sk_k<PREC, 2, 4, 512, 0, 1>(g, nc, s, q); break;
        case 9: if constexpr (!SPLIT) return launch_sk_k<PREC, 4, 2, 512, 0, 1>(g, nc, s, q); break;
        case 10: if constexpr (!SPLIT) return launch_sk_k<PREC, 2, 1, 256, 0>(g, nc, s, q); break;
        case 11: if constexpr (!SPLIT) return launch_sk_k<PREC, 2, 1, 128, 0>(g, nc, s, q); break;
    }
    return fail(CORR_EINVAL, "small-K contraction: tile configuration not available for this precision");
}

int smallk_num_configs() { return kNumSkCfgs; }
int smallk_row_pad(int cfg) { return 32 * kSkCfgs[cfg].wm; }
int smallk_col_pad(int cfg) { return kSkCfgs[cfg].bn; }
// Register budget: split modes keep hi and lo A fragments (one row block
// only); FP32 operands with two row blocks cannot also double-buffer A.
static bool smallk_config_static_ok(int prec, int cfg) {
    if (cfg < 0 || cfg >= kNumSkCfgs) return false;
    const SkCfg& c = kSkCfgs[cfg];
    if (prec_split(prec) && c.wm != 1) return false;
    return true;
}

static int sk_dispatch(const GemmArgs& g, int cfg, int num_cus, hipStream_t s, bool query) {
    switch (g.prec) {
        case CORR_PREC_F32: return launch_sk_p<CORR_PREC_F32>(g, cfg, num_cus, s, query);
        case CORR_PREC_F16: return launch_sk_p<CORR_PREC_F16>(g, cfg, num_cus, s, query);
        case CORR_PREC_BF16: return launch_sk_p<CORR_PREC_BF16>(g, cfg, num_cus, s, query);
        case CORR_PREC_F16X3: return launch_sk_p<CORR_PREC_F16X3>(g, cfg, num_cus, s, query);
        case CORR_PREC_BF16X3: return launch_sk_p<CORR_PREC_BF16X3>(g, cfg, num_cus, s, query);
    }
    return fail(CORR_EUNSUPPORTED, "unknown precision");
}

// A configuration is usable for (prec, K) when it exists for the precision
// and its kernel runs without scratch (answer cached per process).
bool smallk_config_ok(int prec, int cfg, int K) {
    if (!smallk_config_static_ok(prec, cfg) || prec < CORR_PREC_F32 || prec > CORR_PREC_BF16X3) return false;
    const int es = prec == CORR_PREC_F32 ? 4 : 2, parts = prec_split(prec) ? 2 : 1;
    if ((size_t)parts * kSkCfgs[cfg].bn * (K * es + 16) > 160 * 1024) return false;  // B tile must fit LDS
    const int ki = K == 64 ? 0 : (K == 112 ? 1 : (K == 128 ? 2 : -1));
    if (ki < 0) return false;
    // 0 = not queried yet, 1 = usable, -1 = not; the query is idempotent, so
    // concurrent first calls at worst repeat it
    static std::atomic<signed char> cache[5][kNumSkCfgs][3] = {};
    std::atomic<signed char>& c = cache[prec][cfg][ki];
    signed char v = c.load(std::memory_order_relaxed);
    if (v == 0) {
        GemmArgs g{};
        g.prec = prec;
        g.K = K;
        v = sk_dispatch(g, cfg, 0, nullptr, true) == CORR_OK ? 1 : -1;
        c.store(v, std::memory_order_relaxed);
    }
    return v > 0;
}

int launch_gemm_smallk(const GemmArgs& g, int cfg, int num_cus, hipStream_t s) {
    if (g.na == 0 || g.nb == 0) return CORR_OK;
    if (!smallk_config_ok(g.prec, cfg, (int)g.K)) return fail(CORR_EINVAL, "small-K contraction: bad tile configuration");
    return sk_dispatch(g, cfg, num_cus, s, false);
}

}  // namespace corr
