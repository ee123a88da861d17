// Exhaustive Pearson region maximum as one MFMA contraction (Sec. 3: the
// brick-pair indicator is the maximum of all point-to-point correlations
// between the two bricks).
//
// With point-major standardised rows Zhat_A [na][K] and Zhat_B [nb][K]
// (K = members, zero-padded), R = Zhat_A Zhat_B^T holds every r(pA, pB).
// R is never stored: each tile's epilogue folds |r| into a running maximum.
//
// Design (gfx950):
//  - workgroup = 4 waves (2 x 2), workgroup tile 128 (A rows) x 128 (B rows),
//    wave tile 64 x 64 = 2 x 2 blocks of v_mfma_f32_32x32x16_{f16,bf16}
//    (v_mfma_f32_32x32x2_f32 for FP32 operands), FP32 accumulators;
//  - K is consumed in chunks (64 B per row; 128 B for single-pass 16-bit
//    operands) staged through LDS, double-buffered: chunk c+1 is copied into
//    the other stage after chunk c's products are issued, from registers
//    loaded several chunks earlier; LDS rows are padded by 16 bytes so the
//    16-byte operand reads are conflict-free;
//  - split modes hold hi and lo parts and issue hi.hi + hi.lo + lo.hi;
//  - persistent workgroups walk tiles in an XCD-grouped order, and tiles
//    are numbered in 8-row groups, so the workgroups resident on one XCD
//    (one L2) work on an 8 x 8 block of tiles;
//  - epilogue: per-lane max of |r| (v_max3 with abs modifiers), wave max by
//    shuffles; only when a tile beats the wave's best so far (rare after the
//    first tiles) does the wave locate the element, picking the smallest
//    linear index among equal values (the search scans only the 32 x 32
//    blocks whose maximum equals the wave's). One 64-bit atomicMax per wave
//    at the end publishes (|r|, index, sign) -- independent of scheduling
//    order;
//  - single-pass 16-bit operands on bricks large enough to give every CU a
//    256 x 256 tile take the wide-tile kernel further down (one workgroup
//    per CU: 4 waves of 128 x 128 at one tile per CU, 8 waves of 128 x 64
//    from two tiles per CU on).
#include "common.h"

namespace corr {

typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef __bf16 b8_t __attribute__((ext_vector_type(8)));
typedef float f16_t __attribute__((ext_vector_type(16)));
// 16-byte staging word: a native vector, so the staging registers are plain
// SSA values (a struct copy would go through a private-memory temporary)
typedef unsigned int u4_t __attribute__((ext_vector_type(4)));

constexpr int G_BM = 128, G_BN = 128;  // workgroup tile
constexpr int G_WM = 2, G_WN = 2;      // 32x32 blocks per wave
constexpr int G_THREADS = 256;

template <int PREC>
struct GemmTraits {
    static constexpr bool F32 = PREC == CORR_PREC_F32;
    static constexpr bool SPLIT = PREC == CORR_PREC_F16X3 || PREC == CORR_PREC_BF16X3;
    static constexpr bool BF = PREC == CORR_PREC_BF16 || PREC == CORR_PREC_BF16X3;
    static constexpr int ES = F32 ? 4 : 2;              // element bytes
    // chunk length (elements): 64 bytes per row for FP32 and the split
    // modes (two parts), 128 bytes for single-pass 16-bit operands
    static constexpr int KC = F32 ? 16 : (SPLIT ? 32 : 64);
    static constexpr int QW = KC * ES / 16;             // 16-byte words per row and chunk
    static constexpr int ROWB = KC * ES + 16;           // padded LDS row bytes
    static constexpr int PARTS = SPLIT ? 2 : 1;
    static constexpr int STAGE = PARTS * (G_BM + G_BN) * ROWB;  // bytes per LDS stage
    static constexpr int PF = F32 ? 4 : 2;                       // chunks in flight in registers
    static constexpr int NRA = G_BM * QW / G_THREADS;            // A words per thread and part
    static constexpr int NRB = G_BN * QW / G_THREADS;            // B words per thread and part
};

template <int PREC>
__device__ __forceinline__ void mfma_step(f16_t& acc, const char* pa, const char* pb, int e) {
    using T = GemmTraits<PREC>;
    if constexpr (T::F32) {
        float a = reinterpret_cast<const float*>(pa)[e];
        float b = reinterpret_cast<const float*>(pb)[e];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    } else if constexpr (T::BF) {
        b8_t a = *reinterpret_cast<const b8_t*>(pa);
        b8_t b = *reinterpret_cast<const b8_t*>(pb);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    } else {
        h8_t a = *reinterpret_cast<const h8_t*>(pa);
        h8_t b = *reinterpret_cast<const h8_t*>(pb);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc, 0, 0, 0);
    }
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

template <int PREC, int NRB>
__device__ __forceinline__ void g_load(const char* a_hi, const char* a_lo, const char* b_hi, const char* b_lo,
                                       int64_t row0, int64_t col0, int64_t rowb_g, int c, int tid,
                                       u4_t (&ra)[GemmTraits<PREC>::PARTS][GemmTraits<PREC>::NRA],
                                       u4_t (&rb)[GemmTraits<PREC>::PARTS][NRB]) {
    using T = GemmTraits<PREC>;
    const int64_t kb = (int64_t)c * T::KC * T::ES;
#pragma unroll
    for (int q = 0; q < T::PARTS; ++q) {
        const char* sa = q ? a_lo : a_hi;
        const char* sb = q ? b_lo : b_hi;
#pragma unroll
        for (int r = 0; r < T::NRA; ++r) {
            const int v = tid + G_THREADS * r;
            ra[q][r] = *reinterpret_cast<const u4_t*>(sa + (row0 + v / T::QW) * rowb_g + kb + (v % T::QW) * 16);
        }
#pragma unroll
        for (int r = 0; r < NRB; ++r) {
            const int v = tid + G_THREADS * r;
            rb[q][r] = *reinterpret_cast<const u4_t*>(sb + (col0 + v / T::QW) * rowb_g + kb + (v % T::QW) * 16);
        }
    }
}

template <int PREC, int NRB>
__device__ __forceinline__ void s_store(char* smem, int stage, int tid,
                                        const u4_t (&ra)[GemmTraits<PREC>::PARTS][GemmTraits<PREC>::NRA],
                                        const u4_t (&rb)[GemmTraits<PREC>::PARTS][NRB]) {
    using T = GemmTraits<PREC>;
    char* base = smem + stage * T::STAGE;
#pragma unroll
    for (int q = 0; q < T::PARTS; ++q) {
        char* la = base + q * (G_BM + G_BN) * T::ROWB;
        char* lb = la + G_BM * T::ROWB;
#pragma unroll
        for (int r = 0; r < T::NRA; ++r) {
            const int v = tid + G_THREADS * r;
            *reinterpret_cast<u4_t*>(la + (v / T::QW) * T::ROWB + (v % T::QW) * 16) = ra[q][r];
        }
#pragma unroll
        for (int r = 0; r < NRB; ++r) {
            const int v = tid + G_THREADS * r;
            *reinterpret_cast<u4_t*>(lb + (v / T::QW) * T::ROWB + (v % T::QW) * 16) = rb[q][r];
        }
    }
}

// One chunk of a tile: products from LDS stage c & 1, then chunk c + 1
// (held in register set (U + 1) % PF) into the other stage -- its readers
// finished before the barrier that ended the previous chunk -- and that set
// loads chunk c + 1 + PF. U is a template constant so every set index is
// static and the sets stay in registers.
template <int PREC, int NRB, int U>
__device__ __forceinline__ void chunk_step(char* smem, int c, int n_chunks, int wr, int wc, int lane, int tid,
                                           const char* a_hi, const char* a_lo, const char* b_hi, const char* b_lo,
                                           int64_t row0, int64_t col0, int64_t rowb_g,
                                           u4_t (&ra)[GemmTraits<PREC>::PF][GemmTraits<PREC>::PARTS][GemmTraits<PREC>::NRA],
                                           u4_t (&rb)[GemmTraits<PREC>::PF][GemmTraits<PREC>::PARTS][NRB],
                                           f16_t (&acc)[G_WM][G_WN]) {
    using T = GemmTraits<PREC>;
    constexpr int PF = T::PF;
    const int stage = c & 1;
    const char* base = smem + stage * T::STAGE;
    const char* la_hi = base + (wr * 64 + (lane & 31)) * T::ROWB;
    const char* lb_hi = base + G_BM * T::ROWB + (wc * 32 * G_WN + (lane & 31)) * T::ROWB;
    const int half = lane >> 5;
    if constexpr (T::F32) {
        // 8 K-steps of 2 per chunk; lane reads k = 8q + 4*half + e
#pragma unroll
        for (int qq = 0; qq < 2; ++qq) {
            float4 av[G_WM], bv[G_WN];
#pragma unroll
            for (int i = 0; i < G_WM; ++i)
                av[i] = *reinterpret_cast<const float4*>(la_hi + i * 32 * T::ROWB + (qq * 8 + half * 4) * 4);
#pragma unroll
            for (int j = 0; j < G_WN; ++j)
                bv[j] = *reinterpret_cast<const float4*>(lb_hi + j * 32 * T::ROWB + (qq * 8 + half * 4) * 4);
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int i = 0; i < G_WM; ++i)
#pragma unroll
                    for (int j = 0; j < G_WN; ++j)
                        mfma_step<PREC>(acc[i][j], (const char*)&av[i], (const char*)&bv[j], e);
        }
    } else {
#pragma unroll
        for (int s = 0; s < T::KC / 16; ++s) {
            const int off = (s * 16 + half * 8) * 2;
#pragma unroll
            for (int i = 0; i < G_WM; ++i)
#pragma unroll
                for (int j = 0; j < G_WN; ++j) {
                    const char* pa = la_hi + i * 32 * T::ROWB + off;
                    const char* pb = lb_hi + j * 32 * T::ROWB + off;
                    mfma_step<PREC>(acc[i][j], pa, pb, 0);
                    if constexpr (T::SPLIT) {
                        const int lo = (G_BM + G_BN) * T::ROWB;
                        mfma_step<PREC>(acc[i][j], pa, pb + lo, 0);
                        mfma_step<PREC>(acc[i][j], pa + lo, pb, 0);
                    }
                }
        }
    }
    // Unconditional on purpose: after the last chunk the store is a dead
    // copy into the idle stage and the load re-reads the last chunk; a
    // branch here would make the compiler wait for every load in flight.
    constexpr int nx = (U + 1) % PF;
    s_store<PREC, NRB>(smem, stage ^ 1, tid, ra[nx], rb[nx]);
    g_load<PREC, NRB>(a_hi, a_lo, b_hi, b_lo, row0, col0, rowb_g, min(c + 1 + PF, n_chunks - 1), tid, ra[nx], rb[nx]);
    __syncthreads();
}

// Fold |r| of one wave's WM x WN accumulator blocks (the block at (i, j)
// covers rows r_base + 32 i .. and columns c_base + 32 j ..) into the wave's
// running maximum `best` and its key. `edge`: the workgroup tile reaches past
// the valid rows or columns (those are masked, as are self pairs).
template <int WM, int WN>
__device__ __forceinline__ void fold_tile(const f16_t (&acc)[WM][WN], const GemmArgs& g, int64_t r_base,
                                          int64_t c_base, bool edge, int lane, float& best,
                                          unsigned long long& best_key) {
    const bool self = g.self_col != nullptr;
    // 32x32 accumulator layout: register r of lane l holds
    // row 8*(r/4) + 4*(l/32) + r%4, column l%32 of the block.
#define ELEM_ROW(i, r) (r_base + (i) * 32 + 8 * ((r) >> 2) + 4 * (lane >> 5) + ((r) & 3))
#define ELEM_COL(j) (c_base + (j) * 32 + (lane & 31))
    const bool fast = !edge && !self;  // every element valid
    float m = -1.0f;
    float mb[WM][WN];                  // per-block maxima (fast case)
    if (fast) {
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < WN; ++j) {
                float x = -1.0f;
#pragma unroll
                for (int r = 0; r < 16; r += 2) x = fmaxf(x, fmaxf(fabsf(acc[i][j][r]), fabsf(acc[i][j][r + 1])));
                mb[i][j] = x;
                m = fmaxf(m, x);
            }
    } else {
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < WN; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    int64_t row = ELEM_ROW(i, r), col = ELEM_COL(j);
                    bool ok = row < g.na && col < g.nb && !(self && g.self_col[row] == col);
                    if (ok) m = fmaxf(m, fabsf(acc[i][j][r]));
                }
    }
    const float wm = wave_max(m);
    if (wm >= 0.0f && wm >= best) {
        // locate: smallest linear index among elements with |r| == wm
        uint32_t cand = 0xffffffffu;
        uint32_t neg = 0;
        if (fast) {
            // Only the blocks holding wm are scanned, behind a wave-uniform
            // branch, so the code of the others is neither run nor fetched.
            // In a block (one column per lane) the smallest register index
            // is the smallest row; across blocks the smallest index wins.
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j) {
                    if (__builtin_amdgcn_ballot_w64(mb[i][j] == wm) == 0) continue;
                    int rr = -1;
                    float sv = 0.0f;
#pragma unroll
                    for (int r = 15; r >= 0; --r) {
                        const float v = acc[i][j][r];
                        const bool hit = fabsf(v) == wm;
                        rr = hit ? r : rr;
                        sv = hit ? v : sv;
                    }
                    if (rr >= 0) {
                        const uint32_t lin = (uint32_t)(ELEM_ROW(i, rr) * g.nb + ELEM_COL(j));
                        if (lin < cand) {
                            cand = lin;
                            neg = sv < 0.0f ? 1u : 0u;
                        }
                    }
                }
        } else {
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        float v = acc[i][j][r];
                        int64_t row = ELEM_ROW(i, r), col = ELEM_COL(j);
                        bool ok = row < g.na && col < g.nb && !(self && g.self_col[row] == col);
                        uint32_t lin = (uint32_t)(row * g.nb + col);
                        if (ok && fabsf(v) == wm && lin < cand) {
                            cand = lin;
                            neg = v < 0.0f ? 1u : 0u;
                        }
                    }
        }
        unsigned long long k = (cand == 0xffffffffu) ? 0ull : make_key(wm, cand, neg);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            unsigned long long o = __shfl_xor(k, off, 64);
            k = o > k ? o : k;
        }
        best_key = k > best_key ? k : best_key;
        best = wm;
    }
#undef ELEM_ROW
#undef ELEM_COL
}

template <int PREC>
__global__ __launch_bounds__(G_THREADS, 2) void gemm_max_kernel(GemmArgs g, int n_ti, int n_tj) {
    using T = GemmTraits<PREC>;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;  // wave position in the 2 x 2 grid
    const int64_t rowb_g = g.K * T::ES;       // global row bytes
    const int n_chunks = (int)(g.K / T::KC);
    const int64_t n_tiles = (int64_t)n_ti * n_tj;

    // XCD-grouped logical workgroup id: blocks are dealt round-robin to the
    // 8 XCDs, so give the blocks of one XCD consecutive logical ids.
    const int G = gridDim.x;
    const int b = blockIdx.x;
    const int lg = (G % 8 == 0) ? ((b % 8) * (G / 8) + b / 8) : b;

    float best = -1.0f;
    unsigned long long best_key = 0;

    const char* a_hi = (const char*)g.a_hi;
    const char* a_lo = (const char*)g.a_lo;
    const char* b_hi = (const char*)g.b_hi;
    const char* b_lo = (const char*)g.b_lo;

    for (int64_t tile = lg; tile < n_tiles; tile += G) {
        // groups of 8 tile rows walked column by column: 64 consecutive
        // tiles (the workgroups resident on one XCD at a time) form an 8 x 8
        // block and share 8 A and 8 B panels in that XCD's L2
        const int64_t grp = tile / (8 * (int64_t)n_tj);
        const int first = (int)grp * 8, gsz = min(n_ti - first, 8);
        const int64_t in = tile - grp * 8 * (int64_t)n_tj;
        const int ti = first + (int)(in % gsz), tj = (int)(in / gsz);
        const int64_t row0 = (int64_t)ti * G_BM, col0 = (int64_t)tj * G_BN;

        // global -> register staging (per part): A tile = 128 rows x KC
        // elements in 16-byte words, B tile likewise. PF register sets keep the
        // loads of the next PF chunks in flight, so a chunk's copy into LDS
        // waits on a load issued PF chunks earlier (one chunk of products is
        // far shorter than a load's latency).
        constexpr int NRB = T::NRB;
        constexpr int PF = T::PF;
        static_assert(PF == 2 || PF == 4, "register sets: 2 or 4");
        u4_t ra[PF][T::PARTS][T::NRA], rb[PF][T::PARTS][NRB];
        f16_t acc[G_WM][G_WN];
#pragma unroll
        for (int i = 0; i < G_WM; ++i)
#pragma unroll
            for (int j = 0; j < G_WN; ++j) acc[i][j] = f16_t{};

        g_load<PREC, NRB>(a_hi, a_lo, b_hi, b_lo, row0, col0, rowb_g, 0, tid, ra[0], rb[0]);
        s_store<PREC, NRB>(smem, 0, tid, ra[0], rb[0]);
        // chunks 1..PF into sets 1 % PF .. PF % PF (n_chunks is a multiple
        // of PF; a chunk index past the end re-reads the last chunk)
        const int last = n_chunks - 1;
        g_load<PREC, NRB>(a_hi, a_lo, b_hi, b_lo, row0, col0, rowb_g, min(1, last), tid, ra[1 % PF], rb[1 % PF]);
        g_load<PREC, NRB>(a_hi, a_lo, b_hi, b_lo, row0, col0, rowb_g, min(2, last), tid, ra[2 % PF], rb[2 % PF]);
        if constexpr (PF > 2) {
            g_load<PREC, NRB>(a_hi, a_lo, b_hi, b_lo, row0, col0, rowb_g, min(3, last), tid, ra[3 % PF], rb[3 % PF]);
            g_load<PREC, NRB>(a_hi, a_lo, b_hi, b_lo, row0, col0, rowb_g, min(4, last), tid, ra[4 % PF], rb[4 % PF]);
        }
        __syncthreads();
#define CHUNK(U)                                                                                                   \
    chunk_step<PREC, NRB, (U) % PF>(smem, c0 + (U), n_chunks, wr, wc, lane, tid, a_hi, a_lo, b_hi, b_lo, row0, col0, \
                                    rowb_g, ra, rb, acc)
        for (int c0 = 0; c0 < n_chunks; c0 += PF) {
            CHUNK(0);
            CHUNK(1);
            if constexpr (PF > 2) {
                CHUNK(2);
                CHUNK(3);
            }
        }
#undef CHUNK

        // ---- epilogue: fold |r| of this tile into the wave's running max
        fold_tile<G_WM, G_WN>(acc, g, row0 + wr * 64, col0 + wc * 32 * G_WN,
                              (row0 + G_BM > g.na) || (col0 + G_BN > g.nb), lane, best, best_key);
    }
    if (lane == 0 && best >= 0.0f) atomicMax(g.key, best_key);
}

// ---- wide tiles: single-pass 16-bit operands, enough tiles to fill the chip
//
// A workgroup tile of 256 x 256 reads each A and B row once per 256 partner
// rows instead of once per 128: half the L2 traffic per product of the
// 128 x 128 tile. Four waves (2 x 2, each 128 x 128 = 4 x 4 blocks of
// 32x32x16 MFMAs, 256 accumulator registers, one fragment read per two
// MFMAs) when each CU gets one tile; eight waves (2 x 4, each 128 x 64, two
// per SIMD, 0.75 reads per MFMA) when CUs get two or more, where the second
// wave on a SIMD hides the first one's waits (about 10% faster there, 12%
// slower at one tile per CU). K is consumed in 32-element
// chunks (64 B per row) through a ring of three LDS stages: during chunk c
// the waves read stage c mod 3 (the chunk's second K-step) and stage
// (c + 1) mod 3 (the next chunk's first K-step, read while this chunk's
// products run), and copy chunk c + 2 into stage (c + 2) mod 3, whose last
// readers finished before the barrier that ended chunk c - 1 -- one barrier
// per chunk. Two register sets hold the global loads of chunks c + 2 and
// c + 3, issued two chunks before their copy into LDS (four sets measured
// slower: more registers and twice the unrolled loop code).
constexpr int W_BM = 256, W_BN = 256;                   // workgroup tile
constexpr int W_WM = 4;                                 // 32x32 blocks per wave, rows
constexpr int W_KC = 32;                                // chunk length (elements)
constexpr int W_QW = W_KC * 2 / 16;                     // 16-byte words per row and chunk
constexpr int W_ROWB = W_KC * 2 + 16;                   // padded LDS row bytes (conflict-free reads)
constexpr int W_STAGE = (W_BM + W_BN) * W_ROWB;         // bytes per LDS stage
constexpr int W_NST = 3;                                // LDS stages
constexpr int W_PF = 2;                                 // register sets of staged loads

// Wave layout of the tile: 4 waves (2 x 2, each 128 x 128) or 8 waves (2 x 4,
// each 128 x 64, two waves per SIMD).
template <int WAVES>
struct WL {
    static_assert(WAVES == 4 || WAVES == 8, "4 or 8 waves");
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int WAVES_N = WAVES / 2;                   // wave columns
    static constexpr int WN = W_BN / 32 / WAVES_N;              // 32x32 blocks per wave, columns
    static constexpr int NR = (W_BM + W_BN) * W_QW / THREADS;   // staged words per thread and chunk
    static constexpr int RSTEP = THREADS / W_QW;                // rows between a thread's staged words
};

template <int NR>
__device__ __forceinline__ void w_load(const char* const (&src)[NR], int c, u4_t (&set)[NR]) {
#pragma unroll
    for (int r = 0; r < NR; ++r) set[r] = *reinterpret_cast<const u4_t*>(src[r] + c * (W_KC * 2));
}

template <int NR, int RSTEP>
__device__ __forceinline__ void w_store(char* dst, const u4_t (&set)[NR]) {
#pragma unroll
    for (int r = 0; r < NR; ++r) *reinterpret_cast<u4_t*>(dst + r * RSTEP * W_ROWB) = set[r];
}

// Fragments of K-step s (16 elements) of the chunk held in stage `st`.
template <int WN>
__device__ __forceinline__ void w_frags(const char* st, int wr, int wc, int lane, int s, u4_t (&fa)[W_WM],
                                        u4_t (&fb)[WN]) {
    const int off = (s * 16 + (lane >> 5) * 8) * 2;
    const char* pa = st + (wr * 128 + (lane & 31)) * W_ROWB + off;
    const char* pb = st + (W_BM + wc * 32 * WN + (lane & 31)) * W_ROWB + off;
#pragma unroll
    for (int i = 0; i < W_WM; ++i) fa[i] = *reinterpret_cast<const u4_t*>(pa + i * 32 * W_ROWB);
#pragma unroll
    for (int j = 0; j < WN; ++j) fb[j] = *reinterpret_cast<const u4_t*>(pb + j * 32 * W_ROWB);
}

// Instruction order of one chunk, for the scheduler: each of the 32 MFMAs
// is followed by one memory instruction (the next K-step's fragment reads,
// the LDS copy of a later chunk, its global loads), so the matrix pipe
// is never left idle while a block of memory instructions issues (one wave
// per SIMD: no other wave fills the gaps).
template <int WN, int NW>
__device__ __forceinline__ void w_schedule() {
    constexpr int MFMA = 0x008, DS_READ = 0x100, DS_WRITE = 0x200, VMEM_READ = 0x020;
    constexpr int NM = 2 * W_WM * WN, NR = W_WM + WN;  // per chunk: MFMAs, reads per K-step
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        __builtin_amdgcn_sched_group_barrier(MFMA, 1, 0);
        __builtin_amdgcn_sched_group_barrier(DS_READ, 1, 0);
    }
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        __builtin_amdgcn_sched_group_barrier(MFMA, 1, 0);
        __builtin_amdgcn_sched_group_barrier(DS_WRITE, 1, 0);
        __builtin_amdgcn_sched_group_barrier(VMEM_READ, 1, 0);
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        __builtin_amdgcn_sched_group_barrier(MFMA, 1, 0);
        __builtin_amdgcn_sched_group_barrier(DS_READ, 1, 0);
    }
    if constexpr (NM > 2 * NR + NW) __builtin_amdgcn_sched_group_barrier(MFMA, NM - 2 * NR - NW, 0);
}

template <int PREC, int WN>
__device__ __forceinline__ void w_mfma(f16_t (&acc)[W_WM][WN], const u4_t (&fa)[W_WM], const u4_t (&fb)[WN]) {
#pragma unroll
    for (int i = 0; i < W_WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            if constexpr (PREC == CORR_PREC_BF16)
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(b8_t, fa[i]),
                                                                     __builtin_bit_cast(b8_t, fb[j]), acc[i][j], 0, 0, 0);
            else
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(h8_t, fa[i]),
                                                                    __builtin_bit_cast(h8_t, fb[j]), acc[i][j], 0, 0, 0);
        }
}

template <int PREC, int WAVES>
__global__ __launch_bounds__(WL<WAVES>::THREADS, 1) void gemm_max_wide_kernel(GemmArgs g, int n_ti, int n_tj) {
    using L = WL<WAVES>;
    static_assert(PREC == CORR_PREC_F16 || PREC == CORR_PREC_BF16, "single-pass 16-bit operands");
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / L::WAVES_N, wc = wave % L::WAVES_N;  // wave position in the grid
    const int64_t rowb_g = g.K * 2;
    const int n_chunks = (int)(g.K / W_KC);  // a multiple of W_PF: K is a multiple of W_PF * W_KC
    const int last = n_chunks - 1;
    const int64_t n_tiles = (int64_t)n_ti * n_tj;
    const int G = gridDim.x;
    const int b = blockIdx.x;
    const int lg = (G % 8 == 0) ? ((b % 8) * (G / 8) + b / 8) : b;  // XCD-grouped, as above

    // this thread stages the 16-byte word tid % 4 of rows trow + 64 r. A
    // wave's 16 lane groups of 4 take its 16 rows in the order 0, 4, 8, 12,
    // 1, 5, ...: the LDS serves 16 lanes (four rows) at a time, and at the
    // 80-byte row pitch rows r and r + 3 share banks, rows r, r + 4, r + 8,
    // r + 12 do not (each group of 4 lanes still reads one 64-byte segment)
    const int lg4 = (tid & 63) / W_QW;
    const int trow = (tid >> 6) * 16 + (lg4 & 3) * 4 + (lg4 >> 2);
    char* const dst0 = smem + trow * W_ROWB + (tid % W_QW) * 16;

    float best = -1.0f;
    unsigned long long best_key = 0;

    for (int64_t tile = lg; tile < n_tiles; tile += G) {
        const int64_t grp = tile / (8 * (int64_t)n_tj);
        const int first = (int)grp * 8, gsz = min(n_ti - first, 8);
        const int64_t in = tile - grp * 8 * (int64_t)n_tj;
        const int ti = first + (int)(in % gsz), tj = (int)(in / gsz);
        const int64_t row0 = (int64_t)ti * W_BM, col0 = (int64_t)tj * W_BN;

        // source rows, clamped to the padded row counts: a 256-row tile may
        // run past buffers padded to 128 rows; rows past na / nb are masked
        // in the epilogue
        const char* src[L::NR];
#pragma unroll
        for (int r = 0; r < L::NR / 2; ++r) {
            const int64_t ra = min(row0 + trow + L::RSTEP * r, g.na_pad - 1);
            const int64_t rb = min(col0 + trow + L::RSTEP * r, g.nb_pad - 1);
            src[r] = (const char*)g.a_hi + ra * rowb_g + (tid % W_QW) * 16;
            src[L::NR / 2 + r] = (const char*)g.b_hi + rb * rowb_g + (tid % W_QW) * 16;
        }

        u4_t set0[L::NR], set1[L::NR];
        w_load(src, 0, set0);
        w_load(src, min(1, last), set1);
        w_store<L::NR, L::RSTEP>(dst0, set0);
        w_load(src, min(2, last), set0);
        w_store<L::NR, L::RSTEP>(dst0 + W_STAGE, set1);
        w_load(src, min(3, last), set1);
        __syncthreads();

        f16_t acc[W_WM][L::WN];
#pragma unroll
        for (int i = 0; i < W_WM; ++i)
#pragma unroll
            for (int j = 0; j < L::WN; ++j) acc[i][j] = f16_t{};
        u4_t fa0[W_WM], fb0[L::WN], fa1[W_WM], fb1[L::WN];
        w_frags(smem, wr, wc, lane, 0, fa0, fb0);

        // chunk cc in stage st; `set` holds chunk cc + 2 and then takes
        // cc + 2 + W_PF (the two sets hold chunks cc + 2 and cc + 3).
        // Past the last chunk the reads and copies touch idle stages and the
        // loads re-read the last chunk (no branch: a branch here would make
        // the compiler wait for every load in flight).
        int st = 0;
#define W_CHUNK(cc, set)                                                        \
    {                                                                           \
        const int sn = st == W_NST - 1 ? 0 : st + 1;                            \
        const int sw = sn == W_NST - 1 ? 0 : sn + 1;                            \
        w_frags(smem + st * W_STAGE, wr, wc, lane, 1, fa1, fb1);                \
        w_mfma<PREC>(acc, fa0, fb0);                                            \
        w_store<L::NR, L::RSTEP>(dst0 + sw * W_STAGE, set);                                 \
        w_load(src, min((cc) + W_PF + 2, last), set);                           \
        w_frags(smem + sn * W_STAGE, wr, wc, lane, 0, fa0, fb0);                \
        w_mfma<PREC>(acc, fa1, fb1);                                            \
        w_schedule<L::WN, L::NR>();                                                \
        __syncthreads();                                                        \
        st = sn;                                                                \
    }
        for (int c = 0; c < n_chunks; c += W_PF) {
            W_CHUNK(c, set0);
            W_CHUNK(c + 1, set1);
        }
#undef W_CHUNK

        fold_tile<W_WM, L::WN>(acc, g, row0 + wr * 128, col0 + wc * 32 * L::WN,
                              (row0 + W_BM > g.na) || (col0 + W_BN > g.nb), lane, best, best_key);
    }
    if (lane == 0 && best >= 0.0f) atomicMax(g.key, best_key);
}

template <int PREC>
static int launch_p(const GemmArgs& g, int num_cus, hipStream_t s) {
    using T = GemmTraits<PREC>;
    const int n_ti = (int)(g.na_pad / G_BM), n_tj = (int)(g.nb_pad / G_BN);
    const int64_t n_tiles = (int64_t)n_ti * n_tj;
    int64_t grid = (int64_t)num_cus * 2;
    if (grid > n_tiles) grid = n_tiles;
    const size_t lds = 2 * (size_t)T::STAGE;
    if (g.K <= 0 || g.K % (T::KC * T::PF)) return fail(CORR_EINVAL, "contraction: K not a multiple of the chunk group");
    int rc = kernel_setup((const void*)gemm_max_kernel<PREC>, lds, G_THREADS, nullptr);
    if (rc) return rc;
    gemm_max_kernel<PREC><<<dim3((unsigned)grid), G_THREADS, lds, s>>>(g, n_ti, n_tj);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

template <int PREC, int WAVES>
static int launch_wide(const GemmArgs& g, int64_t n_ti, int64_t n_tj, int num_cus, hipStream_t s) {
    const int64_t n_tiles = n_ti * n_tj;
    const int grid = (int)(n_tiles < num_cus ? n_tiles : num_cus);
    const size_t lds = (size_t)W_NST * W_STAGE;
    if (g.K <= 0 || g.K % (W_PF * W_KC)) return fail(CORR_EINVAL, "contraction: K not a multiple of the chunk group");
    int rc = kernel_setup((const void*)gemm_max_wide_kernel<PREC, WAVES>, lds, WL<WAVES>::THREADS, nullptr);
    if (rc) return rc;
    gemm_max_wide_kernel<PREC, WAVES><<<dim3((unsigned)grid), WL<WAVES>::THREADS, lds, s>>>(g, (int)n_ti, (int)n_tj);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

// Wide 256 x 256 tiles when there are enough of them to give every CU one;
// otherwise (and for FP32 and the split modes) the 128 x 128 tiles.
static bool use_wide(const GemmArgs& g, int num_cus, int64_t& n_ti, int64_t& n_tj) {
    if (g.prec != CORR_PREC_F16 && g.prec != CORR_PREC_BF16) return false;
    n_ti = (g.na + W_BM - 1) / W_BM;
    n_tj = (g.nb + W_BN - 1) / W_BN;
    return n_ti * n_tj >= num_cus;
}

int launch_gemm_max(const GemmArgs& g, int num_cus, hipStream_t s) {
    if (g.na == 0 || g.nb == 0) return CORR_OK;
    int64_t n_ti = 0, n_tj = 0;
    if (use_wide(g, num_cus, n_ti, n_tj)) {
        // one tile per CU: 4 waves (its start and epilogue are cheaper);
        // two or more: 8 waves, two per SIMD, which hide each other's waits
        const bool eight = n_ti * n_tj >= 2 * (int64_t)num_cus;
        if (g.prec == CORR_PREC_F16)
            return eight ? launch_wide<CORR_PREC_F16, 8>(g, n_ti, n_tj, num_cus, s)
                         : launch_wide<CORR_PREC_F16, 4>(g, n_ti, n_tj, num_cus, s);
        return eight ? launch_wide<CORR_PREC_BF16, 8>(g, n_ti, n_tj, num_cus, s)
                     : launch_wide<CORR_PREC_BF16, 4>(g, n_ti, n_tj, num_cus, s);
    }
    switch (g.prec) {
        case CORR_PREC_F32: return launch_p<CORR_PREC_F32>(g, num_cus, s);
        case CORR_PREC_F16: return launch_p<CORR_PREC_F16>(g, num_cus, s);
        case CORR_PREC_BF16: return launch_p<CORR_PREC_BF16>(g, num_cus, s);
        case CORR_PREC_F16X3: return launch_p<CORR_PREC_F16X3>(g, num_cus, s);
        case CORR_PREC_BF16X3: return launch_p<CORR_PREC_BF16X3>(g, num_cus, s);
    }
    return fail(CORR_EUNSUPPORTED, "unknown precision");
}

int gemm_row_pad() { return G_BM; }
int gemm_col_pad() { return G_BN; }
int gemm_k_pad(int prec) {
    // K is consumed in groups of PF chunks
    switch (prec) {
        case CORR_PREC_F32: return GemmTraits<CORR_PREC_F32>::KC * GemmTraits<CORR_PREC_F32>::PF;
        case CORR_PREC_F16X3: return GemmTraits<CORR_PREC_F16X3>::KC * GemmTraits<CORR_PREC_F16X3>::PF;
        case CORR_PREC_BF16X3: return GemmTraits<CORR_PREC_BF16X3>::KC * GemmTraits<CORR_PREC_BF16X3>::PF;
        default: return GemmTraits<CORR_PREC_F16>::KC * GemmTraits<CORR_PREC_F16>::PF;
    }
}

}  // namespace corr
