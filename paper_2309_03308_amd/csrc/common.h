// Internal declarations shared by libcorr's translation units (not part of
// the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/corr.h"

namespace corr {

// ---- error plumbing -------------------------------------------------------
void set_error(const std::string& msg);
int fail(int status, const std::string& msg);

#define CORR_HIP(call)                                                                 \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::corr::fail(CORR_EHIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

#define CORR_LAUNCH_CHECK() CORR_HIP(hipGetLastError())

// ---- point sets -------------------------------------------------------------
// A box of grid cells enumerated in local x-fastest order; the whole grid is
// the box (0,0,0,nx,ny,nz).
struct Box {
    int32_t x0, y0, z0, dx, dy, dz;
    int32_t nx, ny;  // grid extent used for global indexing
    __host__ __device__ int64_t count() const { return (int64_t)dx * dy * dz; }
    __host__ __device__ int32_t global(int64_t i) const {
        int32_t lx = (int32_t)(i % dx);
        int64_t r = i / dx;
        int32_t ly = (int32_t)(r % dy);
        int32_t lz = (int32_t)(r / dy);
        return (x0 + lx) + nx * ((y0 + ly) + ny * (z0 + lz));
    }
    // local index of a global point, or -1 if outside
    __host__ __device__ int64_t local(int32_t p) const {
        int32_t x = p % nx, r = p / nx;
        int32_t y = r % ny, z = r / ny;
        x -= x0; y -= y0; z -= z0;
        if (x < 0 || y < 0 || z < 0 || x >= dx || y >= dy || z >= dz) return -1;
        return x + (int64_t)dx * (y + (int64_t)dy * z);
    }
};

// Division of 0 <= n < 2^31 by a divisor 1 <= d < 2^31 fixed for a launch:
// a multiply-high and two shifts instead of a full integer division
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, the unsigned case with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1).
struct FastDiv {
    uint32_t d = 1, m = 1, s1 = 0, s2 = 0;
    __host__ __device__ FastDiv() {}
    __host__ explicit FastDiv(uint32_t dd) {
        d = dd;
        uint32_t l = 0;
        while (l < 32 && (uint64_t(1) << l) < dd) ++l;
        m = (uint32_t)(((uint64_t(1) << 32) * ((uint64_t(1) << l) - dd)) / dd + 1);
        s1 = l == 0 ? 0u : 1u;
        s2 = l == 0 ? 0u : l - 1;
    }
    __host__ __device__ uint32_t div(uint32_t n) const {
#ifdef __HIP_DEVICE_COMPILE__
        const uint32_t t = __umulhi(m, n);
#else
        const uint32_t t = (uint32_t)(((uint64_t)m * n) >> 32);
#endif
        return (t + ((n - t) >> s1)) >> s2;
    }
};

// Local index of global point p in box b (grid divisors dx = nx, dy = ny),
// or -1 if outside; the same as Box::local with invariant divisions.
__host__ __device__ inline int64_t box_local_fast(const Box& b, const FastDiv& dx, const FastDiv& dy, int32_t p) {
    const uint32_t r = dx.div((uint32_t)p);
    const int32_t x = p - (int32_t)(r * dx.d) - b.x0;
    const uint32_t zq = dy.div(r);
    const int32_t y = (int32_t)(r - zq * dy.d) - b.y0;
    const int32_t z = (int32_t)zq - b.z0;
    if (x < 0 || y < 0 || z < 0 || x >= b.dx || y >= b.dy || z >= b.dz) return -1;
    return x + (int64_t)b.dx * (y + (int64_t)b.dy * z);
}

// ---- workspace --------------------------------------------------------------
enum WsSlot {
    WS_STATS_A = 0, WS_STATS_B, WS_Z_A, WS_Z_B, WS_ZH_A, WS_ZH_B, WS_ZL_A, WS_ZL_B,
    WS_PAIRS, WS_MISC, WS_SORT_A, WS_SORT_B, WS_SAMPLES, WS_SVALUES, WS_SBOXES,
    WS_SUB_AH, WS_SUB_AL, WS_SUB_BH, WS_SUB_BL, WS_SUB_KEYS, WS_BOXES, WS_BOX_KEYS, WS_COUNT
};

}  // namespace corr

// One autotuner record. kind 0: fastest small-K tile configuration of the
// exhaustive Pearson contraction for (K, prec, na, nb). kind 1: fastest KSG
// workgroups-per-CU cap for (K = M, prec = k); na = nb = 0.
struct corr_tune_rec {
    int kind;
    int K;
    int prec;
    int64_t na, nb;
    int cfg;
    float ms;
};

struct corr_ctx {
    int device = 0;
    std::vector<corr_tune_rec> tune;
    int num_cus = 256;
    double* psi = nullptr;   // device psi(n), n = 0..psi_max (psi[0] unused)
    int psi_max = 0;
    void* ws[corr::WS_COUNT] = {};
    size_t ws_size[corr::WS_COUNT] = {};
    unsigned long long* keys = nullptr;     // device scratch for max keys
    unsigned long long* keys_host = nullptr;  // pinned host mirror
    void* scratch = nullptr;  // device address of this GPU's fixed scratch (no-allocation calls)
    size_t ws_limit = (size_t)-1;  // cap on the sum of the workspace slots (corr_set_workspace_limit)
    hipStream_t last_stream = nullptr;  // stream of the previous call that used the context's buffers
    bool used = false;
    // kernel timing hook: events per kernel class (see corr_set_timing)
    bool timing = false;
    hipEvent_t ev_start[5] = {};
    hipEvent_t ev_stop[5] = {};
    bool ev_valid[5] = {};
};

namespace corr {

// Grow-only workspace buffer; synchronises `stream` before replacing a buffer.
int ws_get(corr_ctx* ctx, int slot, size_t bytes, hipStream_t stream, void** out);

// Orders a call on `s` after the context's previous call: when the stream
// differs from the previous call's, the device is synchronised first, so two
// streams never use the context's workspaces at the same time.
int ctx_use_stream(corr_ctx* ctx, hipStream_t s);


// ---- statistics layout ------------------------------------------------------
// Per point of a point set, four float arrays of length n (contiguous):
// [0] mu32, [1] inv32 = 1/sigma_pop (KSG), [2] rs32 = 1/sqrt(sum sq dev)
// (Pearson), [3] sigma_pop.
struct Stats {
    float* mu32;
    float* inv32;
    float* rs32;
    float* sigma;
};
inline Stats stats_view(float* base, int64_t n) { return {base, base + n, base + 2 * n, base + 3 * n}; }

// Launchers (standardize.hip). acc64 selects FP64 accumulation.
int launch_stats(const corr_field& f, const Box& box, bool acc64, Stats st, hipStream_t s);

// Output formats of the transpose-normalise kernel.
enum ZFormat { ZF_KSG = 0, ZF_RAW = 1, ZF_F32 = 2, ZF_F16 = 3, ZF_BF16 = 4, ZF_F16X2 = 5, ZF_BF16X2 = 6 };
// Writes rows[i][m] for i in [0, rows_pad) and m in [0, ld); rows i >= count
// and members m >= M are zero. hi / lo as required by the format.
int launch_transpose(const corr_field& f, const Box& box, Stats st, int fmt, void* hi, void* lo,
                     int64_t rows_pad, int64_t ld, hipStream_t s);

int zfmt_for_prec(int prec);
bool prec_split(int prec);
size_t prec_elem_bytes(int prec);

// pairs.hip
// Rows of za/zb are the local indices of the boxes (a whole-grid box makes
// them global indices). key (may be NULL) receives the fused max of |r|.
// Exhaustive max |r| of each of n box pairs (boxes [A boxes n][B boxes n],
// device); keys[t] receives the orderable key of pair t (0: nothing evaluated).
int launch_box_pairs_max(const float* za, const float* zb, int64_t ld, const Box* boxes, int n, int same_field,
                         int max_points, unsigned long long* keys, int num_cus, hipStream_t s);
int launch_pearson_pairs(int prec, const void* za_hi, const void* za_lo, const void* zb_hi, const void* zb_lo,
                         int64_t ld, const int32_t* pairs, int64_t n, float* r_out, const Box& ba, const Box& bb,
                         int same_field, unsigned long long* key, hipStream_t s);

// ksg.hip
struct KsgArgs {
    const float* za;  // point-major rows, row stride ld
    const float* zb;
    int64_t ld;
    const float* inv_a;  // per-point inv32 of the row sets (NULL: raw mode)
    const float* inv_b;
    const int32_t* pairs;  // global indices (NULL: implicit all pairs of the boxes)
    int64_t n;
    int M;
    int k;
    const double* psi;
    float* mi_out;         // may be NULL
    int32_t* counts_out;   // may be NULL
    unsigned long long* key;  // may be NULL: fused region max
    Box ba, bb;            // rows of za/zb are the boxes' local indices
    int same_field;        // skip pA == pB
    const float* sa;       // rows of za / zb sorted ascending, row stride ksg_p2(M), +inf padded
    const float* sb;
    int pw;                // workgroups per CU cap of the resident grid (<= 0: the occupancy limit)
    unsigned long long* work;  // device word the waves take pair chunks from (zeroed by launch_ksg)
    int whole_a, whole_b;  // box covers the whole grid: local index = global index
    FastDiv ax, ay, bx, by;  // grid divisors nx, ny of the boxes' fields (set by launch_ksg)
    FastDiv nbd;             // number of points of box b (implicit all pairs; set by launch_ksg)
};
int launch_ksg(const KsgArgs& a, int num_cus, hipStream_t s);
int ksg_p2(int M);
int ksg_default_pw(int M);
size_t ksg_lds_bytes(int M, int pw);
int launch_sort_rows(const float* z, int64_t ld, int64_t nrows, int M, float* out, int num_cus, hipStream_t s);

// gemm.hip
struct GemmArgs {
    int prec;
    const void* a_hi; const void* a_lo;
    const void* b_hi; const void* b_lo;
    int64_t K;            // padded reduction length (row stride in elements)
    int64_t na, nb;       // valid rows
    int64_t na_pad, nb_pad;
    const int32_t* self_col;  // per A row: local B column of the same point, or -1 (NULL: none)
    unsigned long long* key;
};
int launch_gemm_max(const GemmArgs& g, int num_cus, hipStream_t s);
int gemm_row_pad();
int gemm_col_pad();
int gemm_k_pad(int prec);

// gemm_smallk.hip (members padded to K <= 128; A fragments held in registers)
int launch_gemm_smallk(const GemmArgs& g, int cfg, int num_cus, hipStream_t s);
int smallk_num_configs();
int smallk_row_pad(int cfg);
int smallk_col_pad(int cfg);
int smallk_pad_K(int M);
bool smallk_config_ok(int prec, int cfg, int K);  // exists for prec and runs without scratch at K

// timing hook helpers (api.hip): bracket a launch with events when enabled
enum TimedKernel { TK_GEMM = 0, TK_KSG = 1, TK_PAIRS = 2, TK_STD = 3, TK_AGG = 4, TK_COUNT = 5 };
void timing_begin(corr_ctx* ctx, int which, hipStream_t s);
void timing_end(corr_ctx* ctx, int which, hipStream_t s);

// aggregate.hip: member-major level of f^3 block means (f a power of two <= 64)
int launch_block_means(const corr_field& A, int f, int out_dtype, void* out, int64_t out_stride, hipStream_t s);

// sampling.hip: brick-pair samples and per-pair maxima of sample values
int launch_sample_pairs(const void* boxes, int32_t n_pairs, int32_t n, int sampler, uint64_t seed, int32_t* out,
                        hipStream_t s);
int launch_segment_max(const float* values, const int32_t* pairs, int32_t n_pairs, int32_t n, int use_abs,
                       int same_field, corr_max* out, hipStream_t s);
size_t sample_boxes_bytes(int32_t n_pairs);
void fill_sample_boxes(void* host, const corr_region* regions, const int32_t* region_pairs, int32_t n_pairs,
                       const corr_field& A, const corr_field& B);

// Per-device kernel set-up, done once per (device, kernel, LDS bytes, block
// size) under a lock: raises the kernel's dynamic-LDS limit to `lds` and
// returns the resident workgroups per CU (>= 1) in *per_cu (may be NULL).
// Safe to call from several host threads (api.hip).
int kernel_setup(const void* fn, size_t lds, int threads, int* per_cu);

// small utility kernels (api.hip)
int launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);

// Orderable 32-bit image of a float: monotone in the float's value.
__host__ __device__ inline uint32_t order_bits(float v) {
    uint32_t u;
    __builtin_memcpy(&u, &v, 4);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float from_order_bits(uint32_t o) {
    uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    float v;
    __builtin_memcpy(&v, &u, 4);
    return v;
}

// Max key: [63:32] order_bits(objective), [31:1] 0x7fffffff - lin where lin
// is the local linear pair index la * nb + lb (< 2^31), [0] sign of the
// correlation at that pair. The largest key holds the largest objective and,
// among equal objectives, the smallest lin.
__host__ __device__ inline unsigned long long make_key(float obj, uint32_t lin, uint32_t neg) {
    return ((unsigned long long)order_bits(obj) << 32) |
           ((unsigned long long)((0x7fffffffu - lin) & 0x7fffffffu) << 1) | (unsigned long long)(neg & 1u);
}
__host__ __device__ inline uint32_t key_lin(unsigned long long key) {
    return 0x7fffffffu - (uint32_t)((key >> 1) & 0x7fffffffu);
}

// ------------------------------------------------------------------ Philox
constexpr uint64_t PH_M0 = 0xD2E7470EE14C6C93ull, PH_M1 = 0xCA5A826395121157ull;
constexpr uint64_t PH_W0 = 0x9E3779B97F4A7C15ull, PH_W1 = 0xBB67AE8584CAA73Bull;
constexpr uint64_t KEY_HI = 0x636F7272ull;
enum { ST_INIT = 0, ST_SCHED = 1, ST_UNIF = 2, ST_LOCAL = 3, ST_ROUND = 4 };

// Philox4x64-10 block function (Salmon, Moraes, Dror, Shaw 2011).
__host__ __device__ inline void philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                           uint64_t k1, uint64_t out[4]) {
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += PH_W0;
            k1 += PH_W1;
        }
#ifdef __HIP_DEVICE_COMPILE__
        const uint64_t hi0 = __umul64hi(PH_M0, c0), hi1 = __umul64hi(PH_M1, c2);
#else
        const uint64_t hi0 = (uint64_t)(((unsigned __int128)PH_M0 * c0) >> 64);
        const uint64_t hi1 = (uint64_t)(((unsigned __int128)PH_M1 * c2) >> 64);
#endif
        const uint64_t lo0 = PH_M0 * c0, lo1 = PH_M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

__host__ __device__ inline double ph_u01(uint64_t w) { return (double)(w >> 11) * (1.0 / 9007199254740992.0); }

__host__ __device__ inline double ph_uniform(uint64_t seed, uint64_t pair, uint64_t stream, uint64_t index,
                                             uint64_t axis) {
    uint64_t o[4];
    philox4x64(pair, stream, index, axis, seed, KEY_HI, o);
    return ph_u01(o[0]);
}

}  // namespace corr
