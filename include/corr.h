/*
 * corr.h -- C ABI of libcorr, the MI355X (gfx950) correlation hot path for
 * focus+context correlation views of 3D ensembles (arXiv 2309.03308).
 *
 * What it computes (Sec. 3): an ensemble of M members (the paper's E) on an
 * nx x ny x nz grid; for grid points pA and pB the point-to-point correlation
 * across members is either the Pearson coefficient (PPMCC, Sec. 3.2) or the
 * Kraskov k-nearest-neighbour mutual-information estimate (KSG/"KMI",
 * Sec. 3.2); the indicator of a region (brick) pair is the maximum of these
 * over pA in A and pB in B (Sec. 3). Batched Bayesian optimal sampling of
 * that maximum (Sec. 3.1) is declared in bos.h.
 *
 * Conventions for every call:
 *  - Device pointers are HIP device memory owned by the caller; the library
 *    never frees caller memory. Library objects (corr_ctx) own their
 *    internal workspaces.
 *  - Struct arguments (corr_field, corr_region) are read during the call only.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = legacy default
 *    stream) and the call returns; calls that write HOST outputs synchronise
 *    that stream before returning.
 *  - Arguments are validated on the host before anything is enqueued:
 *    CORR_EINVAL for bad arguments (null pointers, M < 2, k outside
 *    [1, M-1], regions outside the grid, n < 0, fields of different M),
 *    CORR_EUNSUPPORTED for a dtype / precision / size the library does not
 *    handle, CORR_ENOMEM when a workspace cannot be allocated, CORR_EHIP for
 *    a failed HIP call (its message is kept in corr_last_error()).
 *    No C++ exception crosses this ABI.
 *  - One host thread at a time per corr_ctx; separate contexts may be used
 *    from separate threads. Calls run on the calling thread's current HIP
 *    device, which must be the device the context was created for.
 *  - A context's workspaces serve one stream at a time: when a call names a
 *    different stream than the previous call on the same context, the
 *    library first synchronises the device (hipDeviceSynchronize), so work
 *    on two streams never shares the workspaces while in flight. Use one
 *    context per stream to overlap streams without that wait.
 *  - Point indices are global linear indices p = x + nx * (y + ny * z),
 *    int32. A region's local index follows the same x-fastest rule relative
 *    to its origin.
 */
#ifndef CORR_H
#define CORR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A hipStream_t (same underlying type). */
typedef struct ihipStream_t* corr_stream_t;

enum corr_status {
    CORR_OK = 0,
    CORR_EINVAL = 1,
    CORR_EUNSUPPORTED = 2,
    CORR_ENOMEM = 3,
    CORR_EHIP = 4,
    CORR_ESTATE = 5
};

/* Storage type of a field in HBM. FP16 values are upcast exactly to FP32. */
enum corr_dtype { CORR_F32 = 0, CORR_F16 = 1 };

/* Arithmetic of the Pearson contraction. F32: FP32 operands. F16/BF16: one
 * pass with 16-bit operands and FP32 accumulation. F16X3/BF16X3: operands
 * split into hi + lo 16-bit parts, r = hi.hi + hi.lo + lo.hi, FP32
 * accumulation. */
enum corr_prec {
    CORR_PREC_F32 = 0,
    CORR_PREC_F16 = 1,
    CORR_PREC_BF16 = 2,
    CORR_PREC_F16X3 = 3,
    CORR_PREC_BF16X3 = 4
};

enum corr_measure { CORR_PEARSON = 0, CORR_KSG = 1 };

/* Sample sequences over a brick pair's 6-D box (Sec. 3.1): uniform
 * pseudo-random, Halton, and the (six-dimensional) plastic sequence. */
enum corr_sampler { CORR_SAMPLE_UNIFORM = 0, CORR_SAMPLE_HALTON = 1, CORR_SAMPLE_PLASTIC = 2 };

/* Estimation strategy for a brick pair (Sec. 5, sampling strategy). */
enum corr_strategy { CORR_STRATEGY_BOS = 0, CORR_STRATEGY_RANDOM = 1, CORR_STRATEGY_EXHAUSTIVE = 2 };

/* corr_ksg_mi_pairs flag: use the stored values as the KSG samples instead
 * of z-scoring each point first. */
#define CORR_KSG_RAW 1u

typedef struct corr_ctx corr_ctx;

/* An ensemble field (Sec. 3): value(m, p) = data[m * member_stride + p],
 * member-major. member_stride = 0 means nx * ny * nz. */
typedef struct corr_field {
    const void* data;      /* device pointer */
    int32_t dtype;         /* enum corr_dtype */
    int32_t M;             /* ensemble members, >= 2 */
    int32_t nx, ny, nz;    /* grid extent */
    int64_t member_stride; /* elements between consecutive members */
} corr_field;

/* A region (the paper's brick): half-open box of grid cells. */
typedef struct corr_region {
    int32_t x0, y0, z0;
    int32_t dx, dy, dz;
} corr_region;

/* Result of a region-pair maximum. value = max |r| (Pearson) or max MI
 * (KSG); signed_value = r (or MI) at the argmax; pa, pb = global indices
 * of the argmax (-1 if nothing was evaluated); n_evaluated = pairs counted. */
typedef struct corr_max {
    float value;
    float signed_value;
    int32_t pa, pb;
    int64_t n_evaluated;
} corr_max;

/* Library version string. */
const char* corr_version(void);

/* Create a context on HIP device `device`; allocates the digamma table and
 * small device scratch. *out receives the context. */
int corr_create(int device, corr_ctx** out);

/* Wait for the context's work, free its workspaces and the context. NULL ok. */
void corr_destroy(corr_ctx* ctx);

/* Static description of a status code. */
const char* corr_status_str(int status);

/* Last error message of the calling thread ("" if none). */
const char* corr_last_error(void);

/*
 * Cap on the device memory a context keeps in its grow-only workspaces (the
 * sum over all of them), in bytes; 0 removes the cap (the default). A call
 * whose workspaces would grow past the cap returns CORR_ENOMEM before its
 * main kernel (kernels it enqueued up to that point wrote only into the
 * context's own workspaces); the workspaces already held are kept. Prepared
 * fields, BOS states and networks own their buffers and are not counted.
 */
int corr_set_workspace_limit(corr_ctx* ctx, size_t bytes);

/*
 * Per-point statistics of every grid point of field A (Sec. 3.2: Pearson
 * needs only means and variances; KSG works on z-scored samples).
 * Two-pass sums in member order in FP64. Outputs (device, nx*ny*nz floats
 * each, any may be NULL): mu32 = fl32(mean), inv32 = fl32(1 / sigma_pop)
 * (0 for a constant point), sigma = fl32(sigma_pop) (the ensemble spread).
 */
int corr_standardize(corr_ctx* ctx, const corr_field* A, float* mu32, float* inv32, float* sigma,
                     corr_stream_t stream);

/*
 * Pearson r for a list of point pairs (Sec. 3.2):
 *   r_i = sum_m (a_m - mean a)(b_m - mean b) / sqrt(sum (a - mean a)^2 sum (b - mean b)^2)
 * with a = A[:, pairs[i][0]], b = B[:, pairs[i][1]], clamped to [-1, 1];
 * a constant point gives r = 0.
 * pairs: device int32 [n][2] of global indices into A and B.
 * r_out: device float [n]. prec: enum corr_prec.
 */
int corr_pearson_pairs(corr_ctx* ctx, const corr_field* A, const corr_field* B, const int32_t* pairs,
                       int64_t n, int prec, float* r_out, corr_stream_t stream);

/*
 * Kraskov (KSG) mutual information, in nats, for a list of point pairs
 * (Sec. 3.2). For pair (a, b): x_i, y_i are the z-scored samples of a and b
 * (z = fl32(fl32(v - mu32) * inv32), see corr_standardize; raw values with
 * CORR_KSG_RAW); d_ij = max(|x_i - x_j|, |y_i - y_j|) in FP32; eps_i = k-th
 * smallest d_ij over j != i; n_x,i = #{j != i : |x_i - x_j| < eps_i}, n_y,i
 * alike; MI = psi(M) + psi(k) - (1/M) sum_i [psi(n_x,i + 1) + psi(n_y,i + 1)].
 * A constant point gives MI = 0 and zero counts (not with CORR_KSG_RAW).
 * pairs: device int32 [n][2]; mi_out: device float [n];
 * counts_out: NULL or device int32 [n][M][2] receiving (n_x,i, n_y,i).
 * k in [1, min(M-1, 31)].
 */
int corr_ksg_mi_pairs(corr_ctx* ctx, const corr_field* A, const corr_field* B, const int32_t* pairs,
                      int64_t n, int32_t k, uint32_t flags, float* mi_out, int32_t* counts_out,
                      corr_stream_t stream);

/*
 * A field standardised once for many pair-list calls (Sec. 3.2: Pearson
 * needs only each point's mean and variance, KSG its z-scored samples and,
 * here, their sorted marginals). corr_pearson_pairs and corr_ksg_mi_pairs
 * standardise the whole field on every call; a prepared field holds that
 * work, so repeated calls only gather the rows their pairs name.
 *  measure CORR_PEARSON: rows in the format of `prec` (as corr_pearson_pairs
 *    with that prec); CORR_KSG: z-scored FP32 rows, the sorted rows and the
 *    per-point statistics (as corr_ksg_mi_pairs without CORR_KSG_RAW).
 * The handle owns its device buffers (about nx*ny*nz*M*(2 or 4) bytes for
 * Pearson, 2x that plus the sorted rows for KSG) and keeps no reference to
 * A's data: after A changes, prepare again. It is enqueued on `stream`; use
 * it on that stream or after synchronising it.
 */
typedef struct corr_prepared corr_prepared;
int corr_prepare(corr_ctx* ctx, const corr_field* A, int measure, int prec, corr_prepared** out,
                 corr_stream_t stream);
/* Frees the handle's buffers after synchronising the device. NULL is ignored. */
void corr_prepared_destroy(corr_prepared* p);

/*
 * Exhaustive Pearson maxima of many small box pairs in one call (Sec. 3, the
 * brick-pair indicator, for boxes of up to 4096 points each, e.g. the
 * neighbourhoods of candidate cells). For box pair t: the maximum |r| over
 * (pA, pB) in boxes_a[t] x boxes_b[t], with the signed r, the argmax (the
 * smallest local index la * |b| + lb among equal values) and n_evaluated, as
 * corr_region_max returns them; pA == pB is skipped when A and B are the same
 * handle. A and B: prepared for CORR_PEARSON with CORR_PREC_F32 (else
 * CORR_EUNSUPPORTED). boxes_a, boxes_b: HOST corr_region [n] inside the
 * fields' grids; out: HOST corr_max [n]. Synchronises `stream`.
 */
int corr_box_pairs_max(corr_ctx* ctx, const corr_prepared* A, const corr_prepared* B, const corr_region* boxes_a,
                       const corr_region* boxes_b, int32_t n, corr_max* out, corr_stream_t stream);

/*
 * corr_pearson_pairs on prepared fields: A and B (may be the same handle)
 * prepared for CORR_PEARSON with the same member count and precision; the
 * results equal corr_pearson_pairs with that precision bit for bit.
 */
int corr_pearson_pairs_prepared(corr_ctx* ctx, const corr_prepared* A, const corr_prepared* B,
                                const int32_t* pairs, int64_t n, float* r_out, corr_stream_t stream);

/*
 * corr_ksg_mi_pairs on prepared fields (flags 0): A and B (may be the same
 * handle) prepared for CORR_KSG with the same member count; mi and counts
 * equal corr_ksg_mi_pairs's bit for bit.
 */
int corr_ksg_mi_pairs_prepared(corr_ctx* ctx, const corr_prepared* A, const corr_prepared* B,
                               const int32_t* pairs, int64_t n, int32_t k, float* mi_out,
                               int32_t* counts_out, corr_stream_t stream);

/*
 * Region-pair maximum (Sec. 3: the brick-pair indicator is the maximum of
 * the point-to-point correlations between the two bricks).
 *  measure CORR_PEARSON: objective |r|; CORR_KSG: objective MI.
 *  sample_pairs == NULL: every (pA, pB) in ra x rb is evaluated (for Pearson
 *    as one fused MFMA contraction that never stores the correlations);
 *  otherwise: device int32 [n_samples][2] of global indices, each inside
 *    ra resp. rb, and only those pairs are evaluated.
 * When A and B are the same field, pA == pB is skipped. Ties go to the
 * smallest (local pA, local pB) for exhaustive runs. prec applies to
 * Pearson; k to KSG. out: HOST pointer; the call synchronises `stream`.
 * An exhaustive call over 2^31 or more point pairs runs as consecutive
 * pieces of ra (same result and tie-break as one pass); a sampled call over
 * such a region pair returns CORR_EUNSUPPORTED.
 */
int corr_region_max(corr_ctx* ctx, const corr_field* A, const corr_region* ra, const corr_field* B,
                    const corr_region* rb, int measure, int prec, int32_t k, const int32_t* sample_pairs,
                    int64_t n_samples, corr_max* out, corr_stream_t stream);

/*
 * corr_region_max without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc. Same arguments, validation, kernels and results as
 * corr_region_max (out: HOST, the call synchronises `stream`). Its
 * workspaces (statistics, standardised rows, sorted rows, self-pair list)
 * come from a fixed device array of CORR_SCRATCH_BYTES per GPU, owned by the
 * library and held until the process ends, instead of the context's
 * grow-only buffers; the call makes no hipMalloc / hipFree or other
 * allocating call. A call that needs more scratch returns CORR_EINVAL with
 * the size in corr_last_error(). Every context on a GPU shares that GPU's
 * array and it keeps the last call's contents: calls that overlap in time on
 * one GPU (two streams, two host threads) race on it and must be ordered by
 * the caller.
 * Sizes: e.g. exhaustive FP16 Pearson over two 20480-point regions at M = 100
 * needs about 10 MB; KSG over the same regions about 38 MB.
 */
#define CORR_SCRATCH_BYTES ((size_t)64 << 20)
int corr_region_max_noalloc(corr_ctx* ctx, const corr_field* A, const corr_region* ra, const corr_field* B,
                            const corr_region* rb, int measure, int prec, int32_t k, const int32_t* sample_pairs,
                            int64_t n_samples, corr_max* out, corr_stream_t stream);

/*
 * Autotuner for the exhaustive Pearson contraction (tile shapes of the
 * small-ensemble kernel, M <= 128): runs every tile configuration valid for
 * `prec` on the given region pair `reps` times, timing the contraction kernel
 * with HIP events, and records the fastest (median) in the context's table;
 * later corr_region_max calls of the same shape use it. best_cfg / best_ms
 * (HOST, nullable) receive the choice (-1 when M > 128: nothing to tune).
 * Synchronises `stream`.
 */
int corr_autotune(corr_ctx* ctx, const corr_field* A, const corr_region* ra, const corr_field* B,
                  const corr_region* rb, int prec, int reps, int* best_cfg, float* best_ms, corr_stream_t stream);

/*
 * Autotuner for the KSG launch (Sec. 3.2 estimator): times each candidate
 * cap on the workgroups per CU of the resident grid (1, 2, 4, 8, 16; the
 * kernel's occupancy limit applies on top) on the given pair list, as
 * corr_ksg_mi_pairs would run it, and records the fastest for (M, k).
 * best_pw (the cap) / best_ms: HOST, nullable. Synchronises `stream`.
 */
int corr_ksg_autotune(corr_ctx* ctx, const corr_field* A, const corr_field* B, const int32_t* pairs, int64_t n,
                      int32_t k, int reps, int* best_pw, float* best_ms, corr_stream_t stream);

/* Write / read the context's tuning table as JSON lines (one record per
 * line: arch, kind, K, prec, na, nb, cfg, ms). Loading merges into the
 * table; malformed or out-of-range records are skipped. */
int corr_tune_save(corr_ctx* ctx, const char* path);
int corr_tune_load(corr_ctx* ctx, const char* path);

/*
 * Sub-brick maxima: one level of brick refinement of a pair (Sec. 3 and 4.2, the
 * focus view refines a selected brick pair). Brick ra is split into
 * splits_a[0] x splits_a[1] x splits_a[2] sub-bricks and rb into splits_b
 * likewise (each axis as evenly as possible, the first parts one cell
 * larger), and for every (sub-brick i of ra, sub-brick j of rb) the exhaustive
 * Pearson maximum of |r| is computed exactly as corr_region_max does it
 * (same precision modes, the same exclusion of a point paired with itself
 * within one field, the same argmax rule). Both fields are standardised once.
 *   splits_a, splits_b: HOST int32[3], each in [1, the axis extent].
 *   out: HOST corr_max[n_a * n_b], out[i * n_b + j], sub-bricks numbered
 *        x-fastest (x, then y, then z).
 * CORR_EINVAL for bad splits or regions, CORR_EUNSUPPORTED when a sub-brick
 * pair has 2^31 or more point pairs; synchronises `stream`.
 */
int corr_region_submax(corr_ctx* ctx, const corr_field* A, const corr_region* ra, const int32_t* splits_a,
                       const corr_field* B, const corr_region* rb, const int32_t* splits_b, int prec,
                       corr_max* out, corr_stream_t stream);

/*
 * Samples of brick pairs (Sec. 3.1: random or quasi-random sampling of the
 * 6-D box x, y, z in brick A and x, y, z in brick B). For region pair p
 * (regions[region_pairs[2p]], regions[region_pairs[2p+1]]) and sample
 * s in [0, n_samples): u in [0,1)^6 from `sampler` (enum corr_sampler), cell
 * c_j = min(floor(u_j d_j), d_j - 1) with d = the two regions' extents, and
 * out[2 (p n + s)] / out[2 (p n + s) + 1] = the global indices of the A and B
 * points (A's grid for the first, B's for the second).
 *   uniform: u_j = Philox4x64-10 word 0 of counter (p, 5, s, j), key
 *            (seed, 0x636F7272), as (w >> 11) 2^-53;
 *   Halton:  u_j = frac(h_{b_j}(s + 1) + c_j), bases 2, 3, 5, 7, 11, 13;
 *   plastic: u_j = frac(c_j + (s + 1) alpha_j), alpha_j = phi^-j by repeated
 *            division, phi = 1.1127756842787055 (root of x^7 = x + 1);
 *   c_j = the uniform of counter (p, 6, 0, j).
 * regions / region_pairs: HOST arrays ([n_regions], [n_pairs][2]); out:
 * device int32 [n_pairs][n_samples][2]. CORR_EINVAL for bad indices or
 * regions outside their grids, n_pairs < 0, n_samples < 0 or
 * n_pairs * n_samples >= 2^31; CORR_EUNSUPPORTED for an unknown sampler.
 * Synchronises `stream` (the pair boxes are staged from host memory).
 */
int corr_sample_pairs(corr_ctx* ctx, const corr_field* A, const corr_field* B, const corr_region* regions,
                      int32_t n_regions, const int32_t* region_pairs, int32_t n_pairs, int sampler,
                      int32_t n_samples, uint64_t seed, int32_t* out, corr_stream_t stream);

/*
 * Sampled maxima of many brick pairs at once: the samples of
 * corr_sample_pairs, evaluated with corr_pearson_pairs (objective |r|, in
 * precision `prec`) or corr_ksg_mi_pairs (objective MI, k neighbours), and
 * per pair the earliest sample of the largest objective. Within one field
 * (A and B the same) a sample of a point with itself is skipped, as in the
 * exhaustive maxima. out: HOST corr_max[n_pairs] (n_evaluated = the samples
 * counted). Synchronises `stream`.
 */
int corr_sampled_max(corr_ctx* ctx, const corr_field* A, const corr_field* B, const corr_region* regions,
                     int32_t n_regions, const int32_t* region_pairs, int32_t n_pairs, int measure, int prec,
                     int32_t k, int sampler, int32_t n_samples, uint64_t seed, corr_max* out,
                     corr_stream_t stream);

/*
 * Strategy for a pair of bricks with na and nb points (Sec. 5, sampling
 * strategy): CORR_STRATEGY_BOS when both hold at least 16^3 points, else
 * CORR_STRATEGY_EXHAUSTIVE when na * nb / pairs_per_s <= budget_s (the
 * paper's 5 s), else CORR_STRATEGY_RANDOM. pairs_per_s: the exhaustive
 * evaluation rate of the measure at hand (> 0). strategy: HOST int.
 */
int corr_choose_strategy(int64_t na, int64_t nb, double pairs_per_s, double budget_s, int32_t* strategy);

/*
 * One level of the mean tree (Sec. 3.3, sampling from spatial aggregates):
 * for every member m and every block of f x f x f grid points, the mean of
 * A's values over the block. Blocks tile the grid from the origin; a block on
 * a high face holds the min(f, n - f*X) points left on that axis and its
 * mean is over those. The result is an ensemble field of the same M on a
 * ceil(nx/f) x ceil(ny/f) x ceil(nz/f) grid (x fastest), on which every
 * other call of this library can estimate brick-pair maxima (Sec. 5 compares
 * maxima at f = 1, 2 and 4).
 *   f:          a power of two in [1, 64] (else CORR_EINVAL).
 *   out:        device, member-major: value(m, q) = out[m * out_stride + q];
 *               caller-owned, must not overlap A's data.
 *   out_dtype:  CORR_F32 or CORR_F16 (else CORR_EUNSUPPORTED).
 *   out_stride: elements between members; 0 = the level's point count
 *               (smaller non-zero values are CORR_EINVAL).
 * Sums in FP64; the mean is rounded once to out_dtype.
 */
int corr_block_means(corr_ctx* ctx, const corr_field* A, int f, int out_dtype, void* out, int64_t out_stride,
                     corr_stream_t stream);

/*
 * Kernel timing hook (instrumentation, no effect on results). With timing
 * on, the main kernel of each call is bracketed by HIP events recorded on the
 * call's stream. corr_kernel_time_ms waits for the last such kernel of class
 * `which` and returns its duration in milliseconds (-1 if none yet).
 * which: 0 = Pearson contraction (exhaustive region max), 1 = KSG,
 *        2 = Pearson pair list, 3 = standardisation (statistics + layout),
 *        4 = mean-tree level (corr_block_means).
 */
int corr_set_timing(corr_ctx* ctx, int on);
int corr_kernel_time_ms(corr_ctx* ctx, int which, float* ms);

#ifdef __cplusplus
}
#endif

#endif /* CORR_H */
