/*
 * bos.h -- batched Bayesian optimal sampling (BOS) of region-pair maxima on
 * the GPU (arXiv 2309.03308, Sec. 3.1), part of libcorr.
 *
 * For every region pair the maximum correlation between a point of region A
 * and a point of region B is estimated from few evaluated point pairs. A
 * sample position is a point of the 6-D space of (cell in A, cell in B),
 * in cell units. Per pair:
 *   1. an initial design of n_init uniformly drawn cells is evaluated;
 *   2. then, per iteration, a Gaussian process with a Matern-5/2 covariance
 *      (length scale `lengthscale` cells on every axis, unit signal
 *      variance, `jitter` on the diagonal; observations standardised per
 *      pair) is conditioned on the pair's observations, the upper confidence
 *      bound mu + kappa * sigma is maximised over a seeded candidate set
 *      (n_uniform uniform points and n_local Gaussian perturbations of sd
 *      `local_sd` cells around the best cell so far, clipped to the box), a
 *      batch of b picks is chosen by Kriging believer (each pick joins the GP
 *      with its posterior mean as value), each pick is rounded to a cell by
 *      the probabilistic reparameterisation P = floor(theta) +
 *      Ber(theta - floor(theta)) (Sec. 3.1), cells already observed are not
 *      evaluated again (the slot is used), and the new cells are evaluated;
 *   3. batch sizes are uneven per pair: the n_total - n_init acquired
 *      samples are split into batches of 8 * p, p = 1 + floor(u * min(8,
 *      units left)), so 8..64 per batch.
 * Objective: |r| (CORR_PEARSON) or the KSG MI (CORR_KSG), computed as in
 * corr.h. Random numbers: Philox4x64-10, counter (pair, stream, index,
 * axis), key (seed, 0x636f7272); streams 0 initial design, 1 schedule,
 * 2 uniform candidates, 3 local candidates, 4 rounding.
 *
 * All pairs advance together: bos_sample_step runs one iteration for every
 * pair that still has work, as one persistent kernel whose workgroups walk
 * the iteration's pair list (costliest pairs first, static stride) followed
 * by a one-thread kernel that advances the device-side iteration counter.
 * The two launches are captured once into a HIP graph and replayed
 * (BOS_LAUNCH_GRAPH, the default) or launched directly (BOS_LAUNCH_PLAIN);
 * both give bit-identical results.
 * Calls that wait for the GPU (bos_create, bos_run, bos_results,
 * bos_history, bos_save, bos_load, bos_destroy) poll with a deadline
 * (bos_set_launch) and return CORR_EHIP when it passes instead of blocking.
 * Ownership: bos_state owns its device state and workspaces; it borrows the
 * fields (their device memory must stay valid until bos_destroy) and the
 * corr_ctx. Errors as in corr.h.
 */
#ifndef BOS_H
#define BOS_H

#include <stdint.h>

#include "corr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bos_config {
    int32_t measure;    /* CORR_PEARSON or CORR_KSG */
    int32_t k;          /* KSG neighbours (CORR_KSG) */
    int32_t n_init;     /* initial design per pair, >= 2 */
    int32_t n_total;    /* samples per pair, <= 128; n_total - n_init a positive multiple of 8 */
    int32_t n_uniform;  /* uniform candidates per iteration */
    int32_t n_local;    /* local candidates per iteration; n_uniform + n_local in [64, 1024] */
    double kappa;       /* UCB weight (0.5) */
    double lengthscale; /* Matern length scale in cells (3) */
    double local_sd;    /* sd of the local candidates in cells (1) */
    double jitter;      /* diagonal jitter (1e-6) */
    uint64_t seed;
} bos_config;

typedef struct bos_state bos_state;

/* Launch modes of an iteration (bos_set_launch). */
enum { BOS_LAUNCH_GRAPH = 0, BOS_LAUNCH_PLAIN = 1 };

/* Fill a config with the defaults listed above (measure CORR_PEARSON, k 10,
 * n_init 20, n_total 100, n_uniform 384, n_local 128, seed 1). */
void bos_config_default(bos_config* cfg);

/*
 * Create the sampler for `n_pairs` region pairs of fields A (regions on the
 * A side) and B. regions: HOST [n_regions] boxes (inside the grids);
 * region_pairs: HOST int32 [n_pairs][2] indices into regions (A side, B
 * side). Standardises the fields into the state's workspaces on `stream`.
 * No sample is evaluated yet.
 */
int bos_create(corr_ctx* ctx, const corr_field* A, const corr_field* B, const corr_region* regions,
               int32_t n_regions, const int32_t* region_pairs, int32_t n_pairs, const bos_config* cfg,
               bos_state** out, corr_stream_t stream);

/*
 * Proposal prior (the learned proposal): HOST float [n_pairs][6] proposed
 * cell (local coordinates of the A cell, then the B cell) per pair, or a
 * negative first coordinate for none. The cell, rounded and clamped to the
 * box, replaces the first cell of the initial design; like every
 * observation it then steers the GP, and the local candidates are drawn
 * around the incumbent (the best observation so far), which it is as long
 * as nothing better has been seen. Must be called before the first
 * bos_sample_step (CORR_ESTATE otherwise).
 */
int bos_set_prior(bos_state* st, const float* cells);

/*
 * Launch mode (BOS_LAUNCH_GRAPH or BOS_LAUNCH_PLAIN) and the longest time in
 * seconds (> 0; default 300) that a call waits for the GPU before it returns
 * CORR_EHIP. May be called at any time; a captured graph is kept.
 */
int bos_set_launch(bos_state* st, int32_t mode, double timeout_s);

/*
 * One iteration for every pair with work left, enqueued on `stream` (the
 * call does not wait for it): the first call evaluates the initial designs,
 * later calls one batch per pair. n_active_out (HOST, nullable) receives the
 * number of pairs that still have batches left after this iteration; it
 * follows from the schedule, which the host knows, so no read-back is needed.
 * After the last iteration further calls do nothing and report 0.
 */
int bos_sample_step(bos_state* st, corr_stream_t stream, int32_t* n_active_out);

/* Run steps until no pair is active, then wait for them (with the deadline). */
int bos_run(bos_state* st, corr_stream_t stream);

/* Per pair: maximum found (value, signed value at it, global pa/pb) and the
 * number of distinct evaluated point pairs. out: HOST [n_pairs].
 * Synchronises `stream`. */
int bos_results(bos_state* st, corr_max* out, corr_stream_t stream);

/* Evaluated cells (HOST int32 [n_total][6], local coordinates) and values
 * (HOST float [n_total]) of one pair in evaluation order; *n_out receives
 * their number. Synchronises `stream`. */
int bos_history(bos_state* st, int32_t pair, int32_t* cells, float* values, int32_t* n_out,
                corr_stream_t stream);

/* The uneven batch schedule drawn from the seed (Sec. 3.1 batching, the rule
 * in the header comment): sched_out HOST int32 [n_pairs][16] receives each
 * pair's batch sizes in order (unused entries 0), n_batches_out HOST int32
 * [n_pairs] the number of batches. Host-only; no GPU work. */
int bos_schedule(bos_state* st, int32_t* sched_out, int32_t* n_batches_out);

/* Save / restore the sampling state (observations, schedules, iteration)
 * to / from a file; the restored state continues bit-identically. load
 * requires a state created with the same fields, pairs and config. */
int bos_save(bos_state* st, const char* path, corr_stream_t stream);
int bos_load(bos_state* st, const char* path, corr_stream_t stream);

/* Free the state after its enqueued work has finished (waiting with the
 * deadline; if the deadline passes the device buffers are left allocated
 * rather than freed under running work). NULL is allowed. */
void bos_destroy(bos_state* st);

#ifdef __cplusplus
}
#endif

#endif /* BOS_H */
