/*
 * cmflb.h -- C ABI of libcmflb, the MI355X (gfx950) implementation of the
 * fused stream-and-collide step of the fluctuating orthogonal-central-moment
 * lattice Boltzmann method (De Rosis & Zhou, "A fluctuating lattice
 * Boltzmann formulation based on orthogonal central moments",
 * arXiv 2602.16486), for the D2Q9, D3Q27 and D3Q19 lattices on periodic
 * boxes.
 *
 * One time step is the paper's per-site algorithm (Sec. 2.2, "Algorithm of
 * computation"): density and velocity (eq. macro), standard normals for the
 * non-conserved modes, central moments k = T(u) f (Sec. 2.2, 2.3, 2.4), the
 * collision k* = (I - Lambda) k + Lambda k_eq + I~ phi eta (eq. cm_collision)
 * with phi from eq. phi_general, the back transformation f* = T(u)^-1 k*,
 * and the streaming f_i(x + c_i, t + 1) = f*_i(x, t) (eq. streaming).
 *
 * Conventions shared by every entry point:
 *  - Site order is x fastest: s = x + nx * (y + ny * z); nz = 1 for D2Q9.
 *  - Population order is the paper's velocity order (Sec. 2.2 for D2Q9,
 *    Sec. 2.3 for D3Q27; D3Q19, whose order Sec. 2.4 does not give, uses
 *    the D3Q27 order without the eight corners).  "Populations" at the ABI
 *    are the pre-collision populations f_i(x, t) of the current step t, in
 *    FP64, laid out q x N (population-major).
 *  - Noise: the paper asks for independent standard normal variables
 *    (Sec. 2.1, eq. Xi_pop); eta of mode v at site s and step t comes from
 *    Philox4x32-10 (Salmon et al., SC'11) with key (seed low word, seed high
 *    word) and counter (s, t mod 2^32, replica, block + 256 floor(t / 2^32))
 *    -- (s, t, replica, block) for t < 2^32; the counters of all steps below
 *    2^56 are distinct, and no call accepts a step beyond that (about 2
 *    million years of steps at one per microsecond); normal n = v - 3 (D2Q9) or v - 4
 *    (D3Q19, D3Q27), pair p = n / 2 uses block p / 2 and words 2 (p mod 2),
 *    2 (p mod 2) + 1 as (a, b); u1 = ((a >> 8) + 1) 2^-24,
 *    u2 = (b >> 8) 2^-24; the pair is r cos(2 pi u2), r sin(2 pi u2) with
 *    r = sqrt(-2 ln u1) (even n takes the cosine).  Results do not depend
 *    on tiling or launch shape.
 *  - Every function returns CMF_OK (0) or a negative status; the message of
 *    the last failure on the calling thread is cmf_last_error().  No
 *    exception crosses the ABI.
 *  - Host pointers are owned by the caller and are never retained.  Device
 *    memory allocated by cmf_create is owned by the lattice and released by
 *    cmf_destroy.
 *  - Steps are enqueued asynchronously on the HIP stream given at creation
 *    (NULL: the lattice creates a stream of its own, default priority, and
 *    destroys it with the lattice); every call that returns host data
 *    synchronises that stream first.  A lattice lives on the device that is
 *    current when it is created; a stream passed in must belong to it.
 *  - Threads: different lattices and ensembles may be used from different
 *    host threads at the same time (graph capture is thread-local, the
 *    process-wide launch-shape cache is locked); one lattice or ensemble
 *    must not be used by two threads at once.
 */
#ifndef CMFLB_H
#define CMFLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CMF_OK 0
#define CMF_EINVAL -1       /* invalid argument */
#define CMF_ENOMEM -2       /* device or host allocation failed */
#define CMF_EHIP -3         /* a HIP runtime call failed */
#define CMF_ENONFINITE -4   /* a recorded step had non-finite rho or u */
#define CMF_EUNSUPPORTED -5 /* combination not built into this library */

/* Storage type of the populations in HBM.  Populations are stored as
 * deviations f_i - w_i rho0.  F32/F16/BF16 collide in FP32; F64 collides in
 * FP64.  F16/BF16 store (f_i - w_i rho0) / s_i with a per-population
 * power-of-two scale s_i = 2^ceil(log2(sigma_i)),
 * sigma_i = sqrt(rho0 kT w_i / c_s^2) (sigma_i = 1e-2 w_i when kT = 0),
 * rounded to nearest even. */
enum {
  CMF_STORE_F64 = 0,
  CMF_STORE_F32 = 1,
  CMF_STORE_F16 = 2,
  CMF_STORE_BF16 = 3
};

/* desc.flags */
#define CMF_FLAG_NO_GRAPH 1u   /* enqueue launches directly, never capture */
#define CMF_FLAG_NO_STATS 2u   /* skip the per-step statistics finalize */
#define CMF_FLAG_IN_PLACE 4u   /* in-place (AA) streaming on one population
                                  buffer instead of two: the streaming of
                                  eq. (streaming) in another storage order,
                                  half the population memory, the same
                                  results bit for bit (single lattices whose
                                  z planes of q ny nx values take below
                                  4 GiB) */

typedef struct {
  int32_t q;         /* 9 (D2Q9), 19 (D3Q19) or 27 (D3Q27) */
  int32_t nx, ny, nz;/* box edges, >= 1; nz must be 1 for D2Q9 */
  int32_t storage;   /* CMF_STORE_* */
  uint32_t flags;    /* CMF_FLAG_* */
  double rho0;       /* reference density of the deviation storage, > 0 */
  double tau;        /* relaxation time, omega = 1 / tau, tau >= 0.5 */
  double kT;         /* thermal energy per site, >= 0 */
  const double *lambda; /* NULL: the paper's rates (D2Q9: Lambda_4,5 = omega,
                           others 1, Sec. 2.2; D3Q27: Lambda_7-9 = omega,
                           others 1, Sec. 2.3).  Otherwise q host doubles,
                           one rate per mode in [0, 2]; copied. */
  uint64_t seed;     /* Philox key */
  uint32_t replica;  /* third Philox counter word */
  int32_t series_capacity; /* rows kept in the device statistics ring;
                              0 selects 4096 */
} cmf_desc;

/* One row of the per-step statistics, taken from the pre-collision state
 * of step `step` (the state whose density and velocity the collision of
 * that step uses).  Sums run over all N sites and are accumulated in FP64. */
typedef struct {
  double step;      /* step index */
  double sum_rho;   /* sum of rho */
  double sum_j[3];  /* sum of rho u_a */
  double sum_u[3];  /* sum of u_a */
  double sum_u2[3]; /* sum of u_a^2 */
  double nonfinite; /* number of sites whose rho or u is not finite */
} cmf_moments;

typedef struct cmf_lattice cmf_lattice;

/* Version string of the library.  Never fails. */
const char *cmf_version(void);

/* Message of the last failure on the calling thread ("" if none). */
const char *cmf_last_error(void);

/* Number of HIP devices visible (0 when there is none); never fails. */
int cmf_device_count(void);

/* Create a lattice on the current HIP device: validates `desc`, builds the
 * per-mode constants in FP64 (norms b_v, rates Lambda_v, noise prefactors
 * sqrt(kT Lambda_v (2 - Lambda_v) b_v / c_s^2) of eq. phi_general, storage
 * scales) and allocates two population buffers of q x N elements of the
 * storage type plus statistics scratch.  The populations start at rest
 * (f = w rho0) at step 0.  `hip_stream` is a hipStream_t, or NULL for a
 * stream owned by the lattice.
 * Errors: CMF_EINVAL (bad sizes, tau < 0.5, kT < 0, rho0 <= 0, rates out of
 * [0, 2], N >= 2^31, nx >= 2^28), CMF_ENOMEM, CMF_EHIP. */
int cmf_create(const cmf_desc *desc, void *hip_stream, cmf_lattice **out);

/* As cmf_create, but the two population buffers (one with
 * CMF_FLAG_IN_PLACE) live in caller-owned device memory (for instance a
 * torch tensor): dev_ptr, 256-byte aligned, on the current device, holding
 * at least cmf_external_bytes(desc) bytes; buffer 0 starts at dev_ptr,
 * buffer 1 half-way.  Their contents are the library's internal storage
 * (deviations f - w rho0, scaled for 16-bit storage, in a row-interleaved
 * order: for lattice row y + ny z, q rows of nx values, the populations of
 * the 3-D lattices ordered by their velocities (c_z, c_y, c_x), those of
 * D2Q9 in the paper's order; with in-place streaming, in the natural slot order after an even
 * number of steps and in the swapped one after an odd number), not the
 * canonical populations: read those with
 * cmf_get_populations.  The lattice writes the rest state into the buffers,
 * never frees them, and the caller
 * keeps it alive until cmf_destroy.  Statistics scratch is still allocated by
 * the library.  Errors: those of cmf_create, CMF_EINVAL when dev_ptr is NULL,
 * misaligned, too small (the `bytes` given, or what its allocation holds
 * from dev_ptr on, checked with hipMemGetAddressRange) or not device memory
 * of the current device. */
int cmf_create_external(const cmf_desc *desc, void *dev_ptr, size_t bytes, void *hip_stream,
                        cmf_lattice **out);

/* Bytes cmf_create_external needs for `desc` (two population buffers, or
 * one with CMF_FLAG_IN_PLACE, each q x N elements of the storage type
 * rounded up to 256 bytes); 0 when the descriptor is invalid or asks for
 * in-place streaming where it is not supported. */
size_t cmf_external_bytes(const cmf_desc *desc);

/* Release all device memory the lattice allocated (synchronises its
 * stream); caller-owned buffers of cmf_create_external are left alone. */
int cmf_destroy(cmf_lattice *lat);

/* Set the state to the equilibrium f_eq(rho, u) of eq. feq (maximal Hermite
 * order; Sec. 2.2, 2.3) and reset the step counter and statistics.
 * rho: N host doubles or NULL (rho0 everywhere); u: 3 x N host doubles
 * (u_x of all sites, then u_y, then u_z) or NULL (rest).  Synchronous.
 * Errors: CMF_EINVAL (nothing changed) when a density is not positive and
 * finite or a velocity component is not finite. */
int cmf_init_equilibrium(cmf_lattice *lat, const double *rho, const double *u);

/* Overwrite the pre-collision populations f_i(x, t) of the current step
 * (the f of eq. lbe before its collision, Sec. 2.1) with q x N host doubles
 * (canonical layout).  The step counter is unchanged.  Allocates a
 * temporary device buffer of q N doubles.  Synchronous.  Errors: CMF_EINVAL
 * (NULL argument), CMF_ENOMEM, CMF_EHIP. */
int cmf_set_populations(cmf_lattice *lat, const double *f);

/* Copy the pre-collision populations f_i(x, t) of the current step (the f
 * of eq. lbe before its collision, Sec. 2.1) into q x N host doubles
 * (canonical layout).  Allocates a temporary device buffer of q N doubles.
 * Synchronous.  Errors: CMF_EINVAL (NULL argument), CMF_ENOMEM, CMF_EHIP. */
int cmf_get_populations(cmf_lattice *lat, double *f);

/* Pre-collision populations of the current step at `n` sites: out[k*q + i]
 * = f_i(sites[k]).  Site indices must lie in [0, N).  Synchronous. */
int cmf_gather_sites(cmf_lattice *lat, const int64_t *sites, int64_t n,
                     double *out);

/* Enqueue `nsteps` time steps on the lattice's stream.  One step is the
 * paper's per-site algorithm (Sec. 2.2, "Algorithm of computation"; the
 * D3Q27 and D3Q19 forms of Sec. 2.3 and 2.4): density and velocity (eq.
 * macro), normals, central moments, the collision of eq. cm_collision with
 * phi of eq. phi_general, f* = T(u)^-1 k*, and the streaming of eq.
 * streaming on the periodic box; plus, unless CMF_FLAG_NO_STATS, the
 * statistics row of the step (see cmf_stats).  Runs of 32 steps are
 * replayed from captured HIP graphs unless CMF_FLAG_NO_GRAPH.
 * Asynchronous; nsteps >= 0.  Errors: CMF_EINVAL (NULL lattice,
 * nsteps < 0), CMF_EHIP (launch or graph capture failed). */
int cmf_step(cmf_lattice *lat, int64_t nsteps);

/* Diagnostic timing: enqueue `nsteps` steps as direct launches (no graph)
 * with a HIP event pair around every fused-step kernel on the lattice's
 * stream, synchronise, and return in *kernel_ms the summed duration of the
 * step kernels alone, in milliseconds (the statistics reductions run after
 * each batch of up to 8 steps, outside the event pairs, so that only the
 * event markers separate consecutive kernels).  The steps are real steps:
 * the state and the statistics advance. */
int cmf_profile_steps(cmf_lattice *lat, int64_t nsteps, double *kernel_ms);

/* One launch shape of the fused-step kernel: `block` threads per workgroup
 * (a multiple of 64, at most 256; a workgroup covers `block` consecutive
 * sites of an x-row per tile) and `grid` workgroups, each walking tiles
 * blockIdx, blockIdx + grid, ... */
typedef struct {
  int32_t block;
  int32_t grid;
  double ms_per_step; /* measured by cmf_autotune; 0 otherwise */
} cmf_launch;

/* Current launch shape of the lattice's step kernel. */
int cmf_get_launch(cmf_lattice *lat, cmf_launch *out);

/* Set the launch shape: block in {64, 128, 192, 256}, grid >= 1 (capped at
 * the number of tiles).  Results do not depend on it (the noise is keyed by
 * the site), only the speed and the summation order of the statistics.
 * Synchronises; drops captured graphs. */
int cmf_set_launch(cmf_lattice *lat, int32_t block, int32_t grid);

/* Autotuner: time every candidate launch shape (block 64..256 up to the
 * row length; grid 1, 2, 4, 8, 16 and 32 x the compute-unit count, and one
 * tile per workgroup) with `steps_per_trial` real steps each (after one
 * untimed step; a step = fused kernel + statistics finalize), then restore the state, step counter and statistics ring
 * exactly as they were and keep the fastest shape.  The best shape is
 * remembered for the process under (device, q, storage, rates kind, box)
 * and used by later cmf_create calls with the same key; when the environment
 * variable CMFLB_TUNE_CACHE names a file, entries are also read from and
 * appended to it.  Up to `cap` trials are written to `trials` (may be NULL);
 * *n_out (may be NULL) receives the number of trials.  Needs one temporary
 * buffer the size of the population state (also with CMF_FLAG_IN_PLACE, for
 * the duration of the call).  Synchronous. */
int cmf_autotune(cmf_lattice *lat, int32_t steps_per_trial, cmf_launch *trials,
                 int32_t cap, int32_t *n_out);

/* One time step without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  The step is the one cmf_step takes (same kernels,
 * same results), for the lattice `desc` describes, from the state in `src`
 * to `dst`: two different device buffers of the current device, each
 * 256-byte aligned and holding q x N elements of the storage type in the
 * library's internal layout -- the two halves of a cmf_create_external
 * buffer (deviations f - w rho0, scaled for 16-bit storage, row-interleaved;
 * write and read them through such a lattice).  Each buffer, and
 * `stats_dev`, must lie in one device allocation known to HIP (hipMalloc,
 * or an allocator built on it such as PyTorch's) with room for its data
 * from the pointer to the allocation's end; the call checks this on the
 * host (hipPointerGetAttributes, hipMemGetAddressRange) and returns
 * CMF_EINVAL otherwise.  `step` (in [0, 2^56)) is
 * the index whose noise the step draws; the launch shape is (`block`,
 * `grid`) as in cmf_set_launch, with grid at most 65536 (larger grids are
 * rejected: the scratch holds the partial sums of that many workgroups).
 * When `stats_dev` is not NULL it receives the statistics row of the step
 * (12 device doubles, laid out as cmf_moments).  The statistics scratch
 * (partial sums, reduction rows, step counter; about 6.3 MB) is a static
 * device array, one per GPU, held until the process ends; every call on a
 * GPU shares it, so calls that overlap on one GPU (different streams or
 * threads) race and must be serialised by the caller.  Asynchronous on
 * `hip_stream` (NULL: the null stream); launches kernels only (no memset,
 * no allocation).  Errors: CMF_EINVAL (desc, buffers and their sizes, step, launch shape),
 * CMF_EUNSUPPORTED (device index >= 64), CMF_EHIP. */
int cmf_step_noalloc(const cmf_desc *desc, const void *src, void *dst, int64_t step,
                     int32_t block, int32_t grid, double *stats_dev, void *hip_stream);

/* Wait for all work enqueued on the lattice's stream. */
int cmf_synchronize(cmf_lattice *lat);

/* Index of the next step to be computed (synchronises). */
int cmf_get_step(cmf_lattice *lat, int64_t *step);

/* Set the index of the next step to be computed, e.g. to resume a run from
 * saved populations (cmf_get_populations + cmf_get_step, later
 * cmf_set_populations + cmf_set_step continue with the same noise).  Rows
 * of earlier steps are no longer returned by cmf_stats.  Synchronous.
 * Errors: CMF_EINVAL (NULL lattice, step outside [0, 2^56)), CMF_EHIP. */
int cmf_set_step(cmf_lattice *lat, int64_t step);

/* The per-step spatial sums behind the diagnostics of Sec. 3 (the spatial
 * averages <u_a^2> of Tests 3-7 are sum_u2[a] / N; mass and momentum are
 * conserved by the collision and the streaming, eq. cm_collision with
 * Lambda = 1 and I~ = 0 on modes 0-3).
 * Statistics rows of the steps completed since the previous call (or since
 * init), oldest first, at most min(cap, series_capacity) of them (the most
 * recent ones); *n_out receives the count.  Synchronises.  Returns
 * CMF_ENONFINITE (after filling `out`) when one of the returned rows counts
 * non-finite sites, CMF_EINVAL when cap < 0. */
int cmf_stats(cmf_lattice *lat, cmf_moments *out, int64_t cap,
              int64_t *n_out);

/* Write the density and velocity of the current pre-collision state
 * (eq. macro: rho = sum f, rho u = sum c f, evaluated in FP64 and rounded
 * to FP32) into device buffers on the lattice's device: rho_dev (N floats)
 * and u_dev (3 x N floats, u_x block first; u_z = 0 on D2Q9); both are
 * owned by the caller.  Either pointer may be NULL.  Asynchronous on the
 * lattice's stream.  Errors: CMF_EINVAL (NULL lattice; a buffer that is not
 * device memory of the current device or whose allocation holds fewer
 * bytes from the pointer on than it receives, checked on the host before
 * any launch), CMF_EHIP. */
int cmf_sample_macro(cmf_lattice *lat, void *rho_dev, void *u_dev);

/* The density and velocity of the current pre-collision state, computed on
 * the device in FP64 from the stored populations (eq. macro: rho = sum f,
 * rho u = sum c f): rho (N host doubles) and u (3 x N host doubles, u_x
 * block first; u_z = 0 on D2Q9).  Either pointer may be NULL.  Allocates a
 * temporary device buffer of 4 N doubles.  Synchronous. */
int cmf_get_macro(cmf_lattice *lat, double *rho, double *u);

/* Velocity statistics of the current pre-collision state (Test 7, Fig. 8),
 * per component a = x, y, z, with u = sum c f / rho in FP64 per site:
 *   moments[4 a + 0..3] = mean, variance (1/N), skewness m3 / var^1.5 and
 *   kurtosis m4 / var^2 (3 for a Gaussian) -- central moments about the mean;
 *   counts[(nbins + 2) a + b] = histogram of x = (u_a - mean_a) / sqrt(var_a):
 *   b = 0 counts x < -xmax and non-finite x, b = 1..nbins split [-xmax, xmax)
 *   into equal bins, b = nbins + 1 counts x >= xmax (z entries are zero on
 *   D2Q9).  moments (12 doubles) or counts (3 (nbins + 2) int64) may be NULL.
 * Three device passes (means, central moments, histogram), fixed-order FP64
 * sums and integer counts; allocates temporary device buffers.
 * Errors: CMF_EINVAL (nbins outside [1, 4096] or xmax <= 0 with counts).
 * Synchronous. */
int cmf_velocity_pdf(cmf_lattice *lat, int32_t nbins, double xmax, double *moments,
                     int64_t *counts);

/* Diagnostic: the standard normals eta_v the step kernels draw, for the
 * noisy modes of `n` consecutive sites starting at `site0` of step `step`.
 * out: n x q host doubles, zero on the conserved modes.  `fp64` selects
 * the FP64 transform (as in F64 storage) instead of the FP32 one.  Runs a
 * device kernel on the null stream; synchronous.  Errors: CMF_EINVAL (q,
 * step outside [0, 2^56), sites outside [0, 2^32)), CMF_ENOMEM, CMF_EHIP. */
int cmf_noise_sample(int32_t q, uint64_t seed, uint32_t replica, int64_t step,
                     int64_t site0, int64_t n, int32_t fp64, double *out);

/* Diagnostic: Philox4x32-10 words for n counters (ctr[4k..4k+3]) under one
 * key, computed on the device; out receives 4n words.  Synchronous. */
int cmf_philox_words(const uint32_t *ctr, int64_t n, uint32_t key0,
                     uint32_t key1, uint32_t *out);

/* ---- static structure factor (amortized diagnostic) ----------------------
 * S_a(k) = < |sum_x a(x) exp(-i k.x)|^2 > / N over sampled states, for
 * a = drho (= rho - rho0), u_x, u_y, u_z of the pre-collision state; for the
 * equilibrium of the method S_rho = rho0 kT / c_s^2 and S_u = kT / rho0 at
 * every k != 0 (linearised equipartition).  Each sample computes the four
 * FP32 fields on the device, transforms them with hipFFT (real-to-complex)
 * and adds |F(k)|^2 / N to FP64 accumulators; shell averages over
 * |k| = 2 pi sqrt((m_x/n_x)^2 + ...) are reduced in a fixed order. */

/* Allocate (first call) and zero the accumulators, with `nbins` shells of
 * equal width on [0, pi sqrt(d)] (1 <= nbins <= 1024).  Synchronous. */
int cmf_sk_reset(cmf_lattice *lat, int32_t nbins);

/* Add one sample: the current pre-collision state.  Asynchronous on the
 * lattice's stream (call between steps, not inside captured graphs). */
int cmf_sk_accumulate(cmf_lattice *lat);

/* Shell averages of the samples so far: out[6 b + c] for shell b with
 * c = 0 mean |k|, 1 number of modes (k = 0 excluded), 2 S_rho, 3 S_ux,
 * 4 S_uy, 5 S_uz (averaged over samples and over the shell's modes; empty
 * shells have 0 modes and zeros).  *nsamples receives the sample count.
 * Synchronous. */
int cmf_sk_shells(cmf_lattice *lat, double *out, int64_t *nsamples);

/* ---- batched ensembles ------------------------------------------------
 * Many independent replicas (D2Q9, D3Q19 and D3Q27 mixed; uneven boxes;
 * each with its own tau / rates, kT, rho0, seed and replica number) advanced together
 * by ONE fused-step launch per step that covers the tiles of every replica,
 * followed by a per-replica statistics reduction; runs of steps are
 * replayed from captured HIP graphs unless CMF_FLAG_NO_GRAPH.  Each replica
 * evolves exactly as a cmf_lattice created from the same descriptor would
 * (same arithmetic, same noise keys).  All replicas share the storage type
 * and the flags of descs[0] and one step counter. */
typedef struct cmf_ensemble cmf_ensemble;

/* Create an ensemble of n >= 1 replicas from n descriptors (validated as in
 * cmf_create; storage and flags must agree; series_capacity of descs[0]
 * applies to all; each replica's q arrays of N rounded up to 64 values
 * must take below 4 GiB in the storage type).  All replicas start at rest
 * at step 0.  Allocates two population arenas holding every replica (one
 * array per population of each replica, unlike the row-interleaved layout
 * of a cmf_lattice; read and write states with the calls below), the
 * replica records, the tile map and the statistics buffers.  Errors:
 * CMF_EINVAL, CMF_ENOMEM, CMF_EHIP. */
int cmf_ensemble_create(const cmf_desc *descs, int32_t n, void *hip_stream,
                        cmf_ensemble **out);

/* Release the ensemble (synchronises its stream). */
int cmf_ensemble_destroy(cmf_ensemble *ens);

/* Number of replicas, total sites and tiles (any output may be NULL). */
int cmf_ensemble_info(cmf_ensemble *ens, int32_t *n_replicas,
                      int64_t *total_sites, int64_t *n_tiles);

/* Tile shape of the ensemble step kernel: one workgroup of 256 threads per
 * tile, each thread up to spt sites (spt9 for D2Q9 replicas, spt3d for
 * D3Q19 and D3Q27 replicas); a tile is spt x 256 consecutive sites of its
 * replica (x fastest), the last tile of a replica ragged.  Defaults
 * 3 and 1 (environment variables CMF_ENSEMBLE_SPT9 and CMF_ENSEMBLE_SPT27
 * override them at creation). */
typedef struct {
  int32_t spt9;
  int32_t spt3d;
  double ms_per_step; /* measured by cmf_ensemble_autotune; 0 otherwise */
} cmf_ensemble_tiles;

/* Current tile shape. */
int cmf_ensemble_get_tiles(cmf_ensemble *ens, cmf_ensemble_tiles *out);

/* Set the tile shape (both values in [1, 16]).  Results do not depend on
 * it (the noise is keyed by the site), only the speed and the summation
 * order of the statistics.  Synchronises; rebuilds the tile map (may
 * reallocate it and the partial sums: CMF_ENOMEM) and drops captured
 * graphs.  Errors: CMF_EINVAL, CMF_ENOMEM, CMF_EHIP. */
int cmf_ensemble_set_tiles(cmf_ensemble *ens, int32_t spt9, int32_t spt3d);

/* Autotuner of the tile shape (the batched-ensemble configuration of the
 * benchmark asks for tuned tiles): time spt9 in {1, 2, 3, 4, 6, 8} (when
 * there are D2Q9 replicas) x spt3d in {1, 2, 3, 4, 6, 8} (when there are 3-D
 * replicas) with `steps_per_trial` direct steps each (after one untimed
 * step; a step = fused kernel + per-replica statistics), then restore the
 * populations, step counter and statistics rings exactly and keep the
 * fastest shape.  Up to `cap` trials go to `trials` (may be NULL); *n_out
 * (may be NULL) receives their number.  Needs one temporary buffer the size
 * of a population arena.  Synchronous.  Errors: CMF_EINVAL, CMF_ENOMEM,
 * CMF_EHIP (the previous tile shape is kept on error). */
int cmf_ensemble_autotune(cmf_ensemble *ens, int32_t steps_per_trial,
                          cmf_ensemble_tiles *trials, int32_t cap, int32_t *n_out);

/* Replica `index` (creation order) to f_eq(rho, u), with the arguments of
 * cmf_init_equilibrium (and its CMF_EINVAL checks).  The shared step
 * counter is not changed.  Synchronous. */
int cmf_ensemble_init_equilibrium(cmf_ensemble *ens, int32_t index,
                                  const double *rho, const double *u);

/* Pre-collision populations of replica `index` (q x N host doubles, as in
 * cmf_set_populations / cmf_get_populations).  Synchronous. */
int cmf_ensemble_set_populations(cmf_ensemble *ens, int32_t index,
                                 const double *f);
int cmf_ensemble_get_populations(cmf_ensemble *ens, int32_t index, double *f);

/* Enqueue nsteps steps of every replica.  Asynchronous. */
int cmf_ensemble_step(cmf_ensemble *ens, int64_t nsteps);

/* nsteps direct-launch steps with a HIP event pair around every ensemble
 * step kernel; *kernel_ms = summed kernel time.  Synchronous. */
int cmf_ensemble_profile_steps(cmf_ensemble *ens, int64_t nsteps,
                               double *kernel_ms);

/* Wait for the ensemble's stream; index of the next step. */
int cmf_ensemble_synchronize(cmf_ensemble *ens);
int cmf_ensemble_get_step(cmf_ensemble *ens, int64_t *step);

/* Set the shared step counter (as cmf_set_step). */
int cmf_ensemble_set_step(cmf_ensemble *ens, int64_t step);

/* Statistics rows of replica `index` since the previous call for that
 * replica, as cmf_stats. */
int cmf_ensemble_stats(cmf_ensemble *ens, int32_t index, cmf_moments *out,
                       int64_t cap, int64_t *n_out);

/* Diagnostic: practical HBM ceiling.  Allocates two device buffers of
 * `bytes` bytes (rounded up to 16), copies one into the other `reps` times
 * with a plain streaming copy kernel (`cmf_stream_copy_kernel`, 16-byte
 * vector loads and stores, each byte read once and written once), and
 * returns the fastest copy in *best_ms.  Uses the null stream; synchronous;
 * frees its buffers. */
int cmf_stream_copy(size_t bytes, int32_t reps, double *best_ms);

#ifdef __cplusplus
}
#endif

#endif /* CMFLB_H */
