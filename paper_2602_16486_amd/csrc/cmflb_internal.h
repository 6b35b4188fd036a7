// cmflb_internal.h -- declarations shared by the kernel translation unit and
// the C-ABI implementation of libcmflb (not installed, not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmf {

constexpr int kNAcc = 11;      // accumulated statistics per block
constexpr int kPartStride = 12;// doubles per block partial
constexpr int kSeriesStride = 12;
constexpr int kMaxBlock = 256;
// statistics partials beyond this count are first summed by up to
// kMaxLevel2 workgroups (second-level rows); 256 rows per workgroup, one per
// thread (65536 one-tile partials: 256 workgroups, one per CU)
constexpr int kLevel2Threshold = 256;
constexpr int kMaxLevel2 = 256;

// Parameters of one lattice as the step kernels see them (kernel argument,
// so every field lives in scalar registers).
template <typename R>
struct StepParams {
  int32_t nx, ny, nz, nxb;  // box and x-tiles per row
  int32_t ntiles;           // nxb * ny * nz
  int32_t noise;            // kT > 0
  R rho0;
  // phi_v = sqrt(rho) amp1 amp_v (eq. phi_general): amp_v = I~_v
  // sqrt(Lambda_v (2 - Lambda_v) b_v) (sqrt(b_v) when Lambda_v = 1) and
  // amp1 = sqrt(kT / c_s^2)
  R amp[27];
  R amp1;
  R oml[27];   // 1 - Lambda_v
  R lam[27];   // Lambda_v
  // storage scale s and 1 / s of each weight class |c_i|^2 = 0..3 (s_i
  // depends on i through w_i only): 8 values instead of 2 q keeps them in
  // scalar registers
  float scale[4], iscale[4];
  uint32_t key0, key1, replica;
};

// One replica of a batched ensemble as the ensemble kernel sees it (an
// array in device memory; every field is read with scalar loads because a
// workgroup works on one replica).
template <typename R>
struct ReplicaParams {
  int32_t q, nx, ny, nz;
  int32_t nsites, tile0, ntiles, noise;
  int64_t offset;  // element offset of the replica's populations in an arena
  uint32_t key0, key1, replica;
  int32_t spt;     // sites per thread: a tile has spt x kEnsembleBlock sites
  int32_t tsites;  // sites per tile, spt x kEnsembleBlock (the last one ragged)
  int32_t pitch;   // elements from population i to i + 1: nsites rounded up to 64
  // exact division of a site index by nx and of a row index by ny with a
  // multiplier m and shifts s1 | s2 << 8 (see udiv_invariant)
  uint32_t div_nx, div_ny, sh_nx, sh_ny;
  R rho0;
  R amp[27];
  R amp1;
  R oml[27];
  R lam[27];
  float scale[4], iscale[4];  // per weight class, as in StepParams
};

// Where the buffer keeps the pre-collision population f_i(x) of the next
// step: kLayoutPull, slot i of site x - c_i (the post-collision value of
// the step before, not yet streamed; two-buffer pull); with in-place (AA)
// streaming, kLayoutNatural, slot i of site x (after an odd step), or
// kLayoutSwapped, slot opposite(i) of site x - c_i (after an even step).
enum Layout { kLayoutPull = 0, kLayoutNatural = 1, kLayoutSwapped = 2 };

// Streaming form of a step launch: the two-buffer pull, or the two halves
// of in-place streaming.  AA even step: read slot i of own site, write the
// post-collision population i to slot opposite(i) of own site; AA odd
// step: read slot opposite(i) of site x - c_i, write slot i of site
// x + c_i.  Every buffer element is read and written by one site only.
enum StreamMode { kStreamPull = 0, kStreamAAEven = 1, kStreamAAOdd = 2 };

// Parameters of the state conversion kernels (FP64 always).  pitch = 0:
// the row-interleaved layout of a single lattice; pitch > 0: one array per
// population, population i starting at element i pitch (ensemble replicas).
// layout: a Layout value.
struct ConvParams {
  int32_t nx, ny, nz;
  int32_t layout;
  int64_t pitch;
  double rho0;
  double w[27];
  float scale[27], iscale[27];
};

enum Storage { kF64 = 0, kF32 = 1, kF16 = 2, kBF16 = 3 };

// launchers (defined in cmflb_kernels.hip, the ensemble's in cmflb_ensemble.hip);
// all return hipError_t
// nt: non-temporal population stores (rows of whole cache lines), else plain
// The step index of a launch is *step_ptr + step_off: runs of steps
// captured in a graph pass offsets 0, 1, ... and advance *step_ptr once at
// their end (launch_bump_step); a direct step passes 0 and its finalize
// advances *step_ptr by bump = 1.
// mode: a StreamMode value; src == dst for the in-place modes.
hipError_t launch_step(int q, int storage, bool general, bool nt, int mode,
                       const void *params, const void *src, void *dst,
                       const int64_t *step_ptr, int step_off, double *partials,
                       int grid, int block, hipStream_t stream);
hipError_t launch_finalize(const double *partials, int nparts, double *level2,
                           double *series, int cap, int64_t *step_ptr, int step_off,
                           int bump, double mass0, bool stats, hipStream_t stream);
// the statistics rows of `count` consecutive steps (step offsets step_off,
// step_off + 1, ...) whose partial sums start at partials + k pstride
// (k = 0 .. count - 1); level2 holds count kMaxLevel2 rows; bump must be 0
// when count > 1
hipError_t launch_finalize_batch(const double *partials, int64_t pstride, int count, int nparts,
                                 double *level2, double *series, int cap, int64_t *step_ptr,
                                 int step_off, int bump, double mass0, bool stats,
                                 hipStream_t stream);
hipError_t launch_bump_step(int64_t *step_ptr, int64_t by, hipStream_t stream);
hipError_t launch_init_eq(int q, int storage, const ConvParams &cp,
                          const double *rho, const double *u, void *buf,
                          hipStream_t stream);
hipError_t launch_set_state(int q, int storage, const ConvParams &cp,
                            const double *f, void *buf, hipStream_t stream);
hipError_t launch_get_state(int q, int storage, const ConvParams &cp,
                            const void *buf, double *f, hipStream_t stream);
hipError_t launch_gather(int q, int storage, const ConvParams &cp,
                         const void *buf, const int64_t *sites, int64_t n,
                         double *out, hipStream_t stream);
hipError_t launch_macro(int q, int storage, const ConvParams &cp,
                        const void *buf, float *rho, float *u,
                        hipStream_t stream);
hipError_t launch_macro(int q, int storage, const ConvParams &cp,
                        const void *buf, double *rho, double *u,
                        hipStream_t stream);
hipError_t launch_noise(int q, int fp64, uint32_t key0, uint32_t key1,
                        uint32_t replica, uint64_t step, int64_t site0,
                        int64_t n, double *out, hipStream_t stream);
hipError_t launch_philox(const uint32_t *ctr, int64_t n, uint32_t key0,
                         uint32_t key1, uint32_t *out, hipStream_t stream);
hipError_t launch_zero_i64(int64_t *p, int64_t n, hipStream_t stream);
// *p = v by a one-thread kernel (no memset node when captured)
hipError_t launch_set_i64(int64_t *p, int64_t v, hipStream_t stream);
hipError_t launch_stream_copy(const void *src, void *dst, size_t n16,
                              hipStream_t stream);

// velocity statistics (moments about a centre, normalised histograms)
constexpr int kVelCols = 12;      // sum (u_a - c_a)^p, column 4 a + p - 1
constexpr int kVelMaxBins = 4096;
struct VelNorm {
  double centre[3];
  double inv_sigma[3];
};
hipError_t launch_vel_moments(int q, int storage, const ConvParams &cp, const void *buf,
                              const VelNorm &c, int grid, double *partials, double *out,
                              hipStream_t stream);
hipError_t launch_vel_hist(int q, int storage, const ConvParams &cp, const void *buf,
                           const VelNorm &c, int grid, int nbins, double xmax,
                           unsigned long long *counts, hipStream_t stream);

// structure factor
hipError_t launch_macro_dev(int q, int storage, const ConvParams &cp,
                            const void *buf, float *out, hipStream_t stream);
hipError_t launch_sk_accumulate(const void *F, int64_t M, double inv_n,
                                double *acc, hipStream_t stream);
hipError_t launch_sk_shell_index(int nx, int ny, int nz, int nbins, int64_t M,
                                 int32_t *bin, hipStream_t stream);
hipError_t launch_sk_segments(const double *acc, int64_t M, int nx, int ny, int nz,
                              int nbins, const int32_t *perm, const int64_t *off,
                              double *out, hipStream_t stream);

// ensemble
constexpr int kEnsembleBlock = 256;
// default sites per thread of an ensemble tile: a D2Q9 site carries a third
// of the bytes of a D3Q27 one, so its tiles are longer to amortise the
// per-workgroup start (replica record loads) and the partial-sum reduction
constexpr int kEnsembleSpt9 = 3, kEnsembleSpt27 = 1;
// cache-line bytes: a buffer whose population rows are multiples of this
// gets non-temporal stores
constexpr int kLineBytes = 128;
// XCDs of an MI355X (the tile maps assume round-robin dispatch over them)
constexpr int kXcds = 8;
// adjacent ensemble tiles kept on one XCD
constexpr int kXcdChunk = 8;
hipError_t launch_ensemble_step(int storage, bool general, const void *reps,
                                const int32_t *tile_rep, int ntiles,
                                const void *src, void *dst,
                                const int64_t *step_ptr, int step_off, double *partials,
                                hipStream_t stream);
hipError_t launch_ensemble_finalize(int storage, const void *reps, int nrep,
                                    const double *partials, double *series,
                                    int cap, int64_t *step_ptr, int step_off, int bump,
                                    double *mass0, bool stats, hipStream_t stream);

}  // namespace cmf
