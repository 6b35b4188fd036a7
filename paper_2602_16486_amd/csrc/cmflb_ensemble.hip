// cmflb_ensemble.hip -- the batched-ensemble step (one launch per step over
// the tiles of every replica, inlining the collision of cmflb_step.h), its
// per-replica statistics reduction and their launchers, in a translation
// unit of their own.
#include "cmflb_step.h"
#include "cmflb_sums.h"

namespace cmf {

// ---------------------------------------------------------------------------
// batched ensemble: one launch per step over the tiles of every replica
// ---------------------------------------------------------------------------
// Layout of a replica: one array per population (population i of site s at
// element i pitch + s, pitch = the site count rounded up to 64), unlike the
// row-interleaved single lattice.  Replica rows have any length, so rows
// seldom start on a cache line; per-population arrays keep the stores of a
// tile whole, aligned cache lines whatever the row length (64 consecutive
// sites are 128 B or more in every storage type), so they are written
// non-temporally, and only the loads of shifted rows straddle lines.
// A tile is spt x kEnsembleBlock consecutive sites (x fastest) of one
// replica, the last tile of a replica ragged: lanes idle only there.  The
// replica, and with it the lattice type, is uniform per workgroup.
// Replicas are listed 3-D first (heavier tiles dispatched first).

// n / d for any 32-bit n by a multiply-high and two shifts, with m and
// s1 | s2 << 8 precomputed for the divisor d (Granlund and Montgomery,
// "Division by invariant integers using multiplication", PLDI 1994,
// Fig. 4.1): t = mulhi(m, n), q = (t + ((n - t) >> s1)) >> s2, in place of
// a generic 32-bit division, which forms and corrects a reciprocal per lane.
__device__ __forceinline__ uint32_t udiv_invariant(uint32_t n, uint32_t m, uint32_t sh) {
  const uint32_t t = __umulhi(m, n);
  return (t + ((n - t) >> (sh & 255u))) >> (sh >> 8);
}

// One site of an ensemble replica whose populations the resources rs / rd
// cover (q pitch values, below 4 GiB): the vector byte offset carries the
// source site, the scalar offset the population array i pitch.  The rest
// population is read at the site itself, an aligned stream read once, so
// it is loaded non-temporally too.
template <class L, typename S, typename R, bool GENERAL>
__device__ __forceinline__ void ensemble_site(__amdgpu_buffer_rsrc_t rs, __amdgpu_buffer_rsrc_t rd,
                                              const ReplicaParams<R> &p,
                                              int64_t s, uint64_t step,
                                              Acc &acc) {
  using ST = Store<S, R>;
  constexpr uint32_t B = sizeof(S);
  const uint32_t nx = (uint32_t)p.nx, ny = (uint32_t)p.ny;
  const uint32_t us = (uint32_t)s;
  const uint32_t row = udiv_invariant(us, p.div_nx, p.sh_nx);
  const uint32_t x = us - row * nx;
  uint32_t y = row, z = 0;
  if constexpr (L::D == 3) {
    z = udiv_invariant(row, p.div_ny, p.sh_ny);
    y = row - z * ny;
  }
  // byte offsets from site s to the source site x - c along each axis
  // (index c + 1), periodic; unsigned arithmetic wraps, the sums land in
  // [0, N) sites
  const uint32_t plane = nx * ny;
  const uint32_t dx[3] = {(x == nx - 1 ? 0u - (nx - 1) : 1u) * B, 0u,
                          (x == 0 ? nx - 1 : 0u - 1u) * B};
  const uint32_t dy[3] = {(y == ny - 1 ? 0u - (ny - 1) * nx : nx) * B, 0u,
                          (y == 0 ? (ny - 1) * nx : 0u - nx) * B};
  uint32_t dz[3] = {0u, 0u, 0u};
  if constexpr (L::D == 3) {
    const uint32_t nz = (uint32_t)p.nz;
    dz[0] = (z == nz - 1 ? 0u - (nz - 1) * plane : plane) * B;
    dz[2] = (z == 0 ? (nz - 1) * plane : 0u - plane) * B;
  }
  const uint32_t sb = us * B;
  const uint32_t popb = (uint32_t)p.pitch * B;
  R d[L::Q];
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const uint32_t voff = sb + dx[L::cx[i] + 1] + dy[L::cy[i] + 1] + dz[L::cz[i] + 1];
    const float sc = p.scale[weight_class<L>(i)];
    if (L::cx[i] == 0 && L::cy[i] == 0 && L::cz[i] == 0)
      d[i] = ST::from_bits(buf_load<S, true>(rs, voff, (uint32_t)i * popb), sc);
    else
      d[i] = ST::from_bits(buf_load<S, false>(rs, voff, (uint32_t)i * popb), sc);
  }
  collide_site<L, R, GENERAL, sizeof(S) == 2>(d, p, us, step, acc);
#pragma unroll
  for (int i = 0; i < L::Q; ++i)
    buf_store<S, true>(ST::to_bits(d[i], p.iscale[weight_class<L>(i)]), rd, sb, (uint32_t)i * popb);
}

// Workgroups are handed to the XCDs round-robin by id and every XCD has its
// own L2.  Map workgroup b to a tile so that runs of kXcdChunk adjacent
// tiles go to one XCD (chunk c to XCD c mod kXcds): two tiles that split a
// lattice row, or that pull from each other's rows, then mostly meet in the
// same L2, which merges the two parts of a shared cache line before it goes
// to HBM; the chunks rotate over the XCDs, so tiles of different cost (D2Q9
// and D3Q27 replicas) spread evenly.  A bijection on [0, n): the last
// n mod (kXcds kXcdChunk) tiles keep their own ids.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  constexpr int G = kXcds * kXcdChunk;
  if (b >= n / G * G) return b;
  const int j = b % kXcds, k = b / kXcds;
  return ((k / kXcdChunk) * kXcds + j) * kXcdChunk + k % kXcdChunk;
}

template <typename S, typename R, bool GENERAL>
__global__ __launch_bounds__(kEnsembleBlock) void k_ensemble_step(
    const S *__restrict__ src, S *__restrict__ dst,
    const ReplicaParams<R> *__restrict__ reps, const int32_t *__restrict__ tile_rep,
    const int64_t *__restrict__ step_ptr, int step_off, double *__restrict__ partials) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const ReplicaParams<R> &p = reps[tile_rep[tile]];
  const uint64_t step = (uint64_t)(*step_ptr + step_off);
  Acc acc;
#pragma unroll
  for (int k = 0; k < kNAcc; ++k) acc.v[k] = 0.0;
  const int64_t t0 = (int64_t)(tile - p.tile0) * p.tsites;
  const int64_t s0 = t0 + threadIdx.x;
  const int64_t end = t0 + p.tsites < p.nsites ? t0 + p.tsites : p.nsites;
  // the replica's population arrays, below 4 GiB (checked at creation)
  const uint32_t bytes = (uint32_t)((int64_t)p.q * p.pitch * (int64_t)sizeof(S));
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(src + p.offset, bytes);
  const __amdgpu_buffer_rsrc_t rd = make_rsrc(dst + p.offset, bytes);
  if (p.q == 27) {
    for (int j = 0; j < p.spt; ++j) {
      const int64_t s = s0 + (int64_t)j * kEnsembleBlock;
      if (s < end) ensemble_site<D3Q27, S, R, GENERAL>(rs, rd, p, s, step, acc);
    }
  } else if (p.q == 19) {
    for (int j = 0; j < p.spt; ++j) {
      const int64_t s = s0 + (int64_t)j * kEnsembleBlock;
      if (s < end) ensemble_site<D3Q19, S, R, GENERAL>(rs, rd, p, s, step, acc);
    }
  } else {
    for (int j = 0; j < p.spt; ++j) {
      const int64_t s = s0 + (int64_t)j * kEnsembleBlock;
      if (s < end) ensemble_site<D2Q9, S, R, GENERAL>(rs, rd, p, s, step, acc);
    }
  }
  __shared__ double acc_lds[acc_lds_bytes<double>(kEnsembleBlock) / sizeof(double)];
  block_store_acc(acc, partials + (int64_t)tile * kPartStride, acc_lds);
}

// per-replica fixed-order sum of its tiles' partials into its series row
template <typename R>
__global__ __launch_bounds__(256) void k_ensemble_reduce(
    const ReplicaParams<R> *__restrict__ reps, const double *__restrict__ partials,
    double *__restrict__ series, int cap, const int64_t *__restrict__ step_ptr,
    int step_off, const double *__restrict__ mass0) {
  __shared__ double tot[kNAcc];
  const int r = blockIdx.x;
  const ReplicaParams<R> &p = reps[r];
  const int64_t step = *step_ptr + step_off;
  block_sum_rows(partials, p.tile0, p.tile0 + p.ntiles, tot);
  __syncthreads();
  if (threadIdx.x == 0) {
    double *row = series + ((int64_t)r * cap + step % cap) * kSeriesStride;
    row[0] = (double)step;
    row[1] = mass0[r] + tot[0];
#pragma unroll
    for (int k = 1; k < kNAcc; ++k) row[1 + k] = tot[k];
  }
}

namespace {

template <typename S, typename R>
hipError_t ensemble_launch(bool general, const void *reps, const int32_t *tile_rep, int ntiles,
                           const void *src, void *dst, const int64_t *step_ptr, int step_off,
                           double *partials, hipStream_t stream) {
  if (general)
    hipLaunchKernelGGL((k_ensemble_step<S, R, true>), dim3(ntiles), dim3(kEnsembleBlock), 0,
                       stream, static_cast<const S *>(src), static_cast<S *>(dst),
                       static_cast<const ReplicaParams<R> *>(reps), tile_rep, step_ptr,
                       step_off, partials);
  else
    hipLaunchKernelGGL((k_ensemble_step<S, R, false>), dim3(ntiles), dim3(kEnsembleBlock), 0,
                       stream, static_cast<const S *>(src), static_cast<S *>(dst),
                       static_cast<const ReplicaParams<R> *>(reps), tile_rep, step_ptr,
                       step_off, partials);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_ensemble_step(int storage, bool general, const void *reps,
                                const int32_t *tile_rep, int ntiles,
                                const void *src, void *dst,
                                const int64_t *step_ptr, int step_off, double *partials,
                                hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  switch (storage) {
    case kF64:
      return ensemble_launch<double, double>(general, reps, tile_rep, ntiles, src, dst,
                                             step_ptr, step_off, partials, stream);
    case kF32:
      return ensemble_launch<float, float>(general, reps, tile_rep, ntiles, src, dst,
                                           step_ptr, step_off, partials, stream);
    case kF16:
      return ensemble_launch<__half, float>(general, reps, tile_rep, ntiles, src, dst,
                                            step_ptr, step_off, partials, stream);
    case kBF16:
      return ensemble_launch<__hip_bfloat16, float>(general, reps, tile_rep, ntiles, src,
                                                    dst, step_ptr, step_off, partials, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_ensemble_finalize(int storage, const void *reps, int nrep,
                                    const double *partials, double *series,
                                    int cap, int64_t *step_ptr, int step_off, int bump,
                                    double *mass0, bool stats, hipStream_t stream) {
  if (stats) {
    if (storage == kF64)
      hipLaunchKernelGGL(k_ensemble_reduce<double>, dim3(nrep), dim3(256), 0, stream,
                         static_cast<const ReplicaParams<double> *>(reps), partials,
                         series, cap, step_ptr, step_off, mass0);
    else
      hipLaunchKernelGGL(k_ensemble_reduce<float>, dim3(nrep), dim3(256), 0, stream,
                         static_cast<const ReplicaParams<float> *>(reps), partials,
                         series, cap, step_ptr, step_off, mass0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return bump ? launch_bump_step(step_ptr, bump, stream) : hipSuccess;
}

}  // namespace cmf
