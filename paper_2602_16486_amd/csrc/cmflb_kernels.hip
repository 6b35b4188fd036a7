// cmflb_kernels.hip -- gfx950 kernels of libcmflb besides the fused steps
// (cmflb_step.h, cmflb_ensemble.hip): the statistics reductions, the state
// conversion and diagnostic kernels and their launchers.
#include "cmflb_step.h"
#include "cmflb_sums.h"

namespace cmf {

// ---------------------------------------------------------------------------
// statistics finalize: fixed-order FP64 sums of the block partials (in two
// levels when there are many blocks) into the series row of the current
// step, then advance the step counter
// ---------------------------------------------------------------------------
// first level: block (r, y) sums partial rows [r chunk, (r + 1) chunk) of
// step y of a batch (its rows from partials + y pstride) into level-2 row
// y gridDim.x + r
__global__ __launch_bounds__(256) void k_reduce_partials(
    const double *__restrict__ partials, int nparts, int chunk, int64_t pstride,
    double *__restrict__ level2) {
  const int lo = blockIdx.x * chunk;
  const int hi = lo + chunk < nparts ? lo + chunk : nparts;
  block_sum_rows(partials + blockIdx.y * pstride, lo, hi,
                 level2 + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * kPartStride);
}

// The statistics row of step *step_ptr + step_off + y for block y of a
// batch (its nrows rows from rows + y rstride); *step_ptr advances by `bump`
// (0 inside a run of steps, which advances it once at its end; a batch of
// more than one step passes 0).
__global__ __launch_bounds__(256) void k_finalize(
    const double *__restrict__ rows, int nrows, int64_t rstride, double *__restrict__ series,
    int cap, int64_t *__restrict__ step_ptr, int step_off, int bump, double mass0,
    int stats) {
  __shared__ double tot[kNAcc];
  const int64_t base = *step_ptr;
  const int64_t step = base + step_off + blockIdx.x;
  // with a ring shorter than the batch, a later step of the same batch
  // takes the same row: only the latest of them writes it, as if the steps
  // had been reduced one after the other
  if (stats && blockIdx.x + (int64_t)cap >= gridDim.x) {
    block_sum_rows(rows + blockIdx.x * rstride, 0, nrows, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
      double *row = series + (step % cap) * kSeriesStride;
      row[0] = (double)step;
      row[1] = mass0 + tot[0];
#pragma unroll
      for (int k = 1; k < kNAcc; ++k) row[1 + k] = tot[k];
    }
  }
  if (threadIdx.x == 0 && bump) *step_ptr = base + bump;
}

// ---------------------------------------------------------------------------
// state conversion kernels (FP64 arithmetic)
// ---------------------------------------------------------------------------
// element offset of population i at site s in the population buffer (the
// row-interleaved layout, or one array per population when cp.pitch > 0)
template <class L>
__device__ __forceinline__ int64_t pop_site_offset(const ConvParams &cp, int i,
                                                   int64_t s) {
  if (cp.pitch > 0) return (int64_t)i * cp.pitch + s;
  return pop_row_offset<L>(i, s / cp.nx, cp.nx) + s % cp.nx;
}

template <class L>
__device__ __forceinline__ int64_t shifted_site(const ConvParams &cp, int64_t s,
                                                int i, int sign) {
  // site s + sign * c_i, periodic
  const int x = (int)(s % cp.nx);
  const int64_t r = s / cp.nx;
  const int y = (int)(r % cp.ny);
  const int z = (int)(r / cp.ny);
  const int xs = wrap_sub(x, -sign * L::cx[i], cp.nx);
  const int ys = wrap_sub(y, -sign * L::cy[i], cp.ny);
  const int zs = wrap_sub(z, -sign * L::cz[i], cp.nz);
  return xs + (int64_t)cp.nx * (ys + (int64_t)cp.ny * zs);
}

// element offset of the pre-collision population f_i of site s in the
// buffer, for the buffer's layout (cp.layout)
template <class L>
__device__ __forceinline__ int64_t state_offset(const ConvParams &cp, int i, int64_t s) {
  if (cp.layout == kLayoutNatural) return pop_site_offset<L>(cp, i, s);
  const int slot = cp.layout == kLayoutSwapped ? opposite<L>(i) : i;
  return pop_site_offset<L>(cp, slot, shifted_site<L>(cp, s, i, -1));
}

// d_eq = f_eq(rho, u) - w rho0 = T(u)^-1 (rho e_0 - rho0 G(u)), evaluated at
// site s and written to the buffer slot that the next pull reads from.
template <class L, typename S>
__global__ __launch_bounds__(256) void k_init_eq(const ConvParams cp,
                                                 const double *__restrict__ rho,
                                                 const double *__restrict__ u,
                                                 S *__restrict__ buf) {
  using ST = Store<S, double>;
  const int64_t N = (int64_t)cp.nx * cp.ny * cp.nz;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  const double r = rho ? rho[s] : cp.rho0;
  const double ux = u ? u[s] : 0.0, uy = u ? u[N + s] : 0.0,
               uz = u ? u[2 * N + s] : 0.0;
  double t[L::NT];
#pragma unroll
  for (int k = 0; k < L::NT; ++k) t[k] = 0.0;
  t[0] = r;
  if constexpr (L::Q == 19) {
    double dd[19];
    d3q19::shift_inverse(t, ux, uy, uz);
    t[0] = r - cp.rho0;
    d3q19::populations(t, dd);
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
      ST::store(buf + state_offset<L>(cp, i, s), dd[i],
                cp.iscale[i]);
  } else {
    add_rest_moments<L::D, double>(t, -cp.rho0, ux, uy, uz);
    const Axis<double> ax(ux), ay(uy), az(uz);
    tensor_inv<L::D, double>(t, ax, ay, az);
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
      ST::store(buf + state_offset<L>(cp, i, s),
                t[pop_pos<L>(i)], cp.iscale[i]);
  }
}

template <class L, typename S>
__global__ __launch_bounds__(256) void k_set_state(const ConvParams cp,
                                                   const double *__restrict__ f,
                                                   S *__restrict__ buf) {
  using ST = Store<S, double>;
  const int64_t N = (int64_t)cp.nx * cp.ny * cp.nz;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
#pragma unroll
  for (int i = 0; i < L::Q; ++i)
    ST::store(buf + state_offset<L>(cp, i, s),
              f[(int64_t)i * N + s] - cp.w[i] * cp.rho0, cp.iscale[i]);
}

template <class L, typename S>
__global__ __launch_bounds__(256) void k_get_state(const ConvParams cp,
                                                   const S *__restrict__ buf,
                                                   double *__restrict__ f) {
  using ST = Store<S, double>;
  const int64_t N = (int64_t)cp.nx * cp.ny * cp.nz;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
#pragma unroll
  for (int i = 0; i < L::Q; ++i)
    f[(int64_t)i * N + s] =
        cp.w[i] * cp.rho0 +
        ST::load(buf + state_offset<L>(cp, i, s),
                 cp.scale[i]);
}

template <class L, typename S>
__global__ __launch_bounds__(256) void k_gather(const ConvParams cp,
                                                const S *__restrict__ buf,
                                                const int64_t *__restrict__ sites,
                                                int64_t n,
                                                double *__restrict__ out) {
  using ST = Store<S, double>;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t s = sites[k];
#pragma unroll
  for (int i = 0; i < L::Q; ++i)
    out[k * L::Q + i] =
        cp.w[i] * cp.rho0 +
        ST::load(buf + state_offset<L>(cp, i, s),
                 cp.scale[i]);
}

template <class L, typename S, typename T>
__global__ __launch_bounds__(256) void k_macro(const ConvParams cp,
                                               const S *__restrict__ buf,
                                               T *__restrict__ rho_out,
                                               T *__restrict__ u_out) {
  using ST = Store<S, double>;
  const int64_t N = (int64_t)cp.nx * cp.ny * cp.nz;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  double drho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const double d =
        ST::load(buf + state_offset<L>(cp, i, s),
                 cp.scale[i]);
    drho += d;
    j[0] += L::cx[i] * d;
    j[1] += L::cy[i] * d;
    j[2] += L::cz[i] * d;
  }
  const double rho = cp.rho0 + drho;
  if (rho_out) rho_out[s] = (T)rho;
  if (u_out) {
    u_out[s] = (T)(j[0] / rho);
    u_out[N + s] = (T)(j[1] / rho);
    u_out[2 * N + s] = (T)(j[2] / rho);
  }
}

template <class L, typename R>
__global__ __launch_bounds__(256) void k_noise(uint32_t key0, uint32_t key1,
                                               uint32_t replica, uint64_t step,
                                               int64_t site0, int64_t n,
                                               double *__restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  R eta[L::NNOISE];
  site_normals<L, R>((uint32_t)(site0 + k), step, replica, key0, key1, R(1), eta);
  for (int v = 0; v < L::Q; ++v)
    out[k * L::Q + v] =
        v < L::FIRST_NOISY ? 0.0 : (double)eta[v - L::FIRST_NOISY];
}

__global__ __launch_bounds__(256) void k_philox(const uint32_t *__restrict__ ctr,
                                                int64_t n, uint32_t key0,
                                                uint32_t key1,
                                                uint32_t *__restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const U4 w = philox4x32_10(ctr[4 * k], ctr[4 * k + 1], ctr[4 * k + 2],
                             ctr[4 * k + 3], key0, key1);
  out[4 * k] = w.x;
  out[4 * k + 1] = w.y;
  out[4 * k + 2] = w.z;
  out[4 * k + 3] = w.w;
}

// plain streaming copy of n16 16-byte elements (the HBM calibration kernel)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void cmf_stream_copy_kernel(
    const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, size_t n16) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + k), dst + k);
}

__global__ void k_zero_i64(int64_t *p, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0;
}

__global__ void k_set_i64(int64_t *p, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// ---------------------------------------------------------------------------
// structure factor (amortized diagnostic): fields, |FFT|^2 accumulation and
// deterministic shell binning
// ---------------------------------------------------------------------------
// drho = rho - rho0, u_x, u_y, u_z of the pre-collision state as 4 FP32
// planes of N values (FP64 arithmetic, rounded once).
template <class L, typename S>
__global__ __launch_bounds__(256) void k_macro_dev(const ConvParams cp,
                                                   const S *__restrict__ buf,
                                                   float *__restrict__ out) {
  using ST = Store<S, double>;
  const int64_t N = (int64_t)cp.nx * cp.ny * cp.nz;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  double drho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const double d = ST::load(buf + state_offset<L>(cp, i, s),
                              cp.scale[i]);
    drho += d;
    j[0] += L::cx[i] * d;
    j[1] += L::cy[i] * d;
    j[2] += L::cz[i] * d;
  }
  const double rho = cp.rho0 + drho;
  out[s] = (float)drho;
  out[N + s] = (float)(j[0] / rho);
  out[2 * N + s] = (float)(j[1] / rho);
  out[3 * N + s] = (float)(j[2] / rho);
}

// acc[f][m] += |F_f(m)|^2 / N for the 4 transformed fields (M modes each)
__global__ __launch_bounds__(256) void k_sk_accumulate(
    const float2 *__restrict__ F, int64_t M, double inv_n,
    double *__restrict__ acc) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= 4 * M) return;
  const float2 c = F[m];
  acc[m] += ((double)c.x * c.x + (double)c.y * c.y) * inv_n;
}

// shell of half-spectrum mode m (nxh = nx/2 + 1 modes along x), with the
// Hermitian weight of the modes the real transform does not store
struct ShellGeom {
  int nx, ny, nz, nxh, nbins;
  double kmax;
};

__device__ __forceinline__ int shell_of(const ShellGeom &g, int64_t m,
                                        double *weight, double *kmag) {
  const int kx = (int)(m % g.nxh);
  const int64_t r = m / g.nxh;
  const int ky0 = (int)(r % g.ny), kz0 = (int)(r / g.ny);
  const int ky = ky0 <= g.ny / 2 ? ky0 : ky0 - g.ny;
  const int kz = kz0 <= g.nz / 2 ? kz0 : kz0 - g.nz;
  const double two_pi = 6.283185307179586;
  const double ax = two_pi * kx / g.nx, ay = two_pi * ky / g.ny,
               az = two_pi * kz / g.nz;
  const double k = sqrt(ax * ax + ay * ay + az * az);
  *kmag = k;
  const bool self = kx == 0 || (g.nx % 2 == 0 && kx == g.nx / 2);
  *weight = self ? 1.0 : 2.0;
  if (kx == 0 && ky == 0 && kz == 0) return -1;  // k = 0 excluded
  int b = (int)(k / g.kmax * g.nbins);
  return b < g.nbins ? b : g.nbins - 1;
}

// shell index of every half-spectrum mode (-1 for k = 0)
__global__ __launch_bounds__(256) void k_sk_shell_index(const ShellGeom g, int64_t M,
                                                        int32_t *__restrict__ bin) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  double w, k;
  bin[m] = shell_of(g, m, &w, &k);
}

// one workgroup per shell sums its modes (listed contiguously in `perm`,
// shell b in [off[b], off[b + 1])) in a fixed order:
// out[b] = (sum w k, sum w, sum w S_rho, sum w S_ux, sum w S_uy, sum w S_uz)
constexpr int kSkCols = 6;
__global__ __launch_bounds__(256) void k_sk_segments(const double *__restrict__ acc,
                                                     int64_t M, const ShellGeom g,
                                                     const int32_t *__restrict__ perm,
                                                     const int64_t *__restrict__ off,
                                                     double *__restrict__ out) {
  __shared__ double sh[256][kSkCols];
  const int b = blockIdx.x;
  double s[kSkCols] = {0, 0, 0, 0, 0, 0};
  for (int64_t j = off[b] + threadIdx.x; j < off[b + 1]; j += blockDim.x) {
    const int64_t m = perm[j];
    double w, k;
    shell_of(g, m, &w, &k);
    s[0] += w * k;
    s[1] += w;
#pragma unroll
    for (int f = 0; f < 4; ++f) s[2 + f] += w * acc[f * M + m];
  }
#pragma unroll
  for (int c = 0; c < kSkCols; ++c) sh[threadIdx.x][c] = s[c];
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h)
#pragma unroll
      for (int c = 0; c < kSkCols; ++c) sh[threadIdx.x][c] += sh[threadIdx.x + h][c];
    __syncthreads();
  }
  if (threadIdx.x < kSkCols) out[(int64_t)b * kSkCols + threadIdx.x] = sh[0][threadIdx.x];
}

// ---------------------------------------------------------------------------
// velocity statistics of the pre-collision state (Test 7, Fig. 8): moments
// about a given centre and normalised histograms, FP64 per site
// ---------------------------------------------------------------------------
template <class L, typename S>
__device__ __forceinline__ void site_velocity(const ConvParams &cp,
                                              const S *__restrict__ buf,
                                              int64_t s, double u[3]) {
  using ST = Store<S, double>;
  double drho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const double d = ST::load(buf + state_offset<L>(cp, i, s),
                              cp.scale[i]);
    drho += d;
    j[0] += L::cx[i] * d;
    j[1] += L::cy[i] * d;
    j[2] += L::cz[i] * d;
  }
  const double rho = cp.rho0 + drho;
  u[0] = j[0] / rho;
  u[1] = j[1] / rho;
  u[2] = j[2] / rho;
}

// per-block sums of (u_a - c_a)^p, p = 1..4, a = x, y, z (column 4 a + p - 1),
// each block over a fixed set of sites in a fixed order
template <class L, typename S>
__global__ __launch_bounds__(256) void k_vel_moments(const ConvParams cp,
                                                     const S *__restrict__ buf,
                                                     const VelNorm c,
                                                     double *__restrict__ partials) {
  const int64_t N = (int64_t)cp.nx * cp.ny * cp.nz;
  double acc[kVelCols];
#pragma unroll
  for (int k = 0; k < kVelCols; ++k) acc[k] = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < N; s += (int64_t)gridDim.x * 256) {
    double u[3];
    site_velocity<L, S>(cp, buf, s, u);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double v = u[a] - c.centre[a], v2 = v * v;
      acc[4 * a] += v;
      acc[4 * a + 1] += v2;
      acc[4 * a + 2] += v2 * v;
      acc[4 * a + 3] += v2 * v2;
    }
  }
  __shared__ double sh[256][kVelCols];
#pragma unroll
  for (int k = 0; k < kVelCols; ++k) sh[threadIdx.x][k] = acc[k];
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h)
#pragma unroll
      for (int k = 0; k < kVelCols; ++k) sh[threadIdx.x][k] += sh[threadIdx.x + h][k];
    __syncthreads();
  }
  if (threadIdx.x < kVelCols) partials[(int64_t)blockIdx.x * kVelCols + threadIdx.x] = sh[0][threadIdx.x];
}

// one workgroup: fixed-order sum of the block rows
__global__ __launch_bounds__(256) void k_vel_moments_final(const double *__restrict__ partials,
                                                           int nparts, double *__restrict__ out) {
  __shared__ double sh[256][kVelCols];
  double acc[kVelCols];
#pragma unroll
  for (int k = 0; k < kVelCols; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < nparts; b += 256)
#pragma unroll
    for (int k = 0; k < kVelCols; ++k) acc[k] += partials[(int64_t)b * kVelCols + k];
#pragma unroll
  for (int k = 0; k < kVelCols; ++k) sh[threadIdx.x][k] = acc[k];
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h)
#pragma unroll
      for (int k = 0; k < kVelCols; ++k) sh[threadIdx.x][k] += sh[threadIdx.x + h][k];
    __syncthreads();
  }
  if (threadIdx.x < kVelCols) out[threadIdx.x] = sh[0][threadIdx.x];
}

// histogram of x = (u_a - centre_a) / sigma_a: bin 0 counts x < -xmax (and
// non-finite x), bins 1..nbins split [-xmax, xmax) evenly, bin nbins + 1
// counts x >= xmax; LDS counters per block, integer totals (order-free)
template <class L, typename S>
__global__ __launch_bounds__(256) void k_vel_hist(const ConvParams cp,
                                                  const S *__restrict__ buf,
                                                  const VelNorm c, int dims, int nbins,
                                                  double xmax,
                                                  unsigned long long *__restrict__ counts) {
  extern __shared__ uint32_t hist[];
  const int nb2 = nbins + 2;
  for (int k = threadIdx.x; k < 3 * nb2; k += 256) hist[k] = 0u;
  __syncthreads();
  const int64_t N = (int64_t)cp.nx * cp.ny * cp.nz;
  const double width = 2.0 * xmax / nbins;
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < N; s += (int64_t)gridDim.x * 256) {
    double u[3];
    site_velocity<L, S>(cp, buf, s, u);
    for (int a = 0; a < dims; ++a) {
      const double x = (u[a] - c.centre[a]) * c.inv_sigma[a];
      int b;
      if (!(x >= -xmax)) {
        b = 0;
      } else if (x >= xmax) {
        b = nbins + 1;
      } else {
        b = 1 + (int)floor((x + xmax) / width);
        b = b > nbins ? nbins : b;
      }
      atomicAdd(&hist[a * nb2 + b], 1u);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < 3 * nb2; k += 256)
    if (hist[k]) atomicAdd(&counts[k], (unsigned long long)hist[k]);
}

__global__ void k_bump_step(int64_t *step_ptr, int64_t by) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step_ptr = *step_ptr + by;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_step(int q, int storage, bool general, bool nt, int mode,
                       const void *params, const void *src, void *dst,
                       const int64_t *step_ptr, int step_off, double *partials,
                       int grid, int block, hipStream_t stream) {
  if (mode == kStreamPull)
    return launch_step_pull(q, storage, general, nt, params, src, dst, step_ptr, step_off,
                            partials, grid, block, stream);
  if (mode == kStreamAAEven || mode == kStreamAAOdd)
    return launch_step_in_place(q, storage, general, nt, mode == kStreamAAOdd, params, dst,
                                step_ptr, step_off, partials, grid, block, stream);
  return hipErrorInvalidValue;
}

hipError_t launch_finalize(const double *partials, int nparts, double *level2,
                           double *series, int cap, int64_t *step_ptr, int step_off,
                           int bump, double mass0, bool stats, hipStream_t stream) {
  return launch_finalize_batch(partials, 0, 1, nparts, level2, series, cap, step_ptr, step_off,
                               bump, mass0, stats, stream);
}

hipError_t launch_finalize_batch(const double *partials, int64_t pstride, int count, int nparts,
                                 double *level2, double *series, int cap, int64_t *step_ptr,
                                 int step_off, int bump, double mass0, bool stats,
                                 hipStream_t stream) {
  if (count < 1 || (count > 1 && bump != 0)) return hipErrorInvalidValue;
  const double *rows = partials;
  int nrows = nparts;
  int64_t rstride = pstride;
  if (stats && nparts > kLevel2Threshold) {
    int nb = (nparts + kLevel2Threshold - 1) / kLevel2Threshold;
    if (nb > kMaxLevel2) nb = kMaxLevel2;
    const int chunk = (nparts + nb - 1) / nb;
    nb = (nparts + chunk - 1) / chunk;
    hipLaunchKernelGGL(k_reduce_partials, dim3(nb, count), dim3(256), 0, stream, partials,
                       nparts, chunk, pstride, level2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    rows = level2;
    nrows = nb;
    rstride = (int64_t)nb * kPartStride;
  }
  hipLaunchKernelGGL(k_finalize, dim3(count), dim3(256), 0, stream, rows, nrows, rstride,
                     series, cap, step_ptr, step_off, bump, mass0, stats ? 1 : 0);
  return hipGetLastError();
}

template <class T>
struct Tag {
  using type = T;
};

// call f(Tag<Lattice>, Tag<StorageType>) for a runtime (q, storage)
template <class F>
hipError_t with_lattice_storage(int q, int storage, F &&f) {
  auto by_storage = [&](auto lt) -> hipError_t {
    switch (storage) {
      case kF64: return f(lt, Tag<double>{});
      case kF32: return f(lt, Tag<float>{});
      case kF16: return f(lt, Tag<__half>{});
      case kBF16: return f(lt, Tag<__hip_bfloat16>{});
    }
    return hipErrorInvalidValue;
  };
  if (q == 9) return by_storage(Tag<D2Q9>{});
  if (q == 19) return by_storage(Tag<D3Q19>{});
  if (q == 27) return by_storage(Tag<D3Q27>{});
  return hipErrorInvalidValue;
}

hipError_t launch_init_eq(int q, int storage, const ConvParams &cp,
                          const double *rho, const double *u, void *buf,
                          hipStream_t stream) {
  const int64_t N = (int64_t)cp.nx * cp.ny * cp.nz;
  return with_lattice_storage(q, storage, [&](auto lt, auto stt) {
    using L = typename decltype(lt)::type;
    using S = typename decltype(stt)::type;
    hipLaunchKernelGGL((k_init_eq<L, S>), dim3(blocks_for(N, 256)), dim3(256),
                       0, stream, cp, rho, u, static_cast<S *>(buf));
    return hipGetLastError();
  });
}

hipError_t launch_set_state(int q, int storage, const ConvParams &cp,
                            const double *f, void *buf, hipStream_t stream) {
  const int64_t N = (int64_t)cp.nx * cp.ny * cp.nz;
  return with_lattice_storage(q, storage, [&](auto lt, auto stt) {
    using L = typename decltype(lt)::type;
    using S = typename decltype(stt)::type;
    hipLaunchKernelGGL((k_set_state<L, S>), dim3(blocks_for(N, 256)),
                       dim3(256), 0, stream, cp, f, static_cast<S *>(buf));
    return hipGetLastError();
  });
}

hipError_t launch_get_state(int q, int storage, const ConvParams &cp,
                            const void *buf, double *f, hipStream_t stream) {
  const int64_t N = (int64_t)cp.nx * cp.ny * cp.nz;
  return with_lattice_storage(q, storage, [&](auto lt, auto stt) {
    using L = typename decltype(lt)::type;
    using S = typename decltype(stt)::type;
    hipLaunchKernelGGL((k_get_state<L, S>), dim3(blocks_for(N, 256)),
                       dim3(256), 0, stream, cp, static_cast<const S *>(buf), f);
    return hipGetLastError();
  });
}

hipError_t launch_gather(int q, int storage, const ConvParams &cp,
                         const void *buf, const int64_t *sites, int64_t n,
                         double *out, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  return with_lattice_storage(q, storage, [&](auto lt, auto stt) {
    using L = typename decltype(lt)::type;
    using S = typename decltype(stt)::type;
    hipLaunchKernelGGL((k_gather<L, S>), dim3(blocks_for(n, 256)), dim3(256), 0,
                       stream, cp, static_cast<const S *>(buf), sites, n, out);
    return hipGetLastError();
  });
}

template <typename T>
hipError_t macro_t(int q, int storage, const ConvParams &cp, const void *buf, T *rho,
                   T *u, hipStream_t stream) {
  const int64_t N = (int64_t)cp.nx * cp.ny * cp.nz;
  return with_lattice_storage(q, storage, [&](auto lt, auto stt) {
    using L = typename decltype(lt)::type;
    using S = typename decltype(stt)::type;
    hipLaunchKernelGGL((k_macro<L, S, T>), dim3(blocks_for(N, 256)), dim3(256), 0,
                       stream, cp, static_cast<const S *>(buf), rho, u);
    return hipGetLastError();
  });
}

hipError_t launch_macro(int q, int storage, const ConvParams &cp,
                        const void *buf, float *rho, float *u,
                        hipStream_t stream) {
  return macro_t<float>(q, storage, cp, buf, rho, u, stream);
}

hipError_t launch_macro(int q, int storage, const ConvParams &cp,
                        const void *buf, double *rho, double *u,
                        hipStream_t stream) {
  return macro_t<double>(q, storage, cp, buf, rho, u, stream);
}

hipError_t launch_noise(int q, int fp64, uint32_t key0, uint32_t key1,
                        uint32_t replica, uint64_t step, int64_t site0,
                        int64_t n, double *out, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const unsigned g = blocks_for(n, 256);
  if (q == 9) {
    if (fp64)
      hipLaunchKernelGGL((k_noise<D2Q9, double>), dim3(g), dim3(256), 0, stream,
                         key0, key1, replica, step, site0, n, out);
    else
      hipLaunchKernelGGL((k_noise<D2Q9, float>), dim3(g), dim3(256), 0, stream,
                         key0, key1, replica, step, site0, n, out);
  } else if (q == 19) {
    if (fp64)
      hipLaunchKernelGGL((k_noise<D3Q19, double>), dim3(g), dim3(256), 0,
                         stream, key0, key1, replica, step, site0, n, out);
    else
      hipLaunchKernelGGL((k_noise<D3Q19, float>), dim3(g), dim3(256), 0, stream,
                         key0, key1, replica, step, site0, n, out);
  } else if (q == 27) {
    if (fp64)
      hipLaunchKernelGGL((k_noise<D3Q27, double>), dim3(g), dim3(256), 0,
                         stream, key0, key1, replica, step, site0, n, out);
    else
      hipLaunchKernelGGL((k_noise<D3Q27, float>), dim3(g), dim3(256), 0, stream,
                         key0, key1, replica, step, site0, n, out);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, int64_t n, uint32_t key0,
                         uint32_t key1, uint32_t *out, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox, dim3(blocks_for(n, 256)), dim3(256), 0, stream,
                     ctr, n, key0, key1, out);
  return hipGetLastError();
}

hipError_t launch_stream_copy(const void *src, void *dst, size_t n16,
                              hipStream_t stream) {
  if (n16 == 0) return hipSuccess;
  // one 16-byte element per thread (a grid-stride loop only beyond 2^30
  // workgroups): the fastest plain copy measured on gfx950
  size_t blocks = (n16 + 255) / 256;
  if (blocks > ((size_t)1 << 30)) blocks = (size_t)1 << 30;
  hipLaunchKernelGGL(cmf_stream_copy_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     stream, static_cast<const u32x4 *>(src),
                     static_cast<u32x4 *>(dst), n16);
  return hipGetLastError();
}

hipError_t launch_bump_step(int64_t *step_ptr, int64_t by, hipStream_t stream) {
  hipLaunchKernelGGL(k_bump_step, dim3(1), dim3(64), 0, stream, step_ptr, by);
  return hipGetLastError();
}

hipError_t launch_macro_dev(int q, int storage, const ConvParams &cp,
                            const void *buf, float *out, hipStream_t stream) {
  const int64_t N = (int64_t)cp.nx * cp.ny * cp.nz;
  return with_lattice_storage(q, storage, [&](auto lt, auto stt) {
    using L = typename decltype(lt)::type;
    using S = typename decltype(stt)::type;
    hipLaunchKernelGGL((k_macro_dev<L, S>), dim3(blocks_for(N, 256)), dim3(256), 0,
                       stream, cp, static_cast<const S *>(buf), out);
    return hipGetLastError();
  });
}

hipError_t launch_sk_accumulate(const void *F, int64_t M, double inv_n,
                                double *acc, hipStream_t stream) {
  hipLaunchKernelGGL(k_sk_accumulate, dim3(blocks_for(4 * M, 256)), dim3(256), 0,
                     stream, static_cast<const float2 *>(F), M, inv_n, acc);
  return hipGetLastError();
}

ShellGeom shell_geom(int nx, int ny, int nz, int nbins) {
  ShellGeom g;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.nxh = nx / 2 + 1;
  g.nbins = nbins;
  const double pi = 3.141592653589793;
  g.kmax = pi * sqrt((nx > 1 ? 1.0 : 0.0) + (ny > 1 ? 1.0 : 0.0) + (nz > 1 ? 1.0 : 0.0)) *
           (1.0 + 1e-12);
  return g;
}

hipError_t launch_sk_shell_index(int nx, int ny, int nz, int nbins, int64_t M,
                                 int32_t *bin, hipStream_t stream) {
  hipLaunchKernelGGL(k_sk_shell_index, dim3(blocks_for(M, 256)), dim3(256), 0, stream,
                     shell_geom(nx, ny, nz, nbins), M, bin);
  return hipGetLastError();
}

hipError_t launch_sk_segments(const double *acc, int64_t M, int nx, int ny, int nz,
                              int nbins, const int32_t *perm, const int64_t *off,
                              double *out, hipStream_t stream) {
  hipLaunchKernelGGL(k_sk_segments, dim3(nbins), dim3(256), 0, stream, acc, M,
                     shell_geom(nx, ny, nz, nbins), perm, off, out);
  return hipGetLastError();
}

hipError_t launch_vel_moments(int q, int storage, const ConvParams &cp, const void *buf,
                              const VelNorm &c, int grid, double *partials, double *out,
                              hipStream_t stream) {
  hipError_t e = with_lattice_storage(q, storage, [&](auto lt, auto stt) {
    using L = typename decltype(lt)::type;
    using S = typename decltype(stt)::type;
    hipLaunchKernelGGL((k_vel_moments<L, S>), dim3(grid), dim3(256), 0, stream, cp,
                       static_cast<const S *>(buf), c, partials);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vel_moments_final, dim3(1), dim3(256), 0, stream, partials, grid, out);
  return hipGetLastError();
}

hipError_t launch_vel_hist(int q, int storage, const ConvParams &cp, const void *buf,
                           const VelNorm &c, int grid, int nbins, double xmax,
                           unsigned long long *counts, hipStream_t stream) {
  const size_t lds = sizeof(uint32_t) * 3 * (size_t)(nbins + 2);
  const int dims = q == 9 ? 2 : 3;
  return with_lattice_storage(q, storage, [&](auto lt, auto stt) {
    using L = typename decltype(lt)::type;
    using S = typename decltype(stt)::type;
    hipLaunchKernelGGL((k_vel_hist<L, S>), dim3(grid), dim3(256), lds, stream, cp,
                       static_cast<const S *>(buf), c, dims, nbins, xmax, counts);
    return hipGetLastError();
  });
}

hipError_t launch_set_i64(int64_t *p, int64_t v, hipStream_t stream) {
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, stream, p, v);
  return hipGetLastError();
}

hipError_t launch_zero_i64(int64_t *p, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_i64, dim3(blocks_for(n, 256)), dim3(256), 0, stream,
                     p, n);
  return hipGetLastError();
}

}  // namespace cmf
