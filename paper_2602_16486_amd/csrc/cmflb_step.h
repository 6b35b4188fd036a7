// cmflb_step.h -- the fused step of libcmflb for gfx950: the per-site
// collision (D2Q9, D3Q19, D3Q27), the block reduction of its statistics, the
// single-lattice step kernels (two-buffer pull and in-place pair) and their
// launch templates.  Included by cmflb_ensemble.hip (the ensemble step
// inlines the same collision), by cmflb_kernels.hip (launch_step) and by the
// two translation units that instantiate the launches.
//
// Method: De Rosis & Zhou, "A fluctuating lattice Boltzmann formulation based
// on orthogonal central moments" (arXiv 2602.16486), Sec. 2.2 (D2Q9),
// Sec. 2.3 (D3Q27) and Sec. 2.4 (D3Q19).  The per-site work follows the
// paper's "Algorithm of computation": macroscopic moments (eq. macro),
// normals, pre-collision central moments, collision (eq. cm_collision with
// phi of eq. phi_general), back transformation f* = T(u)^-1 k*, streaming
// (eq. streaming).
//
// Memory layout: populations are stored as deviations d_i = f_i - w_i rho0
// in a row-interleaved structure of arrays (pop_row_offset): for lattice row
// (y, z) the Q rows of nx values are contiguous, in the order of the
// velocities (c_z, c_y, c_x) (pop_slot).  The buffer of step t
// holds post-collision values of step t - 1 at their source site; step t
// pulls d_i(x - c_i), collides, and writes d*_i(x) to the other buffer
// (two-buffer pull scheme), or, with in-place streaming, the even and odd
// steps of a pair read and write one buffer.  Every value is read once and
// written once per step, so the step is HBM-bound at 2 Q sizeof(storage)
// bytes per site.
//
// Work decomposition: a tile is BX consecutive sites of one x-row
// (BX = blockDim.x, a multiple of 64); a block walks tiles
// blockIdx.x, blockIdx.x + gridDim.x, ... (or has exactly one) and keeps its
// statistics in registers until the end, so the partial-sum traffic is one
// row per block.
#pragma once

#include "cmflb_d3q19.h"
#include "cmflb_device.h"
#include "cmflb_internal.h"

#include <type_traits>

namespace cmf {

// ---------------------------------------------------------------------------
// per-site collision
// ---------------------------------------------------------------------------

// Per-thread statistics of the sites a thread processes: drho, j(3), u(3),
// u^2(3), non-finite count.  Acc sums them in FP64 over several sites;
// SiteStats holds the compute-type values of a single site (a thread that
// processes one site), which the block reduction converts to FP64 exactly.
// Both give the same FP64 sums for one site per thread.
struct Acc {
  using lds_type = double;
  double v[kNAcc];
  template <typename R>
  __device__ __forceinline__ void record(R drho, R jx, R jy, R jz, R ux, R uy, R uz,
                                         bool finite) {
    v[0] += (double)drho;
    v[1] += (double)jx;
    v[2] += (double)jy;
    v[3] += (double)jz;
    v[4] += (double)ux;
    v[5] += (double)uy;
    v[6] += (double)uz;
    v[7] += (double)(ux * ux);
    v[8] += (double)(uy * uy);
    v[9] += (double)(uz * uz);
    v[10] += finite ? 0.0 : 1.0;
  }
};

template <typename R>
struct SiteStats {
  using lds_type = R;
  R v[kNAcc] = {};
  __device__ __forceinline__ void record(R drho, R jx, R jy, R jz, R ux, R uy, R uz,
                                         bool finite) {
    v[0] = drho;
    v[1] = jx;
    v[2] = jy;
    v[3] = jz;
    v[4] = ux;
    v[5] = uy;
    v[6] = uz;
    v[7] = ux * ux;
    v[8] = uy * uy;
    v[9] = uz * uz;
    v[10] = finite ? R(0) : R(1);
  }
};

// 1 / rho: the hardware reciprocal in FP32 (within 1 ulp; the FP32 path's
// error budget is set by its storage rounding), a division in FP64
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

template <typename R>
__device__ __forceinline__ bool finite4(R a, R b, R c, R d) {
  return __builtin_isfinite(a) && __builtin_isfinite(b) &&
         __builtin_isfinite(c) && __builtin_isfinite(d);
}

// d: the Q pulled deviations (population order) in, the post-collision
// deviations out.  GENERAL selects the full forward transform for arbitrary
// Lambda; otherwise the rates follow the paper's pattern (Lambda = 1 except
// the modes relaxed at omega: D2Q9 v = 4, 5; D3Q27 v = 7, 8, 9) and only
// those pre-collision central moments are formed, as the paper does.
// P is any parameter record with the fields of StepParams (rho0, amp, oml,
// lam, noise, replica, key0, key1): the single-lattice kernel passes its
// kernel argument, the ensemble kernel a replica record in global memory.
// LEAN (16-bit storage, issue-bound): the noise amplitude of a mode relaxed
// at rate 1 is formed as amp1 sqrt(b_v) with sqrt(b_v) a compile-time
// constant, instead of being kept per mode in scalar registers (which then
// spill into vector lanes); the wider storages, bound by HBM, measured
// slightly faster with the per-mode values.
template <class L, typename R, bool GENERAL, bool LEAN, class P, class A>
__device__ __forceinline__ void collide_tensor(R *d, const P &p,
                                               uint32_t site, uint64_t step,
                                               A &acc) {
  constexpr int Q = L::Q;
  // step 1: rho = rho0 + sum d, rho u = sum c d (eq. macro).  D3Q27 forms
  // them from per-row partial sums (sum and difference along x of each
  // (c_y, c_z) row, then along y), which also yields the off-diagonal sums
  // sxy, sxz, syz of the pre-collision k_7..k_9.
  R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
  R sxy = R(0), sxz = R(0), syz = R(0);
  if constexpr (Q == 27) {
    constexpr PosTable<L> tab{};
    R s0[9], s1[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const R gm = d[tab.pop[3 * r]], g0 = d[tab.pop[3 * r + 1]],
              gp = d[tab.pop[3 * r + 2]];
      s0[r] = (gm + gp) + g0;  // sum over c_x
      s1[r] = gp - gm;         // sum of c_x d
    }
    R t0[3], t1[3], u0[3], v1[3];
#pragma unroll
    for (int z = 0; z < 3; ++z) {
      t0[z] = (s0[3 * z] + s0[3 * z + 2]) + s0[3 * z + 1];
      t1[z] = s0[3 * z + 2] - s0[3 * z];
      u0[z] = (s1[3 * z] + s1[3 * z + 2]) + s1[3 * z + 1];
      v1[z] = s1[3 * z + 2] - s1[3 * z];
    }
    drho = (t0[0] + t0[2]) + t0[1];
    jx = (u0[0] + u0[2]) + u0[1];
    jy = (t1[0] + t1[2]) + t1[1];
    jz = t0[2] - t0[0];
    sxy = (v1[0] + v1[2]) + v1[1];
    sxz = u0[2] - u0[0];
    syz = t1[2] - t1[0];
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      drho += d[i];
      if (L::cx[i] > 0) jx += d[i];
      if (L::cx[i] < 0) jx -= d[i];
      if (L::cy[i] > 0) jy += d[i];
      if (L::cy[i] < 0) jy -= d[i];
    }
  }
  const R rho = p.rho0 + drho;
  const R irho = recip(rho);
  const R ux = jx * irho, uy = jy * irho, uz = jz * irho;

  acc.record(drho, jx, jy, jz, ux, uy, uz, finite4(rho, ux, uy, uz));

  // step 2: normals of the noisy modes.  phi_v = a1 amp_v with the site's
  // noise scale a1 = sqrt(rho kT / c_s^2) (eq. phi_general with the local
  // rho) and the mode factors amp_v = sqrt(Lambda_v (2 - Lambda_v) b_v).
  // The issue-bound 16-bit kernels (LEAN) draw the plain normals, which do
  // not wait for the loaded populations, and scale each mode by a1 amp_v;
  // the others draw them times a1 (one multiply per pair of modes instead
  // of one per mode: FP32 256^3 step 1.3 % faster)
  const R a1 = p.amp1 * sqrt(rho);
  R eta[L::NNOISE];
  if (p.noise) {
    site_normals<L, R>(site, step, p.replica, p.key0, p.key1, LEAN ? R(1) : a1, eta);
  } else {
#pragma unroll
    for (int n = 0; n < L::NNOISE; ++n) eta[n] = R(0);
  }

  R t[L::NT];
  if constexpr (!GENERAL) {
    // steps 3-4 with the paper's rates: only the modes relaxed at omega
    // need their pre-collision value; every other noisy mode is pure noise
    // around k_eq = 0.
    if constexpr (Q == 27) {
      // k_7, k_8, k_9 (Sec. 2.3): sum f c_a c_b - rho u_a u_b; the rest
      // weights do not contribute to the off-diagonal sums.
      const R k7 = sxy - jx * uy, k8 = sxz - jx * uz, k9 = syz - jy * uz;
      t[0] = rho;
      t[1] = R(0);
      t[3] = R(0);
      t[9] = R(0);
#pragma unroll
      for (int n = 0; n < L::NNOISE; ++n) {
        const int v = L::FIRST_NOISY + n;
        R val;
        if (v == 7)
          val = p.oml[7] * k7 + (LEAN ? a1 * p.amp[7] : p.amp[7]) * eta[n];
        else if (v == 8)
          val = p.oml[8] * k8 + (LEAN ? a1 * p.amp[8] : p.amp[8]) * eta[n];
        else if (v == 9)
          val = p.oml[9] * k9 + (LEAN ? a1 * p.amp[9] : p.amp[9]) * eta[n];
        else if constexpr (LEAN)
          val = a1 * R(sqrt_norm<L>(v)) * eta[n];
        else
          val = p.amp[v] * eta[n];
        t[L::mode_pos[v]] = val;
      }
    } else {
      R sd = R(0);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int dd = L::cx[i] * L::cx[i] - L::cy[i] * L::cy[i];
        const int pxy = L::cx[i] * L::cy[i];
        if (dd > 0) sd += d[i];
        if (dd < 0) sd -= d[i];
        if (pxy > 0) sxy += d[i];
        if (pxy < 0) sxy -= d[i];
      }
      // k_4 = r_4 - rho (u_x^2 - u_y^2), k_5 = r_5 - rho u_x u_y (Sec. 2.2)
      const R k4 = sd - (jx * ux - jy * uy);
      const R k5 = sxy - jx * uy;
      auto amp_eta = [&](int v, R e) { return LEAN ? a1 * R(sqrt_norm<L>(v)) * e : p.amp[v] * e; };
      const R k3s = amp_eta(3, eta[0]);
      const R k4s = p.oml[4] * k4 + (LEAN ? a1 * p.amp[4] : p.amp[4]) * eta[1];
      const R k5s = p.oml[5] * k5 + (LEAN ? a1 * p.amp[5] : p.amp[5]) * eta[2];
      t[0] = rho;
      t[1] = R(0);
      t[3] = R(0);
      t[2] = R(0.5) * (k3s + k4s);  // P2(x) P0(y)
      t[6] = R(0.5) * (k3s - k4s);  // P0(x) P2(y)
      t[4] = k5s;
      t[5] = amp_eta(6, eta[3]);
      t[7] = amp_eta(7, eta[4]);
      t[8] = amp_eta(8, eta[5]);
    }
  } else {
    // steps 3-4 for arbitrary rates: k = T(u) f = T(u) d + rho0 G(u), then
    // k*_v = (1 - Lambda_v) k_v + Lambda_v k_eq_v + I~_v phi_v eta_v with
    // k_eq = (rho, 0, ..., 0).
    const Axis<R> ax(ux), ay(uy), az(uz);
#pragma unroll
    for (int i = 0; i < Q; ++i) t[pop_pos<L>(i)] = d[i];
    tensor_fwd<L::D, R>(t, ax, ay, az);
    add_rest_moments<L::D, R>(t, p.rho0, ux, uy, uz);
    if constexpr (Q == 27) {
      R k[27];
#pragma unroll
      for (int v = 0; v < 27; ++v) k[v] = t[L::mode_pos[v]];
#pragma unroll
      for (int v = 0; v < 27; ++v) {
        R val = p.oml[v] * k[v];
        if (v == 0) val += p.lam[0] * rho;
        if (v >= L::FIRST_NOISY) val += (LEAN ? a1 * p.amp[v] : p.amp[v]) * eta[v - L::FIRST_NOISY];
        t[L::mode_pos[v]] = val;
      }
    } else {
      R k[9];
      k[0] = t[0];
      k[1] = t[1];
      k[2] = t[3];
      k[3] = t[2] + t[6];
      k[4] = t[2] - t[6];
      k[5] = t[4];
      k[6] = t[5];
      k[7] = t[7];
      k[8] = t[8];
      R ks[9];
#pragma unroll
      for (int v = 0; v < 9; ++v) {
        R val = p.oml[v] * k[v];
        if (v == 0) val += p.lam[0] * rho;
        if (v >= L::FIRST_NOISY) val += (LEAN ? a1 * p.amp[v] : p.amp[v]) * eta[v - L::FIRST_NOISY];
        ks[v] = val;
      }
      t[0] = ks[0];
      t[1] = ks[1];
      t[3] = ks[2];
      t[2] = R(0.5) * (ks[3] + ks[4]);
      t[6] = R(0.5) * (ks[3] - ks[4]);
      t[4] = ks[5];
      t[5] = ks[6];
      t[7] = ks[7];
      t[8] = ks[8];
    }
  }
  // steps 5-6: d* = T(u)^-1 (k* - rho0 G(u)).  The zeroth entry is
  // k*_0 - rho0 = rho - rho0 = drho exactly (mode 0 is conserved); it is set
  // directly rather than as (rho0 + drho) - rho0, which would round drho to
  // the spacing of FP32 numbers near rho0.
  // LEAN: the one-axis maps skip their halvings, so d_i comes out as
  // 2^|c_i|^2 d*_i; the 16-bit store scales of these lattices carry the
  // factor 2^-|c_i|^2 (exact: the stored values are unchanged)
  add_rest_moments<L::D, R>(t, -p.rho0, ux, uy, uz);
  t[0] = drho;
  {
    const Axis<R> ax(ux), ay(uy), az(uz);
    tensor_inv<L::D, R, LEAN>(t, ax, ay, az);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) d[i] = t[pop_pos<L>(i)];
}

// D3Q19 (Sec. 2.4): r = M d (basis raw moments of the deviations), then the
// same steps with k = N(u) r and f* = M^-1 N(u)^-1 k* (cmflb_d3q19.h).  With
// the paper's rates only k_7..k_9 = r_7..r_9 - rho u_a u_b are needed
// (M_7 = c_x c_y, M_8 = c_y c_z, M_9 = c_x c_z); k_eq = (rho, 0, ..., 0).
template <typename R, bool GENERAL, bool LEAN, class P, class A>
__device__ __forceinline__ void collide_d3q19(R *d, const P &p, uint32_t site,
                                              uint64_t step, A &acc) {
  using L = D3Q19;
  R r[19];
  d3q19::raw_moments(d, r);
  const R drho = r[0], jx = r[1], jy = r[2], jz = r[3];
  const R rho = p.rho0 + drho;
  const R irho = recip(rho);
  const R ux = jx * irho, uy = jy * irho, uz = jz * irho;

  acc.record(drho, jx, jy, jz, ux, uy, uz, finite4(rho, ux, uy, uz));

  const R a1 = p.amp1 * sqrt(rho);  // as in collide_tensor
  R eta[L::NNOISE];
  if (p.noise) {
    site_normals<L, R>(site, step, p.replica, p.key0, p.key1, LEAN ? R(1) : a1, eta);
  } else {
#pragma unroll
    for (int n = 0; n < L::NNOISE; ++n) eta[n] = R(0);
  }

  R k[19];
  if constexpr (!GENERAL) {
    const R k7 = r[7] - jx * uy, k8 = r[8] - jy * uz, k9 = r[9] - jx * uz;
    k[0] = rho;
    k[1] = R(0);
    k[2] = R(0);
    k[3] = R(0);
#pragma unroll
    for (int n = 0; n < L::NNOISE; ++n) {
      const int v = L::FIRST_NOISY + n;
      R val;
      if (v == 7)
        val = p.oml[7] * k7 + (LEAN ? a1 * p.amp[7] : p.amp[7]) * eta[n];
      else if (v == 8)
        val = p.oml[8] * k8 + (LEAN ? a1 * p.amp[8] : p.amp[8]) * eta[n];
      else if (v == 9)
        val = p.oml[9] * k9 + (LEAN ? a1 * p.amp[9] : p.amp[9]) * eta[n];
      else if constexpr (LEAN)
        val = a1 * R(sqrt_norm<L>(v)) * eta[n];
      else
        val = p.amp[v] * eta[n];
      k[v] = val;
    }
  } else {
    // raw moments of f = d + w rho0 differ from those of d in r_0 only
    r[0] = rho;
    d3q19::shift_forward(r, ux, uy, uz);
#pragma unroll
    for (int v = 0; v < 19; ++v) {
      R val = p.oml[v] * r[v];
      if (v == 0) val += p.lam[0] * rho;
      if (v >= L::FIRST_NOISY) val += (LEAN ? a1 * p.amp[v] : p.amp[v]) * eta[v - L::FIRST_NOISY];
      k[v] = val;
    }
  }
  // raw moments of f* (k*_1..k*_3 are the central first moments, zero by
  // construction, and are not read), then those of d* = f* - w rho0: r_0 =
  // k*_0 - rho0 = drho and r_1..r_3 = rho u = j exactly (mass and momentum
  // are conserved), set directly rather than re-rounded; then the populations
  d3q19::shift_inverse(k, ux, uy, uz);
  k[0] = drho;
  k[1] = jx;
  k[2] = jy;
  k[3] = jz;
  d3q19::populations(k, d);
}

template <class L, typename R, bool GENERAL, bool LEAN, class P, class A>
__device__ __forceinline__ void collide_site(R *d, const P &p, uint32_t site,
                                             uint64_t step, A &acc) {
  if constexpr (L::Q == 19)
    collide_d3q19<R, GENERAL, LEAN>(d, p, site, step, acc);
  else
    collide_tensor<L, R, GENERAL, LEAN>(d, p, site, step, acc);
}

// ---------------------------------------------------------------------------
// block reduction of the statistics accumulators (fixed order)
// ---------------------------------------------------------------------------
// LDS bytes used by block_store_acc for a workgroup of nt threads whose
// per-thread values have type T
template <typename T>
__host__ __device__ constexpr int acc_lds_bytes(int nt) {
  return kNAcc * nt * (int)sizeof(T) + kNAcc * (nt / 16) * (int)sizeof(double);
}

// Every thread writes its kNAcc values to LDS, accumulator-major; then
// (accumulator, part) pairs, P = nt / 16 parts per accumulator, sum the 16
// entries part, part + P, ..., part + 15 P in FP64 (the lanes of a wave read
// consecutive entries), and kNAcc threads add the P part sums in order.  The
// order depends only on nt (a multiple of 16).  Compared with a butterfly of
// wave shuffles this takes kNAcc + 2 additions per thread instead of
// 6 kNAcc, which matters when a workgroup processes a single tile (the
// single-lattice step in one-tile launches, every ensemble tile; with the
// shuffles the 320-replica FP16 ensemble step took 2.7 % longer).
template <class A>
__device__ __forceinline__ void block_store_acc(const A &acc, double *out, void *lds) {
  using T = typename A::lds_type;
  const int tid = threadIdx.x, nt = blockDim.x, parts = nt >> 4;
  T *vals = static_cast<T *>(lds);
#pragma unroll
  for (int k = 0; k < kNAcc; ++k) vals[k * nt + tid] = acc.v[k];
  __syncthreads();
  double *part = reinterpret_cast<double *>(vals + kNAcc * nt);
  for (int w = tid; w < kNAcc * parts; w += nt) {
    const int k = w / parts, pp = w - k * parts;
    const T *col = vals + k * nt + pp;
    double s = (double)col[0];
#pragma unroll
    for (int j = 1; j < 16; ++j) s += (double)col[j * parts];
    part[w] = s;
  }
  __syncthreads();
  if (tid < kNAcc) {
    double s = part[tid * parts];
    for (int pp = 1; pp < parts; ++pp) s += part[tid * parts + pp];
    out[tid] = s;
  }
}

// ---------------------------------------------------------------------------
// the fused step
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wrap_sub(int a, int c, int n) {
  // (a - c) mod n for c in {-1, 0, 1}
  int r = a - c;
  r = r < 0 ? r + n : r;
  r = r >= n ? r - n : r;
  return r;
}

// Pull the Q populations of site (x, y, z) of a box (nx, ny, nz) whose
// buffer starts at src: f_i(x) <- f*_i(x - c_i), periodic, with 64-bit
// addresses (the single-lattice step when a z plane of the buffer spans
// 4 GiB or more; otherwise load_site_buf).  y and z are wave-uniform (one
// lattice row per tile), so the row part of every address is scalar.
// NT_C0: non-temporal loads for the populations with c_x = 0, only when
// every population row is a whole number of cache lines (then tiles, which
// start at a row or at a multiple of 256 sites of a row, never share a
// line of such a row).
template <class L, typename S, typename R, bool NT_C0 = false>
__device__ __forceinline__ void load_site(R *d, const S *__restrict__ src,
                                          const float *scale, int nx, int ny,
                                          int nz, int x, int y, int z) {
  using ST = Store<S, R>;
  const uint32_t xs[3] = {(uint32_t)(x == nx - 1 ? 0 : x + 1), (uint32_t)x,
                          (uint32_t)(x == 0 ? nx - 1 : x - 1)};
  int64_t srow[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const int ys = wrap_sub(y, a - 1, ny);
      const int zs = L::D == 3 ? wrap_sub(z, b - 1, nz) : z;
      srow[a][b] = (int64_t)ys + (int64_t)ny * zs;
    }
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const S *base = src + pop_row_offset<L>(i, srow[L::cy[i] + 1][L::cz[i] + 1], nx);
    const float sc = scale[weight_class<L>(i)];
    // (the condition is a compile-time constant once the loop is unrolled)
    if (NT_C0 && L::cx[i] == 0)
      d[i] = ST::template load<true>(base + xs[1], sc);
    else
      d[i] = ST::template load<false>(base + xs[L::cx[i] + 1], sc);
  }
}

// Write the Q post-collision populations of site x of lattice row `row`
// (64-bit addresses, as load_site; NT selects the store kind).
template <class L, typename S, typename R, bool NT>
__device__ __forceinline__ void store_site(const R *d, S *__restrict__ dst,
                                           const float *iscale, int nx, int x,
                                           int64_t row) {
  using ST = Store<S, R>;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    S *base = dst + pop_row_offset<L>(i, row, nx);
    ST::template store<NT>(base + (uint32_t)x, d[i], iscale[weight_class<L>(i)]);
  }
}

// Buffer-addressed forms of load_site / store_site for the single-lattice
// step (BUF): one resource per source plane z - c_z (its Q ny rows of nx
// values, below 4 GiB), the row of population i of source row y - c_y as a
// scalar byte offset, and one vector byte offset per x shift.
template <class L, typename S, typename R, bool NT_C0>
__device__ __forceinline__ void load_site_buf(R *d, const S *__restrict__ src,
                                              const float *scale, int nx, int ny,
                                              int nz, int x, int y, int z) {
  using ST = Store<S, R>;
  constexpr uint32_t B = sizeof(S);
  const int64_t plane = (int64_t)ny * L::Q * nx;
  const uint32_t pbytes = (uint32_t)(plane * B);
  __amdgpu_buffer_rsrc_t rs[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int zs = L::D == 3 ? wrap_sub(z, b - 1, nz) : z;
    rs[b] = make_rsrc(src + (int64_t)zs * plane, pbytes);
  }
  const uint32_t xs[3] = {(uint32_t)(x == nx - 1 ? 0 : x + 1) * B, (uint32_t)x * B,
                          (uint32_t)(x == 0 ? nx - 1 : x - 1) * B};
  uint32_t ys[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) ys[a] = (uint32_t)wrap_sub(y, a - 1, ny);
  const uint32_t rowb = (uint32_t)nx * B;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const uint32_t soff = (ys[L::cy[i] + 1] * (uint32_t)L::Q + (uint32_t)pop_slot<L>(i)) * rowb;
    const float sc = scale[weight_class<L>(i)];
    if (NT_C0 && L::cx[i] == 0)
      d[i] = ST::from_bits(buf_load<S, true>(rs[L::cz[i] + 1], xs[1], soff), sc);
    else
      d[i] = ST::from_bits(buf_load<S, false>(rs[L::cz[i] + 1], xs[L::cx[i] + 1], soff), sc);
  }
}

template <class L, typename S, typename R, bool NT>
__device__ __forceinline__ void store_site_buf(const R *d, S *__restrict__ dst,
                                               const float *iscale, int nx, int ny, int x,
                                               int y, int z) {
  using ST = Store<S, R>;
  constexpr uint32_t B = sizeof(S);
  const int64_t plane = (int64_t)ny * L::Q * nx;
  const __amdgpu_buffer_rsrc_t r = make_rsrc(dst + (int64_t)z * plane, (uint32_t)(plane * B));
  const uint32_t rowb = (uint32_t)nx * B;
  const uint32_t blk = (uint32_t)y * (uint32_t)L::Q;
#pragma unroll
  for (int i = 0; i < L::Q; ++i)
    buf_store<S, NT>(ST::to_bits(d[i], iscale[weight_class<L>(i)]), r, (uint32_t)x * B,
                     (blk + (uint32_t)pop_slot<L>(i)) * rowb);
}

struct TileXY {
  int x, y, z;
};

__device__ __forceinline__ TileXY tile_coords(int tile, int nxb, int ny, int bx) {
  const int xb = tile % nxb;
  const int row = tile / nxb;
  return TileXY{xb * bx + (int)threadIdx.x, row % ny, row / ny};
}

// ONE: the grid has one workgroup per tile (every thread processes at most
// one site, and its statistics go to the block reduction as compute-type
// values); otherwise workgroups stride over the tiles and accumulate in FP64.
// BUF: buffer-addressed population accesses (every z plane of the buffer
// below 4 GiB); otherwise 64-bit addresses.
template <class L, typename S, typename R, bool GENERAL, bool NT, bool ONE, bool BUF>
__global__ __launch_bounds__(kMaxBlock) void k_step(
    const S *__restrict__ src, S *__restrict__ dst, const StepParams<R> p,
    const int64_t *__restrict__ step_ptr, int step_off, double *__restrict__ partials) {
  constexpr int Q = L::Q;
  const uint64_t step = (uint64_t)(*step_ptr + step_off);
  const int BX = blockDim.x;
  const int nx = p.nx, ny = p.ny;
  using A = typename std::conditional<ONE, SiteStats<R>, Acc>::type;
  A acc{};

  for (int tile = blockIdx.x; tile < p.ntiles; tile += gridDim.x) {
    const TileXY c = tile_coords(tile, p.nxb, ny, BX);
    if (c.x < nx) {
      R d[Q];
      if constexpr (BUF)
        load_site_buf<L, S, R, NT>(d, src, p.scale, nx, ny, p.nz, c.x, c.y, c.z);
      else
        load_site<L, S, R, NT>(d, src, p.scale, nx, ny, p.nz, c.x, c.y, c.z);
      const int64_t row = (int64_t)c.y + (int64_t)ny * c.z;
      const int site = (int)(c.x + nx * row);
      collide_site<L, R, GENERAL, sizeof(S) == 2>(d, p, (uint32_t)site, step, acc);
      if constexpr (BUF)
        store_site_buf<L, S, R, NT>(d, dst, p.iscale, nx, ny, c.x, c.y, c.z);
      else
        store_site<L, S, R, NT>(d, dst, p.iscale, nx, c.x, row);
    }
    if constexpr (ONE) break;
  }
  extern __shared__ double acc_lds[];
  block_store_acc(acc, partials + (int64_t)blockIdx.x * kPartStride, acc_lds);
}

// In-place (AA) streaming, buffer-addressed like load_site_buf (every z
// plane below 4 GiB).  Even step (ODD = false): the populations of the
// site's own slots in, post-collision population i out to slot
// opposite(i) of the same site.  Odd step: slot opposite(i) of site
// x - c_i in (where the even step left f*_i), slot i of site x + c_i out.
// NT (population rows of whole cache lines): non-temporal accesses where a
// tile covers whole rows, every access of the even step and the c_x = 0
// accesses of the odd step.
template <class L, typename S, typename R, bool NT, bool ODD>
__device__ __forceinline__ void load_site_aa(R *d, const S *buf, const float *scale, int nx,
                                             int ny, int nz, int x, int y, int z) {
  using ST = Store<S, R>;
  constexpr uint32_t B = sizeof(S);
  const int64_t plane = (int64_t)ny * L::Q * nx;
  const uint32_t pbytes = (uint32_t)(plane * B);
  const uint32_t rowb = (uint32_t)nx * B;
  if constexpr (!ODD) {
    const __amdgpu_buffer_rsrc_t r = make_rsrc(buf + (int64_t)z * plane, pbytes);
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
      d[i] = ST::from_bits(buf_load<S, NT>(r, (uint32_t)x * B, ((uint32_t)y * L::Q + pop_slot<L>(i)) * rowb),
                           scale[weight_class<L>(i)]);
  } else {
    __amdgpu_buffer_rsrc_t rs[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const int zs = L::D == 3 ? wrap_sub(z, b - 1, nz) : z;
      rs[b] = make_rsrc(buf + (int64_t)zs * plane, pbytes);
    }
    const uint32_t xs[3] = {(uint32_t)(x == nx - 1 ? 0 : x + 1) * B, (uint32_t)x * B,
                            (uint32_t)(x == 0 ? nx - 1 : x - 1) * B};
    uint32_t ys[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) ys[a] = (uint32_t)wrap_sub(y, a - 1, ny);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
      const uint32_t soff =
          (ys[L::cy[i] + 1] * (uint32_t)L::Q + (uint32_t)pop_slot<L>(opposite<L>(i))) * rowb;
      const float sc = scale[weight_class<L>(i)];
      if (NT && L::cx[i] == 0)
        d[i] = ST::from_bits(buf_load<S, true>(rs[L::cz[i] + 1], xs[1], soff), sc);
      else
        d[i] = ST::from_bits(buf_load<S, false>(rs[L::cz[i] + 1], xs[L::cx[i] + 1], soff), sc);
    }
  }
}

template <class L, typename S, typename R, bool NT, bool ODD>
__device__ __forceinline__ void store_site_aa(const R *d, S *buf, const float *iscale, int nx,
                                              int ny, int nz, int x, int y, int z) {
  using ST = Store<S, R>;
  constexpr uint32_t B = sizeof(S);
  const int64_t plane = (int64_t)ny * L::Q * nx;
  const uint32_t pbytes = (uint32_t)(plane * B);
  const uint32_t rowb = (uint32_t)nx * B;
  if constexpr (!ODD) {
    const __amdgpu_buffer_rsrc_t r = make_rsrc(buf + (int64_t)z * plane, pbytes);
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
      buf_store<S, NT>(ST::to_bits(d[i], iscale[weight_class<L>(i)]), r, (uint32_t)x * B,
                       ((uint32_t)y * L::Q + (uint32_t)pop_slot<L>(opposite<L>(i))) * rowb);
  } else {
    // destination plane z + c_z, row y + c_y, column x + c_x (index c + 1)
    __amdgpu_buffer_rsrc_t rd[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const int zd = L::D == 3 ? wrap_sub(z, 1 - b, nz) : z;
      rd[b] = make_rsrc(buf + (int64_t)zd * plane, pbytes);
    }
    const uint32_t xd[3] = {(uint32_t)(x == 0 ? nx - 1 : x - 1) * B, (uint32_t)x * B,
                            (uint32_t)(x == nx - 1 ? 0 : x + 1) * B};
    uint32_t yd[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) yd[a] = (uint32_t)wrap_sub(y, 1 - a, ny);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
      const uint32_t soff = (yd[L::cy[i] + 1] * (uint32_t)L::Q + (uint32_t)pop_slot<L>(i)) * rowb;
      const R v = d[i];
      if (NT && L::cx[i] == 0)
        buf_store<S, true>(ST::to_bits(v, iscale[weight_class<L>(i)]), rd[L::cz[i] + 1], xd[1], soff);
      else
        buf_store<S, false>(ST::to_bits(v, iscale[weight_class<L>(i)]), rd[L::cz[i] + 1],
                            xd[L::cx[i] + 1], soff);
    }
  }
}

// The fused step with in-place streaming on one buffer (the even or the odd
// half of a pair of steps); tiles, statistics and ONE as in k_step.  Every
// element is read and then written by the same thread only, and each store
// depends on every load of its site through the collision.
template <class L, typename S, typename R, bool GENERAL, bool NT, bool ONE, bool ODD>
__global__ __launch_bounds__(kMaxBlock) void k_step_aa(
    S *buf, const StepParams<R> p, const int64_t *__restrict__ step_ptr, int step_off,
    double *__restrict__ partials) {
  constexpr int Q = L::Q;
  const uint64_t step = (uint64_t)(*step_ptr + step_off);
  const int BX = blockDim.x;
  const int nx = p.nx, ny = p.ny;
  using A = typename std::conditional<ONE, SiteStats<R>, Acc>::type;
  A acc{};

  for (int tile = blockIdx.x; tile < p.ntiles; tile += gridDim.x) {
    const TileXY c = tile_coords(tile, p.nxb, ny, BX);
    if (c.x < nx) {
      R d[Q];
      load_site_aa<L, S, R, NT, ODD>(d, buf, p.scale, nx, ny, p.nz, c.x, c.y, c.z);
      const int64_t row = (int64_t)c.y + (int64_t)ny * c.z;
      const int site = (int)(c.x + nx * row);
      collide_site<L, R, GENERAL, sizeof(S) == 2>(d, p, (uint32_t)site, step, acc);
      store_site_aa<L, S, R, NT, ODD>(d, buf, p.iscale, nx, ny, p.nz, c.x, c.y, c.z);
    }
    if constexpr (ONE) break;
  }
  extern __shared__ double acc_lds[];
  block_store_acc(acc, partials + (int64_t)blockIdx.x * kPartStride, acc_lds);
}

// ---------------------------------------------------------------------------
// launch of the fused step: the two-buffer pull family (IN_PLACE = false) or
// the in-place pair (IN_PLACE = true), instantiated in translation units of
// their own (cmflb_step_pull.hip, cmflb_step_aa.hip) so that they compile in
// parallel
// ---------------------------------------------------------------------------
namespace step_launch {

// MODE: a StreamMode (the in-place modes only with BUF)
template <class L, typename S, typename R, bool G, bool NT, bool BUF, int MODE>
hipError_t shape(const StepParams<R> &p, const void *src, void *dst,
                 const int64_t *step_ptr, int step_off, double *partials, int grid,
                 int block, hipStream_t stream) {
  auto go = [&](auto one, int nblocks, size_t lds) {
    constexpr bool ONE = decltype(one)::value;
    if constexpr (MODE == kStreamPull)
      hipLaunchKernelGGL((k_step<L, S, R, G, NT, ONE, BUF>), dim3(nblocks), dim3(block), lds,
                         stream, static_cast<const S *>(src), static_cast<S *>(dst), p, step_ptr,
                         step_off, partials);
    else
      hipLaunchKernelGGL((k_step_aa<L, S, R, G, NT, ONE, MODE == kStreamAAOdd>), dim3(nblocks),
                         dim3(block), lds, stream, static_cast<S *>(dst), p, step_ptr, step_off,
                         partials);
    return hipGetLastError();
  };
  // one workgroup per tile: per-site statistics (measured faster for D2Q9,
  // 4096^2 FP32 0.218 -> 0.205 ms; 1-2% slower for the 3-D lattices, whose
  // kernels then keep the FP64 accumulation)
  if constexpr (L::Q == 9)
    if (grid >= p.ntiles) return go(std::true_type{}, p.ntiles, acc_lds_bytes<R>(block));
  return go(std::false_type{}, grid, acc_lds_bytes<double>(block));
}

// mode: kStreamPull for the pull family; kStreamAAEven / kStreamAAOdd for
// the in-place one (src == dst)
template <bool IN_PLACE, class L, typename S, typename R, bool G, bool NT>
hipError_t one(int mode, const void *params, const void *src, void *dst,
               const int64_t *step_ptr, int step_off, double *partials, int grid, int block,
               hipStream_t stream) {
  const StepParams<R> &p = *static_cast<const StepParams<R> *>(params);
  // buffer-addressed accesses when every z plane (ny Q nx values) of a
  // population buffer spans less than 4 GiB (always so for in-place
  // streaming, which the library accepts only then)
  const bool buf = (int64_t)p.ny * L::Q * p.nx * (int64_t)sizeof(S) < ((int64_t)1 << 32);
  if constexpr (IN_PLACE) {
    if (!buf || src != dst) return hipErrorInvalidValue;
    return mode == kStreamAAEven
               ? shape<L, S, R, G, NT, true, kStreamAAEven>(p, src, dst, step_ptr, step_off,
                                                            partials, grid, block, stream)
               : shape<L, S, R, G, NT, true, kStreamAAOdd>(p, src, dst, step_ptr, step_off,
                                                           partials, grid, block, stream);
  } else {
    if (buf)
      return shape<L, S, R, G, NT, true, kStreamPull>(p, src, dst, step_ptr, step_off, partials,
                                                      grid, block, stream);
    return shape<L, S, R, G, NT, false, kStreamPull>(p, src, dst, step_ptr, step_off, partials,
                                                     grid, block, stream);
  }
}

template <bool IN_PLACE, class L, typename S, typename R>
hipError_t by_rates(bool general, bool nt, int mode, const void *params, const void *src,
                    void *dst, const int64_t *step_ptr, int off, double *partials, int grid,
                    int block, hipStream_t stream) {
  if (general)
    return nt ? one<IN_PLACE, L, S, R, true, true>(mode, params, src, dst, step_ptr, off, partials,
                                                   grid, block, stream)
              : one<IN_PLACE, L, S, R, true, false>(mode, params, src, dst, step_ptr, off, partials,
                                                    grid, block, stream);
  return nt ? one<IN_PLACE, L, S, R, false, true>(mode, params, src, dst, step_ptr, off, partials,
                                                  grid, block, stream)
            : one<IN_PLACE, L, S, R, false, false>(mode, params, src, dst, step_ptr, off, partials,
                                                   grid, block, stream);
}

template <bool IN_PLACE, class L>
hipError_t by_storage(int storage, bool general, bool nt, int mode, const void *params,
                      const void *src, void *dst, const int64_t *step_ptr, int off,
                      double *partials, int grid, int block, hipStream_t stream) {
  switch (storage) {
    case kF64:
      return by_rates<IN_PLACE, L, double, double>(general, nt, mode, params, src, dst, step_ptr,
                                                   off, partials, grid, block, stream);
    case kF32:
      return by_rates<IN_PLACE, L, float, float>(general, nt, mode, params, src, dst, step_ptr,
                                                 off, partials, grid, block, stream);
    case kF16:
      return by_rates<IN_PLACE, L, __half, float>(general, nt, mode, params, src, dst, step_ptr,
                                                  off, partials, grid, block, stream);
    case kBF16:
      return by_rates<IN_PLACE, L, __hip_bfloat16, float>(general, nt, mode, params, src, dst,
                                                          step_ptr, off, partials, grid, block,
                                                          stream);
  }
  return hipErrorInvalidValue;
}

template <bool IN_PLACE>
hipError_t by_lattice(int q, int storage, bool general, bool nt, int mode, const void *params,
                      const void *src, void *dst, const int64_t *step_ptr, int off,
                      double *partials, int grid, int block, hipStream_t stream) {
  if (q == 9)
    return by_storage<IN_PLACE, D2Q9>(storage, general, nt, mode, params, src, dst, step_ptr, off,
                                      partials, grid, block, stream);
  if (q == 19)
    return by_storage<IN_PLACE, D3Q19>(storage, general, nt, mode, params, src, dst, step_ptr,
                                       off, partials, grid, block, stream);
  if (q == 27)
    return by_storage<IN_PLACE, D3Q27>(storage, general, nt, mode, params, src, dst, step_ptr,
                                       off, partials, grid, block, stream);
  return hipErrorInvalidValue;
}

}  // namespace step_launch

// the two families (cmflb_step_pull.hip, cmflb_step_aa.hip); launch_step
// (cmflb_kernels.hip) picks one by the stream mode
hipError_t launch_step_pull(int q, int storage, bool general, bool nt, const void *params,
                            const void *src, void *dst, const int64_t *step_ptr, int step_off,
                            double *partials, int grid, int block, hipStream_t stream);
hipError_t launch_step_in_place(int q, int storage, bool general, bool nt, bool odd,
                                const void *params, void *buf, const int64_t *step_ptr,
                                int step_off, double *partials, int grid, int block,
                                hipStream_t stream);

}  // namespace cmf
