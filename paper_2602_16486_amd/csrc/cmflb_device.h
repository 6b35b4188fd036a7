// cmflb_device.h -- device building blocks of the fused CM-FLBM step for
// gfx950: lattice traits, Philox4x32-10 + Box-Muller normals, storage
// conversions, and the per-site collision written as tensor-product passes.
//
// Method: De Rosis & Zhou, "A fluctuating lattice Boltzmann formulation based
// on orthogonal central moments" (arXiv 2602.16486).
//
// Factorisation used here (a property of the paper's bases, not a step the
// paper prints): every D3Q27 basis row of Sec. 2.3 is a product
// P_px(c_x) P_py(c_y) P_pz(c_z) of the one-dimensional polynomials
// P_0 = 1, P_1 = c, P_2 = c^2 - c_s^2 (row 15 read as (c_y^2 - c_s^2) c_z);
// the D2Q9 basis of Sec. 2.2 is the same tensor basis in 2-D except that
// rows 3 and 4 are P_2 P_0 + P_0 P_2 and P_2 P_0 - P_0 P_2.  Shifting c by u
// keeps that structure, so T(u) = T1(u_x) (x) T1(u_y) (x) T1(u_z) and both
// k = T(u) f and f* = T(u)^-1 k* are three (two) passes of 3x3 one-axis maps
// instead of a dense 27x27 (9x9) product.
//
// Deviation form: the step stores d_i = f_i - w_i rho0.  With
// g(u) = (1, -u, u^2) the one-axis central moments of the rest weights,
// T(u) (rho0 w) = rho0 g(u_x) (x) g(u_y) (x) g(u_z), so
//   k   = T(u) d + rho0 G(u)        and
//   d*  = T(u)^-1 (k* - rho0 G(u)),
// which keeps every intermediate O(fluctuation) in FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace cmf {

// ---------------------------------------------------------------------------
// Lattices, in the paper's velocity order.
// ---------------------------------------------------------------------------

struct D2Q9 {
  static constexpr int Q = 9;
  static constexpr int D = 2;
  static constexpr int NT = 9;          // tensor positions 3^D
  static constexpr int FIRST_NOISY = 3; // I~ = diag[0,0,0,1,...] (Sec. 2.2)
  static constexpr int NNOISE = 6;
  static constexpr int NBLOCKS = 2;     // Philox blocks per site and step
  // Sec. 2.2: c_x = [0,1,0,-1,0,1,-1,-1,1], c_y = [0,0,1,0,-1,1,1,-1,-1]
  static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
};

struct D3Q27 {
  static constexpr int Q = 27;
  static constexpr int D = 3;
  static constexpr int NT = 27;
  static constexpr int FIRST_NOISY = 4; // I~_0-3 = 0 (Sec. 2.3)
  static constexpr int NNOISE = 23;
  static constexpr int NBLOCKS = 6;
  // Sec. 2.3, component lists of the 27 velocities
  static constexpr int cx[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1,
                                 -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
  static constexpr int cy[27] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0,
                                 0, 1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1};
  static constexpr int cz[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1,
                                 -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1};
  // tensor index px + 3 py + 9 pz of mode v (Sec. 2.3 rows as products of
  // P_0, P_1, P_2 per axis)
  static constexpr int mode_pos[27] = {
      0,            // 1
      1, 3, 9,      // c_x, c_y, c_z
      2, 6, 18,     // P2(x), P2(y), P2(z)
      4, 10, 12,    // xy, xz, yz
      5, 11,        // P2(x) y, P2(x) z
      7, 19,        // x P2(y), x P2(z)
      21, 15,       // y P2(z), P2(y) z
      13,           // xyz
      8, 20, 24,    // P2 P2 0, P2 0 P2, 0 P2 P2
      22, 16, 14,   // x y P2(z), x P2(y) z, P2(x) y z
      23, 17, 25,   // P2 y P2, P2 P2 z, x P2 P2
      26};          // P2 P2 P2
};

// D3Q19 (Sec. 2.4): {-1, 0, 1}^3 without the eight corners, in the D3Q27
// order above with the corners left out.  Its basis is not a tensor
// product; the transforms are in cmflb_d3q19.h.
struct D3Q19 {
  static constexpr int Q = 19;
  static constexpr int D = 3;
  static constexpr int NT = 19;
  static constexpr int FIRST_NOISY = 4; // I~_0-3 = 0, I~_4-18 = 1 (Sec. 2.4)
  static constexpr int NNOISE = 15;
  static constexpr int NBLOCKS = 4;
  static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
};

// sqrt(b_v), the square roots of the modal norms of the paper's bases, as
// compile-time constants: the noise amplitude of a mode relaxed at rate 1 is
// sqrt(kT / c_s^2) sqrt(b_v), so the paper-rate kernels need one runtime
// amplitude instead of one per mode.  D3Q27: products of the one-axis norms
// 1, 1/3, 2/9 over the mode's tensor position; D2Q9 (Sec. 2.2) and D3Q19
// (Sec. 2.4) tabulated.
constexpr double kSqrtAxisNorm[3] = {1.0, 0.57735026918962576, 0.47140452079103168};
template <class L>
__host__ __device__ constexpr double sqrt_norm(int v) {
  if constexpr (L::Q == 27) {
    return kSqrtAxisNorm[L::mode_pos[v] % 3] * kSqrtAxisNorm[(L::mode_pos[v] / 3) % 3] *
           kSqrtAxisNorm[L::mode_pos[v] / 9];
  } else if constexpr (L::Q == 9) {
    // b = 1, 1/3, 1/3, 4/9, 4/9, 1/9, 2/27, 2/27, 4/81
    constexpr double t[9] = {1.0, 0.57735026918962576, 0.57735026918962576,
                             0.66666666666666667, 0.66666666666666667, 0.33333333333333333,
                             0.27216552697590868, 0.27216552697590868, 0.22222222222222222};
    return t[v];
  } else {
    // b = 1, 1/3 (x3), 2/3, 4/3, 4/9, 1/9 (x3), 2/3 (x3), 2/9 (x3), 2, 4/3, 4/9
    constexpr double t[19] = {1.0, 0.57735026918962576, 0.57735026918962576,
                              0.57735026918962576, 0.81649658092772603, 1.1547005383792515,
                              0.66666666666666667, 0.33333333333333333, 0.33333333333333333,
                              0.33333333333333333, 0.81649658092772603, 0.81649658092772603,
                              0.81649658092772603, 0.47140452079103168, 0.47140452079103168,
                              0.47140452079103168, 1.4142135623730951, 1.1547005383792515,
                              0.66666666666666667};
    return t[v];
  }
}

// weight class |c_i|^2 of population i (the weights, and with them the
// storage scales, depend on i through it only)
template <class L>
__host__ __device__ constexpr int weight_class(int i) {
  return L::cx[i] * L::cx[i] + L::cy[i] * L::cy[i] + L::cz[i] * L::cz[i];
}

// the population whose velocity is -c_i (every lattice here lists both
// directions of each velocity)
template <class L>
__host__ __device__ constexpr int opposite(int i) {
  for (int j = 0; j < L::Q; ++j)
    if (L::cx[j] == -L::cx[i] && L::cy[j] == -L::cy[i] && L::cz[j] == -L::cz[i]) return j;
  return -1;
}
static_assert(opposite<D2Q9>(5) == 7 && opposite<D3Q27>(0) == 0 && opposite<D3Q19>(1) == 2,
              "opposite velocities");

// tensor position (c_x + 1) + 3 (c_y + 1) [+ 9 (c_z + 1) in 3-D] of
// population i
template <class L>
__host__ __device__ constexpr int pop_pos(int i) {
  return (L::cx[i] + 1) + 3 * (L::cy[i] + 1) +
         (L::D == 3 ? 9 * (L::cz[i] + 1) : 0);
}
static_assert(pop_pos<D2Q9>(8) == 2 && pop_pos<D2Q9>(7) == 0, "D2Q9 positions");

// population index at each tensor position (inverse of pop_pos)
template <class L>
struct PosTable {
  int pop[L::NT];
  constexpr PosTable() : pop() {
    for (int i = 0; i < L::Q; ++i) pop[pop_pos<L>(i)] = i;
  }
};
static_assert(pop_pos<D3Q27>(26) == 0 && pop_pos<D3Q27>(19) == 26, "D3Q27 positions");

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): per round, the 64-bit
// products of words 0 and 2 with 0xD2511F53 and 0xCD9E8D57 give the new
// words (hi(2) ^ w1 ^ k0, lo(2), hi(0) ^ w3 ^ k1, lo(0)); the key advances by
// (0x9E3779B9, 0xBB67AE85) between rounds.
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1,
                                            uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // each 64-bit product is one v_mad_u64_u32, which costs about as much
    // as one of the two 32-bit high/low multiplies it replaces (measured on
    // gfx950: about 3 full-rate VALU slots each)
    const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
    const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
    // three-input xor in one instruction (truth table 0x96 = a ^ b ^ c)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// Box-Muller pair from two Philox words (a -> radius, b -> angle), times a
// scale s: (z0, z1) = s (r cos theta, r sin theta).  The FP32 and FP64 step
// kernels pass the site's noise amplitude, which then costs one multiply
// per pair of modes instead of one per mode.
template <typename R>
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, R s, R &z0,
                                           R &z1);

// FP32: the hardware transcendentals.  v_log_f32 gives log2, so
// r = sqrt(-2 ln u1) = sqrt(2 ln 2) sqrt(-log2 u1); v_sin_f32 / v_cos_f32
// take their argument in revolutions, so sin(2 pi u2) is v_sin_f32(u2) with
// no range reduction.  Over all 2^24 possible u1 and u2 the radius
// sqrt(-2 ln 2 log2 u1) is within 4.9e-7 and sine and cosine within 1.3e-7
// of the exact values (exhaustive check on gfx950), i.e.
// |eta_fp32 - eta| <= 1.2e-6; the form used here rounds the factor
// sqrt(2 ln 2) s separately (one more rounding of r, 6e-8 relative).
template <>
__device__ __forceinline__ void box_muller<float>(uint32_t a, uint32_t b, float s,
                                                  float &z0, float &z1) {
  // ((a >> 8) + 1) 2^-24 as one multiply-add of exact operands (exact)
  const float u1 = __builtin_fmaf((float)(a >> 8), 0x1p-24f, 0x1p-24f);  // (0, 1]
  const float u2 = (float)(b >> 8) * 0x1p-24f;         // [0, 1), exact
  const float r = __builtin_amdgcn_sqrtf(-__builtin_amdgcn_logf(u1)) * (s * 1.17741002f);
  z0 = r * __builtin_amdgcn_cosf(u2);
  z1 = r * __builtin_amdgcn_sinf(u2);
}

template <>
__device__ __forceinline__ void box_muller<double>(uint32_t a, uint32_t b, double s,
                                                   double &z0, double &z1) {
  const double u1 = (double)((a >> 8) + 1u) * 0x1p-24;
  const double u2 = (double)(b >> 8) * 0x1p-24;
  const double r = sqrt(-2.0 * log(u1)) * s;
  double sn, cs;
  sincospi(2.0 * u2, &sn, &cs);
  z0 = r * cs;
  z1 = r * sn;
}

// The NNOISE normals of one site and step, eta[n] for mode FIRST_NOISY + n.
// Counter (site, step mod 2^32, replica, block + 2^8 floor(step / 2^32)):
// the block index takes 8 bits, so the counters of all steps below 2^56
// are distinct, and steps below 2^32 keep the plain (site, step, replica,
// block) counter.  The step is wave-uniform, so its two words cost scalar
// operations only.
// scale: every normal comes out multiplied by it (1 for the normals
// themselves).
template <class L, typename R>
__device__ __forceinline__ void site_normals(uint32_t site, uint64_t step,
                                             uint32_t replica, uint32_t k0,
                                             uint32_t k1, R scale, R *eta) {
  const uint32_t step_lo = (uint32_t)step;
  const uint32_t blk_hi = (uint32_t)(step >> 32) << 8;
#pragma unroll
  for (int blk = 0; blk < L::NBLOCKS; ++blk) {
    const U4 w = philox4x32_10(site, step_lo, replica, (uint32_t)blk | blk_hi, k0, k1);
    const int n0 = 4 * blk;
    R a, b;
    box_muller<R>(w.x, w.y, scale, a, b);
    if (n0 < L::NNOISE) eta[n0] = a;
    if (n0 + 1 < L::NNOISE) eta[n0 + 1] = b;
    if (n0 + 2 < L::NNOISE) {
      R c, d;
      box_muller<R>(w.z, w.w, scale, c, d);
      eta[n0 + 2] = c;
      if (n0 + 3 < L::NNOISE) eta[n0 + 3] = d;
    }
  }
}

// ---------------------------------------------------------------------------
// One-axis maps between populations (c = -1, 0, +1) and central moments
// (P_0, P_1, P_2 of c - u), in place.
// ---------------------------------------------------------------------------
template <typename R>
struct Axis {
  R u, twou, u2mcs2, cs2pu2;
  __device__ __forceinline__ explicit Axis(R uu) {
    const R cs2 = R(1) / R(3);
    u = uu;
    twou = uu + uu;
    u2mcs2 = uu * uu - cs2;
    cs2pu2 = uu * uu + cs2;
  }
  // (g-, g0, g+) -> (m0, m1, m2)
  __device__ __forceinline__ void fwd(R &a0, R &a1, R &a2) const {
    const R m0 = a0 + a1 + a2;
    const R d = a2 - a0;
    const R s = a2 + a0;
    a0 = m0;
    a1 = d - u * m0;
    a2 = s - twou * d + u2mcs2 * m0;
  }
  // (m0, m1, m2) -> (g-, g0, g+); DOUBLED: (2 g-, g0, 2 g+), leaving the
  // halving of the moving populations to the caller
  template <bool DOUBLED = false>
  __device__ __forceinline__ void inv(R &a0, R &a1, R &a2) const {
    const R r1 = a1 + u * a0;
    const R r2 = a2 + cs2pu2 * a0 + twou * a1;
    const R g0 = a0 - r2;
    if constexpr (DOUBLED) {
      a0 = r2 - r1;
      a2 = r2 + r1;
    } else {
      a0 = R(0.5) * (r2 - r1);
      a2 = R(0.5) * (r2 + r1);
    }
    a1 = g0;
  }
};

// passes over a 3^D tensor t[px + 3 py + 9 pz]
template <int D, typename R>
__device__ __forceinline__ void tensor_fwd(R *t, const Axis<R> &ax,
                                           const Axis<R> &ay,
                                           const Axis<R> &az) {
  constexpr int NZ = D == 3 ? 3 : 1;
#pragma unroll
  for (int k = 0; k < 3 * NZ; ++k) ax.fwd(t[3 * k], t[3 * k + 1], t[3 * k + 2]);
#pragma unroll
  for (int z = 0; z < NZ; ++z)
#pragma unroll
    for (int x = 0; x < 3; ++x)
      ay.fwd(t[x + 9 * z], t[x + 3 + 9 * z], t[x + 6 + 9 * z]);
  if constexpr (D == 3) {
#pragma unroll
    for (int k = 0; k < 9; ++k) az.fwd(t[k], t[k + 9], t[k + 18]);
  }
}

// DOUBLED: every one-axis map leaves out its halving, so population i comes
// out multiplied by 2^(|c_ix| + |c_iy| + |c_iz|) = 2^|c_i|^2, an exact power
// of two that the 16-bit stores fold into their per-weight-class scale.
template <int D, typename R, bool DOUBLED = false>
__device__ __forceinline__ void tensor_inv(R *t, const Axis<R> &ax,
                                           const Axis<R> &ay,
                                           const Axis<R> &az) {
  constexpr int NZ = D == 3 ? 3 : 1;
  if constexpr (D == 3) {
#pragma unroll
    for (int k = 0; k < 9; ++k) az.template inv<DOUBLED>(t[k], t[k + 9], t[k + 18]);
  }
#pragma unroll
  for (int z = 0; z < NZ; ++z)
#pragma unroll
    for (int x = 0; x < 3; ++x)
      ay.template inv<DOUBLED>(t[x + 9 * z], t[x + 3 + 9 * z], t[x + 6 + 9 * z]);
#pragma unroll
  for (int k = 0; k < 3 * NZ; ++k) ax.template inv<DOUBLED>(t[3 * k], t[3 * k + 1], t[3 * k + 2]);
}

// t[p] += s * G(u)[p], G = g(u_x) (x) g(u_y) (x) g(u_z), g(u) = (1, -u, u^2)
template <int D, typename R>
__device__ __forceinline__ void add_rest_moments(R *t, R s, R ux, R uy, R uz) {
  const R gx[3] = {s, -s * ux, s * ux * ux};
  const R gy[3] = {R(1), -uy, uy * uy};
  if constexpr (D == 3) {
    const R gz[3] = {R(1), -uz, uz * uz};
#pragma unroll
    for (int z = 0; z < 3; ++z)
#pragma unroll
      for (int y = 0; y < 3; ++y) {
        const R gyz = gy[y] * gz[z];
#pragma unroll
        for (int x = 0; x < 3; ++x) t[x + 3 * y + 9 * z] += gx[x] * gyz;
      }
  } else {
    (void)uz;
#pragma unroll
    for (int y = 0; y < 3; ++y)
#pragma unroll
      for (int x = 0; x < 3; ++x) t[x + 3 * y] += gx[x] * gy[y];
  }
}

// ---------------------------------------------------------------------------
// Storage conversions.  F16/BF16 hold d_i / s_i (s_i a power of two).
// ---------------------------------------------------------------------------
// Cache policy of the population traffic: stores are non-temporal (written
// once, read by the next step long after); loads of the x-shifted rows go
// through the caches so that the cache lines shared by the +-1 x-shifted
// reads of neighbouring waves are fetched from HBM once (non-temporal loads
// of every row measured 1.26x the algorithmic read bytes, cached loads
// 1.10x); the rows with c_x = 0 are read line-aligned, each line by one wave
// only, and go non-temporal when rows are whole cache lines (they then do
// not displace the shared lines: D3Q19 256^3 FP32 0.441 -> 0.430 ms).
// NT: non-temporal load, for lines that no other wave reads (see load_site)
template <bool NT = false, typename T>
__device__ __forceinline__ T cmf_ld(const T *p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
// NT: non-temporal (streaming) store, used when every population row of
// the buffer is a whole number of cache lines, so a wave writes whole lines;
// otherwise a plain store, so that the two parts of a line shared by two
// rows merge in L2 before they go to HBM.
template <bool NT, typename T>
__device__ __forceinline__ void cmf_st(T v, T *p) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Population layout in HBM (row-interleaved structure of arrays): the Q
// rows of nx elements that the Q populations of one lattice row (y, z) hold
// are stored back to back, row = y + ny z; on the 3-D lattices in the order
// of their velocities (c_z, c_y, c_x) (pop_slot), on D2Q9 in the paper's
// population order.  A step then reads 9 blocks of Q rows, on the 3-D
// lattices from each the 3 adjacent rows of the populations with that
// (c_y, c_z), and writes one block of Q rows per lattice row, instead of
// 27 + 27 rows spread over Q planes.  On gfx950 the row blocks measured 10 %
// faster than one plane per population, and the velocity order within a
// block 1.7-3 % faster than the paper's order on D3Q27 and D3Q19 (FP32;
// 16-bit storage unchanged), while D2Q9 was 1 % slower with it.
//
// Slot of population i within its row block: on the 3-D lattices its rank
// in the order of (c_z, c_y, c_x), i.e. of the tensor position pop_pos; on
// D2Q9, i.
template <class L>
__host__ __device__ constexpr int pop_slot(int i) {
  if (L::D == 2) return i;
  int s = 0;
  for (int j = 0; j < L::Q; ++j) s += pop_pos<L>(j) < pop_pos<L>(i) ? 1 : 0;
  return s;
}

// Offset of the first element (x = 0) of population i in lattice row `row`.
template <class L>
__host__ __device__ __forceinline__ int64_t pop_row_offset(int i, int64_t row,
                                                           int nx) {
  return (row * L::Q + pop_slot<L>(i)) * (int64_t)nx;
}

template <typename S, typename R>
struct Store;

// Each Store<S, R> also converts between the compute type and the stored
// bits (from_bits / to_bits, the same arithmetic as load / store), for the
// buffer-addressed accesses of the single-lattice step (buf_load, buf_store).
template <typename R>
struct Store<double, R> {
  static constexpr bool scaled = false;
  using bits_t = unsigned long long;
  __device__ __forceinline__ static R from_bits(bits_t b, float) {
    return (R)__longlong_as_double((long long)b);
  }
  __device__ __forceinline__ static bits_t to_bits(R v, float) {
    return (bits_t)__double_as_longlong((double)v);
  }
  template <bool NT = false>
  __device__ __forceinline__ static R load(const double *p, float) {
    return (R)cmf_ld<NT>(p);
  }
  template <bool NT = true>
  __device__ __forceinline__ static void store(double *p, R v, float) {
    cmf_st<NT>((double)v, p);
  }
};

template <typename R>
struct Store<float, R> {
  static constexpr bool scaled = false;
  using bits_t = unsigned int;
  __device__ __forceinline__ static R from_bits(bits_t b, float) { return (R)__uint_as_float(b); }
  __device__ __forceinline__ static bits_t to_bits(R v, float) { return __float_as_uint((float)v); }
  template <bool NT = false>
  __device__ __forceinline__ static R load(const float *p, float) {
    return (R)cmf_ld<NT>(p);
  }
  template <bool NT = true>
  __device__ __forceinline__ static void store(float *p, R v, float) {
    cmf_st<NT>((float)v, p);
  }
};

template <typename R>
struct Store<__half, R> {
  static constexpr bool scaled = true;
  using bits_t = unsigned short;
  __device__ __forceinline__ static R from_bits(bits_t b, float scale) {
    return (R)__builtin_fmaf(__half2float(__ushort_as_half(b)), scale, 0.0f);
  }
  __device__ __forceinline__ static bits_t to_bits(R v, float iscale) {
    return __half_as_ushort(__float2half_rn((float)v * iscale));
  }
  template <bool NT = false>
  __device__ __forceinline__ static R load(const __half *p, float scale) {
    const unsigned short bits =
        cmf_ld<NT>(reinterpret_cast<const unsigned short *>(p));
    // h s + 0 as one fused multiply-add of a half and a float operand (one
    // v_fma_mix_f32 instead of a conversion and a multiply); the zero addend
    // turns a -0 product into +0, which is the same deviation
    return (R)__builtin_fmaf(__half2float(__ushort_as_half(bits)), scale, 0.0f);
  }
  template <bool NT = true>
  __device__ __forceinline__ static void store(__half *p, R v, float iscale) {
    const __half h = __float2half_rn((float)v * iscale);
    cmf_st<NT>(__half_as_ushort(h), reinterpret_cast<unsigned short *>(p));
  }
};

template <typename R>
struct Store<__hip_bfloat16, R> {
  static constexpr bool scaled = true;
  using bits_t = unsigned short;
  __device__ __forceinline__ static R from_bits(bits_t b, float scale) {
    return (R)(__uint_as_float(((unsigned int)b) << 16) * scale);
  }
  __device__ __forceinline__ static bits_t to_bits(R v, float iscale) {
    const __hip_bfloat16 h = __float2bfloat16((float)v * iscale);
    unsigned short bits;
    __builtin_memcpy(&bits, &h, sizeof(bits));
    return bits;
  }
  template <bool NT = false>
  __device__ __forceinline__ static R load(const __hip_bfloat16 *p,
                                           float scale) {
    const unsigned short bits =
        cmf_ld<NT>(reinterpret_cast<const unsigned short *>(p));
    return (R)(__uint_as_float(((unsigned int)bits) << 16) * scale);
  }
  template <bool NT = true>
  __device__ __forceinline__ static void store(__hip_bfloat16 *p, R v,
                                               float iscale) {
    const __hip_bfloat16 h = __float2bfloat16((float)v * iscale);
    unsigned short bits;
    __builtin_memcpy(&bits, &h, sizeof(bits));
    cmf_st<NT>(bits, reinterpret_cast<unsigned short *>(p));
  }
};

// ---------------------------------------------------------------------------
// Buffer-resource accesses (gfx9 MUBUF): address = resource base + scalar
// offset (soffset) + vector offset (voffset), all in bytes, the resource
// covering `bytes` bytes (at most 4 GiB).  The per-lane part of a
// population row access is then one 32-bit offset shared by every row with
// the same x shift, and the row offsets are scalar, so a site's 2 Q accesses
// take no vector address arithmetic.  NT selects the non-temporal policy.
// ---------------------------------------------------------------------------
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9)

template <typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const S *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<S *>(base), (short)0, (int)bytes,
                                           kRsrcWord3);
}

template <typename S, bool NT>
__device__ __forceinline__ typename Store<S, float>::bits_t buf_load(__amdgpu_buffer_rsrc_t r,
                                                                     uint32_t voff, uint32_t soff) {
  constexpr int aux = NT ? 2 : 0;
  if constexpr (sizeof(S) == 2) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, aux);
  } else if constexpr (sizeof(S) == 4) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, aux);
  } else {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, aux);
    return (unsigned long long)v[0] | ((unsigned long long)v[1] << 32);
  }
}

// Non-temporal stores carry the system-scope bits as well (cache policy
// sc0 nt sc1: streamed past the caches to memory); measured 0.5-1 % faster
// than nt alone on every step kernel, and results do not depend on it.
template <typename S, bool NT>
__device__ __forceinline__ void buf_store(typename Store<S, float>::bits_t b,
                                          __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  constexpr int aux = NT ? (1 | 2 | 16) : 0;
  if constexpr (sizeof(S) == 2) {
    __builtin_amdgcn_raw_buffer_store_b16(b, r, (int)voff, (int)soff, aux);
  } else if constexpr (sizeof(S) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(b, r, (int)voff, (int)soff, aux);
  } else {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    u2 v;
    v[0] = (unsigned int)b;
    v[1] = (unsigned int)(b >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)voff, (int)soff, aux);
  }
}

}  // namespace cmf
