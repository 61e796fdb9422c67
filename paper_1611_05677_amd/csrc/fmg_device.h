// Device-side building blocks of the FMG solver for gfx950 (wave64).
//
// Level layout: one nodal array per level, (n+1)^d nodes including the
// Dirichlet ring (held at zero), x fastest, rows padded to a pitch of 16
// elements so that every row starts on a 128-byte boundary in float64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fmg.h"

namespace fmg {

constexpr int kMaxY = 64;           // max unknowns of the augmented problem (N_1 + 1)
constexpr int kBlock = 256;         // threads per block of the grid kernels

struct Grid {
  int n;        // cells per side; interior node indices 1..n-1
  int px;       // x pitch in elements
  int pz;       // plane pitch in elements (3D), 0 in 2D
};

__host__ __device__ inline int pitch_for(int n) { return ((n + 1) + 15) & ~15; }

template <int DIM>
__device__ __forceinline__ int gidx(const Grid& g, int i, int j, int l) {
  return DIM == 2 ? j * g.px + i : l * g.pz + j * g.px + i;
}

// ---------------------------------------------------------------------------
// Nonlinearity catalogue: value f, derivative f', antiderivative F (F(0)=0).
// Every entry is nondecreasing in u (Assumption A, Section 2).
// ---------------------------------------------------------------------------
template <int KIND> struct NL;

template <> struct NL<FMG_F_ZERO> {
  __device__ static double f(double, double) { return 0.0; }
  __device__ static void all(double, double, double& f, double& df, double& F) { f = df = F = 0.0; }
};
template <> struct NL<FMG_F_LINEAR> {
  __device__ static double f(double u, double c) { return c * u; }
  __device__ static void all(double u, double c, double& f, double& df, double& F) {
    f = c * u; df = c; F = 0.5 * c * u * u;
  }
};
template <> struct NL<FMG_F_CUBIC> {
  __device__ static double f(double u, double) { return u * u * u; }
  __device__ static void all(double u, double, double& f, double& df, double& F) {
    double u2 = u * u; f = u2 * u; df = 3.0 * u2; F = 0.25 * u2 * u2;
  }
};
template <> struct NL<FMG_F_U_PLUS_SIN> {
  __device__ static double f(double u, double) { return u + sin(u); }
  __device__ static void all(double u, double, double& f, double& df, double& F) {
    double s, c; sincos(u, &s, &c);
    f = u + s; df = 1.0 + c; F = 0.5 * u * u + (1.0 - c);
  }
};
template <> struct NL<FMG_F_ABS_U_U> {
  __device__ static double f(double u, double) { return fabs(u) * u; }
  __device__ static void all(double u, double, double& f, double& df, double& F) {
    double a = fabs(u); f = a * u; df = 2.0 * a; F = a * a * a * (1.0 / 3.0);
  }
};
// sign(u)|u|^q; the exponent q = 3/2 of the paper's Example 3 takes |u|^{1/2}
// from sqrt (correctly rounded) instead of pow's logarithm and exponential.
template <> struct NL<FMG_F_SIGNED_POW> {
  __device__ static double f(double u, double q) {
    const double a = fabs(u);
    return copysign(q == 1.5 ? a * sqrt(a) : pow(a, q), u);
  }
  __device__ static void all(double u, double q, double& f, double& df, double& F) {
    double a = fabs(u);
    double p = q == 1.5 ? sqrt(a) : pow(a, q - 1.0);   // |u|^{q-1}
    double aq = p * a;                                  // |u|^q
    f = copysign(aq, u); df = q * p; F = aq * a / (q + 1.0);
  }
};
template <> struct NL<FMG_F_NEG_EXP> {
  __device__ static double f(double u, double) { return -exp(-u); }
  __device__ static void all(double u, double, double& f, double& df, double& F) {
    double e = exp(-u); f = -e; df = e; F = e - 1.0;
  }
};

// ---------------------------------------------------------------------------
// Coarse-cell geometry.  A fine node of level k lies in coarse cell
// c = min(i >> log2r, nH - 1) per axis (r = 2^(k-1) fine cells per coarse
// cell) at local coordinate t = (i - c r)/r in [0,1].  The coarse P1 hat
// function of cell vertex a (bit i of a = offset along axis i) on the Kuhn
// split of the cell is
//     phi_a(t) = max(0, min_{i in a} t_i - max_{i not in a} t_i)
// (min over an empty set = 1, max over an empty set = 0): inside the simplex
// ordered by decreasing t these are its barycentric coordinates, elsewhere 0.
// ---------------------------------------------------------------------------
template <int DIM>
__device__ __forceinline__ void kuhn_phi(const double* t, double* phi) {
  constexpr int NV = 1 << DIM;
#pragma unroll
  for (int a = 0; a < NV; ++a) {
    double mn = 1.0, mx = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      if (a & (1 << i)) mn = fmin(mn, t[i]);
      else mx = fmax(mx, t[i]);
    }
    phi[a] = fmax(0.0, mn - mx);
  }
}

// Pairs (a, b) of cell vertices with a a subset of b: exactly the pairs that
// can share a Kuhn simplex (phi_a phi_b is identically zero otherwise).
template <int DIM> struct Pairs;
template <> struct Pairs<2> {
  static constexpr int N = 9;
  __device__ static int a(int p) { constexpr int A[9] = {0, 0, 0, 0, 1, 1, 2, 2, 3}; return A[p]; }
  __device__ static int b(int p) { constexpr int B[9] = {0, 1, 2, 3, 1, 3, 2, 3, 3}; return B[p]; }
};
template <> struct Pairs<3> {
  static constexpr int N = 27;
  __device__ static int a(int p) {
    constexpr int A[27] = {0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2, 2, 3, 3, 4, 4, 4, 4, 5, 5, 6, 6, 7};
    return A[p];
  }
  __device__ static int b(int p) {
    constexpr int B[27] = {0, 1, 2, 3, 4, 5, 6, 7, 1, 3, 5, 7, 2, 3, 6, 7, 3, 7, 4, 5, 6, 7, 5, 7, 6, 7, 7};
    return B[p];
  }
};

// Accumulator layouts of the augmented-space passes (per coarse cell).
template <int DIM> struct Acc {
  static constexpr int NV = 1 << DIM;
  static constexpr int NP = Pairs<DIM>::N;
  // quadrature pass at (w, alpha): sum over fine nodes of
  //   f(z) phi_a | f(z) u~ | f'(z) phi_a phi_b | f'(z) phi_a u~ | f'(z) u~^2 | F(z)
  static constexpr int Q_NH = 0, Q_NU = NV, Q_K = NV + 1, Q_KHU = NV + 1 + NP,
                       Q_KUU = 2 * NV + 1 + NP, Q_E = 2 * NV + 2 + NP, NQ = 2 * NV + 3 + NP;
  // setup pass: (A u~) phi_a | (A u~) u~ | g phi_a | g u~
  static constexpr int S_BH = 0, S_C = NV, S_GH = NV + 1, S_GU = 2 * NV + 1, NS = 2 * NV + 2;
};

// ---------------------------------------------------------------------------
// Cross-lane operations on doubles.  Reductions use DPP data movement (VALU
// operands permuted within quads, rotated within 16-lane rows, and broadcast
// from row to row) instead of LDS-routed shuffles; broadcasts from a fixed
// lane use v_readlane.  All 64 lanes must be active.  The order of additions
// is fixed, so results are bitwise reproducible run to run.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_value(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes, returned to every lane.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xb1>(v);         // quad_perm [1,0,3,2]
  v += dpp_move<0x4e>(v);         // quad_perm [2,3,0,1]: quad sums
  v += dpp_move<0x124>(v);        // row_ror 4
  v += dpp_move<0x128>(v);        // row_ror 8: 16-lane row sums in every lane
  v += dpp_move<0x142, 0xa>(v);   // row_bcast 15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);   // row_bcast 31 into rows 2 and 3: lane 63 holds the total
  return lane_value(v, 63);
}

// N independent sums over the 64 lanes, each returned to every lane; every
// stage of the DPP tree is applied to all N values before the next, so the
// N reductions overlap (same additions, in the same order, as wave_sum).
template <int N>
__device__ __forceinline__ void wave_sum_n(double (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<0xb1>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<0x4e>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<0x124>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<0x128>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<0x142, 0xa>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<0x143, 0xc>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = lane_value(v[i], 63);
}

// Sum over aligned segments of LPC lanes (LPC = 4, 8, 16, 32 or 64); the
// last lane of each segment receives its segment's total (LPC <= 16: every
// lane of the segment does).
template <int LPC>
__device__ __forceinline__ double seg_sum(double v) {
  static_assert(LPC == 4 || LPC == 8 || LPC == 16 || LPC == 32 || LPC == 64, "segment size");
  v += dpp_move<0xb1>(v);                        // quad_perm [1,0,3,2]
  v += dpp_move<0x4e>(v);                        // quad_perm [2,3,0,1]: quad sums
  if (LPC >= 8) v += dpp_move<0x141>(v);         // row_half_mirror: the other quad of the half-row
  if (LPC >= 16) v += dpp_move<0x140>(v);        // row_mirror: the other half of the row
  if (LPC >= 32) v += dpp_move<0x142, 0xa>(v);   // row_bcast 15 into rows 1 and 3
  if (LPC >= 64) v += dpp_move<0x143, 0xc>(v);   // row_bcast 31 into rows 2 and 3
  return v;
}

// 1 / sqrt(d) for d > 0: the hardware estimate refined by two Newton steps
// (quadratic convergence from ~2^-29 relative error to full double accuracy),
// a short dependent chain in place of the correctly rounded sqrt and divide.
__device__ __forceinline__ double fast_rsqrt(double d) {
  double y = __builtin_amdgcn_rsq(d);
  const double hd = 0.5 * d;
  y = y * (1.5 - hd * y * y);
  y = y * (1.5 - hd * y * y);
  return y;
}

// 1 / d for d != 0: the hardware estimate refined by two Newton steps
// (e <- 1 - d y, y <- y + y e), full double accuracy in a short dependent chain.
__device__ __forceinline__ double fast_rcp(double d) {
  double y = __builtin_amdgcn_rcp(d);
  double e = fma(-d, y, 1.0);
  y = fma(y, e, y);
  e = fma(-d, y, 1.0);
  y = fma(y, e, y);
  return y;
}

// Maximum over the 64 lanes (inputs >= 0), returned to every lane.
__device__ __forceinline__ double wave_max_nonneg(double v) {
  v = fmax(v, dpp_move<0xb1>(v));
  v = fmax(v, dpp_move<0x4e>(v));
  v = fmax(v, dpp_move<0x124>(v));
  v = fmax(v, dpp_move<0x128>(v));
  v = fmax(v, dpp_move<0x142, 0xa>(v));
  v = fmax(v, dpp_move<0x143, 0xc>(v));
  return lane_value(v, 63);
}

// N independent maxima over the 64 lanes (inputs >= 0), as wave_sum_n.
template <int N>
__device__ __forceinline__ void wave_max_n(double (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = fmax(v[i], dpp_move<0xb1>(v[i]));
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = fmax(v[i], dpp_move<0x4e>(v[i]));
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = fmax(v[i], dpp_move<0x124>(v[i]));
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = fmax(v[i], dpp_move<0x128>(v[i]));
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = fmax(v[i], dpp_move<0x142, 0xa>(v[i]));
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = fmax(v[i], dpp_move<0x143, 0xc>(v[i]));
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = lane_value(v[i], 63);
}

// Sum NACC per-thread accumulators over the block; thread t < NACC receives
// the block total of accumulator t.  lds must hold (blockDim/64) * NACC doubles.
template <int NACC>
__device__ __forceinline__ double block_sum_many(const double* acc, double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NACC; ++q) {
    double v = wave_sum(acc[q]);
    if (lane == 0) lds[wave * NACC + q] = v;
  }
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x < NACC)
    for (int w = 0; w < nw; ++w) s += lds[w * NACC + threadIdx.x];
  __syncthreads();
  return s;
}

}  // namespace fmg
