// Element quadrature of the L2 pairings (f(u), v) and (g, v): the element
// reading of the integrals in the discrete problem (Section 2, eq.
// "FEM_form") and in the augmented problem of Algorithm 3.1 (eq. "coarse
// problem"), in place of the vertex rule.  On every fine simplex the integrand
// is evaluated at the d+1 points of a symmetric rule exact for polynomials of
// degree 2 (barycentric coordinates (A, B, .., B) and permutations), with u_h,
// the test functions and the load taken as P1 interpolants.
//
// Fine cells are the unit squares / cubes of the level grid; fine cell t of a
// coarse cell has lower corner node t (local coordinates 0..r-1), so the node
// ranges of the vertex-rule passes become cell ranges.  Its d! Kuhn simplices
// are the vertex chains 0, e_a0, e_a0 + e_a1, ..., 1..1 over the axis orders
// (a0, a1, ..); every point has the weight |T| omega = h^d / (d! (d+1)), i.e.
// ElemRule::W times the lumped mass h^d by which the sums are scaled later.
#pragma once

#include "fmg_device.h"

namespace fmg {

template <int DIM> struct ElemRule;
template <> struct ElemRule<2> {
  static constexpr double A = 2.0 / 3.0, B = 1.0 / 6.0;
  static constexpr double W = 1.0 / 6.0;       // 1 / (2! 3)
  static constexpr int NS = 2;                 // simplices per fine cell
};
template <> struct ElemRule<3> {
  static constexpr double kSqrt5 = 2.23606797749978969641;
  static constexpr double A = (5.0 + 3.0 * kSqrt5) / 20.0, B = (5.0 - kSqrt5) / 20.0;
  static constexpr double W = 1.0 / 24.0;      // 1 / (3! 4)
  static constexpr int NS = 6;
};

// Axis order of Kuhn simplex s of a fine cell (compile time): the chain adds
// axis a0, then a1, then a2.
template <int DIM, int S>
struct KuhnChain {
  static constexpr int a0 = DIM == 2 ? S : S / 2;
  static constexpr int r0 = a0 == 0 ? 1 : 0;   // the two remaining axes, ascending
  static constexpr int r1 = a0 == 2 ? 1 : 2;
  static constexpr int a1 = DIM == 2 ? 1 - S : ((S & 1) ? r1 : r0);
  static constexpr int a2 = DIM == 2 ? 2 : ((S & 1) ? r0 : r1);
  static constexpr int v1 = 1 << a0;
  static constexpr int v2 = v1 | (1 << a1);
  static constexpr int vl = (1 << DIM) - 1;    // last vertex 1..1
};

// Coordinates (in fine-cell units) of point p of chain KC inside the cell:
// along the k-th axis of the chain, the sum of the barycentric coordinates of
// the chain vertices from k on.
template <int DIM, typename KC>
__device__ __forceinline__ void elem_point(int p, double (&s)[3]) {
  using R = ElemRule<DIM>;
  constexpr double D = R::A - R::B;
  const double s1 = DIM * R::B + (p >= 1 ? D : 0.0);
  const double s2 = (DIM - 1) * R::B + (p >= 2 ? D : 0.0);
  const double s3 = DIM == 3 ? R::B + (p >= 3 ? D : 0.0) : 0.0;
  s[KC::a0] = s1;
  s[KC::a1] = s2;
  if (DIM == 3) s[KC::a2] = s3;
}

// Value at point p of the P1 interpolant with chain-vertex values v[0..d].
// The vertex value v[p] is picked by 0/1 weights, not by a select chain: the
// compiler turns such a chain into an indexed load from a private array.
template <int DIM>
__device__ __forceinline__ double elem_interp(const double (&v)[DIM + 1], double vsum, int p) {
  using R = ElemRule<DIM>;
  double vp = 0.0;
#pragma unroll
  for (int k = 0; k <= DIM; ++k) vp = fma(p == k ? 1.0 : 0.0, v[k], vp);
  return R::B * vsum + (R::A - R::B) * vp;
}

// Visit the fine cells of one block's share of a coarse cell:
// fn(i, j, l of the lower corner, local corner coordinates, corner values
// uc[e] of u at corner e (bit a = +1 along axis a)).
template <int DIM, typename Fn>
__device__ __forceinline__ void for_cell_cells(const Grid& g, const AugShape& s, int cx, int cy, int cz, int t0,
                                               int t1, int tid, int nthreads, const double* __restrict__ u,
                                               Fn&& fn) {
  const int r = 1 << s.log2r, mask = r - 1;
  for (int t = t0 + tid; t < t1; t += nthreads) {
    const int lx = t & mask, ly = (t >> s.log2r) & mask, lz = DIM == 3 ? t >> (2 * s.log2r) : 0;
    const int i = cx * r + lx, j = cy * r + ly, l = cz * r + lz;
    double uc[1 << DIM];
#pragma unroll
    for (int e = 0; e < (1 << DIM); ++e)
      uc[e] = u[gidx<DIM>(g, i + (e & 1), j + ((e >> 1) & 1), DIM == 3 ? l + ((e >> 2) & 1) : 0)];
    fn(i, j, l, lx, ly, lz, uc);
  }
}

// Quadrature sums of one fine cell (unweighted; the caller scales by W):
// every point of every Kuhn simplex, z = Q w + alpha u~ there.  SETUP adds the
// load terms W g phi_a, W g u~ to acc_s (the g values at the corners in gc).
template <int DIM, int KIND, bool SETUP, int S>
__device__ __forceinline__ void elem_simplex(const double* tl0, double inv_r, const double* uc, const double* gc,
                                             const double* wv, double alpha, double param, double* acc_q,
                                             double* acc_s) {
  using AC = Acc<DIM>;
  using R = ElemRule<DIM>;
  using KC = KuhnChain<DIM, S>;
  double uv[DIM + 1], gv[DIM + 1];
  uv[0] = uc[0]; uv[1] = uc[KC::v1]; uv[DIM] = uc[KC::vl];
  if (DIM == 3) uv[2] = uc[KC::v2];
  double usum = 0.0, gsum = 0.0;
#pragma unroll
  for (int k = 0; k <= DIM; ++k) usum += uv[k];
  if (SETUP) {
    gv[0] = gc[0]; gv[1] = gc[KC::v1]; gv[DIM] = gc[KC::vl];
    if (DIM == 3) gv[2] = gc[KC::v2];
#pragma unroll
    for (int k = 0; k <= DIM; ++k) gsum += gv[k];
  }
#pragma unroll 1
  for (int p = 0; p <= DIM; ++p) {
    double sp[3] = {0.0, 0.0, 0.0};
    elem_point<DIM, KC>(p, sp);
    double tl[3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) tl[a] = tl0[a] + sp[a] * inv_r;
    double phi[AC::NV];
    kuhn_phi<DIM>(tl, phi);
    const double uq = elem_interp<DIM>(uv, usum, p);
    double z = alpha * uq;
#pragma unroll
    for (int a = 0; a < AC::NV; ++a) z += wv[a] * phi[a];
    quad_node<DIM, KIND>(phi, z, uq, param, acc_q);
    if (SETUP) {
      const double gq = R::W * elem_interp<DIM>(gv, gsum, p);
#pragma unroll
      for (int a = 0; a < AC::NV; ++a) acc_s[AC::S_GH + a] += gq * phi[a];
      acc_s[AC::S_GU] += gq * uq;
    }
  }
}

template <int DIM, int KIND, bool SETUP>
__device__ __forceinline__ void elem_cell(const AugShape& s, int lx, int ly, int lz, const double* uc,
                                          const double* gc, const double* wv, double alpha, double param,
                                          double* acc_q, double* acc_s) {
  const double inv_r = 1.0 / (1 << s.log2r);
  const double tl0[3] = {lx * inv_r, ly * inv_r, lz * inv_r};
  elem_simplex<DIM, KIND, SETUP, 0>(tl0, inv_r, uc, gc, wv, alpha, param, acc_q, acc_s);
  elem_simplex<DIM, KIND, SETUP, 1>(tl0, inv_r, uc, gc, wv, alpha, param, acc_q, acc_s);
  if constexpr (DIM == 3) {
    elem_simplex<DIM, KIND, SETUP, 2>(tl0, inv_r, uc, gc, wv, alpha, param, acc_q, acc_s);
    elem_simplex<DIM, KIND, SETUP, 3>(tl0, inv_r, uc, gc, wv, alpha, param, acc_q, acc_s);
    elem_simplex<DIM, KIND, SETUP, 4>(tl0, inv_r, uc, gc, wv, alpha, param, acc_q, acc_s);
    elem_simplex<DIM, KIND, SETUP, 5>(tl0, inv_r, uc, gc, wv, alpha, param, acc_q, acc_s);
  }
}

}  // namespace fmg
