// Kernels of the nonlinear parts of the method (float64 throughout):
//   * linearised right-hand side b = M (g - f(u))        (Alg. 3.1, eq. "linearized")
//   * Newton solve on level 1                            (Alg. 3.2, step 1)
//   * augmented-space problem on V_H + span{u~}          (Alg. 3.1, step 2,
//     eq. "coarse problem"): one setup pass, then per Newton iteration one
//     fine quadrature pass and one single-workgroup step, then the update
//     u = Q_k w + alpha u~.
//
// Quadrature: the vertex rule on the current finest level k (m_j = h_k^d), so
// every coefficient of the small problem is a sum over the fine nodes:
//   R_H = A_1 w + alpha Q^T A u~ + Q^T M f(z) - Q^T M g
//   R_u = (Q^T A u~).w + alpha u~^T A u~ + u~^T M f(z) - u~^T M g
//   J   = [[A_1 + Q^T M f'(z) Q, Q^T A u~ + Q^T M f'(z) u~], [sym, u~^T A u~ + u~^T M f'(z) u~]]
//   E   = 1/2 a(z,z) + sum_j m F(z_j) - (g, z)_h,    z = Q w + alpha u~.
// Q^T v at coarse node a is sum_j phi_a(x_j) v_j; the fine nodes are grouped
// by coarse cell and the per-cell sums are reduced in a fixed order.
#pragma once

#include "fmg_device.h"
#include "fmg_kernels_coef.h"
#include "fmg_kernels_mg.h"

namespace fmg {

struct ProblemSlot {
  const double* g;        // finest nodal load, packed (nf+1)^d
  double* u_out;          // packed (nf+1)^d output
  fmg_report* rep_out;    // optional device-writable report copy
  const double* c;        // weight c(x) of f(x, u) = c f(u) at the finest nodes (packed), or nullptr (c = 1)
  double param;           // nonlinearity parameter
  int kind;
  // set when the hierarchy is created (not per problem)
  int nf1;                // finest nodes per side
  CoefLevels coef;        // stencil arrays of the variable-coefficient operator (w[k] = nullptr: A = I)
};

struct NewtonState {
  double y[kMaxY];        // accepted iterate (w_1..w_N1, alpha)
  double ytry[kMaxY];     // point evaluated by the next quadrature pass
  double d[kMaxY];        // Newton direction
  double bH[kMaxY];       // Q^T A u~
  double GH[kMaxY];       // Q^T M g
  double c, Gu;           // u~^T A u~, u~^T M g
  double E, Escale, slope, t;
  int iter, passes, halvings, done, ok, level;
};

struct AugShape {
  int nH;        // coarse cells per side
  int log2r;     // fine cells per coarse cell per side = 2^log2r
  int bpc_log;   // blocks per coarse cell = 2^bpc_log
  int npb_log;   // fine node slots per block = 2^npb_log
  int N1;        // interior coarse nodes
  int general;   // 1: A_1 is a general matrix (variable coefficient), not the constant stencil
};

constexpr double kArmijo = 1e-4;
constexpr double kEnergyRounding = 1e-12;
constexpr int kMaxHalvings = 40;
constexpr double kSchurDrop = 1e-12;

__device__ __forceinline__ void report_status(fmg_report* rep, int code) {
  atomicCAS(&rep->status, 0, code);
}

// Dense coarse interior index of vertex a of coarse cell (cx, cy, cz), or -1.
template <int DIM>
__device__ __forceinline__ int coarse_vertex(int nH, int cx, int cy, int cz, int a) {
  const int x = cx + (a & 1), y = cy + ((a >> 1) & 1), z = DIM == 3 ? cz + ((a >> 2) & 1) : 1;
  if (x < 1 || x > nH - 1 || y < 1 || y > nH - 1 || (DIM == 3 && (z < 1 || z > nH - 1))) return -1;
  const int m = nH - 1;
  return (x - 1) + m * (y - 1) + (DIM == 3 ? m * m * (z - 1) : 0);
}

template <int DIM>
__device__ __forceinline__ void cell_of(int cell, int nH, int& cx, int& cy, int& cz) {
  cx = cell % nH;
  cy = (cell / nH) % nH;
  cz = DIM == 3 ? cell / (nH * nH) : 0;
}

// Visit the fine nodes of one block's share of a coarse cell:
// fn(grid index c, local coordinates t[DIM], i, j, l, u[c]).  The values
// u[c] are loaded kNodePrefetch visits ahead (from clamped, in-bounds
// addresses), so each wave keeps several loads in flight instead of waiting
// for one per node.  All threads of a block make the same number of visits
// unless the block's share is smaller than its thread count.
constexpr int kNodePrefetch = 4;

template <int DIM, typename Fn>
__device__ __forceinline__ void for_cell_nodes(const Grid& g, const AugShape& s, int cx, int cy, int cz,
                                               int t0, int t1, int tid, int nthreads,
                                               const double* __restrict__ u, Fn&& fn) {
  const int r = 1 << s.log2r, mask = r - 1;
  const double inv_r = 1.0 / r;
  auto index_of = [&](int t, int& i, int& j, int& l) {
    const int lx = t & mask, ly = (t >> s.log2r) & mask, lz = DIM == 3 ? t >> (2 * s.log2r) : 0;
    i = cx * r + lx; j = cy * r + ly; l = cz * r + lz;
    return gidx<DIM>(g, i, j, l);
  };
  auto load = [&](int t) {
    int i, j, l;
    return u[index_of(t < t1 ? t : t1 - 1, i, j, l)];
  };
  double q[kNodePrefetch];
#pragma unroll
  for (int p = 0; p < kNodePrefetch; ++p) q[p] = load(t0 + tid + p * nthreads);
  for (int tb = t0 + tid; tb < t1; tb += kNodePrefetch * nthreads) {
#pragma unroll
    for (int p = 0; p < kNodePrefetch; ++p) {
      const int t = tb + p * nthreads;
      const double uc = q[p];
      q[p] = load(t + kNodePrefetch * nthreads);
      if (t < t1) {
        int i, j, l;
        const int c = index_of(t, i, j, l);
        if (i != 0 && j != 0 && (DIM == 2 || l != 0)) {   // skip the Dirichlet nodes
          const int lx = i - cx * r, ly = j - cy * r, lz = DIM == 3 ? l - cz * r : 0;
          double tl[3] = {lx * inv_r, ly * inv_r, lz * inv_r};
          fn(c, tl, i, j, l, uc);
        }
      }
    }
  }
}

__device__ __forceinline__ long long fine_load_index(int nf1, int s, int i, int j, int l) {
  return ((long long)l * s * nf1 + (long long)j * s) * nf1 + (long long)i * s;
}

// The values the setup pass needs at one fine node: u~ at the node (c) and at
// its 2d axis neighbours (west, east, south, north, down, up), and the load g.
struct StencilVals {
  double c, w, e, s, n, d, u, g;
};

// (A u~) at the node from its stencil values: apply_A_at's expression, in the
// same order.
template <int DIM>
__device__ __forceinline__ double apply_A_vals(const StencilVals& v, double scale) {
  double s = (v.w + v.e) + (v.s + v.n);
  if (DIM == 3) s += v.d + v.u;
  return scale * (double(2 * DIM) * v.c - s);
}

// for_cell_nodes for the 3D setup pass: the node's stencil values and its
// load are loaded kSetupPrefetch visits ahead (from clamped, in-bounds
// addresses; the values of the skipped Dirichlet nodes are never used), not
// at their use, where each node waited for a round trip of its own (256^3
// solve 2.414 -> 2.391 ms; 250 registers).  The 2D setup pass keeps its loads
// at their use: its 1024-thread blocks leave 128 registers, and the ring made
// the u + sin u instance spill more.
constexpr int kSetupPrefetch = 3;

template <int DIM, typename Fn>
__device__ __forceinline__ void for_cell_nodes_stencil(const Grid& g, const AugShape& s, int cx, int cy, int cz,
                                                       int t0, int t1, int tid, int nthreads,
                                                       const double* __restrict__ u,
                                                       const double* __restrict__ gl, int nf1, int fs, Fn&& fn) {
  const int r = 1 << s.log2r, mask = r - 1;
  const double inv_r = 1.0 / r;
  auto index_of = [&](int t, int& i, int& j, int& l) {
    const int lx = t & mask, ly = (t >> s.log2r) & mask, lz = DIM == 3 ? t >> (2 * s.log2r) : 0;
    i = cx * r + lx; j = cy * r + ly; l = cz * r + lz;
    return gidx<DIM>(g, i, j, l);
  };
  auto load = [&](int t) {
    int i, j, l;
    const int c = index_of(t < t1 ? t : t1 - 1, i, j, l);
    StencilVals v;
    v.c = u[c];
    v.w = u[max(c - 1, 0)];
    v.e = u[c + 1];
    v.s = u[max(c - g.px, 0)];
    v.n = u[c + g.px];
    v.d = DIM == 3 ? u[max(c - g.pz, 0)] : 0.0;
    v.u = DIM == 3 ? u[c + g.pz] : 0.0;
    v.g = gl[fine_load_index(nf1, fs, i, j, l)];
    return v;
  };
  StencilVals q[kSetupPrefetch];
#pragma unroll
  for (int p = 0; p < kSetupPrefetch; ++p) q[p] = load(t0 + tid + p * nthreads);
  for (int tb = t0 + tid; tb < t1; tb += kSetupPrefetch * nthreads) {
#pragma unroll
    for (int p = 0; p < kSetupPrefetch; ++p) {
      const int t = tb + p * nthreads;
      const StencilVals v = q[p];
      q[p] = load(t + kSetupPrefetch * nthreads);
      if (t < t1) {
        int i, j, l;
        const int c = index_of(t, i, j, l);
        if (i != 0 && j != 0 && (DIM == 2 || l != 0)) {   // skip the Dirichlet nodes
          const int lx = i - cx * r, ly = j - cy * r, lz = DIM == 3 ? l - cz * r : 0;
          double tl[3] = {lx * inv_r, ly * inv_r, lz * inv_r};
          fn(c, tl, i, j, l, v);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Linearised right-hand side: b_j = m (g_j - f(u_j)) at level-k interior nodes.
// ---------------------------------------------------------------------------
// CW: f(x, u) = c(x) f(u) with c at the finest nodes (slot->c; nullptr means
// c = 1).  A separate instance, so that the c = 1 kernel keeps its own
// arithmetic (the compiler fuses g - f(u) differently once a weight may enter).
template <int DIM, int KIND, bool CW = false>
__global__ void __launch_bounds__(kBlock) k_rhs(Grid g, const ProblemSlot* __restrict__ slot, int nf1, int s,
                                                const double* __restrict__ u, double* __restrict__ b, double m) {
  int i, j, l;
  if (!node_of_thread<DIM>(g, i, j, l)) return;
  const int c = gidx<DIM>(g, i, j, l);
  const long long fi = fine_load_index(nf1, s, i, j, l);
  const double gv = slot->g[fi];
  if constexpr (CW) {
    const double* __restrict__ cw = slot->c;
    b[c] = m * (gv - (cw ? cw[fi] : 1.0) * NL<KIND>::f(u[c], slot->param));
  } else {
    b[c] = m * (gv - NL<KIND>::f(u[c], slot->param));
  }
}

// Per-cell setup sums for one block's node range:
//   sum phi_a (A u~)_j, sum u~_j (A u~)_j, sum phi_a g_j, sum u~_j g_j.
// Setup sums of one fine node (Alg. 3.1 step 2: the linear terms of the
// augmented problem): (A u~) phi_a, (A u~) u~, g phi_a, g u~.
template <int DIM>
__device__ __forceinline__ void setup_node(const double* phi, double u, double au, double gv, double* acc) {
  using AC = Acc<DIM>;
#pragma unroll
  for (int a = 0; a < AC::NV; ++a) {
    acc[AC::S_BH + a] += phi[a] * au;
    acc[AC::S_GH + a] += phi[a] * gv;
  }
  acc[AC::S_C] += u * au;
  acc[AC::S_GU] += u * gv;
}

// Quadrature sums of one fine node at z (the nonlinear terms and their
// derivatives): f phi_a, f' phi_a u~, f' phi_a phi_b, f u~, f' u~^2, F.
// CW: the sums are weighted by c(x_j) (cj) of f(x, u) = c(x) f(u).
template <int DIM, int KIND, bool CW = false>
__device__ __forceinline__ void quad_node(const double* phi, double z, double u, double param, double* acc,
                                          double cj = 1.0) {
  using AC = Acc<DIM>;
  using PR = Pairs<DIM>;
  double f, df, F;
  NL<KIND>::all(z, param, f, df, F);
  if (CW) { f *= cj; df *= cj; F *= cj; }
  double dphi[AC::NV];
#pragma unroll
  for (int a = 0; a < AC::NV; ++a) {
    acc[AC::Q_NH + a] += f * phi[a];
    dphi[a] = df * phi[a];
    acc[AC::Q_KHU + a] += dphi[a] * u;
  }
#pragma unroll
  for (int p = 0; p < PR::N; ++p) acc[AC::Q_K + p] += dphi[PR::a(p)] * phi[PR::b(p)];
  acc[AC::Q_NU] += f * u;
  acc[AC::Q_KUU] += df * u * u;
  acc[AC::Q_E] += F;
}

template <int DIM>
__device__ __forceinline__ void setup_accumulate(const Grid& g, const AugShape& s, const double* __restrict__ ut,
                                                 const double* __restrict__ gl, int nf1, int fs, double scale,
                                                 int cell, int t0, int t1, int tid, int nthreads, double* acc) {
  int cx, cy, cz;
  cell_of<DIM>(cell, s.nH, cx, cy, cz);
  for_cell_nodes<DIM>(g, s, cx, cy, cz, t0, t1, tid, nthreads, ut,
                      [&](int c, const double* tl, int i, int j, int l, double u) {
    double phi[Acc<DIM>::NV];
    kuhn_phi<DIM>(tl, phi);
    setup_node<DIM>(phi, u, apply_A_at<DIM>(ut, c, g, scale), gl[fine_load_index(nf1, fs, i, j, l)], acc);
  });
}

// The same with the variable-coefficient stencil (W, plane) and, when cw is
// set, the weight c(x) in the quadrature sums at z = u~.
template <int DIM, int KIND>
__device__ __forceinline__ void setup_quad_accumulate_var(const Grid& g, const AugShape& s,
                                                          const double* __restrict__ ut,
                                                          const double* __restrict__ gl,
                                                          const double* __restrict__ cw, int nf1, int fs,
                                                          const double* __restrict__ W, long long plane,
                                                          double param, int cell, int t0, int t1, int tid,
                                                          int nthreads, double* acc_s, double* acc_q) {
  int cx, cy, cz;
  cell_of<DIM>(cell, s.nH, cx, cy, cz);
  for_cell_nodes<DIM>(g, s, cx, cy, cz, t0, t1, tid, nthreads, ut,
                      [&](int c, const double* tl, int i, int j, int l, double u) {
    double phi[Acc<DIM>::NV];
    kuhn_phi<DIM>(tl, phi);
    const long long fi = fine_load_index(nf1, fs, i, j, l);
    double diag;
    setup_node<DIM>(phi, u, apply_Aw_at<DIM>(ut, c, g, W, plane, diag), gl[fi], acc_s);
    quad_node<DIM, KIND, true>(phi, u, u, param, acc_q, cw ? cw[fi] : 1.0);
  });
}

// Setup sums and the quadrature sums at the Newton start y0 = (0, .., 0, 1)
// (z = u~) in one visit of the nodes.
template <int DIM, int KIND>
__device__ __forceinline__ void setup_quad_accumulate(const Grid& g, const AugShape& s, const double* __restrict__ ut,
                                                      const double* __restrict__ gl, int nf1, int fs, double scale,
                                                      double param, int cell, int t0, int t1, int tid,
                                                      int nthreads, double* acc_s, double* acc_q) {
  int cx, cy, cz;
  cell_of<DIM>(cell, s.nH, cx, cy, cz);
  if constexpr (DIM == 3) {
    for_cell_nodes_stencil<DIM>(g, s, cx, cy, cz, t0, t1, tid, nthreads, ut, gl, nf1, fs,
                                [&](int, const double* tl, int, int, int, const StencilVals& v) {
      double phi[Acc<DIM>::NV];
      kuhn_phi<DIM>(tl, phi);
      setup_node<DIM>(phi, v.c, apply_A_vals<DIM>(v, scale), v.g, acc_s);
      quad_node<DIM, KIND>(phi, v.c, v.c, param, acc_q);
    });
  } else {
    for_cell_nodes<DIM>(g, s, cx, cy, cz, t0, t1, tid, nthreads, ut,
                        [&](int c, const double* tl, int i, int j, int l, double u) {
      double phi[Acc<DIM>::NV];
      kuhn_phi<DIM>(tl, phi);
      setup_node<DIM>(phi, u, apply_A_at<DIM>(ut, c, g, scale), gl[fine_load_index(nf1, fs, i, j, l)], acc_s);
      quad_node<DIM, KIND>(phi, u, u, param, acc_q);
    });
  }
}

// Newton state at the start of an augmented solve: y = (0, ..., 0, 1), i.e. z = u~.
__device__ __forceinline__ void newton_state_reset(NewtonState* ns, int N1, int level) {
  for (int q = 0; q < N1; ++q) { ns->y[q] = 0.0; ns->ytry[q] = 0.0; ns->d[q] = 0.0; }
  ns->y[N1] = 1.0;
  ns->ytry[N1] = 1.0;
  ns->d[N1] = 0.0;
  ns->iter = 0; ns->passes = 0; ns->halvings = 0; ns->done = 0; ns->ok = 0; ns->level = level;
  ns->t = 1.0; ns->E = 0.0; ns->Escale = 0.0; ns->slope = 0.0;
}

// Per-cell quadrature sums at z = Q w + alpha u~ for one block's node range.
template <int DIM, int KIND>
__device__ __forceinline__ void quad_accumulate(const Grid& g, const AugShape& s, const double* __restrict__ ut,
                                                const double* ytry, double param, int cell, int t0, int t1,
                                                int tid, int nthreads, double* acc) {
  using AC = Acc<DIM>;
  int cx, cy, cz;
  cell_of<DIM>(cell, s.nH, cx, cy, cz);
  double wv[AC::NV];
#pragma unroll
  for (int a = 0; a < AC::NV; ++a) {
    const int gi = coarse_vertex<DIM>(s.nH, cx, cy, cz, a);
    wv[a] = gi >= 0 ? ytry[gi] : 0.0;
  }
  const double alpha = ytry[s.N1];
  for_cell_nodes<DIM>(g, s, cx, cy, cz, t0, t1, tid, nthreads, ut,
                      [&](int, const double* tl, int, int, int, double u) {
    double phi[AC::NV];
    kuhn_phi<DIM>(tl, phi);
    double z = alpha * u;
#pragma unroll
    for (int a = 0; a < AC::NV; ++a) z += wv[a] * phi[a];
    quad_node<DIM, KIND>(phi, z, u, param, acc);
  });
}

// quad_accumulate with the weight c(x) of f(x, u) = c(x) f(u) (cw: finest
// nodal c, nf1 / fs as for the load).
template <int DIM, int KIND>
__device__ __forceinline__ void quad_accumulate_cw(const Grid& g, const AugShape& s, const double* __restrict__ ut,
                                                   const double* ytry, double param, const double* __restrict__ cw,
                                                   int nf1, int fs, int cell, int t0, int t1, int tid, int nthreads,
                                                   double* acc) {
  using AC = Acc<DIM>;
  int cx, cy, cz;
  cell_of<DIM>(cell, s.nH, cx, cy, cz);
  double wv[AC::NV];
#pragma unroll
  for (int a = 0; a < AC::NV; ++a) {
    const int gi = coarse_vertex<DIM>(s.nH, cx, cy, cz, a);
    wv[a] = gi >= 0 ? ytry[gi] : 0.0;
  }
  const double alpha = ytry[s.N1];
  for_cell_nodes<DIM>(g, s, cx, cy, cz, t0, t1, tid, nthreads, ut,
                      [&](int, const double* tl, int i, int j, int l, double u) {
    double phi[AC::NV];
    kuhn_phi<DIM>(tl, phi);
    double z = alpha * u;
#pragma unroll
    for (int a = 0; a < AC::NV; ++a) z += wv[a] * phi[a];
    quad_node<DIM, KIND, true>(phi, z, u, param, acc, cw[fine_load_index(nf1, fs, i, j, l)]);
  });
}

// Quadrature sums of the variable-coefficient solves: weighted when c is given.
template <int DIM, int KIND>
__device__ __forceinline__ void quad_accumulate_var(const Grid& g, const AugShape& s, const double* __restrict__ ut,
                                                    const double* ytry, double param, const double* __restrict__ cw,
                                                    int nf1, int cell, int t0, int t1, int tid, int nthreads,
                                                    double* acc) {
  if (cw) quad_accumulate_cw<DIM, KIND>(g, s, ut, ytry, param, cw, nf1, (nf1 - 1) / g.n, cell, t0, t1, tid,
                                        nthreads, acc);
  else quad_accumulate<DIM, KIND>(g, s, ut, ytry, param, cell, t0, t1, tid, nthreads, acc);
}

}  // namespace fmg

#include "fmg_elem.h"

namespace fmg {

// Element rule: per-cell quadrature sums at z = Q w + alpha u~ for one block's
// range of fine cells, unweighted (the caller scales them by ElemRule::W).
template <int DIM, int KIND>
__device__ __forceinline__ void quad_accumulate_elem(const Grid& g, const AugShape& s, const double* __restrict__ ut,
                                                     const double* ytry, double param, int cell, int t0, int t1,
                                                     int tid, int nthreads, double* acc) {
  using AC = Acc<DIM>;
  int cx, cy, cz;
  cell_of<DIM>(cell, s.nH, cx, cy, cz);
  double wv[AC::NV];
#pragma unroll
  for (int a = 0; a < AC::NV; ++a) {
    const int gi = coarse_vertex<DIM>(s.nH, cx, cy, cz, a);
    wv[a] = gi >= 0 ? ytry[gi] : 0.0;
  }
  const double alpha = ytry[s.N1];
  for_cell_cells<DIM>(g, s, cx, cy, cz, t0, t1, tid, nthreads, ut,
                      [&](int, int, int, int lx, int ly, int lz, const double* uc) {
    elem_cell<DIM, KIND, false>(s, lx, ly, lz, uc, nullptr, wv, alpha, param, acc, nullptr);
  });
}

// Element rule, setup pass: the stiffness terms (A u~) phi_a, (A u~) u~ at the
// cell's lower corner node (as in the vertex rule: they are exact matrix
// products), the load terms W g phi_a, W g u~ at the points, and the
// (unweighted) quadrature sums at the Newton start z = u~.
template <int DIM, int KIND>
__device__ __forceinline__ void setup_quad_accumulate_elem(const Grid& g, const AugShape& s,
                                                           const double* __restrict__ ut,
                                                           const double* __restrict__ gl, int nf1, int fs,
                                                           double scale, double param, int cell, int t0, int t1,
                                                           int tid, int nthreads, double* acc_s, double* acc_q) {
  using AC = Acc<DIM>;
  int cx, cy, cz;
  cell_of<DIM>(cell, s.nH, cx, cy, cz);
  double wv[AC::NV];
#pragma unroll
  for (int a = 0; a < AC::NV; ++a) wv[a] = 0.0;
  const double inv_r = 1.0 / (1 << s.log2r);
  for_cell_cells<DIM>(g, s, cx, cy, cz, t0, t1, tid, nthreads, ut,
                      [&](int i, int j, int l, int lx, int ly, int lz, const double* uc) {
    if (i != 0 && j != 0 && (DIM == 2 || l != 0)) {
      const double tl[3] = {lx * inv_r, ly * inv_r, lz * inv_r};
      double phi[AC::NV];
      kuhn_phi<DIM>(tl, phi);
      const double au = apply_A_at<DIM>(ut, gidx<DIM>(g, i, j, l), g, scale);
#pragma unroll
      for (int a = 0; a < AC::NV; ++a) acc_s[AC::S_BH + a] += phi[a] * au;
      acc_s[AC::S_C] += uc[0] * au;
    }
    double gc[AC::NV];
#pragma unroll
    for (int e = 0; e < AC::NV; ++e)
      gc[e] = gl[fine_load_index(nf1, fs, i + (e & 1), j + ((e >> 1) & 1), DIM == 3 ? l + ((e >> 2) & 1) : 0)];
    elem_cell<DIM, KIND, true>(s, lx, ly, lz, uc, gc, wv, 1.0, param, acc_q, acc_s);
  });
}

// Linearised right-hand side with the element rule (Alg. 3.1 step 1),
// b = (g_I - f(u_h), phi) at every interior node, in two launches: every fine
// cell evaluates g - f(u) once at each point of its Kuhn simplices and
// writes, per corner, the sum of those values times the corner's barycentric
// coordinate there (contrib[corner][cell]); every interior node then adds the
// 2^d contributions of the cells around it (it is corner e of cell node - e),
// in ascending e, times m W.
template <int DIM, int KIND, int S>
__device__ __forceinline__ void rhs_elem_simplex(const double* uc, const double* gc, double param, double* acc) {
  using R = ElemRule<DIM>;
  using KC = KuhnChain<DIM, S>;
  double uv[DIM + 1], gv[DIM + 1];
  uv[0] = uc[0]; uv[1] = uc[KC::v1]; uv[DIM] = uc[KC::vl];
  gv[0] = gc[0]; gv[1] = gc[KC::v1]; gv[DIM] = gc[KC::vl];
  if (DIM == 3) { uv[2] = uc[KC::v2]; gv[2] = gc[KC::v2]; }
  double usum = 0.0, gsum = 0.0;
#pragma unroll
  for (int k = 0; k <= DIM; ++k) { usum += uv[k]; gsum += gv[k]; }
  double vsum = 0.0, own[DIM + 1];
#pragma unroll
  for (int k = 0; k <= DIM; ++k) own[k] = 0.0;
#pragma unroll 1
  for (int p = 0; p <= DIM; ++p) {
    const double val = elem_interp<DIM>(gv, gsum, p) - NL<KIND>::f(elem_interp<DIM>(uv, usum, p), param);
    vsum += val;
#pragma unroll
    for (int k = 0; k <= DIM; ++k) own[k] = fma(p == k ? 1.0 : 0.0, val, own[k]);
  }
  // chain vertex k: coordinate A at its own point, B at the others
  constexpr double D = R::A - R::B;
  acc[0] += R::B * vsum + D * own[0];
  acc[KC::v1] += R::B * vsum + D * own[1];
  if (DIM == 3) acc[KC::v2] += R::B * vsum + D * own[2];
  acc[KC::vl] += R::B * vsum + D * own[DIM];
}

template <int DIM, int KIND>
__global__ void __launch_bounds__(kBlock) k_rhs_elem_cells(Grid g, const ProblemSlot* __restrict__ slot, int nf1,
                                                           int s, const double* __restrict__ u,
                                                           double* __restrict__ contrib) {
  constexpr int NV = 1 << DIM;
  const long long n = g.n;
  const long long ncells = DIM == 2 ? n * n : n * n * n;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  const int i = (int)(c % n), j = (int)((c / n) % n), l = DIM == 3 ? (int)(c / (n * n)) : 0;
  const double* __restrict__ gl = slot->g;
  double uc[NV], gc[NV], acc[NV];
#pragma unroll
  for (int e = 0; e < NV; ++e) {
    const int x = i + (e & 1), y = j + ((e >> 1) & 1), z = DIM == 3 ? l + ((e >> 2) & 1) : 0;
    uc[e] = u[gidx<DIM>(g, x, y, z)];
    gc[e] = gl[fine_load_index(nf1, s, x, y, z)];
    acc[e] = 0.0;
  }
  const double param = slot->param;
  rhs_elem_simplex<DIM, KIND, 0>(uc, gc, param, acc);
  rhs_elem_simplex<DIM, KIND, 1>(uc, gc, param, acc);
  if constexpr (DIM == 3) {
    rhs_elem_simplex<DIM, KIND, 2>(uc, gc, param, acc);
    rhs_elem_simplex<DIM, KIND, 3>(uc, gc, param, acc);
    rhs_elem_simplex<DIM, KIND, 4>(uc, gc, param, acc);
    rhs_elem_simplex<DIM, KIND, 5>(uc, gc, param, acc);
  }
#pragma unroll
  for (int e = 0; e < NV; ++e) contrib[e * ncells + c] = acc[e];
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_rhs_elem_nodes(Grid g, const double* __restrict__ contrib,
                                                           double* __restrict__ b, double mw) {
  int i, j, l;
  if (!node_of_thread<DIM>(g, i, j, l)) return;
  const long long n = g.n;
  const long long ncells = DIM == 2 ? n * n : n * n * n;
  double sum = 0.0;
#pragma unroll
  for (int e = 0; e < (1 << DIM); ++e) {
    const long long cell = (i - (e & 1)) + n * ((j - ((e >> 1) & 1)) + (DIM == 3 ? n * (l - ((e >> 2) & 1)) : 0));
    sum += contrib[e * ncells + cell];
  }
  b[gidx<DIM>(g, i, j, l)] = mw * sum;
}

// ---------------------------------------------------------------------------
// Small dense linear algebra in LDS, executed by the first wavefront of the
// block (n <= 64 = wave size).  Lanes of one wavefront issue their LDS
// operations in program order; wave_sync() keeps the compiler from moving
// LDS accesses across the phase boundaries.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Right-looking Cholesky steps k = 0..kend-1 of the n x n matrix L (row-major,
// lower part; lanes own rows).  After kend = n-1 steps, L[n-1][n-1] holds the
// Schur complement of the leading block.  col: LDS scratch of n doubles
// holding the current column (kept apart from L so that the row updates of a
// lane can be issued without waiting on one another).  rdiag receives the
// reciprocals of the computed diagonal entries.
__device__ __forceinline__ void chol_steps_wave(double* __restrict__ L, double* __restrict__ col,
                                       double* __restrict__ rdiag, int n, int kend) {
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  for (int k = 0; k < kend; ++k) {
    wave_sync();
    const double s = sqrt(L[k * n + k]);
    const double rs = 1.0 / s;
    double lik = 0.0;
    if (lane > k && lane < n) lik = L[lane * n + k] * rs;
    if (lane > k && lane < n) { col[lane] = lik; L[lane * n + k] = lik; }
    if (lane == k) { L[k * n + k] = s; rdiag[k] = rs; }
    wave_sync();
    if (lane > k && lane < n)
      for (int j = k + 1; j <= lane; ++j) L[lane * n + j] -= lik * col[j];
  }
  wave_sync();
}

// Solve L L^T x = x for the leading nn rows (nn <= 64), lanes own entries;
// rdiag holds 1/L[j][j].
__device__ __forceinline__ void chol_solve_wave(const double* __restrict__ L, const double* __restrict__ rdiag, int n,
                                       int nn, double* __restrict__ x) {
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  wave_sync();
  double v = lane < nn ? x[lane] : 0.0;
  for (int j = 0; j < nn; ++j) {
    const double lij = (lane > j && lane < nn) ? L[lane * n + j] : 0.0;
    if (lane == j) v *= rdiag[j];
    const double xj = lane_value(v, j);
    v -= lij * xj;
  }
  for (int j = nn - 1; j >= 0; --j) {
    const double lji = lane < j ? L[j * n + lane] : 0.0;
    if (lane == j) v *= rdiag[j];
    const double xj = lane_value(v, j);
    v -= lji * xj;
  }
  if (lane < nn) x[lane] = v;
  wave_sync();
}

// Parallel copy of a trivially copyable struct (multiple of 8 bytes) by the
// lanes of one wavefront.
template <typename S>
__device__ __forceinline__ void wave_copy(S* dst, const S* src) {
  static_assert(sizeof(S) % 8 == 0, "8-byte words");
  const double* a = reinterpret_cast<const double*>(src);
  double* b = reinterpret_cast<double*>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(S) / 8); i += 64) b[i] = a[i];
}

__device__ __forceinline__ double wave_allsum(double v) { return wave_sum(v); }
__device__ __forceinline__ double wave_allmax(double v) { return wave_max_nonneg(v); }

// LDS doubles newton_core needs besides the per-cell sums.
__host__ __device__ constexpr int newton_scratch_doubles(int N1) {
  return (int)(sizeof(NewtonState) / 8) + N1 * N1 + (N1 + 1) * (N1 + 1) + 5 * (N1 + 1) + 8;
}

// Pair index p with {a, b} = {Pairs::a(p), Pairs::b(p)} for comparable cell
// vertices a, b (one a subset of the other), or -1.
template <int DIM>
__device__ __forceinline__ int pair_index(int a, int b) {
  if (a > b) { const int t = a; a = b; b = t; }
  if ((a & b) != a) return -1;
  for (int p = 0; p < Pairs<DIM>::N; ++p)
    if (Pairs<DIM>::a(p) == a && Pairs<DIM>::b(p) == b) return p;
  return -1;
}

// Coarse interior node A (dense index) -> grid coordinates (1-based).
template <int DIM>
__device__ __forceinline__ void coarse_coords(int nH, int A, int& x, int& y, int& z) {
  const int m = nH - 1;
  x = 1 + A % m;
  y = 1 + (A / m) % m;
  z = DIM == 3 ? 1 + A / (m * m) : 0;
}

// ---------------------------------------------------------------------------
// Newton step of the augmented problem, executed by the first wavefront of
// the block (the others return at once; the caller synchronises the block
// before and after).  Inputs: per-cell quadrature sums `cs` (LDS, ncell x NQ)
// at the point ns->ytry.  Damped Newton with Armijo backtracking on E as a
// state machine, one evaluation per call: accept or halve the trial step,
// test convergence (|t d|_inf <= tol max(1, |y|_inf)), otherwise compute the
// next direction d = -J^{-1} R (dropping the u~ direction when its Schur
// complement is <= 1e-12 of J_uu) and the next trial point; a direction with
// |d|_inf <= tol max(1, |y|_inf) is applied in full and ends the iteration
// without another evaluation (it changes E only at rounding level).  Every entry of
// J and R gathers the contributions of the (at most 2^d) coarse cells that
// touch it, cells in ascending order.
// LDS scratch `sm` (newton_scratch_doubles): state | A_1 | J | R | A_1 w | col | rdiag | 8.
// ---------------------------------------------------------------------------
template <int DIM>
__device__ __forceinline__ void newton_core(const AugShape& s, const double* cs, const double* __restrict__ A1g, double m,
                            NewtonState* nsg, fmg_report* rep, int newton_max, double tol, double* sm) {
  if (threadIdx.x >= 64) return;
  using AC = Acc<DIM>;
  const int lane = threadIdx.x;
  const int N1 = s.N1, ny = N1 + 1, nH = s.nH;
  const int ncell = DIM == 2 ? nH * nH : nH * nH * nH;
  NewtonState* ns = reinterpret_cast<NewtonState*>(sm);
  double* A1 = sm + sizeof(NewtonState) / 8;
  double* J = A1 + N1 * N1;
  double* R = J + ny * ny;
  double* Aw = R + ny;
  double* col = Aw + ny;
  double* rdiag = col + ny;
  double* dsave = rdiag + ny;
  wave_copy(ns, nsg);
  for (int idx = lane; idx < N1 * N1; idx += 64) A1[idx] = A1g[idx];
  wave_sync();
  const double* y = ns->ytry;
  const double alpha = y[N1];
  // A_1 w, R_H, J_Hu (lanes over coarse nodes)
  for (int A = lane; A < N1; A += 64) {
    double t = 0.0;
    for (int B = 0; B < N1; ++B) t += A1[A * N1 + B] * y[B];
    Aw[A] = t;
    int ax, ay, az;
    coarse_coords<DIM>(nH, A, ax, ay, az);
    double nh = 0.0, khu = 0.0;
    for (int e = 0; e < AC::NV; ++e) {     // cells c = A - e containing A as vertex e
      const int cx = ax - (e & 1), cy = ay - ((e >> 1) & 1), cz = DIM == 3 ? az - ((e >> 2) & 1) : 0;
      const int cell = cx + nH * (cy + nH * cz);
      nh += cs[cell * AC::NQ + AC::Q_NH + e];
      khu += cs[cell * AC::NQ + AC::Q_KHU + e];
    }
    R[A] = t + alpha * ns->bH[A] - ns->GH[A] + m * nh;
    J[A * ny + N1] = ns->bH[A] + m * khu;
    J[N1 * ny + A] = J[A * ny + N1];
  }
  // J_HH = A_1 + m sum f'(z) phi_A phi_B (lanes over entries)
  for (int idx = lane; idx < N1 * N1; idx += 64) {
    const int A = idx / N1, B = idx % N1;
    int ax, ay, az, bx, by, bz;
    coarse_coords<DIM>(nH, A, ax, ay, az);
    coarse_coords<DIM>(nH, B, bx, by, bz);
    double k = 0.0;
    if (abs(ax - bx) <= 1 && abs(ay - by) <= 1 && abs(az - bz) <= 1) {
      for (int e = 0; e < AC::NV; ++e) {
        const int cx = ax - (e & 1), cy = ay - ((e >> 1) & 1), cz = DIM == 3 ? az - ((e >> 2) & 1) : 0;
        const int fx = bx - cx, fy = by - cy, fz = DIM == 3 ? bz - cz : 0;
        if (fx < 0 || fx > 1 || fy < 0 || fy > 1 || fz < 0 || fz > 1) continue;
        const int p = pair_index<DIM>(e, fx | (fy << 1) | (fz << 2));
        if (p < 0) continue;
        k += cs[(cx + nH * (cy + nH * cz)) * AC::NQ + AC::Q_K + p];
      }
    }
    J[A * ny + B] = A1[idx] + m * k;
  }
  // scalars: sums over cells and over coarse nodes
  double nu = 0.0, kuu = 0.0, sF = 0.0;
  for (int c = lane; c < ncell; c += 64) {
    nu += cs[c * AC::NQ + AC::Q_NU];
    kuu += cs[c * AC::NQ + AC::Q_KUU];
    sF += cs[c * AC::NQ + AC::Q_E];
  }
  double bw = 0.0, gw = 0.0, wAw = 0.0;
  for (int A = lane; A < N1; A += 64) {
    bw += ns->bH[A] * y[A];
    gw += ns->GH[A] * y[A];
    wAw += y[A] * Aw[A];
  }
  nu = wave_allsum(nu); kuu = wave_allsum(kuu); sF = wave_allsum(sF);
  bw = wave_allsum(bw); gw = wave_allsum(gw); wAw = wave_allsum(wAw);
  const double Juu = ns->c + m * kuu;
  const double Ru = bw + alpha * ns->c + m * nu - ns->Gu;
  if (lane == 0) { J[N1 * ny + N1] = Juu; R[N1] = Ru; }
  const double t1 = 0.5 * wAw + alpha * bw + 0.5 * alpha * alpha * ns->c;
  const double t2 = m * sF;
  const double t3 = gw + alpha * ns->Gu;
  const double Etry = t1 + t2 - t3, Stry = fabs(t1) + fabs(t2) + fabs(t3);
  wave_sync();
  // ---- state machine (decisions are uniform across the wavefront) ----
  bool finite = isfinite(Etry);
  for (int A = lane; A < ny; A += 64) finite = finite && isfinite(R[A]);
  finite = __all(finite);
  const int passes = ns->passes, iter = ns->iter;
  const double E = ns->E, Escale = ns->Escale, slope0 = ns->slope, t = ns->t;
  int newdir = 0, done = 0, ok = 0, halve = 0;
  if (!finite) {
    done = 1;
  } else if (passes == 0) {
    newdir = 1;
  } else if (Etry <= E + kArmijo * t * slope0 + kEnergyRounding * fmax(Escale, Stry)) {
    double stepmax = 0.0, ymax = 0.0;
    for (int A = lane; A < ny; A += 64) {
      stepmax = fmax(stepmax, fabs(t * ns->d[A]));
      ymax = fmax(ymax, fabs(y[A]));
    }
    stepmax = wave_allmax(stepmax);
    ymax = wave_allmax(ymax);
    if (stepmax <= tol * fmax(1.0, ymax)) { done = 1; ok = 1; }
    else newdir = 1;
  } else {
    halve = 1;
  }
  const bool accept = finite && !halve;
  if (newdir && iter >= newton_max) { done = 1; ok = 0; newdir = 0; }
  wave_sync();
  if (accept)
    for (int A = lane; A < ny; A += 64) ns->y[A] = y[A];
  if (halve) {
    const double tn = 0.5 * t;
    for (int A = lane; A < ny; A += 64) ns->ytry[A] = ns->y[A] + tn * ns->d[A];
  }
  wave_sync();
  if (lane == 0) {
    if (accept) { ns->E = Etry; ns->Escale = Stry; }
    if (halve) {
      ns->t = 0.5 * t;
      if (++ns->halvings > kMaxHalvings * newton_max) { done = 1; ok = 0; }
    }
    ns->passes = passes + 1;
  }
  done = __builtin_amdgcn_readlane(done, 0);
  ok = __builtin_amdgcn_readlane(ok, 0);
  if (newdir) {
    // ---- new direction: J d = -R at the accepted point (y == ytry here) ----
    for (int A = lane; A < ny; A += 64) dsave[A] = -R[A];
    chol_steps_wave(J, col, rdiag, ny, N1);   // leading block factored, J[N1][N1] = Schur complement
    const double schur = J[N1 * ny + N1];
    const bool drop = !(schur > kSchurDrop * Juu);
    if (!drop && lane == 0) { const double r = sqrt(schur); J[N1 * ny + N1] = r; rdiag[N1] = 1.0 / r; }
    wave_sync();
    chol_solve_wave(J, rdiag, ny, drop ? N1 : ny, dsave);
    if (drop && lane == 0) dsave[N1] = 0.0;
    wave_sync();
    double sl = 0.0;
    for (int A = lane; A < ny; A += 64) {
      ns->d[A] = dsave[A];
      sl += R[A] * dsave[A];
      ns->ytry[A] = ns->y[A] + dsave[A];
    }
    sl = wave_allsum(sl);
    if (lane == 0) { ns->slope = sl; ns->t = 1.0; ns->iter = iter + 1; }
    // a small direction is applied in full without evaluating the energy there
    double dmax = 0.0, ymax = 0.0;
    bool dfin = true;
    for (int A = lane; A < ny; A += 64) {
      dmax = fmax(dmax, fabs(dsave[A]));
      ymax = fmax(ymax, fabs(ns->y[A]));
      dfin = dfin && isfinite(dsave[A]);
    }
    dmax = wave_allmax(dmax);
    ymax = wave_allmax(ymax);
    dfin = __all(dfin);
    if (dfin && dmax <= tol * fmax(1.0, ymax)) {
      done = 1;
      ok = 1;
      for (int A = lane; A < ny; A += 64) ns->y[A] = ns->ytry[A];
    }
  }
  wave_sync();
  if (lane == 0) {
    const int iter_new = iter + (newdir ? 1 : 0);
    ns->done = done;
    ns->ok = ok;
    if (done) {
      const int k = ns->level - 1;
      rep->newton_iters[k] = iter_new;
      rep->newton_total[k] += iter_new;
      rep->alpha[k] = ns->y[N1];
      if (k == 0) rep->level1_iters = iter_new;   // level 1 solved as the augmented problem with u~ = 0
      if (!finite) report_status(rep, FMG_E_NONFINITE);
      else if (!ok) report_status(rep, FMG_E_NOT_CONVERGED);
    }
  }
  wave_sync();
  wave_copy(nsg, ns);
}

// Partial-sum units per thread kept in flight by the last block of a pass.
template <int DIM>
__host__ __device__ constexpr int sum_units() { return DIM == 2 ? 4 : 12; }

// Reduce the per-block partials of one pass into per-cell sums: every
// (cell, accumulator) item is split into segments of consecutive blocks so
// that all threads take part; segment sums are combined in a fixed order.
// The partials were written by blocks on other XCDs, so each load is a trip
// to the memory side: a thread keeps the loads of kSumUnits items (two
// blocks' partials of each) in flight at once instead of one at a time;
// kSumUnits is smaller where the block's register budget is (1024 threads).
// tmp: LDS of at least blockDim doubles.
template <int NACC, int kSumUnits>
__device__ __forceinline__ void cell_sums_from_partials(const double* __restrict__ partials, int ncell, int bpc,
                                                        double* cs, double* tmp) {
  const int W = ncell * NACC;
  const int S = max(1, min(bpc, (int)blockDim.x / W));
  const int seg = (bpc + S - 1) / S;
  const int U = W * S;
  for (int u0 = threadIdx.x; u0 < U; u0 += kSumUnits * blockDim.x) {
    const double* p[kSumUnits];
    int n[kSumUnits];
    double t0[kSumUnits], t1[kSumUnits];
#pragma unroll
    for (int k = 0; k < kSumUnits; ++k) {
      const int u = u0 + k * blockDim.x;
      const int uc = u < U ? u : 0;
      const int item = uc % W, sg = uc / W;
      const int b0 = sg * seg;
      n[k] = u < U ? max(0, min(bpc, b0 + seg) - b0) : 0;
      p[k] = partials + ((size_t)(item / NACC) * bpc + min(b0, bpc - 1)) * NACC + item % NACC;
      t0[k] = 0.0;
      t1[k] = 0.0;
    }
    for (int b = 0; b < seg; b += 2) {
      double x0[kSumUnits], x1[kSumUnits];
#pragma unroll
      for (int k = 0; k < kSumUnits; ++k) {
        x0[k] = b < n[k] ? p[k][(size_t)b * NACC] : 0.0;
        x1[k] = b + 1 < n[k] ? p[k][(size_t)(b + 1) * NACC] : 0.0;
      }
      // every load is issued before the first add waits for one
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < kSumUnits; ++k) {
        t0[k] += x0[k];
        t1[k] += x1[k];
      }
    }
#pragma unroll
    for (int k = 0; k < kSumUnits; ++k) {
      const int u = u0 + k * blockDim.x;
      if (u < U) {
        const int item = u % W, sg = u / W;
        if (S == 1) cs[item] = t0[k] + t1[k];
        else tmp[sg * W + item] = t0[k] + t1[k];
      }
    }
  }
  __syncthreads();
  if (S > 1) {
    for (int item = threadIdx.x; item < W; item += blockDim.x) {
      double t = 0.0;
      for (int sg = 0; sg < S; ++sg) t += tmp[sg * W + item];
      cs[item] = t;
    }
    __syncthreads();
  }
}

// Fold per-cell setup sums into Q^T A u~, u~^T A u~, Q^T M g, u~^T M g: each
// coarse node gathers the 2^d cells that touch it (vertex e of cell A - e),
// in ascending e; the two scalars are sums over the cells by one wavefront.
template <int DIM>
__device__ __forceinline__ void setup_scatter(const AugShape& s, const double* cs, double m, NewtonState* ns) {
  using AC = Acc<DIM>;
  const int nH = s.nH;
  const int ncell = DIM == 2 ? nH * nH : nH * nH * nH;
  for (int A = threadIdx.x; A < s.N1; A += blockDim.x) {
    int ax, ay, az;
    coarse_coords<DIM>(nH, A, ax, ay, az);
    double bh = 0.0, gh = 0.0;
#pragma unroll
    for (int e = 0; e < AC::NV; ++e) {
      const int cx = ax - (e & 1), cy = ay - ((e >> 1) & 1), cz = DIM == 3 ? az - ((e >> 2) & 1) : 0;
      const double* cc = cs + (cx + nH * (cy + nH * cz)) * AC::NS;
      bh += cc[AC::S_BH + e];
      gh += cc[AC::S_GH + e];
    }
    ns->bH[A] = bh;
    ns->GH[A] = m * gh;
  }
  if (threadIdx.x < 64) {
    double v[2] = {0.0, 0.0};
    for (int cell = threadIdx.x; cell < ncell; cell += 64) {
      v[0] += cs[cell * AC::NS + AC::S_C];
      v[1] += cs[cell * AC::NS + AC::S_GU];
    }
    wave_sum_n<2>(v);
    if (threadIdx.x == 0) {
      ns->c = v[0];
      ns->Gu = m * v[1];
    }
  }
  __syncthreads();
}

template <int DIM>
__device__ __forceinline__ void setup_reduce(const AugShape& s, const double* __restrict__ partials_s, double m,
                                    NewtonState* ns, double* cs, double* tmp) {
  using AC = Acc<DIM>;
  const int ncell = DIM == 2 ? s.nH * s.nH : s.nH * s.nH * s.nH;
  cell_sums_from_partials<AC::NS, sum_units<DIM>()>(partials_s, ncell, 1 << s.bpc_log, cs, tmp);
  setup_scatter<DIM>(s, cs, m, ns);
}

// Threads per block of the fine quadrature passes: 256, or on levels with at
// least 2^aug_wide_nodes_log fine nodes per coarse cell 1024 (2D) / 512 (3D),
// so fewer blocks: fewer release/ticket operations and fewer partials for the
// last block to reduce.  The 3D quadrature needs more registers per thread and
// stops at 512; the element-rule passes (d+1 points on each of d! simplices
// per fine cell) always take 256, so that they never spill.
constexpr int kAugMaxThreads = 1024;
template <int DIM>
__host__ __device__ constexpr int aug_threads() { return DIM == 2 ? kAugMaxThreads : 512; }
template <int DIM>
__host__ __device__ constexpr int aug_wide_nodes_log() { return DIM == 2 ? 12 : 15; }

// The 2D passes that also finish the Newton solve (FINISH) run 512 threads
// over the node range of a 1024-thread block: with the completion code in the
// same kernel, the 1024-thread bound (128 registers) spilled 116-300 bytes per
// lane; at 512 none (2048^2 solve 1.083 -> 1.077 ms).

// LDS doubles of k_newton_step / k_newton_finish for a block of `threads`.
__host__ __device__ constexpr int newton_kernel_lds_doubles(int ncell, int NQ, int N1, int threads) {
  return ncell * NQ + newton_scratch_doubles(N1) + threads;
}

template <int DIM, bool GEN = false>
__device__ __forceinline__ void newton_step_dev(const AugShape& s, const double* cs, const double* __restrict__ A1,
                                                double m, NewtonState* ns, fmg_report* rep, int newton_max,
                                                double tol, double* sm);

template <int DIM, int KIND, bool ELEM = false, bool VAR = false>
__device__ __forceinline__ void quad_cells_by_waves(const Grid& g, const AugShape& s, const double* __restrict__ ut,
                                           const double* ytry, double param, double* cs,
                                           const ProblemSlot* __restrict__ slot = nullptr);

// One pass of the augmented Newton iteration in one launch.  Every block
// accumulates its share of the fine quadrature sums at ns->ytry (SETUP: the
// setup sums plus the sums at y0 = (0,..,0,1), i.e. z = u~) and writes them
// as per-block partials.  The last block to finish (atomic ticket,
// release/acquire at device scope) reduces all partials, cell by cell in a
// fixed block order, into the cell sums and performs the Newton step.
// tickets[0]: zero between launches.  ELEM: the element rule (the block's
// node range is a range of fine cells); the completion of a Newton solve that
// needs more passes is then left to k_newton_finish.  VAR: the variable-
// coefficient operator (the setup pass applies the level's stencil arrays)
// and the weight c(x) of f(x, u) = c(x) f(u) when the problem gives one; the
// completion is left to k_newton_finish as well.
// LDS: newton_kernel_lds_doubles(ncell, NQ, N1, blockDim).
template <int DIM, int KIND, bool SETUP, bool FINISH, bool ELEM = false, bool VAR = false>
__global__ void __launch_bounds__((ELEM || VAR ? kBlock : DIM == 2 && FINISH ? 512 : aug_threads<DIM>())) k_aug_pass(Grid g, AugShape s, const double* __restrict__ ut,
                                                     const ProblemSlot* __restrict__ slot, int nf1, int fs,
                                                     double scale, double m, const double* __restrict__ A1,
                                                     NewtonState* __restrict__ ns, fmg_report* __restrict__ rep,
                                                     double* __restrict__ pq, double* __restrict__ ps,
                                                     unsigned* __restrict__ tickets, int level, int newton_max,
                                                     double tol) {
  static_assert(!(ELEM && FINISH), "element-rule passes leave the completion to k_newton_finish");
  static_assert(!(VAR && (FINISH || ELEM)), "variable-coefficient passes: vertex rule, separate completion");
  using AC = Acc<DIM>;
  extern __shared__ double smem[];
  __shared__ int is_last;
  // the state loads are issued together; a solve already done skips the pass
  const int done_in = SETUP ? 0 : ns->done;
  const double param = slot->param;
  if (!SETUP && done_in) return;
  const int bpc = 1 << s.bpc_log;
  const int cell = blockIdx.x >> s.bpc_log, chunk = blockIdx.x & (bpc - 1);
  const int t0 = chunk << s.npb_log, t1 = t0 + (1 << s.npb_log);
  if (SETUP) {
    // setup sums and the sums at y0 = (0, .., 0, 1) in one visit of the nodes
    double acc[AC::NS + AC::NQ];
#pragma unroll
    for (int q = 0; q < AC::NS + AC::NQ; ++q) acc[q] = 0.0;
    if (ELEM)
      setup_quad_accumulate_elem<DIM, KIND>(g, s, ut, slot->g, nf1, fs, scale, param, cell, t0, t1, threadIdx.x,
                                            blockDim.x, acc, acc + AC::NS);
    else if (VAR)
      setup_quad_accumulate_var<DIM, KIND>(g, s, ut, slot->g, slot->c, nf1, fs, slot->coef.w[level],
                                           slot->coef.plane[level], param, cell, t0, t1, threadIdx.x, blockDim.x,
                                           acc, acc + AC::NS);
    else
      setup_quad_accumulate<DIM, KIND>(g, s, ut, slot->g, nf1, fs, scale, param, cell, t0, t1, threadIdx.x,
                                       blockDim.x, acc, acc + AC::NS);
    double tot = block_sum_many<AC::NS + AC::NQ>(acc, smem);
    if (ELEM && threadIdx.x >= AC::NS) tot *= ElemRule<DIM>::W;
    if (threadIdx.x < AC::NS) ps[(size_t)blockIdx.x * AC::NS + threadIdx.x] = tot;
    else if (threadIdx.x < AC::NS + AC::NQ) pq[(size_t)blockIdx.x * AC::NQ + threadIdx.x - AC::NS] = tot;
  } else {
    double acc[AC::NQ];
#pragma unroll
    for (int q = 0; q < AC::NQ; ++q) acc[q] = 0.0;
    if (ELEM)
      quad_accumulate_elem<DIM, KIND>(g, s, ut, ns->ytry, param, cell, t0, t1, threadIdx.x, blockDim.x, acc);
    else if (VAR)
      quad_accumulate_var<DIM, KIND>(g, s, ut, ns->ytry, param, slot->c, nf1, cell, t0, t1, threadIdx.x,
                                     blockDim.x, acc);
    else
      quad_accumulate<DIM, KIND>(g, s, ut, ns->ytry, param, cell, t0, t1, threadIdx.x, blockDim.x, acc);
    double tot = block_sum_many<AC::NQ>(acc, smem);
    if (ELEM) tot *= ElemRule<DIM>::W;
    if (threadIdx.x < AC::NQ) pq[(size_t)blockIdx.x * AC::NQ + threadIdx.x] = tot;
  }
  // ---- the last block reduces every cell's partials and takes the Newton step ----
  __syncthreads();
  if (threadIdx.x == 0)
    is_last = __hip_atomic_fetch_add(&tickets[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) ==
              gridDim.x - 1u;
  __syncthreads();
  if (!is_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const int ncell = DIM == 2 ? s.nH * s.nH : s.nH * s.nH * s.nH;
  double* cs = smem;
  double* sm = cs + ncell * AC::NQ;
  double* tmp = sm + newton_scratch_doubles(s.N1);
  if (SETUP) {
    if (threadIdx.x == 0) newton_state_reset(ns, s.N1, level);
    setup_reduce<DIM>(s, ps, m, ns, cs, tmp);
  }
  cell_sums_from_partials<AC::NQ, sum_units<DIM>()>(pq, ncell, bpc, cs, tmp);
  newton_step_dev<DIM, VAR>(s, cs, A1, m, ns, rep, newton_max, tol, sm);
  if (FINISH) {
    // last pass of the launch sequence: this block completes the Newton solve
    // if it needs more passes, evaluating the fine quadrature by itself
    while (true) {
      __syncthreads();
      if (ns->done) break;
      quad_cells_by_waves<DIM, KIND>(g, s, ut, ns->ytry, param, cs);
      newton_step_dev<DIM>(s, cs, A1, m, ns, rep, newton_max, tol, sm);
    }
  }
  if (threadIdx.x == 0) __hip_atomic_store(&tickets[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-cell sums of all cells by one block.  A cell's r^d fine nodes are
// spread over a segment of LPC = min(64, r^d) lanes, so a wavefront holds
// 64 / LPC cells and reduces each accumulator over its segment only; the last
// lane of a segment writes the cell's sums.  No block barrier inside.
template <int DIM, int KIND, int LPC, bool ELEM, bool VAR>
__device__ __forceinline__ void quad_cells_seg(const Grid& g, const AugShape& s, const double* __restrict__ ut,
                                               const double* ytry, double param, double* cs,
                                               const ProblemSlot* __restrict__ slot) {
  using AC = Acc<DIM>;
  constexpr int CPW = 64 / LPC;
  const int ncell = DIM == 2 ? s.nH * s.nH : s.nH * s.nH * s.nH;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int sub = lane % LPC;
  const int nodes = 1 << (DIM * s.log2r);
  for (int c0 = wave * CPW; c0 < ncell; c0 += nw * CPW) {
    const int cell = c0 + lane / LPC;
    double acc[AC::NQ];
#pragma unroll
    for (int q = 0; q < AC::NQ; ++q) acc[q] = 0.0;
    if (cell < ncell) {
      if (ELEM) quad_accumulate_elem<DIM, KIND>(g, s, ut, ytry, param, cell, 0, nodes, sub, LPC, acc);
      else if (VAR)
        quad_accumulate_var<DIM, KIND>(g, s, ut, ytry, param, slot->c, slot->nf1, cell, 0, nodes, sub, LPC, acc);
      else quad_accumulate<DIM, KIND>(g, s, ut, ytry, param, cell, 0, nodes, sub, LPC, acc);
    }
#pragma unroll
    for (int q = 0; q < AC::NQ; ++q) {
      const double v = seg_sum<LPC>(acc[q]) * (ELEM ? ElemRule<DIM>::W : 1.0);
      if (sub == LPC - 1 && cell < ncell) cs[cell * AC::NQ + q] = v;
    }
  }
  __syncthreads();
}

template <int DIM, int KIND, bool ELEM, bool VAR>
__device__ __forceinline__ void quad_cells_by_waves(const Grid& g, const AugShape& s, const double* __restrict__ ut,
                                           const double* ytry, double param, double* cs,
                                           const ProblemSlot* __restrict__ slot) {
  const int nodes_log = DIM * s.log2r;
  if (nodes_log <= 2) quad_cells_seg<DIM, KIND, 4, ELEM, VAR>(g, s, ut, ytry, param, cs, slot);
  else if (nodes_log == 3) quad_cells_seg<DIM, KIND, 8, ELEM, VAR>(g, s, ut, ytry, param, cs, slot);
  else if (nodes_log == 4) quad_cells_seg<DIM, KIND, 16, ELEM, VAR>(g, s, ut, ytry, param, cs, slot);
  else if (nodes_log == 5) quad_cells_seg<DIM, KIND, 32, ELEM, VAR>(g, s, ut, ytry, param, cs, slot);
  else quad_cells_seg<DIM, KIND, 64, ELEM, VAR>(g, s, ut, ytry, param, cs, slot);
}

template <int DIM, int LPC>
__device__ __forceinline__ void setup_cells_seg(const Grid& g, const AugShape& s, const double* __restrict__ ut,
                                                const double* __restrict__ gl, int nf1, int fs, double scale,
                                                double* cs) {
  using AC = Acc<DIM>;
  constexpr int CPW = 64 / LPC;
  const int ncell = DIM == 2 ? s.nH * s.nH : s.nH * s.nH * s.nH;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int sub = lane % LPC;
  const int nodes = 1 << (DIM * s.log2r);
  for (int c0 = wave * CPW; c0 < ncell; c0 += nw * CPW) {
    const int cell = c0 + lane / LPC;
    double acc[AC::NS];
#pragma unroll
    for (int q = 0; q < AC::NS; ++q) acc[q] = 0.0;
    if (cell < ncell) setup_accumulate<DIM>(g, s, ut, gl, nf1, fs, scale, cell, 0, nodes, sub, LPC, acc);
#pragma unroll
    for (int q = 0; q < AC::NS; ++q) {
      const double v = seg_sum<LPC>(acc[q]);
      if (sub == LPC - 1 && cell < ncell) cs[cell * AC::NS + q] = v;
    }
  }
  __syncthreads();
}

template <int DIM>
__device__ __forceinline__ void setup_cells_by_waves(const Grid& g, const AugShape& s, const double* __restrict__ ut,
                                            const double* __restrict__ gl, int nf1, int fs, double scale,
                                            double* cs) {
  const int nodes_log = DIM * s.log2r;
  if (nodes_log <= 2) setup_cells_seg<DIM, 4>(g, s, ut, gl, nf1, fs, scale, cs);
  else if (nodes_log == 3) setup_cells_seg<DIM, 8>(g, s, ut, gl, nf1, fs, scale, cs);
  else if (nodes_log == 4) setup_cells_seg<DIM, 16>(g, s, ut, gl, nf1, fs, scale, cs);
  else if (nodes_log == 5) setup_cells_seg<DIM, 32>(g, s, ut, gl, nf1, fs, scale, cs);
  else setup_cells_seg<DIM, 64>(g, s, ut, gl, nf1, fs, scale, cs);
}

// Setup sums (to cs_s) and the quadrature sums at the Newton start z = u~ (to
// cs_q) of all cells in one visit of the nodes, segmented as quad_cells_seg.
template <int DIM, int KIND, int LPC>
__device__ __forceinline__ void setup_quad_cells_seg(const Grid& g, const AugShape& s, const double* __restrict__ ut,
                                                     const double* __restrict__ gl, int nf1, int fs, double scale,
                                                     double param, double* cs_s, double* cs_q) {
  using AC = Acc<DIM>;
  constexpr int CPW = 64 / LPC;
  const int ncell = DIM == 2 ? s.nH * s.nH : s.nH * s.nH * s.nH;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int sub = lane % LPC;
  const int nodes = 1 << (DIM * s.log2r);
  for (int c0 = wave * CPW; c0 < ncell; c0 += nw * CPW) {
    const int cell = c0 + lane / LPC;
    double acc[AC::NS + AC::NQ];
#pragma unroll
    for (int q = 0; q < AC::NS + AC::NQ; ++q) acc[q] = 0.0;
    if (cell < ncell)
      setup_quad_accumulate<DIM, KIND>(g, s, ut, gl, nf1, fs, scale, param, cell, 0, nodes, sub, LPC, acc,
                                       acc + AC::NS);
#pragma unroll
    for (int q = 0; q < AC::NS + AC::NQ; ++q) {
      const double v = seg_sum<LPC>(acc[q]);
      if (sub == LPC - 1 && cell < ncell) {
        if (q < AC::NS) cs_s[cell * AC::NS + q] = v;
        else cs_q[cell * AC::NQ + q - AC::NS] = v;
      }
    }
  }
  __syncthreads();
}

template <int DIM, int KIND>
__device__ __forceinline__ void setup_quad_cells_by_waves(const Grid& g, const AugShape& s,
                                                          const double* __restrict__ ut, const double* __restrict__ gl,
                                                          int nf1, int fs, double scale, double param, double* cs_s,
                                                          double* cs_q) {
  const int nodes_log = DIM * s.log2r;
  if (nodes_log <= 2) setup_quad_cells_seg<DIM, KIND, 4>(g, s, ut, gl, nf1, fs, scale, param, cs_s, cs_q);
  else if (nodes_log == 3) setup_quad_cells_seg<DIM, KIND, 8>(g, s, ut, gl, nf1, fs, scale, param, cs_s, cs_q);
  else if (nodes_log == 4) setup_quad_cells_seg<DIM, KIND, 16>(g, s, ut, gl, nf1, fs, scale, param, cs_s, cs_q);
  else if (nodes_log == 5) setup_quad_cells_seg<DIM, KIND, 32>(g, s, ut, gl, nf1, fs, scale, param, cs_s, cs_q);
  else setup_quad_cells_seg<DIM, KIND, 64>(g, s, ut, gl, nf1, fs, scale, param, cs_s, cs_q);
}

// Completes a Newton solve that the passes of the launch sequence did not
// finish: one block evaluates the fine quadrature itself (3D, and the element
// rule in 2D).
template <int DIM, int KIND, bool ELEM = false, bool VAR = false>
__global__ void __launch_bounds__(kBlock) k_newton_finish(Grid g, AugShape s, const double* __restrict__ ut,
                                                          const ProblemSlot* __restrict__ slot,
                                                          const double* __restrict__ A1, double m,
                                                          NewtonState* __restrict__ ns, fmg_report* __restrict__ rep,
                                                          int newton_max, double tol) {
  using AC = Acc<DIM>;
  extern __shared__ double smem[];
  const int ncell = DIM == 2 ? s.nH * s.nH : s.nH * s.nH * s.nH;
  double* cs = smem;
  double* sm = smem + ncell * AC::NQ;
  while (true) {
    __syncthreads();
    if (ns->done) return;
    quad_cells_by_waves<DIM, KIND, ELEM, VAR>(g, s, ut, ns->ytry, slot->param, cs, slot);
    newton_step_dev<DIM, VAR>(s, cs, A1, m, ns, rep, newton_max, tol, sm);
  }
}

// z = Q w + alpha u~ at node (i, j, l) of the level (0 on the boundary, where
// u~ and every interior coarse hat function vanish).
// Q w + alpha v at fine interior node (i, j, l) of a level with augmented-pass
// shape s, given the value v of u~ there.  The node lies in the Kuhn simplex
// of its coarse cell that follows the axes in order of decreasing local
// coordinate; only that simplex's d+1 vertices have nonzero hats there (the
// same values, added in the same vertex order, as the max/min hat formula).
template <int DIM>
__device__ __forceinline__ void kuhn_weights(const AugShape& s, int i, int j, int l, int& cx, int& cy, int& cz,
                                             int (&vtx)[DIM + 1], double (&lam)[DIM + 1]) {
  const int r = 1 << s.log2r;
  cx = min(i >> s.log2r, s.nH - 1);
  cy = min(j >> s.log2r, s.nH - 1);
  cz = DIM == 3 ? min(l >> s.log2r, s.nH - 1) : 0;
  // Local coordinates in units of the fine step; the barycentric weights are
  // their differences times 1/r = 2^-log2r (exact).
  const int t[3] = {i - cx * r, j - cy * r, DIM == 3 ? l - cz * r : 0};
  const double inv_r = __longlong_as_double((long long)(1023 - s.log2r) << 52);
  // axes by decreasing coordinate (ties keep the lower axis first)
  int p0 = 0, p1 = 1, p2 = 2;
  if (t[p1] > t[p0]) { const int q = p0; p0 = p1; p1 = q; }
  if (DIM == 3) {
    if (t[p2] > t[p1]) { const int q = p1; p1 = p2; p2 = q; }
    if (t[p1] > t[p0]) { const int q = p0; p0 = p1; p1 = q; }
  }
  vtx[0] = 0;
  lam[0] = (r - t[p0]) * inv_r;
  vtx[1] = 1 << p0;
  lam[1] = (t[p0] - t[p1]) * inv_r;
  if constexpr (DIM == 2) {
    vtx[2] = 3;
    lam[2] = t[p1] * inv_r;
  } else {
    vtx[2] = vtx[1] | (1 << p1);
    lam[2] = (t[p1] - t[p2]) * inv_r;
    vtx[3] = 7;
    lam[3] = t[p2] * inv_r;
  }
}

// The coefficients and weights of Q w + alpha v at fine node (i, j, l): all
// d+1 loads are issued before any is used (boundary vertices read y[0] and get
// weight 0), so a wave waits for one round trip, not d+1.
template <int DIM>
struct AugTerms {
  double w[DIM + 1], lam[DIM + 1], alpha;
};

template <int DIM>
__device__ __forceinline__ AugTerms<DIM> aug_gather(const AugShape& s, const double* __restrict__ y, int i, int j,
                                                    int l) {
  AugTerms<DIM> t;
  int cx, cy, cz, vtx[DIM + 1];
  kuhn_weights<DIM>(s, i, j, l, cx, cy, cz, vtx, t.lam);
#pragma unroll
  for (int c = 0; c <= DIM; ++c) {
    const int gi = coarse_vertex<DIM>(s.nH, cx, cy, cz, vtx[c]);
    t.w[c] = y[max(gi, 0)];
    if (gi < 0) t.lam[c] = 0.0;
  }
  t.alpha = y[s.N1];
  return t;
}

template <int DIM>
__device__ __forceinline__ double aug_apply(const AugTerms<DIM>& t, double v) {
  double z = t.alpha * v;
#pragma unroll
  for (int c = 0; c <= DIM; ++c) z += t.w[c] * t.lam[c];
  return z;
}

template <int DIM>
__device__ __forceinline__ double aug_combine(const AugShape& s, const double* __restrict__ y, double v, int i,
                                              int j, int l) {
  return aug_apply<DIM>(aug_gather<DIM>(s, y, i, j, l), v);
}

template <int DIM>
__device__ __forceinline__ double aug_value(const Grid& g, const AugShape& s, const double* __restrict__ y,
                                            const double* __restrict__ ut, int i, int j, int l) {
  return aug_combine<DIM>(s, y, ut[gidx<DIM>(g, i, j, l)], i, j, l);
}

// Level transition of Algorithm 3.2: u_k^(0) = P u_{k-1} (natural inclusion)
// and b_k = M_k (g - f(u_k^(0))).  With use_aug, u_{k-1} is the result of the
// last correction step on level k-1, Q w + alpha u~; since Q w lies in V_H,
// P (Q w + alpha u~) = Q w + alpha P u~, with Q w evaluated at the fine node
// (sf: the augmented-pass shape of level k).
// The transition's arguments: fine level (grid gf, augmented-pass shape sf,
// arrays uf, bf, load stride fs, mass m) from coarse u~ (grid gc, array uc).
struct TransitionArgs {
  Grid gc, gf;
  AugShape sf;
  const double* uc;
  double* uf;
  double* bf;
  int use_aug, nf1, fs;
  double m;
};

// AUG: a.use_aug, as a template argument so that the node's code has no
// branch and every load is issued before the first use.  CW: the weight c(x)
// of f(x, u) = c(x) f(u) (slot->c, nullptr means c = 1), as for k_rhs.
// STORE_U = false: only b is written (the first sweep pair of the level forms
// u_k^(0) itself).
template <int DIM, int KIND, bool AUG, bool CW = false, bool STORE_U = true>
__device__ __forceinline__ void transition_node(const TransitionArgs& a, const double* __restrict__ y,
                                                const ProblemSlot* __restrict__ slot, int i, int j, int l) {
  const int si = i & 1, sj = j & 1, sl = DIM == 3 ? (l & 1) : 0;
  const int pi = i >> 1, pj = j >> 1, pl = l >> 1;
  const long long fi = fine_load_index(a.nf1, a.fs, i, j, l);
  const double gv = slot->g[fi];
  AugTerms<DIM> t;
  if constexpr (AUG) t = aug_gather<DIM>(a.sf, y, i, j, l);
  // both coarse values are loaded; at a coarse node they are the same value,
  // and 0.5 (v0 + v0) = v0 exactly
  const double v0 = a.uc[gidx<DIM>(a.gc, pi, pj, pl)];
  const double v1 = a.uc[gidx<DIM>(a.gc, pi + si, pj + sj, pl + sl)];
  double v = 0.5 * (v0 + v1);
  if constexpr (AUG) v = aug_apply<DIM>(t, v);
  const int q = gidx<DIM>(a.gf, i, j, l);
  if (STORE_U) a.uf[q] = v;
  if constexpr (CW) {
    const double* __restrict__ cw = slot->c;
    a.bf[q] = a.m * (gv - (cw ? cw[fi] : 1.0) * NL<KIND>::f(v, slot->param));
  } else {
    a.bf[q] = a.m * (gv - NL<KIND>::f(v, slot->param));
  }
}

template <int DIM, int KIND, bool AUG, bool CW = false>
__global__ void __launch_bounds__(kBlock) k_transition(TransitionArgs a, const NewtonState* __restrict__ ns,
                                                       const ProblemSlot* __restrict__ slot) {
  int i, j, l;
  if (!node_of_thread<DIM>(a.gf, i, j, l)) return;
  transition_node<DIM, KIND, AUG, CW>(a, ns->y, slot, i, j, l);
}

// The transition's right-hand side b = M (g - f(P u_{k-1})) alone (3D float64
// sweep-pair levels, where the first pre-smoothing pair starts from P u_{k-1}).
template <int DIM, int KIND>
__global__ void __launch_bounds__(kBlock) k_transition_rhs(TransitionArgs a, const ProblemSlot* __restrict__ slot) {
  int i, j, l;
  if (!node_of_thread<DIM>(a.gf, i, j, l)) return;
  transition_node<DIM, KIND, false, false, false>(a, nullptr, slot, i, j, l);
}

// The same transition by the threads of one block (small fine levels, at the
// end of the single-workgroup kernel of the coarser level); y may be in LDS.
template <int DIM, int KIND>
__device__ __forceinline__ void transition_block(const TransitionArgs& a, const double* y,
                                                 const ProblemSlot* __restrict__ slot) {
  const int mm = a.gf.n - 1;
  const int total = DIM == 2 ? mm * mm : mm * mm * mm;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int i = 1 + t % mm, j = 1 + (t / mm) % mm, l = DIM == 3 ? 1 + t / (mm * mm) : 0;
    if (a.use_aug) transition_node<DIM, KIND, true>(a, y, slot, i, j, l);
    else transition_node<DIM, KIND, false>(a, y, slot, i, j, l);
  }
}

// u = Q w + alpha u~ at fine interior node (i, j, l) (in place on u~).
template <int DIM>
__device__ __forceinline__ void update_node(const Grid& g, const AugShape& s, const NewtonState* __restrict__ ns,
                                            double* __restrict__ ut, int i, int j, int l) {
  const double z = aug_value<DIM>(g, s, ns->y, ut, i, j, l);
  ut[gidx<DIM>(g, i, j, l)] = z;
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_aug_update(Grid g, AugShape s, const NewtonState* __restrict__ ns,
                                                       double* __restrict__ ut) {
  int i, j, l;
  if (!node_of_thread<DIM>(g, i, j, l)) return;
  update_node<DIM>(g, s, ns, ut, i, j, l);
}

// ---------------------------------------------------------------------------
// Algorithm 3.2, step 1: Newton on A_1 U + m_1 f(U) = m_1 g on level 1 (one
// block; same damping and stopping rules as the augmented solve).
// ---------------------------------------------------------------------------
// LDS doubles of level1_newton_dev.
__host__ __device__ constexpr int level1_lds_doubles(int N1) { return 2 * N1 * N1 + 8 * N1 + 4; }

template <int DIM, int KIND>
__device__ __forceinline__ void level1_newton_dev(const Grid& g1, int N1, const double* __restrict__ A1g, double m1,
                                  const ProblemSlot* __restrict__ slot, int nf1, int fs, double* __restrict__ x1,
                                  fmg_report* __restrict__ rep, int newton_max, double tol, double* smem) {
  double* A1 = smem;                // N1*N1
  double* J = A1 + N1 * N1;         // N1*N1
  double* R = J + N1 * N1;          // N1
  double* U = R + N1;               // N1
  double* G = U + N1;               // N1 (m g)
  double* D = G + N1;               // N1
  double* T = D + N1;               // N1 trial
  double* col = T + N1;             // N1 Cholesky column
  double* rdiag = col + N1;         // N1 reciprocal pivots
  double* sc = rdiag + N1;          // scalars: [0]=E [1]=scale [2]=done
  double* MC = sc + 4;              // N1: m c(x) at the nodes (c = 1 unless the problem gives c)
  const double q = slot->param;
  const double* __restrict__ cw = slot->c;
  for (int idx = threadIdx.x; idx < N1 * N1; idx += blockDim.x) A1[idx] = A1g[idx];
  for (int r = threadIdx.x; r < N1; r += blockDim.x) {
    const int mm = g1.n - 1;
    const int i = 1 + r % mm, j = 1 + (r / mm) % mm, l = DIM == 3 ? 1 + r / (mm * mm) : 0;
    const long long fi = fine_load_index(nf1, fs, i, j, l);
    G[r] = m1 * slot->g[fi];
    MC[r] = cw ? m1 * cw[fi] : m1;
    U[r] = 0.0;
  }
  __syncthreads();
  auto energy = [&](const double* V, double& E, double& S) {   // one thread
    double t1 = 0.0, t2 = 0.0, t3 = 0.0;
    for (int a = 0; a < N1; ++a) {
      double t = 0.0;
      for (int b = 0; b < N1; ++b) t += A1[a * N1 + b] * V[b];
      t1 += V[a] * t;
      double f, df, F;
      NL<KIND>::all(V[a], q, f, df, F);
      t2 += MC[a] * F;
      t3 += G[a] * V[a];
    }
    t1 *= 0.5;
    E = t1 + t2 - t3;
    S = fabs(t1) + fabs(t2) + fabs(t3);
  };
  if (threadIdx.x == 0) {
    energy(U, sc[0], sc[1]);
    sc[2] = 0.0;
  }
  __syncthreads();
  int it = 0;
  bool ok = false;
  for (it = 1; it <= newton_max; ++it) {
    for (int idx = threadIdx.x; idx < N1 * N1; idx += blockDim.x) J[idx] = A1[idx];
    __syncthreads();
    for (int a = threadIdx.x; a < N1; a += blockDim.x) {
      double t = 0.0;
      for (int b = 0; b < N1; ++b) t += A1[a * N1 + b] * U[b];
      double f, df, F;
      NL<KIND>::all(U[a], q, f, df, F);
      R[a] = t + MC[a] * f - G[a];
      J[a * N1 + a] += MC[a] * df;
      D[a] = -R[a];
    }
    __syncthreads();
    chol_steps_wave(J, col, rdiag, N1, N1);
    chol_solve_wave(J, rdiag, N1, N1, D);
    __syncthreads();
    if (threadIdx.x == 0) {
      // a small direction is applied in full without evaluating the energy there
      double dmax = 0.0, umax0 = 0.0;
      bool dfin = true;
      for (int a = 0; a < N1; ++a) {
        dmax = fmax(dmax, fabs(D[a]));
        umax0 = fmax(umax0, fabs(U[a]));
        dfin = dfin && isfinite(D[a]);
      }
      const bool small = dfin && dmax <= tol * fmax(1.0, umax0);
      double slope = 0.0;
      for (int a = 0; a < N1; ++a) slope += R[a] * D[a];
      double t = 1.0, E = sc[0], S = sc[1], Et = 0.0, St = 0.0;
      if (small) {
        for (int a = 0; a < N1; ++a) U[a] += D[a];
        sc[2] = 1.0;
      } else {
        for (int h = 0; h < kMaxHalvings; ++h) {
          for (int a = 0; a < N1; ++a) T[a] = U[a] + t * D[a];
          energy(T, Et, St);
          if (Et <= E + kArmijo * t * slope + kEnergyRounding * fmax(S, St)) break;
          t *= 0.5;
        }
        double stepmax = 0.0, umax = 0.0;
        for (int a = 0; a < N1; ++a) {
          stepmax = fmax(stepmax, fabs(T[a] - U[a]));
          U[a] = T[a];
          umax = fmax(umax, fabs(U[a]));
        }
        sc[0] = Et; sc[1] = St;
        sc[2] = (stepmax <= tol * fmax(1.0, umax)) ? 1.0 : 0.0;
        if (!isfinite(Et)) sc[2] = 2.0;
      }
    }
    __syncthreads();
    if (sc[2] != 0.0) { ok = sc[2] == 1.0; break; }
  }
  for (int r = threadIdx.x; r < N1; r += blockDim.x) x1[level1_node<DIM>(g1, r)] = U[r];
  if (threadIdx.x == 0) {
    rep->level1_iters = ok ? it : newton_max;
    if (!ok) report_status(rep, sc[2] == 2.0 ? FMG_E_NONFINITE : FMG_E_NOT_CONVERGED);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Solve bookkeeping
// ---------------------------------------------------------------------------
static __global__ void k_set_slot(ProblemSlot* slot, const double* g, double* u_out, fmg_report* rep_out, double param,
                           int kind, const double* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    slot->g = g; slot->u_out = u_out; slot->rep_out = rep_out; slot->param = param; slot->kind = kind;
    slot->c = c;
  }
}

// The hierarchy's part of the slot: finest nodes per side and the stencil
// arrays of the variable-coefficient operator (all nullptr for A = I).
static __global__ void k_init_slot(ProblemSlot* slot, int nf1, CoefLevels coef) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    slot->nf1 = nf1;
    slot->coef = coef;
    slot->c = nullptr;
  }
}

__device__ __forceinline__ void begin_solve_dev(fmg_report* rep, int levels, int* flag) {
  const int t = threadIdx.x;
  if (t == 0) {
    rep->status = 0; rep->levels = levels; rep->level1_iters = 0; rep->extra_steps = 0;
    rep->last_update_rel = 0.0;
    *flag = 0;
  }
  if (t < FMG_MAX_LEVELS) { rep->newton_iters[t] = 0; rep->newton_total[t] = 0; rep->alpha[t] = 0.0; }
}

static __global__ void k_begin_solve(fmg_report* rep, int levels, int* flag) { begin_solve_dev(rep, levels, flag); }

// Copy the finest solution out (packed layout, zero boundary) and flag
// NaN/Inf.  Blocks take whole grid rows (one division per row, none per
// node); with AUG the level's last update was deferred and Q w + alpha u~ is
// written directly.
template <int DIM, bool AUG>
__device__ __forceinline__ void output_rows(const Grid& g, const AugShape& s, const NewtonState* __restrict__ ns,
                                            const double* __restrict__ x, const ProblemSlot* __restrict__ slot,
                                            int* __restrict__ flag) {
  const int n1 = g.n + 1;
  const int rows = DIM == 2 ? n1 : n1 * n1;
  double* __restrict__ out = slot->u_out;
  int bad = 0;
  for (int r = blockIdx.x; r < rows; r += gridDim.x) {
    const int j = r % n1, l = DIM == 3 ? r / n1 : 0;
    const bool bnd_row = j == 0 || j == g.n || (DIM == 3 && (l == 0 || l == g.n));
    double* __restrict__ orow = out + (size_t)r * n1;
    for (int i = threadIdx.x; i < n1; i += blockDim.x) {
      double v = 0.0;
      if (!bnd_row && i != 0 && i != g.n)
        v = AUG ? aug_value<DIM>(g, s, ns->y, x, i, j, l) : x[gidx<DIM>(g, i, j, l)];
      bad |= !isfinite(v);
      orow[i] = v;
    }
  }
  if (bad) atomicOr(flag, 1);
}

// One block per grid row, so that all rows are in flight at once (a block that
// walked many rows would wait on each row's loads in turn).
template <int DIM>
inline int output_blocks(const Grid& g) { return DIM == 2 ? g.n + 1 : (g.n + 1) * (g.n + 1); }

template <int DIM>
__global__ void k_output(Grid g, const double* __restrict__ x, const ProblemSlot* __restrict__ slot,
                         int* __restrict__ flag) {
  output_rows<DIM, false>(g, AugShape{}, nullptr, x, slot, flag);
}

// Output of the final level when its last update was deferred.
template <int DIM>
__global__ void k_output_update(Grid g, AugShape s, const NewtonState* __restrict__ ns,
                                const double* __restrict__ ut, const ProblemSlot* __restrict__ slot,
                                int* __restrict__ flag) {
  output_rows<DIM, true>(g, s, ns, ut, slot, flag);
}

static __global__ void k_end_solve(fmg_report* rep, const int* flag, const ProblemSlot* slot) {
  if (threadIdx.x != 0) return;
  if (*flag) report_status(rep, FMG_E_NONFINITE);
  fmg_report* out = slot->rep_out;
  if (out) *out = *rep;
}

// Deterministic two-pass norms for the converged mode: block partials of
// sum (x - y)^2 and sum x^2 over interior nodes.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_diff_norm_partials(Grid g, const double* __restrict__ x,
                                                               const double* __restrict__ y,
                                                               double* __restrict__ partials) {
  __shared__ double lds[(kBlock / 64) * 2];
  int i, j, l;
  double acc[2] = {0.0, 0.0};
  if (node_of_thread<DIM>(g, i, j, l)) {
    const int c = gidx<DIM>(g, i, j, l);
    const double d = x[c] - y[c];
    acc[0] = d * d;
    acc[1] = x[c] * x[c];
  }
  const double t = block_sum_many<2>(acc, lds);
  if (threadIdx.x < 2) partials[(size_t)blockIdx.x * 2 + threadIdx.x] = t;
}

static __global__ void k_sum_pairs(const double* __restrict__ partials, size_t count, double* __restrict__ out) {
  __shared__ double lds[(kBlock / 64) * 2];
  double acc[2] = {0.0, 0.0};
  for (size_t b = threadIdx.x; b < count; b += blockDim.x) {
    acc[0] += partials[2 * b];
    acc[1] += partials[2 * b + 1];
  }
  const double t = block_sum_many<2>(acc, lds);
  if (threadIdx.x < 2) out[threadIdx.x] = t;
}

}  // namespace fmg
