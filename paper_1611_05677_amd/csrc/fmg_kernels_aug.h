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
#include "fmg_kernels_mg.h"

namespace fmg {

struct ProblemSlot {
  const double* g;        // finest nodal load, packed (nf+1)^d
  double* u_out;          // packed (nf+1)^d output
  fmg_report* rep_out;    // optional device-writable report copy
  double param;           // nonlinearity parameter
  int kind;
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
// fn(grid index c, local coordinates t[DIM], i, j, l).
template <int DIM, typename Fn>
__device__ __forceinline__ void for_cell_nodes(const Grid& g, const AugShape& s, int cx, int cy, int cz,
                                               int t0, int t1, int tid, int nthreads, Fn&& fn) {
  const int r = 1 << s.log2r, mask = r - 1;
  const double inv_r = 1.0 / r;
  for (int t = t0 + tid; t < t1; t += nthreads) {
    const int lx = t & mask, ly = (t >> s.log2r) & mask, lz = DIM == 3 ? t >> (2 * s.log2r) : 0;
    const int i = cx * r + lx, j = cy * r + ly, l = cz * r + lz;
    if (i == 0 || j == 0 || (DIM == 3 && l == 0)) continue;   // Dirichlet nodes
    double tl[3] = {lx * inv_r, ly * inv_r, lz * inv_r};
    fn(gidx<DIM>(g, i, j, l), tl, i, j, l);
  }
}

__device__ __forceinline__ long long fine_load_index(int nf1, int s, int i, int j, int l) {
  return ((long long)l * s * nf1 + (long long)j * s) * nf1 + (long long)i * s;
}

// ---------------------------------------------------------------------------
// Linearised right-hand side: b_j = m (g_j - f(u_j)) at level-k interior nodes.
// ---------------------------------------------------------------------------
template <int DIM, int KIND>
__global__ void __launch_bounds__(kBlock) k_rhs(Grid g, const ProblemSlot* __restrict__ slot, int nf1, int s,
                                                const double* __restrict__ u, double* __restrict__ b, double m) {
  int i, j, l;
  if (!node_of_thread<DIM>(g, i, j, l)) return;
  const int c = gidx<DIM>(g, i, j, l);
  const double gv = slot->g[fine_load_index(nf1, s, i, j, l)];
  b[c] = m * (gv - NL<KIND>::f(u[c], slot->param));
}

// ---------------------------------------------------------------------------
// Setup pass (once per correction step): per coarse cell
//   sum phi_a (A u~)_j, sum u~_j (A u~)_j, sum phi_a g_j, sum u~_j g_j.
// Block 0 also resets the Newton state to y = (0, ..., 0, 1), i.e. z = u~.
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_aug_setup(Grid g, AugShape s, const double* __restrict__ ut,
                                                      const ProblemSlot* __restrict__ slot, int nf1, int fs,
                                                      double scale, double* __restrict__ partials,
                                                      NewtonState* __restrict__ ns, int level) {
  using AC = Acc<DIM>;
  __shared__ double lds[(kBlock / 64) * AC::NS];
  const int cell = blockIdx.x >> s.bpc_log, chunk = blockIdx.x & ((1 << s.bpc_log) - 1);
  int cx, cy, cz;
  cell_of<DIM>(cell, s.nH, cx, cy, cz);
  double acc[AC::NS];
#pragma unroll
  for (int q = 0; q < AC::NS; ++q) acc[q] = 0.0;
  const int t0 = chunk << s.npb_log;
  const double* __restrict__ gl = slot->g;
  for_cell_nodes<DIM>(g, s, cx, cy, cz, t0, t0 + (1 << s.npb_log), threadIdx.x, blockDim.x,
                      [&](int c, const double* tl, int i, int j, int l) {
    double phi[AC::NV];
    kuhn_phi<DIM>(tl, phi);
    const double u = ut[c];
    const double au = apply_A_at<DIM>(ut, c, g, scale);
    const double gv = gl[fine_load_index(nf1, fs, i, j, l)];
#pragma unroll
    for (int a = 0; a < AC::NV; ++a) {
      acc[AC::S_BH + a] += phi[a] * au;
      acc[AC::S_GH + a] += phi[a] * gv;
    }
    acc[AC::S_C] += u * au;
    acc[AC::S_GU] += u * gv;
  });
  const double tot = block_sum_many<AC::NS>(acc, lds);
  if (threadIdx.x < AC::NS) partials[(size_t)blockIdx.x * AC::NS + threadIdx.x] = tot;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int q = 0; q < s.N1; ++q) { ns->y[q] = 0.0; ns->ytry[q] = 0.0; ns->d[q] = 0.0; }
    ns->y[s.N1] = 1.0;
    ns->ytry[s.N1] = 1.0;
    ns->d[s.N1] = 0.0;
    ns->iter = 0; ns->passes = 0; ns->halvings = 0; ns->done = 0; ns->ok = 0; ns->level = level;
    ns->t = 1.0; ns->E = 0.0; ns->Escale = 0.0; ns->slope = 0.0;
  }
}

// Per-cell quadrature sums at z = Q w + alpha u~ for one block's node range.
template <int DIM, int KIND>
__device__ __forceinline__ void quad_accumulate(const Grid& g, const AugShape& s, const double* __restrict__ ut,
                                                const double* ytry, double param, int cell, int t0, int t1,
                                                int tid, int nthreads, double* acc) {
  using AC = Acc<DIM>;
  using PR = Pairs<DIM>;
  int cx, cy, cz;
  cell_of<DIM>(cell, s.nH, cx, cy, cz);
  double wv[AC::NV];
#pragma unroll
  for (int a = 0; a < AC::NV; ++a) {
    const int gi = coarse_vertex<DIM>(s.nH, cx, cy, cz, a);
    wv[a] = gi >= 0 ? ytry[gi] : 0.0;
  }
  const double alpha = ytry[s.N1];
  for_cell_nodes<DIM>(g, s, cx, cy, cz, t0, t1, tid, nthreads, [&](int c, const double* tl, int, int, int) {
    double phi[AC::NV];
    kuhn_phi<DIM>(tl, phi);
    const double u = ut[c];
    double z = alpha * u;
#pragma unroll
    for (int a = 0; a < AC::NV; ++a) z += wv[a] * phi[a];
    double f, df, F;
    NL<KIND>::all(z, param, f, df, F);
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
  });
}

template <int DIM, int KIND>
__global__ void __launch_bounds__(kBlock) k_aug_quad(Grid g, AugShape s, const double* __restrict__ ut,
                                                     const ProblemSlot* __restrict__ slot,
                                                     const NewtonState* __restrict__ ns,
                                                     double* __restrict__ partials) {
  using AC = Acc<DIM>;
  if (ns->done) return;
  __shared__ double lds[(kBlock / 64) * AC::NQ];
  const int cell = blockIdx.x >> s.bpc_log, chunk = blockIdx.x & ((1 << s.bpc_log) - 1);
  double acc[AC::NQ];
#pragma unroll
  for (int q = 0; q < AC::NQ; ++q) acc[q] = 0.0;
  const int t0 = chunk << s.npb_log;
  quad_accumulate<DIM, KIND>(g, s, ut, ns->ytry, slot->param, cell, t0, t0 + (1 << s.npb_log), threadIdx.x,
                             blockDim.x, acc);
  const double tot = block_sum_many<AC::NQ>(acc, lds);
  if (threadIdx.x < AC::NQ) partials[(size_t)blockIdx.x * AC::NQ + threadIdx.x] = tot;
}

// ---------------------------------------------------------------------------
// Small dense linear algebra in LDS, one block.
// ---------------------------------------------------------------------------

// Right-looking Cholesky steps k = 0..kend-1 of the n x n matrix L (row-major,
// lower part used).  After kend = n-1 steps, L[n-1][n-1] is the Schur
// complement of the leading block.
__device__ inline void chol_steps(double* L, int n, int kend) {
  for (int k = 0; k < kend; ++k) {
    __syncthreads();
    const double s = sqrt(L[k * n + k]);
    __syncthreads();
    if (threadIdx.x == 0) L[k * n + k] = s;
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) L[i * n + k] /= s;
    __syncthreads();
    const int m = n - k - 1;
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
      const int i = k + 1 + idx / m, j = k + 1 + idx % m;
      if (j <= i) L[i * n + j] -= L[i * n + k] * L[j * n + k];
    }
  }
  __syncthreads();
}

// Solve L L^T x = rhs for the leading nn rows (thread 0; nn <= 64).
__device__ inline void chol_solve_serial(const double* L, int n, int nn, double* x) {
  if (threadIdx.x != 0) return;
  for (int i = 0; i < nn; ++i) {
    double s = x[i];
    for (int j = 0; j < i; ++j) s -= L[i * n + j] * x[j];
    x[i] = s / L[i * n + i];
  }
  for (int i = nn - 1; i >= 0; --i) {
    double s = x[i];
    for (int j = i + 1; j < nn; ++j) s -= L[j * n + i] * x[j];
    x[i] = s / L[i * n + i];
  }
}

// ---------------------------------------------------------------------------
// Newton step of the augmented problem (one block).  Inputs: per-cell
// quadrature sums `cs` (LDS, ncell x NQ) at the point ns->ytry.  Implements
// damped Newton with Armijo backtracking on E as a state machine, one
// evaluation per call: accept or halve the trial step, test convergence
// (|t d|_inf <= tol max(1, |y|_inf)), otherwise compute the next direction
// d = -J^{-1} R (dropping the u~ direction when its Schur complement is
// <= 1e-12 of J_uu) and the next trial point.
// LDS scratch `sm`: J (ny*ny) | R (ny) | 8 scalars.
// ---------------------------------------------------------------------------
template <int DIM>
__device__ void newton_core(const AugShape& s, const double* cs, const double* __restrict__ A1, double m,
                            NewtonState* ns, fmg_report* rep, int newton_max, double tol, double* sm) {
  using AC = Acc<DIM>;
  using PR = Pairs<DIM>;
  const int N1 = s.N1, ny = N1 + 1;
  const int ncell = DIM == 2 ? s.nH * s.nH : s.nH * s.nH * s.nH;
  double* J = sm;
  double* R = J + ny * ny;
  double* scal = R + ny;   // [0]=Nu [1]=kuu [2]=sumF [3]=E [4]=Escale [5]=schur [6]=Juu [7]=flag
  const double* y = ns->ytry;
  const double alpha = y[N1];

  // J <- A_1, R <- A_1 w (+ terms below)
  for (int idx = threadIdx.x; idx < ny * ny; idx += blockDim.x) J[idx] = 0.0;
  __syncthreads();
  for (int idx = threadIdx.x; idx < N1 * N1; idx += blockDim.x) {
    const int a = idx / N1, b = idx % N1;
    J[a * ny + b] = A1[idx];
  }
  for (int a = threadIdx.x; a < N1; a += blockDim.x) {
    double t = 0.0;
    for (int b = 0; b < N1; ++b) t += A1[a * N1 + b] * y[b];
    R[a] = t + alpha * ns->bH[a] - ns->GH[a];
  }
  __syncthreads();
  // scatter the per-cell sums, cells grouped in 2^d colours (cells of one
  // colour share no vertex), colours in a fixed order
  for (int colour = 0; colour < (1 << DIM); ++colour) {
    const int per = AC::NV + PR::N;
    for (int idx = threadIdx.x; idx < ncell * per; idx += blockDim.x) {
      const int cell = idx / per, item = idx % per;
      int cx, cy, cz;
      cell_of<DIM>(cell, s.nH, cx, cy, cz);
      const int col = (cx & 1) | ((cy & 1) << 1) | (DIM == 3 ? (cz & 1) << 2 : 0);
      if (col != colour) continue;
      const double* c = cs + cell * AC::NQ;
      if (item < AC::NV) {
        const int A = coarse_vertex<DIM>(s.nH, cx, cy, cz, item);
        if (A >= 0) {
          R[A] += m * c[AC::Q_NH + item];
          J[A * ny + N1] += m * c[AC::Q_KHU + item];
        }
      } else {
        const int p = item - AC::NV;
        const int A = coarse_vertex<DIM>(s.nH, cx, cy, cz, PR::a(p));
        const int B = coarse_vertex<DIM>(s.nH, cx, cy, cz, PR::b(p));
        if (A >= 0 && B >= 0) {
          const double v = m * c[AC::Q_K + p];
          J[A * ny + B] += v;
          if (A != B) J[B * ny + A] += v;
        }
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double Nu = 0.0, kuu = 0.0, sF = 0.0;
    for (int cell = 0; cell < ncell; ++cell) {
      Nu += cs[cell * AC::NQ + AC::Q_NU];
      kuu += cs[cell * AC::NQ + AC::Q_KUU];
      sF += cs[cell * AC::NQ + AC::Q_E];
    }
    double bw = 0.0, gw = 0.0, wAw = 0.0;
    for (int a = 0; a < N1; ++a) {
      bw += ns->bH[a] * y[a];
      gw += ns->GH[a] * y[a];
      double t = 0.0;
      for (int b = 0; b < N1; ++b) t += A1[a * N1 + b] * y[b];
      wAw += y[a] * t;
    }
    for (int a = 0; a < N1; ++a) {
      J[a * ny + N1] += ns->bH[a];
      J[N1 * ny + a] = J[a * ny + N1];
    }
    J[N1 * ny + N1] = ns->c + m * kuu;
    R[N1] = bw + alpha * ns->c + m * Nu - ns->Gu;
    const double t1 = 0.5 * wAw + alpha * bw + 0.5 * alpha * alpha * ns->c;
    const double t2 = m * sF;
    const double t3 = gw + alpha * ns->Gu;
    scal[3] = t1 + t2 - t3;
    scal[4] = fabs(t1) + fabs(t2) + fabs(t3);
    scal[6] = J[N1 * ny + N1];
    // ---- state machine: accept / reject the evaluated point ----
    int newdir = 0;
    const double Etry = scal[3], Stry = scal[4];
    bool finite = isfinite(Etry);
    for (int a = 0; a < ny; ++a) finite = finite && isfinite(R[a]);
    if (!finite) {
      ns->done = 1; ns->ok = 0;
      report_status(rep, FMG_E_NONFINITE);
    } else if (ns->passes == 0) {
      ns->E = Etry; ns->Escale = Stry;
      newdir = 1;
    } else if (Etry <= ns->E + kArmijo * ns->t * ns->slope + kEnergyRounding * fmax(ns->Escale, Stry)) {
      double stepmax = 0.0, ymax = 0.0;
      for (int a = 0; a < ny; ++a) {
        ns->y[a] = y[a];
        stepmax = fmax(stepmax, fabs(ns->t * ns->d[a]));
        ymax = fmax(ymax, fabs(y[a]));
      }
      ns->E = Etry; ns->Escale = Stry;
      if (stepmax <= tol * fmax(1.0, ymax)) { ns->done = 1; ns->ok = 1; }
      else newdir = 1;
    } else {
      ns->t *= 0.5;
      if (++ns->halvings > kMaxHalvings * newton_max) { ns->done = 1; ns->ok = 0; }
      for (int a = 0; a < ny; ++a) ns->ytry[a] = ns->y[a] + ns->t * ns->d[a];
    }
    if (newdir && ns->iter >= newton_max) { ns->done = 1; ns->ok = 0; newdir = 0; }
    scal[7] = newdir;
    ns->passes += 1;
    if (ns->done) {
      const int k = ns->level - 1;
      rep->newton_iters[k] = ns->iter;
      rep->newton_total[k] += ns->iter;
      rep->alpha[k] = ns->y[N1];
      if (!ns->ok) report_status(rep, FMG_E_NOT_CONVERGED);
    }
  }
  __syncthreads();
  if (scal[7] == 0.0) return;
  // ---- new direction: J d = -R at the accepted point (y == ytry here) ----
  chol_steps(J, ny, N1);                // leading block factored, J[N1][N1] = Schur complement
  if (threadIdx.x == 0) {
    const double schur = J[N1 * ny + N1];
    const bool drop = !(schur > kSchurDrop * scal[6]);
    scal[5] = drop ? 1.0 : 0.0;
    if (!drop) J[N1 * ny + N1] = sqrt(schur);
    for (int a = 0; a < ny; ++a) ns->d[a] = -R[a];
    const int nn = drop ? N1 : ny;
    chol_solve_serial(J, ny, nn, ns->d);
    if (drop) ns->d[N1] = 0.0;
    double slope = 0.0;
    for (int a = 0; a < ny; ++a) slope += R[a] * ns->d[a];
    ns->slope = slope;
    ns->t = 1.0;
    ns->iter += 1;
    for (int a = 0; a < ny; ++a) ns->ytry[a] = ns->y[a] + ns->d[a];
  }
  __syncthreads();
}

// Reduce the per-block partials of one pass into per-cell sums (fixed order).
template <int NACC>
__device__ inline void cell_sums_from_partials(const double* __restrict__ partials, int ncell, int bpc,
                                               double* cs) {
  for (int idx = threadIdx.x; idx < ncell * NACC; idx += blockDim.x) {
    const int cell = idx / NACC, q = idx % NACC;
    double t = 0.0;
    const double* p = partials + (size_t)cell * bpc * NACC + q;
    for (int b = 0; b < bpc; ++b) t += p[(size_t)b * NACC];
    cs[idx] = t;
  }
  __syncthreads();
}

// Fold the setup partials into Q^T A u~, u~^T A u~, Q^T M g, u~^T M g.
template <int DIM>
__device__ inline void setup_reduce(const AugShape& s, const double* __restrict__ partials_s, double m,
                                    NewtonState* ns, double* cs) {
  using AC = Acc<DIM>;
  const int ncell = DIM == 2 ? s.nH * s.nH : s.nH * s.nH * s.nH;
  cell_sums_from_partials<AC::NS>(partials_s, ncell, 1 << s.bpc_log, cs);
  for (int a = threadIdx.x; a < s.N1; a += blockDim.x) { ns->bH[a] = 0.0; ns->GH[a] = 0.0; }
  __syncthreads();
  for (int colour = 0; colour < (1 << DIM); ++colour) {
    for (int idx = threadIdx.x; idx < ncell * AC::NV; idx += blockDim.x) {
      const int cell = idx / AC::NV, a = idx % AC::NV;
      int cx, cy, cz;
      cell_of<DIM>(cell, s.nH, cx, cy, cz);
      const int col = (cx & 1) | ((cy & 1) << 1) | (DIM == 3 ? (cz & 1) << 2 : 0);
      if (col != colour) continue;
      const int A = coarse_vertex<DIM>(s.nH, cx, cy, cz, a);
      if (A < 0) continue;
      ns->bH[A] += cs[cell * AC::NS + AC::S_BH + a];
      ns->GH[A] += m * cs[cell * AC::NS + AC::S_GH + a];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double c = 0.0, gu = 0.0;
    for (int cell = 0; cell < ncell; ++cell) {
      c += cs[cell * AC::NS + AC::S_C];
      gu += cs[cell * AC::NS + AC::S_GU];
    }
    ns->c = c;
    ns->Gu = m * gu;
  }
  __syncthreads();
}

// One Newton step from the partials of the preceding quadrature pass.
template <int DIM>
__global__ void __launch_bounds__(256) k_newton_step(AugShape s, const double* __restrict__ partials_q,
                                                     const double* __restrict__ partials_s,
                                                     const double* __restrict__ A1, double m,
                                                     NewtonState* __restrict__ ns, fmg_report* __restrict__ rep,
                                                     int newton_max, double tol) {
  using AC = Acc<DIM>;
  if (ns->done) return;
  extern __shared__ double smem[];
  const int ncell = DIM == 2 ? s.nH * s.nH : s.nH * s.nH * s.nH;
  double* cs = smem;                        // ncell * max(NQ, NS)
  double* sm = smem + ncell * AC::NQ;
  if (ns->passes == 0) setup_reduce<DIM>(s, partials_s, m, ns, cs);
  cell_sums_from_partials<AC::NQ>(partials_q, ncell, 1 << s.bpc_log, cs);
  newton_core<DIM>(s, cs, A1, m, ns, rep, newton_max, tol, sm);
}

// Completes a Newton solve that the fixed number of passes did not finish:
// one block evaluates the fine quadrature itself, cell by cell.
template <int DIM, int KIND>
__global__ void __launch_bounds__(256) k_newton_finish(Grid g, AugShape s, const double* __restrict__ ut,
                                                       const ProblemSlot* __restrict__ slot,
                                                       const double* __restrict__ A1, double m,
                                                       NewtonState* __restrict__ ns, fmg_report* __restrict__ rep,
                                                       int newton_max, double tol) {
  using AC = Acc<DIM>;
  extern __shared__ double smem[];
  const int ncell = DIM == 2 ? s.nH * s.nH : s.nH * s.nH * s.nH;
  double* cs = smem;
  double* sm = smem + ncell * AC::NQ;
  double* red = sm + (s.N1 + 1) * (s.N1 + 1) + (s.N1 + 1) + 8;   // (256/64) * NQ
  const int nodes = 1 << (DIM * s.log2r);
  while (true) {
    __syncthreads();
    if (ns->done) return;
    for (int cell = 0; cell < ncell; ++cell) {
      double acc[AC::NQ];
#pragma unroll
      for (int q = 0; q < AC::NQ; ++q) acc[q] = 0.0;
      quad_accumulate<DIM, KIND>(g, s, ut, ns->ytry, slot->param, cell, 0, nodes, threadIdx.x, blockDim.x, acc);
      const double tot = block_sum_many<AC::NQ>(acc, red);
      if (threadIdx.x < AC::NQ) cs[cell * AC::NQ + threadIdx.x] = tot;
    }
    __syncthreads();
    newton_core<DIM>(s, cs, A1, m, ns, rep, newton_max, tol, sm);
  }
}

// u = Q w + alpha u~ at the fine interior nodes (in place on u~).
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_aug_update(Grid g, AugShape s, const NewtonState* __restrict__ ns,
                                                       double* __restrict__ ut) {
  int i, j, l;
  if (!node_of_thread<DIM>(g, i, j, l)) return;
  using AC = Acc<DIM>;
  const int r = 1 << s.log2r;
  const double inv_r = 1.0 / r;
  const int cx = min(i >> s.log2r, s.nH - 1), cy = min(j >> s.log2r, s.nH - 1),
            cz = DIM == 3 ? min(l >> s.log2r, s.nH - 1) : 0;
  double tl[3] = {(i - cx * r) * inv_r, (j - cy * r) * inv_r, DIM == 3 ? (l - cz * r) * inv_r : 0.0};
  double phi[AC::NV];
  kuhn_phi<DIM>(tl, phi);
  const int c = gidx<DIM>(g, i, j, l);
  double z = ns->y[s.N1] * ut[c];
#pragma unroll
  for (int a = 0; a < AC::NV; ++a) {
    const int gi = coarse_vertex<DIM>(s.nH, cx, cy, cz, a);
    if (gi >= 0) z += ns->y[gi] * phi[a];
  }
  ut[c] = z;
}

// ---------------------------------------------------------------------------
// Algorithm 3.2, step 1: Newton on A_1 U + m_1 f(U) = m_1 g on level 1 (one
// block; same damping and stopping rules as the augmented solve).
// ---------------------------------------------------------------------------
template <int DIM, int KIND>
__global__ void __launch_bounds__(256) k_level1_newton(Grid g1, int N1, const double* __restrict__ A1, double m1,
                                                       const ProblemSlot* __restrict__ slot, int nf1, int fs,
                                                       double* __restrict__ x1, fmg_report* __restrict__ rep,
                                                       int newton_max, double tol) {
  extern __shared__ double smem[];
  double* J = smem;                 // N1*N1
  double* R = J + N1 * N1;          // N1
  double* U = R + N1;               // N1
  double* G = U + N1;               // N1 (m g)
  double* D = G + N1;               // N1
  double* T = D + N1;               // N1 trial
  double* sc = T + N1;              // scalars: [0]=E [1]=scale [2]=done [3]=it
  const double q = slot->param;
  for (int r = threadIdx.x; r < N1; r += blockDim.x) {
    const int mm = g1.n - 1;
    const int i = 1 + r % mm, j = 1 + (r / mm) % mm, l = DIM == 3 ? 1 + r / (mm * mm) : 0;
    G[r] = m1 * slot->g[fine_load_index(nf1, fs, i, j, l)];
    U[r] = 0.0;
  }
  __syncthreads();
  auto energy = [&](const double* V, double& E, double& S) {   // thread 0
    double t1 = 0.0, t2 = 0.0, t3 = 0.0;
    for (int a = 0; a < N1; ++a) {
      double t = 0.0;
      for (int b = 0; b < N1; ++b) t += A1[a * N1 + b] * V[b];
      t1 += V[a] * t;
      double f, df, F;
      NL<KIND>::all(V[a], q, f, df, F);
      t2 += m1 * F;
      t3 += G[a] * V[a];
    }
    t1 *= 0.5;
    E = t1 + t2 - t3;
    S = fabs(t1) + fabs(t2) + fabs(t3);
  };
  if (threadIdx.x == 0) {
    energy(U, sc[0], sc[1]);
    sc[2] = 0.0;
    sc[3] = 0.0;
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
      R[a] = t + m1 * f - G[a];
      J[a * N1 + a] += m1 * df;
    }
    __syncthreads();
    chol_steps(J, N1, N1);
    if (threadIdx.x == 0) {
      for (int a = 0; a < N1; ++a) D[a] = -R[a];
      chol_solve_serial(J, N1, N1, D);
      double slope = 0.0;
      for (int a = 0; a < N1; ++a) slope += R[a] * D[a];
      double t = 1.0, E = sc[0], S = sc[1], Et = 0.0, St = 0.0;
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
    __syncthreads();
    if (sc[2] != 0.0) { ok = sc[2] == 1.0; break; }
  }
  for (int r = threadIdx.x; r < N1; r += blockDim.x) x1[level1_node<DIM>(g1, r)] = U[r];
  if (threadIdx.x == 0) {
    rep->level1_iters = ok ? it : newton_max;
    if (!ok) report_status(rep, sc[2] == 2.0 ? FMG_E_NONFINITE : FMG_E_NOT_CONVERGED);
  }
}

// ---------------------------------------------------------------------------
// Solve bookkeeping
// ---------------------------------------------------------------------------
__global__ void k_set_slot(ProblemSlot* slot, const double* g, double* u_out, fmg_report* rep_out, double param,
                           int kind) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    slot->g = g; slot->u_out = u_out; slot->rep_out = rep_out; slot->param = param; slot->kind = kind;
  }
}

__global__ void k_begin_solve(fmg_report* rep, int levels, int* flag) {
  const int t = threadIdx.x;
  if (t == 0) {
    rep->status = 0; rep->levels = levels; rep->level1_iters = 0; rep->extra_steps = 0;
    rep->last_update_rel = 0.0;
    *flag = 0;
  }
  if (t < FMG_MAX_LEVELS) { rep->newton_iters[t] = 0; rep->newton_total[t] = 0; rep->alpha[t] = 0.0; }
}

// Copy the finest solution out (packed layout, zero boundary) and flag NaN/Inf.
template <int DIM>
__global__ void k_output(Grid g, const double* __restrict__ x, const ProblemSlot* __restrict__ slot,
                         int* __restrict__ flag) {
  const int n1 = g.n + 1;
  const size_t total = DIM == 2 ? (size_t)n1 * n1 : (size_t)n1 * n1 * n1;
  double* __restrict__ out = slot->u_out;
  int bad = 0;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(p % n1), j = (int)((p / n1) % n1), l = DIM == 3 ? (int)(p / ((size_t)n1 * n1)) : 0;
    const bool bnd = i == 0 || j == 0 || i == g.n || j == g.n || (DIM == 3 && (l == 0 || l == g.n));
    const double v = bnd ? 0.0 : x[gidx<DIM>(g, i, j, l)];
    bad |= !isfinite(v);
    out[p] = v;
  }
  if (bad) atomicOr(flag, 1);
}

__global__ void k_end_solve(fmg_report* rep, const int* flag, const ProblemSlot* slot) {
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
  const size_t b = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  if (threadIdx.x < 2) partials[b * 2 + threadIdx.x] = t;
}

__global__ void k_sum_pairs(const double* __restrict__ partials, size_t count, double* __restrict__ out) {
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
