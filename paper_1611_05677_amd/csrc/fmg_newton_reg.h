// Register-resident small dense Newton solves for a coarse grid of 4 cells per
// side (N_1 = 9 unknowns in 2D, 27 in 3D), executed by one wavefront.  Lane A
// owns coarse unknown A (and lane N_1 the coefficient alpha of u~): its row
// of the Newton matrix lives in registers, A_1 w comes from the coarse
// stencil through lane shuffles, and Gauss-Jordan elimination broadcasts the
// pivot row with lane reads, so no backward substitution is needed.
// Same damping, stopping and degenerate-direction rules as newton_core.
#pragma once

#include "fmg_kernels_aug.h"

namespace fmg {

// Coarse-stencil product (A_1 v)_A = s1 (2d v_A - sum of axis neighbours) for
// the lane's own node A (mm = nH - 1 nodes per side); lanes >= N1 return 0.
template <int DIM>
__device__ __forceinline__ double stencil_shfl(double v, int A, int ax, int ay, int az, int mm, bool node,
                                               double s1) {
  const int lane = threadIdx.x;
  auto sh = [&](int src, bool ok) {
    const double r = __shfl(v, ok ? src : lane, 64);
    return ok ? r : 0.0;
  };
  double nb = (sh(A - 1, ax > 1) + sh(A + 1, ax < mm)) + (sh(A - mm, ay > 1) + sh(A + mm, ay < mm));
  if (DIM == 3) nb += sh(A - mm * mm, az > 1) + sh(A + mm * mm, az < mm);
  return node ? s1 * (2.0 * DIM * v - nb) : 0.0;
}

// A general A_1 (variable coefficient): on the Kuhn meshes row A couples only
// nodes at offsets in {-1,0,1}^d, so the lane keeps those entries, a1q[q] at
// box offset q = (dx+1) + 3 (dy+1) (+ 9 (dz+1)), zero outside the grid.
template <int DIM> constexpr int box_size() { return DIM == 2 ? 9 : 27; }

template <int DIM>
__device__ __forceinline__ void box_row(const double* __restrict__ A1g, int N1, int A, int ax, int ay, int az,
                                        int mm, bool node, double (&a1q)[box_size<DIM>()]) {
#pragma unroll
  for (int q = 0; q < box_size<DIM>(); ++q) {
    const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = DIM == 3 ? q / 9 - 1 : 0;
    const int bx = ax + dx, by = ay + dy, bz = az + dz;
    const bool in = node && bx >= 1 && bx <= mm && by >= 1 && by <= mm && (DIM == 2 || (bz >= 1 && bz <= mm));
    const int B = A + dx + mm * dy + mm * mm * dz;
    a1q[q] = in ? A1g[(size_t)A * N1 + B] : 0.0;
  }
}

// (A_1 v)_A from the lane's box row (lanes without a node return 0).
template <int DIM>
__device__ __forceinline__ double box_apply_shfl(double v, int A, int mm, const double (&a1q)[box_size<DIM>()]) {
  const int lane = threadIdx.x;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < box_size<DIM>(); ++q) {
    const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = DIM == 3 ? q / 9 - 1 : 0;
    const int B = A + dx + mm * dy + mm * mm * dz;
    const double r = __shfl(v, (B >= 0 && B < 64) ? B : lane, 64);
    s += a1q[q] * r;
  }
  return s;
}

// Gauss-Jordan elimination without pivoting of the symmetric positive definite
// NY x NY system J x = b whose row `lane` is jr[] (full rows; lanes >= NY
// hold zero rows) and whose right-hand side entry `lane` is v.  Steps
// k = 0..NY-2 eliminate column k from every other row (rows above the pivot
// too, so no backward substitution follows); all pivots are positive, being
// those of the Cholesky factorisation squared.  On exit lane i < NY-1 holds
// its pivot in piv and, in jr[NY-1], its remaining coupling to the last
// unknown; the return value, in every lane, is the last pivot: the Schur
// complement of the leading (NY-1) x (NY-1) block.  gj_finish then gives x.
template <int NY>
__device__ __forceinline__ double gj_elim_reg(double (&jr)[NY], double& piv, double& v) {
  const int lane = threadIdx.x;
#pragma unroll
  for (int k = 0; k < NY - 1; ++k) {
    const double pk = lane_value(jr[k], k);
    const double f = lane == k ? 0.0 : jr[k] * fast_rcp(pk);
    if (lane == k) piv = pk;
    v -= f * lane_value(v, k);
#pragma unroll
    for (int j = k + 1; j < NY; ++j) jr[j] -= f * lane_value(jr[j], k);
  }
  const double schur = lane_value(jr[NY - 1], NY - 1);
  if (lane == NY - 1) piv = schur;
  return schur;
}

// Solution entry of lane `lane` after gj_elim_reg: the last unknown is
// v_last / schur, or 0 when keep_last is false (the other entries then solve
// the leading (NY-1) x (NY-1) system alone); 0 for lanes >= NY.
template <int NY>
__device__ __forceinline__ double gj_finish(const double (&jr)[NY], double piv, double v, bool keep_last) {
  const int lane = threadIdx.x;
  const double xl = keep_last ? lane_value(v, NY - 1) / lane_value(piv, NY - 1) : 0.0;
  if (lane == NY - 1) return xl;
  return lane < NY ? (v - jr[NY - 1] * xl) / piv : 0.0;
}

// Pair index of cell vertices (a, b), a subset of b, as a constant expression.
template <int DIM>
__host__ __device__ constexpr int pair_of(int a, int b) {
  int p = 0;
  for (int x = 0; x < (1 << DIM); ++x)
    for (int y = x; y < (1 << DIM); ++y)
      if ((x & y) == x) {
        if (x == a && y == b) return p;
        ++p;
      }
  return -1;
}

// Newton step (see newton_core) with the state in registers.  LDS: J ((NY + 1) rows of NY | 1).
// GEN: A_1 is the general matrix A1g (variable coefficient), not the stencil.
template <int DIM, int NY, bool GEN = false>
__device__ __forceinline__ void newton_core_reg(const AugShape& s, const double* cs, double m, NewtonState* nsg,
                                                fmg_report* rep, int newton_max, double tol, double* sm,
                                                const double* __restrict__ A1g = nullptr) {
  if (threadIdx.x >= 64) return;
  using AC = Acc<DIM>;
  constexpr int N1 = NY - 1;
  constexpr int NV = AC::NV;
  const int lane = threadIdx.x;
  const int nH = s.nH, mm = nH - 1;
  const int ncell = DIM == 2 ? nH * nH : nH * nH * nH;
  const double s1 = DIM == 2 ? 1.0 : 1.0 / nH;
  const bool act = lane < NY, node = lane < N1;
  double* J = sm;
  constexpr int JS = NY | 1;   // odd row stride: lanes reading their rows hit distinct LDS banks
  // ---- state ----
  const double yt = act ? nsg->ytry[lane] : 0.0;
  const double yold = act ? nsg->y[lane] : 0.0;
  const double dold = act ? nsg->d[lane] : 0.0;
  const double bh = node ? nsg->bH[lane] : 0.0;
  const double gh = node ? nsg->GH[lane] : 0.0;
  const double c = nsg->c, Gu = nsg->Gu, E = nsg->E, Escale = nsg->Escale, slope0 = nsg->slope, t = nsg->t;
  const int iter = nsg->iter, passes = nsg->passes;
  const double alpha = lane_value(yt, N1);
  const double w = node ? yt : 0.0;
  const int A = node ? lane : 0;
  int ax, ay, az;
  coarse_coords<DIM>(nH, A, ax, ay, az);
  // ---- residual and the J column of u~ ----
  double a1q[box_size<DIM>()];
  if constexpr (GEN) box_row<DIM>(A1g, N1, A, ax, ay, az, mm, node, a1q);
  const double Aw = GEN ? box_apply_shfl<DIM>(w, A, mm, a1q) : stencil_shfl<DIM>(w, A, ax, ay, az, mm, node, s1);
  double nh = 0.0, khu = 0.0;
  double st[DIM == 2 ? 9 : 27];   // m f' phi_A phi_B by offset B - A in {-1,0,1}^d
#pragma unroll
  for (int q = 0; q < (DIM == 2 ? 9 : 27); ++q) st[q] = 0.0;
  if (node) {
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      const int cx = ax - (e & 1), cy = ay - ((e >> 1) & 1), cz = DIM == 3 ? az - ((e >> 2) & 1) : 0;
      const double* cc = cs + (cx + nH * (cy + nH * cz)) * AC::NQ;
      nh += cc[AC::Q_NH + e];
      khu += cc[AC::Q_KHU + e];
#pragma unroll
      for (int f = 0; f < NV; ++f) {
        const int lo = e < f ? e : f, hi = e < f ? f : e;
        if ((lo & hi) != lo) continue;                  // not in a common simplex
        const int p = pair_of<DIM>(lo, hi);
        const int dx = (f & 1) - (e & 1), dy = ((f >> 1) & 1) - ((e >> 1) & 1),
                  dz = DIM == 3 ? ((f >> 2) & 1) - ((e >> 2) & 1) : 0;
        const int q = (dx + 1) + 3 * (dy + 1) + (DIM == 3 ? 9 * (dz + 1) : 0);
        st[q] += cc[AC::Q_K + p];
      }
    }
  }
  const double R = node ? Aw + alpha * bh - gh + m * nh : 0.0;
  const double jAu = node ? bh + m * khu : 0.0;      // J[A][N1]
  // ---- scalars (wave sums) ----
  double nu = 0.0, kuu = 0.0, sF = 0.0;
  for (int cidx = lane; cidx < ncell; cidx += 64) {
    nu += cs[cidx * AC::NQ + AC::Q_NU];
    kuu += cs[cidx * AC::NQ + AC::Q_KUU];
    sF += cs[cidx * AC::NQ + AC::Q_E];
  }
  double sums[6] = {nu, kuu, sF, bh * w, gh * w, w * Aw};
  wave_sum_n<6>(sums);
  nu = sums[0]; kuu = sums[1]; sF = sums[2];
  const double bw = sums[3], gw = sums[4], wAw = sums[5];
  const double Juu = c + m * kuu;
  const double Ru = bw + alpha * c + m * nu - Gu;
  const double Rl = lane == N1 ? Ru : R;
  const double t1 = 0.5 * wAw + alpha * bw + 0.5 * alpha * alpha * c;
  const double t2 = m * sF;
  const double t3 = gw + alpha * Gu;
  const double Etry = t1 + t2 - t3, Stry = fabs(t1) + fabs(t2) + fabs(t3);
  // ---- state machine (uniform decisions) ----
  const bool finite = __all(isfinite(Etry) && isfinite(Rl));
  int newdir = 0, done = 0, ok = 0, halve = 0;
  if (!finite) {
    done = 1;
  } else if (passes == 0) {
    newdir = 1;
  } else if (Etry <= E + kArmijo * t * slope0 + kEnergyRounding * fmax(Escale, Stry)) {
    double mx[2] = {act ? fabs(t * dold) : 0.0, act ? fabs(yt) : 0.0};
    wave_max_n<2>(mx);
    if (mx[0] <= tol * fmax(1.0, mx[1])) { done = 1; ok = 1; }
    else newdir = 1;
  } else {
    halve = 1;
  }
  if (newdir && iter >= newton_max) { done = 1; ok = 0; newdir = 0; }
  const bool accept = finite && !halve;
  double ynew = accept ? yt : yold;                  // accepted iterate
  double ytry_new = yt, dnew = dold, tnew = t, slope = slope0;
  int halvings = nsg->halvings;
  if (halve) {
    tnew = 0.5 * t;
    ytry_new = ynew + tnew * dold;
    if (++halvings > kMaxHalvings * newton_max) { done = 1; ok = 0; }
  }
  if (newdir) {
    // rows of J in LDS, then in registers; the lanes without a row use a
    // scratch row NY (zeros), so no store or load needs a lane mask
    const int row = act ? lane : NY;
#pragma unroll
    for (int B = 0; B < NY; ++B) J[row * JS + B] = 0.0;
    wave_sync();
    if (node) {
#pragma unroll
      for (int q = 0; q < (DIM == 2 ? 9 : 27); ++q) {
        const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = DIM == 3 ? q / 9 - 1 : 0;
        const int bx = ax + dx, by = ay + dy, bz = az + dz;
        if (bx < 1 || bx > mm || by < 1 || by > mm || (DIM == 3 && (bz < 1 || bz > mm))) continue;
        const int B = A + dx + mm * dy + mm * mm * dz;
        const int nz = (dx != 0) + (dy != 0) + (dz != 0);
        const double a1 = GEN ? a1q[q] : (nz == 0 ? 2.0 * DIM * s1 : (nz == 1 ? -s1 : 0.0));
        J[A * JS + B] = a1 + m * st[q];
      }
      J[A * JS + N1] = jAu;
      J[N1 * JS + A] = jAu;
    }
    if (lane == N1) J[N1 * JS + N1] = Juu;
    wave_sync();
    double jr[NY];
#pragma unroll
    for (int B = 0; B < NY; ++B) jr[B] = J[row * JS + B];
    wave_sync();
    double piv = 1.0, v = act ? -Rl : 0.0;
    const double schur = gj_elim_reg<NY>(jr, piv, v);
    const bool drop = !(schur > kSchurDrop * Juu);
    const double dv = gj_finish<NY>(jr, piv, v, !drop);
    dnew = dv;
    slope = wave_allsum(Rl * dv);
    tnew = 1.0;
    ytry_new = ynew + dv;
    // a small direction is applied in full without evaluating the energy there
    const bool dfin = __all(isfinite(dv));
    double mx[2] = {act ? fabs(dv) : 0.0, act ? fabs(ynew) : 0.0};
    wave_max_n<2>(mx);
    if (dfin && mx[0] <= tol * fmax(1.0, mx[1])) {
      ynew = ytry_new;
      done = 1;
      ok = 1;
    }
  }
  const int iter_new = iter + (newdir ? 1 : 0);
  // ---- write back ----
  if (act) {
    nsg->y[lane] = ynew;
    nsg->ytry[lane] = ytry_new;
    nsg->d[lane] = dnew;
  }
  const double alpha_new = lane_value(ynew, N1);
  if (lane == 0) {
    if (accept) { nsg->E = Etry; nsg->Escale = Stry; }
    nsg->t = tnew;
    nsg->slope = slope;
    nsg->halvings = halvings;
    nsg->passes = passes + 1;
    nsg->iter = iter_new;
    nsg->done = done;
    nsg->ok = ok;
    if (done) {
      const int k = nsg->level - 1;
      rep->newton_iters[k] = iter_new;
      rep->newton_total[k] += iter_new;
      rep->alpha[k] = alpha_new;
      if (k == 0) rep->level1_iters = iter_new;   // level 1 solved as the augmented problem with u~ = 0
      if (!finite) report_status(rep, FMG_E_NONFINITE);
      else if (!ok) report_status(rep, FMG_E_NOT_CONVERGED);
    }
  }
}

// Algorithm 3.2, step 1 with the state in registers (see level1_newton_dev):
// lane A owns U_A; N1 = 9 (2D) or 27 (3D), i.e. 4 coarse cells per side.
// GEN: A_1 is the general matrix A1g and f is weighted by c(x) (slot->c).
template <int DIM, int KIND, int N1, bool GEN = false>
__device__ __forceinline__ void level1_newton_reg(const Grid& g1, double m1, const ProblemSlot* __restrict__ slot,
                                                  int nf1, int fs, double* __restrict__ x1,
                                                  fmg_report* __restrict__ rep, int newton_max, double tol,
                                                  double* sm, const double* __restrict__ A1g = nullptr) {
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  const bool node = lane < N1;
  const int nH = g1.n, mm = nH - 1;
  const double s1 = DIM == 2 ? 1.0 : 1.0 / nH;
  const double q = slot->param;
  const int A = node ? lane : 0;
  int ax, ay, az;
  coarse_coords<DIM>(nH, A, ax, ay, az);
  const long long fi = fine_load_index(nf1, fs, ax, ay, az);
  const double G = node ? m1 * slot->g[fi] : 0.0;
  double arow[GEN ? N1 : 1];        // row A of the general A_1 (GEN)
  double cA = 1.0;                 // c(x_A) (GEN)
  if constexpr (GEN) {
#pragma unroll
    for (int B = 0; B < N1; ++B) arow[B] = node ? A1g[(size_t)A * N1 + B] : 0.0;
    if (slot->c && node) cA = slot->c[fi];
  }
  auto apply = [&](double V) {
    if constexpr (GEN) {
      double sum = 0.0;
#pragma unroll
      for (int B = 0; B < N1; ++B) sum += arow[B] * lane_value(V, B);
      return node ? sum : 0.0;
    } else {
      return stencil_shfl<DIM>(V, A, ax, ay, az, mm, node, s1);
    }
  };
  auto energy = [&](double V, double& Eo, double& So) {
    const double AV = apply(V);
    double f, df, F;
    NL<KIND>::all(V, q, f, df, F);
    double sums[3] = {node ? V * AV : 0.0, node ? (GEN ? cA * F : F) : 0.0, G * V};
    wave_sum_n<3>(sums);
    const double t1 = 0.5 * sums[0];
    const double t2 = m1 * sums[1];
    const double t3 = sums[2];
    Eo = t1 + t2 - t3;
    So = fabs(t1) + fabs(t2) + fabs(t3);
  };
  double U = 0.0, E, S;
  energy(U, E, S);
  int it = 0, status = 0;   // 1 converged, 2 non-finite
  for (it = 1; it <= newton_max; ++it) {
    double f, df, F;
    NL<KIND>::all(U, q, f, df, F);
    if (GEN) { f *= cA; df *= cA; }
    const double R = node ? apply(U) + m1 * f - G : 0.0;
    double jr[N1];
#pragma unroll
    for (int B = 0; B < N1; ++B) {
      const int bx = 1 + B % 3, by = 1 + (B / 3) % 3, bz = DIM == 3 ? 1 + B / 9 : 0;
      const int nz = abs(bx - ax) + abs(by - ay) + abs(bz - az);
      if constexpr (GEN) {
        jr[B] = !node ? 0.0 : arow[B] + (nz == 0 ? m1 * df : 0.0);
      } else {
        jr[B] = !node ? 0.0 : (nz == 0 ? 2.0 * DIM * s1 + m1 * df : (nz == 1 ? -s1 : 0.0));
      }
    }
    double piv = 1.0, v = node ? -R : 0.0;
    gj_elim_reg<N1>(jr, piv, v);
    const double D = gj_finish<N1>(jr, piv, v, true);
    {   // a small direction is applied in full without evaluating the energy there
      const bool dfin = __all(isfinite(D));
      double mx[2] = {node ? fabs(D) : 0.0, node ? fabs(U) : 0.0};
      wave_max_n<2>(mx);
      if (dfin && mx[0] <= tol * fmax(1.0, mx[1])) {
        U = U + D;
        status = 1;
        break;
      }
    }
    const double slope = wave_allsum(R * D);
    double t = 1.0, Et = 0.0, St = 0.0, T = U;
    for (int h = 0; h < kMaxHalvings; ++h) {
      T = U + t * D;
      energy(T, Et, St);
      if (Et <= E + kArmijo * t * slope + kEnergyRounding * fmax(S, St)) break;
      t *= 0.5;
    }
    double mx[2] = {node ? fabs(T - U) : 0.0, node ? fabs(T) : 0.0};
    wave_max_n<2>(mx);
    const double stepmax = mx[0], umax = mx[1];
    U = T;
    E = Et;
    S = St;
    if (!isfinite(Et)) { status = 2; break; }
    if (stepmax <= tol * fmax(1.0, umax)) { status = 1; break; }
  }
  if (node) x1[gidx<DIM>(g1, ax, ay, az)] = U;
  if (lane == 0) {
    rep->level1_iters = status == 1 ? it : newton_max;
    if (status != 1) report_status(rep, status == 2 ? FMG_E_NONFINITE : FMG_E_NOT_CONVERGED);
  }
}

template <int DIM, int KIND>
__device__ __forceinline__ void level1_dispatch(const Grid& g1, int N1, const double* __restrict__ A1g, double m1,
                                                const ProblemSlot* __restrict__ slot, int nf1, int fs,
                                                double* __restrict__ x1, fmg_report* __restrict__ rep,
                                                int newton_max, double tol, double* smem) {
  // A = I and c = 1: the stencil; otherwise the general A_1 (and c(x))
  const bool plain = slot->coef.w[1] == nullptr && slot->c == nullptr;
  if (DIM == 2 && N1 == 9 && plain)
    level1_newton_reg<DIM, KIND, 9>(g1, m1, slot, nf1, fs, x1, rep, newton_max, tol, smem);
  else if (DIM == 3 && N1 == 27 && plain)
    level1_newton_reg<DIM, KIND, 27>(g1, m1, slot, nf1, fs, x1, rep, newton_max, tol, smem);
  else if (DIM == 2 && N1 == 9)
    level1_newton_reg<DIM, KIND, 9, true>(g1, m1, slot, nf1, fs, x1, rep, newton_max, tol, smem, A1g);
  else if (DIM == 3 && N1 == 27)
    level1_newton_reg<DIM, KIND, 27, true>(g1, m1, slot, nf1, fs, x1, rep, newton_max, tol, smem, A1g);
  else level1_newton_dev<DIM, KIND>(g1, N1, A1g, m1, slot, nf1, fs, x1, rep, newton_max, tol, smem);
  __syncthreads();
}

// Dispatch: register-resident step for the 4-cell coarse grids, LDS step
// otherwise.  GEN (the variable-coefficient kernels): the register step with
// the general A_1.
template <int DIM, bool GEN>
__device__ __forceinline__ void newton_step_dev(const AugShape& s, const double* cs, const double* __restrict__ A1,
                                                double m, NewtonState* ns, fmg_report* rep, int newton_max,
                                                double tol, double* sm) {
  if (DIM == 2 && s.N1 == 9 && (GEN || !s.general))
    newton_core_reg<DIM, 10, GEN>(s, cs, m, ns, rep, newton_max, tol, sm, A1);
  else if (DIM == 3 && s.N1 == 27 && (GEN || !s.general))
    newton_core_reg<DIM, 28, GEN>(s, cs, m, ns, rep, newton_max, tol, sm, A1);
  else newton_core<DIM>(s, cs, A1, m, ns, rep, newton_max, tol, sm);
}

// First kernel of a solve: resets the report (as k_begin_solve), then
// Algorithm 3.2, step 1, then (fold) the transition into level 2.
template <int DIM, int KIND>
__global__ void __launch_bounds__(256) k_level1_newton(Grid g1, int N1, const double* __restrict__ A1, double m1,
                                                       const ProblemSlot* __restrict__ slot, int nf1, int fs,
                                                       double* __restrict__ x1, fmg_report* __restrict__ rep,
                                                       int newton_max, double tol, int levels, int* flag, int fold,
                                                       TransitionArgs next) {
  extern __shared__ double smem[];
  begin_solve_dev(rep, levels, flag);
  __syncthreads();
  level1_dispatch<DIM, KIND>(g1, N1, A1, m1, slot, nf1, fs, x1, rep, newton_max, tol, smem);
  if (fold) transition_block<DIM, KIND>(next, nullptr, slot);
}

}  // namespace fmg
