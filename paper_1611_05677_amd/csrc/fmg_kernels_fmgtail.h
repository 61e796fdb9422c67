// Algorithm 3.2 on the first few (small) levels in ONE single-workgroup
// launch: level-1 Newton solve, then for every level k <= top the
// prolongation, the linearised right-hand side, the m V-cycles, the augmented
// problem (setup sums, damped Newton with per-cell quadrature done by the
// workgroup itself, update).  Same arithmetic per node as the grid kernels.
#pragma once

#include "fmg_kernels_aug.h"
#include "fmg_kernels_tail.h"
#include "fmg_newton_reg.h"

namespace fmg {

struct FmgTailParams {
  TailArgs<double> v64;              // float64 level arrays (canonical roles), weights, A_1^{-1}
  TailArgs<float> v32;               // float32 level arrays of the mixed mode
  AugShape aug[kTailLevels + 1];
  double m[kTailLevels + 1];         // lumped mass h_k^d
  const double* A1;
  NewtonState* ns;
  fmg_report* rep;
  const ProblemSlot* slot;
  int top, nlev, nf1, m_vcycles, p_steps, newton_max;
  double newton_tol;
};

template <int DIM, int KIND>
__device__ __forceinline__ void blk_rhs(const Grid& g, const ProblemSlot* __restrict__ slot, int nf1, int fs,
                        const double* __restrict__ u, double* __restrict__ b, double m) {
  const int total = interior_count<DIM>(g);
  const int mm = g.n - 1;
  const double* __restrict__ gl = slot->g;
  const double q = slot->param;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int i = 1 + t % mm, j = 1 + (t / mm) % mm, l = DIM == 3 ? 1 + t / (mm * mm) : 0;
    const int c = gidx<DIM>(g, i, j, l);
    b[c] = m * (gl[fine_load_index(nf1, fs, i, j, l)] - NL<KIND>::f(u[c], q));
  }
  __syncthreads();
}

template <int DIM, typename T>
__device__ __forceinline__ void blk_prolong_plain(const Grid& cg, const Grid& f, const T* __restrict__ xc, T* __restrict__ xf) {
  const int total = interior_count<DIM>(f);
  const int m = f.n - 1;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int i = 1 + t % m, j = 1 + (t / m) % m, l = DIM == 3 ? 1 + t / (m * m) : 0;
    const int si = i & 1, sj = j & 1, sl = DIM == 3 ? (l & 1) : 0;
    const int pi = i >> 1, pj = j >> 1, pl = l >> 1;
    T v = xc[gidx<DIM>(cg, pi, pj, pl)];
    if (si | sj | sl) v = T(0.5) * (v + xc[gidx<DIM>(cg, pi + si, pj + sj, pl + sl)]);
    xf[gidx<DIM>(f, i, j, l)] = v;
  }
  __syncthreads();
}

template <int DIM>
__device__ __forceinline__ void blk_resid_to_f32(const Grid& g, const double* __restrict__ u, const double* __restrict__ b,
                                 float* __restrict__ r, double scale) {
  const int total = interior_count<DIM>(g);
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int c = interior_node<DIM>(g, t);
    r[c] = (float)(b[c] - apply_A_at<DIM>(u, c, g, scale));
  }
  __syncthreads();
}

template <int DIM>
__device__ __forceinline__ void blk_add_f32(const Grid& g, double* __restrict__ u, const float* __restrict__ e) {
  const int total = interior_count<DIM>(g);
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int c = interior_node<DIM>(g, t);
    u[c] += (double)e[c];
  }
  __syncthreads();
}

// Augmented problem of Algorithm 3.1, step 2, solved entirely by this workgroup.
// LDS: cs (ncell*NQ) | Newton scratch (newton_scratch_doubles).
template <int DIM, int KIND>
__device__ __forceinline__ void aug_solve_dev(const Grid& g, const AugShape& s, double* __restrict__ ut,
                              const ProblemSlot* __restrict__ slot, int nf1, int fs, double scale, double m,
                              const double* __restrict__ A1, NewtonState* ns, fmg_report* rep, int level,
                              int newton_max, double tol, double* smem, bool do_update = true) {
  using AC = Acc<DIM>;
  const int ncell = DIM == 2 ? s.nH * s.nH : s.nH * s.nH * s.nH;
  double* cs = smem;
  double* sm = cs + ncell * AC::NQ;
  if (threadIdx.x == 0) newton_state_reset(ns, s.N1, level);
  __syncthreads();
  // 2D: the setup sums (held in the Newton scratch until scattered) and the
  // sums at the start y0 = (0, .., 0, 1) in one visit; 3D: two visits (the
  // fused accumulators would not fit the registers of a 1024-thread block)
  bool have_sums = DIM == 2;
  if (DIM == 2) {
    setup_quad_cells_by_waves<DIM, KIND>(g, s, ut, slot->g, nf1, fs, scale, slot->param, sm, cs);
    setup_scatter<DIM>(s, sm, m, ns);
  } else {
    setup_cells_by_waves<DIM>(g, s, ut, slot->g, nf1, fs, scale, cs);
    setup_scatter<DIM>(s, cs, m, ns);
  }
  while (true) {
    __syncthreads();
    if (ns->done) break;
    if (!have_sums) quad_cells_by_waves<DIM, KIND>(g, s, ut, ns->ytry, slot->param, cs);
    have_sums = false;
    newton_step_dev<DIM>(s, cs, A1, m, ns, rep, newton_max, tol, sm);
  }
  __syncthreads();
  if (!do_update) return;
  const int total = interior_count<DIM>(g);
  const int mm = g.n - 1;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int i = 1 + t % mm, j = 1 + (t / mm) % mm, l = DIM == 3 ? 1 + t / (mm * mm) : 0;
    update_node<DIM>(g, s, ns, ut, i, j, l);
  }
  __syncthreads();
}

// Threads of the single-workgroup augmented solve: 512, so that the per-node
// accumulators and the Newton step get the registers that a 1024-thread block
// (128 per thread) would make them spill.
template <int DIM>
__host__ __device__ constexpr int aug_small_threads() { return 512; }

// The augmented problem of one correction step on a small level, solved by
// one workgroup in one launch (setup sums, every Newton iteration, and the
// update unless the caller defers it).
// With fold, the block then also performs the transition into the next
// (small) level, reading (w, alpha) from LDS.
template <int DIM, int KIND>
__global__ void __launch_bounds__(aug_small_threads<DIM>()) k_aug_solve_small(Grid g, AugShape s, double* __restrict__ ut,
                                                                  const ProblemSlot* __restrict__ slot, int nf1,
                                                                  int fs, double scale, double m,
                                                                  const double* __restrict__ A1, NewtonState* ns,
                                                                  fmg_report* rep, int level, int newton_max,
                                                                  double tol, int do_update, int fold,
                                                                  TransitionArgs next) {
  extern __shared__ double smem[];
  // the Newton state lives in LDS for the whole solve (its many small,
  // dependent reads and writes then cost LDS latency, not L2 latency) and is
  // copied out once at the end for the kernels that consume it
  __shared__ NewtonState nsl;
  aug_solve_dev<DIM, KIND>(g, s, ut, slot, nf1, fs, scale, m, A1, &nsl, rep, level, newton_max, tol, smem,
                           do_update != 0);
  if (fold) transition_block<DIM, KIND>(next, nsl.y, slot);
  const double* src = reinterpret_cast<const double*>(&nsl);
  double* dst = reinterpret_cast<double*>(ns);
  static_assert(sizeof(NewtonState) % sizeof(double) == 0, "NewtonState copied as doubles");
  for (int i = threadIdx.x; i < (int)(sizeof(NewtonState) / sizeof(double)); i += blockDim.x) dst[i] = src[i];
}

template <int DIM, int KIND, bool MIXED>
__global__ void __launch_bounds__(kTailThreads) k_fmg_tail(const FmgTailParams* __restrict__ P) {
  extern __shared__ double smem[];
  const int top = P->top;
  double* x64[kTailLevels + 1];
  double* t64[kTailLevels + 1];
  float* x32[kTailLevels + 1];
  float* t32[kTailLevels + 1];
  for (int k = 1; k <= top; ++k) {
    x64[k] = P->v64.x[k]; t64[k] = P->v64.t[k];
    x32[k] = P->v32.x[k]; t32[k] = P->v32.t[k];
  }
  const TailArgs<double>& V = P->v64;
  // Algorithm 3.2, step 1
  level1_dispatch<DIM, KIND>(V.g[1], V.N1, P->A1, P->m[1], P->slot, P->nf1, 1 << (P->nlev - 1), x64[1], P->rep,
                               P->newton_max, P->newton_tol, smem);
  // step 2 on levels 2..top
  for (int k = 2; k <= top; ++k) {
    blk_prolong_plain<DIM, double>(V.g[k - 1], V.g[k], x64[k - 1], x64[k]);
    const int fs = 1 << (P->nlev - k);
    for (int l = 0; l < P->p_steps; ++l) {
      blk_rhs<DIM, KIND>(V.g[k], P->slot, P->nf1, fs, x64[k], V.b[k], P->m[k]);
      for (int c = 0; c < P->m_vcycles; ++c) {
        if (!MIXED) {
          vcycle_tail_dev<DIM, double>(V, x64, t64, k, false);
        } else {
          // float32 cycles on the correction equation: the float64 residual
          // before the first, the float64 update after the last
          if (c == 0) blk_resid_to_f32<DIM>(V.g[k], x64[k], V.b[k], P->v32.b[k], V.scale[k]);
          vcycle_tail_dev<DIM, float>(P->v32, x32, t32, k, c == 0);
          if (c == P->m_vcycles - 1) blk_add_f32<DIM>(V.g[k], x64[k], x32[k]);
        }
      }
      aug_solve_dev<DIM, KIND>(V.g[k], P->aug[k], x64[k], P->slot, P->nf1, fs, V.scale[k], P->m[k], P->A1, P->ns,
                               P->rep, k, P->newton_max, P->newton_tol, smem);
    }
  }
}

}  // namespace fmg
