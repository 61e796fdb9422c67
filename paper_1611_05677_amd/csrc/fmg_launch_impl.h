// Definitions of the launchers declared in fmg_launch.h, and the macro that
// instantiates them for one dimension and one nonlinearity.
#pragma once

#include "fmg_launch.h"
#include "fmg_newton_reg.h"

namespace fmg {

template <int DIM, int KIND, bool CW>
void launch_rhs(dim3 grid, hipStream_t st, Grid g, const ProblemSlot* slot, int nf1, int fs, const double* u,
                double* b, double m) {
  k_rhs<DIM, KIND, CW><<<grid, kBlock, 0, st>>>(g, slot, nf1, fs, u, b, m);
}

template <int DIM, int KIND>
void launch_aug_small(size_t lds, hipStream_t st, Grid g, AugShape s, double* ut, const ProblemSlot* slot,
                      int nf1, int fs, double scale, double m, const double* A1, NewtonState* ns, fmg_report* rep,
                      int level, int newton_max, double tol, int do_update, int fold, TransitionArgs next) {
  k_aug_solve_small<DIM, KIND><<<1, aug_small_threads<DIM>(), lds, st>>>(g, s, ut, slot, nf1, fs, scale, m, A1, ns, rep, level,
                                                             newton_max, tol, do_update, fold, next);
}

// grid: the node grid of the level (second launch); the first launch takes
// one thread per fine cell.  contrib: 2^d n^d doubles.
template <int DIM, int KIND>
void launch_rhs_elem(dim3 grid, hipStream_t st, Grid g, const ProblemSlot* slot, int nf1, int fs, const double* u,
                     double* contrib, double* b, double m) {
  const long long ncells = DIM == 2 ? (long long)g.n * g.n : (long long)g.n * g.n * g.n;
  k_rhs_elem_cells<DIM, KIND><<<(unsigned)((ncells + kBlock - 1) / kBlock), kBlock, 0, st>>>(g, slot, nf1, fs, u,
                                                                                             contrib);
  k_rhs_elem_nodes<DIM><<<grid, kBlock, 0, st>>>(g, contrib, b, m * ElemRule<DIM>::W);
}

template <int DIM, int KIND, bool SETUP, bool FINISH, bool ELEM, bool VAR>
void launch_aug_pass(int blocks, int threads, size_t lds, hipStream_t st, Grid g, AugShape s, const double* ut,
                     const ProblemSlot* slot, int nf1, int fs, double scale, double m, const double* A1,
                     NewtonState* ns, fmg_report* rep, double* pq, double* ps, unsigned* tickets, int level,
                     int newton_max, double tol) {
  if (DIM == 2 && FINISH && threads > 512) threads = 512;
  k_aug_pass<DIM, KIND, SETUP, FINISH, ELEM, VAR><<<blocks, threads, lds, st>>>(g, s, ut, slot, nf1, fs, scale, m, A1, ns,
                                                                           rep, pq, ps, tickets, level, newton_max,
                                                                           tol);
}

template <int DIM, int KIND, bool ELEM, bool VAR>
void launch_newton_finish(size_t lds, hipStream_t st, Grid g, AugShape s, const double* ut,
                          const ProblemSlot* slot, const double* A1, double m, NewtonState* ns, fmg_report* rep,
                          int newton_max, double tol) {
  k_newton_finish<DIM, KIND, ELEM, VAR><<<1, kBlock, lds, st>>>(g, s, ut, slot, A1, m, ns, rep, newton_max, tol);
}

template <int DIM, int KIND, bool MIXED>
void launch_fmg_tail(size_t lds, hipStream_t st, const FmgTailParams* P) {
  k_fmg_tail<DIM, KIND, MIXED><<<1, kTailThreads, lds, st>>>(P);
}

template <int DIM, int KIND>
void launch_level1(size_t lds, hipStream_t st, Grid g1, int N1, const double* A1, double m1,
                   const ProblemSlot* slot, int nf1, int fs, double* x1, fmg_report* rep, int newton_max,
                   double tol, int levels, int* flag, int fold, TransitionArgs next) {
  k_level1_newton<DIM, KIND><<<1, 256, lds, st>>>(g1, N1, A1, m1, slot, nf1, fs, x1, rep, newton_max, tol, levels,
                                                  flag, fold, next);
}

template <int DIM, int KIND, bool AUG, bool CW>
void launch_transition(dim3 grid, hipStream_t st, TransitionArgs a, const NewtonState* ns,
                       const ProblemSlot* slot) {
  k_transition<DIM, KIND, AUG, CW><<<grid, kBlock, 0, st>>>(a, ns, slot);
}
template <int DIM, int KIND>
void launch_transition_rhs(dim3 grid, hipStream_t st, TransitionArgs a, const ProblemSlot* slot) {
  k_transition_rhs<DIM, KIND><<<grid, kBlock, 0, st>>>(a, slot);
}

}  // namespace fmg

// Every launcher for dimension D and nonlinearity K (the 2D recorder never
// launches the separate Newton finisher or the separate transition right-hand
// side, so those are only instantiated in 3D, by FMG_INSTANTIATE_FINISH).
#define FMG_INSTANTIATE_KIND(D, K)                                                                   \
  namespace fmg {                                                                                    \
  template void launch_rhs<D, K>(dim3, hipStream_t, Grid, const ProblemSlot*, int, int, const double*, \
                                 double*, double);                                                   \
  template void launch_aug_small<D, K>(size_t, hipStream_t, Grid, AugShape, double*, const ProblemSlot*, \
                                       int, int, double, double, const double*, NewtonState*,         \
                                       fmg_report*, int, int, double, int, int, TransitionArgs);       \
  template void launch_aug_pass<D, K, true, true>(int, int, size_t, hipStream_t, Grid, AugShape,       \
                                                  const double*, const ProblemSlot*, int, int, double,  \
                                                  double, const double*, NewtonState*, fmg_report*,     \
                                                  double*, double*, unsigned*, int, int, double);       \
  template void launch_aug_pass<D, K, true, false>(int, int, size_t, hipStream_t, Grid, AugShape,      \
                                                   const double*, const ProblemSlot*, int, int, double, \
                                                   double, const double*, NewtonState*, fmg_report*,    \
                                                   double*, double*, unsigned*, int, int, double);      \
  template void launch_aug_pass<D, K, false, true>(int, int, size_t, hipStream_t, Grid, AugShape,      \
                                                   const double*, const ProblemSlot*, int, int, double, \
                                                   double, const double*, NewtonState*, fmg_report*,    \
                                                   double*, double*, unsigned*, int, int, double);      \
  template void launch_aug_pass<D, K, false, false>(int, int, size_t, hipStream_t, Grid, AugShape,     \
                                                    const double*, const ProblemSlot*, int, int, double, \
                                                    double, const double*, NewtonState*, fmg_report*,   \
                                                    double*, double*, unsigned*, int, int, double);     \
  template void launch_fmg_tail<D, K, false>(size_t, hipStream_t, const FmgTailParams*);              \
  template void launch_fmg_tail<D, K, true>(size_t, hipStream_t, const FmgTailParams*);               \
  template void launch_level1<D, K>(size_t, hipStream_t, Grid, int, const double*, double,             \
                                    const ProblemSlot*, int, int, double*, fmg_report*, int, double,   \
                                    int, int*, int, TransitionArgs);                                   \
  template void launch_transition<D, K, true>(dim3, hipStream_t, TransitionArgs, const NewtonState*,   \
                                              const ProblemSlot*);                                     \
  template void launch_transition<D, K, false>(dim3, hipStream_t, TransitionArgs, const NewtonState*,  \
                                               const ProblemSlot*);                                    \
  }

#define FMG_INSTANTIATE_FINISH(D, K)                                                                 \
  namespace fmg {                                                                                    \
  template void launch_newton_finish<D, K>(size_t, hipStream_t, Grid, AugShape, const double*,         \
                                           const ProblemSlot*, const double*, double, NewtonState*,   \
                                           fmg_report*, int, double);                                 \
  template void launch_transition_rhs<D, K>(dim3, hipStream_t, TransitionArgs, const ProblemSlot*);   \
  }

// The element-rule kernels for dimension D and nonlinearity K: right-hand
// side, setup and quadrature passes, and the Newton finisher (both
// dimensions).  Instantiated in fmg_kind_{2d,3d}_e.hip.
#define FMG_INSTANTIATE_ELEM(D, K)                                                                   \
  namespace fmg {                                                                                    \
  template void launch_rhs_elem<D, K>(dim3, hipStream_t, Grid, const ProblemSlot*, int, int,          \
                                      const double*, double*, double*, double);                     \
  template void launch_aug_pass<D, K, true, false, true>(int, int, size_t, hipStream_t, Grid, AugShape, \
                                                         const double*, const ProblemSlot*, int, int,  \
                                                         double, double, const double*, NewtonState*,  \
                                                         fmg_report*, double*, double*, unsigned*, int, \
                                                         int, double);                                 \
  template void launch_aug_pass<D, K, false, false, true>(int, int, size_t, hipStream_t, Grid, AugShape, \
                                                          const double*, const ProblemSlot*, int, int, \
                                                          double, double, const double*, NewtonState*, \
                                                          fmg_report*, double*, double*, unsigned*, int, \
                                                          int, double);                                \
  template void launch_newton_finish<D, K, true>(size_t, hipStream_t, Grid, AugShape, const double*,   \
                                                 const ProblemSlot*, const double*, double, NewtonState*, \
                                                 fmg_report*, int, double);                           \
  }

// The variable-coefficient kernels for dimension D and nonlinearity K: the
// weighted right-hand side and transitions, setup and quadrature passes and
// the Newton finisher.  Instantiated in fmg_kind_{2d,3d}_v.hip.
#define FMG_INSTANTIATE_VAR(D, K)                                                                    \
  namespace fmg {                                                                                    \
  template void launch_rhs<D, K, true>(dim3, hipStream_t, Grid, const ProblemSlot*, int, int,        \
                                       const double*, double*, double);                              \
  template void launch_transition<D, K, true, true>(dim3, hipStream_t, TransitionArgs,               \
                                                    const NewtonState*, const ProblemSlot*);         \
  template void launch_transition<D, K, false, true>(dim3, hipStream_t, TransitionArgs,              \
                                                     const NewtonState*, const ProblemSlot*);        \
  template void launch_aug_pass<D, K, true, false, false, true>(int, int, size_t, hipStream_t, Grid,  \
                                                                AugShape, const double*,             \
                                                                const ProblemSlot*, int, int, double, \
                                                                double, const double*, NewtonState*,  \
                                                                fmg_report*, double*, double*,        \
                                                                unsigned*, int, int, double);         \
  template void launch_aug_pass<D, K, false, false, false, true>(int, int, size_t, hipStream_t, Grid, \
                                                                 AugShape, const double*,            \
                                                                 const ProblemSlot*, int, int, double, \
                                                                 double, const double*, NewtonState*, \
                                                                 fmg_report*, double*, double*,       \
                                                                 unsigned*, int, int, double);        \
  template void launch_newton_finish<D, K, false, true>(size_t, hipStream_t, Grid, AugShape,           \
                                                        const double*, const ProblemSlot*,             \
                                                        const double*, double, NewtonState*,           \
                                                        fmg_report*, int, double);                    \
  }
