// Launchers of the kernels that depend on the nonlinearity (template argument
// KIND).  They are defined in fmg_launch_impl.h and instantiated in the
// translation units fmg_kind_*.hip, one per dimension and group of
// nonlinearities, so that those kernels (the bulk of the device code) are
// compiled in parallel and each instance lives in exactly one code object.
// The host recorder in fmg.hip only calls these functions.
#pragma once

#include "fmg_kernels_aug.h"
#include "fmg_kernels_fmgtail.h"

namespace fmg {

template <int DIM, int KIND, bool CW = false>
void launch_rhs(dim3 grid, hipStream_t st, Grid g, const ProblemSlot* slot, int nf1, int fs, const double* u,
                double* b, double m);

template <int DIM, int KIND>
void launch_aug_small(size_t lds, hipStream_t st, Grid g, AugShape s, double* ut, const ProblemSlot* slot,
                      int nf1, int fs, double scale, double m, const double* A1, NewtonState* ns, fmg_report* rep,
                      int level, int newton_max, double tol, int do_update, int fold, TransitionArgs next);

template <int DIM, int KIND>
void launch_rhs_elem(dim3 grid, hipStream_t st, Grid g, const ProblemSlot* slot, int nf1, int fs, const double* u,
                     double* contrib, double* b, double m);

template <int DIM, int KIND, bool SETUP, bool FINISH, bool ELEM = false, bool VAR = false>
void launch_aug_pass(int blocks, int threads, size_t lds, hipStream_t st, Grid g, AugShape s, const double* ut,
                     const ProblemSlot* slot, int nf1, int fs, double scale, double m, const double* A1,
                     NewtonState* ns, fmg_report* rep, double* pq, double* ps, unsigned* tickets, int level,
                     int newton_max, double tol);

template <int DIM, int KIND, bool ELEM = false, bool VAR = false>
void launch_newton_finish(size_t lds, hipStream_t st, Grid g, AugShape s, const double* ut,
                          const ProblemSlot* slot, const double* A1, double m, NewtonState* ns, fmg_report* rep,
                          int newton_max, double tol);

template <int DIM, int KIND, bool MIXED>
void launch_fmg_tail(size_t lds, hipStream_t st, const FmgTailParams* P);

template <int DIM, int KIND>
void launch_level1(size_t lds, hipStream_t st, Grid g1, int N1, const double* A1, double m1,
                   const ProblemSlot* slot, int nf1, int fs, double* x1, fmg_report* rep, int newton_max,
                   double tol, int levels, int* flag, int fold, TransitionArgs next);

template <int DIM, int KIND, bool AUG, bool CW = false>
void launch_transition(dim3 grid, hipStream_t st, TransitionArgs a, const NewtonState* ns,
                       const ProblemSlot* slot);

// The transition's right-hand side alone (3D).
template <int DIM, int KIND>
void launch_transition_rhs(dim3 grid, hipStream_t st, TransitionArgs a, const ProblemSlot* slot);

}  // namespace fmg
