// Host side of the FMG library: workspace planning, the launch sequence of
// Algorithm 3.2 / Algorithm 3.1, optional hipGraph capture, and the C ABI of
// include/fmg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/fmg.h"
#include "fmg_device.h"
#include "fmg_kernels_aug.h"
#include "fmg_kernels_mg.h"
#include "fmg_kernels_tail.h"
#include "fmg_kernels_fmgtail.h"
#include "fmg_kernels_fused2d.h"
#include "fmg_kernels_stream2d.h"
#include "fmg_kernels_stream3d.h"
#include "fmg_kernels_pair3d.h"
#include "fmg_kernels_restrict3d.h"
#include "fmg_launch.h"

using namespace fmg;

namespace {

constexpr size_t kAlign = 256;

// Static device scratch of fmg_solve_noalloc: the workspace of one solve, in
// a file-scope array that every GPU the library runs on holds until the
// process ends (host code never uses the array's name as an address: it
// takes the device address from hipGetSymbolAddress, per device).
constexpr size_t kScratchBytes = FMG_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_tail_attr_set = false;
// Converged mode: a stop on a non-shrinking update counts as converged only
// within this factor of the tolerance.
constexpr double kStagnationFloor = 1e3;
constexpr int kNormBlocksMax = 1 << 20;

inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }
inline int ilog2(long long v) { int r = 0; while ((1LL << (r + 1)) <= v) ++r; return r; }

struct Resolved {          // options with defaults applied
  fmg_options o;
  int smoother;
  double pre[16], post[16];
};

struct LevelInfo {
  Grid g;
  size_t count;            // elements per level array (incl. padding)
  double scale;            // h^{d-2}: A_k = scale * (2d, -1 ...)
  double m;                // lumped mass h^d
  AugShape aug;            // augmented-pass tiling (levels >= 2)
  int aug_blocks;
  int aug_threads;          // threads per block of the augmented passes
};

struct Plan {
  int dim, nH, nlev, N1;
  int tail_top;            // deepest level handled by the single-workgroup tail (0: none)
  int tail_dense;          // 1: levels <= tail_top apply the V-cycle as a dense operator
  size_t off_tailB[FMG_MAX_LEVELS + 1];   // B_k (N_k x N_k float64, row-major), k = 2..tail_top
  LevelInfo lev[FMG_MAX_LEVELS + 1];   // 1-based
  size_t off_state, off_report, off_slot, off_flag, off_norm_out, off_norm_part;
  size_t off_A1, off_A1inv, off_A1inv_f, off_pq, off_ps;
  size_t off_x[FMG_MAX_LEVELS + 1], off_b[FMG_MAX_LEVELS + 1], off_t[FMG_MAX_LEVELS + 1];
  size_t off_xs[FMG_MAX_LEVELS + 1], off_bs[FMG_MAX_LEVELS + 1], off_ts[FMG_MAX_LEVELS + 1];
  size_t off_uprev;
  size_t off_fmgtail;
  size_t off_ticket;
  size_t off_econtrib;     // element rule: per-corner cell contributions of the right-hand side
  int var;                 // variable coefficient: the arrays below are in use
  size_t off_w[FMG_MAX_LEVELS + 1];     // forward-edge weight planes of level k
  long long wplane[FMG_MAX_LEVELS + 1];  // elements between the planes (the level's array size)
  size_t off_sm[FMG_MAX_LEVELS + 1];    // per-simplex matrices of level k < n
  size_t norm_blocks;
  size_t total;
};

int resolve(int dim, const fmg_options* in, Resolved& r) {
  fmg_options o;
  if (in) o = *in; else fmg_default_options(dim, &o);
  if (o.precision != FMG_FP64 && o.precision != FMG_MIXED) return FMG_E_INVALID;
  if (o.m_vcycles < 1 || o.p_steps < 1 || o.nu_pre < 0 || o.nu_post < 0 || o.nu_pre > 16 || o.nu_post > 16)
    return FMG_E_INVALID;
  if (o.smoother < 0 || o.smoother > 2 || o.omega < 0 || !(o.cheb_lo > 0) || !(o.cheb_hi > o.cheb_lo))
    return FMG_E_INVALID;
  if (o.newton_max < 1 || !(o.newton_tol > 0) || o.newton_passes < 1 || o.newton_passes > 64)
    return FMG_E_INVALID;
  if (o.mode != FMG_PAPER && o.mode != FMG_CONVERGED) return FMG_E_INVALID;
  if (o.mode == FMG_CONVERGED && (o.converged_max_steps < 1 || !(o.converged_tol > 0))) return FMG_E_INVALID;
  if (o.tail_max_nodes < 0 || (o.fuse_small_levels != 0 && o.fuse_small_levels != 1)) return FMG_E_INVALID;
  if (o.aug_max_blocks < 64 || o.aug_max_blocks > 16384 || o.aug_small_nodes < 0) return FMG_E_INVALID;
  if (o.sweep_rows < -1 || (o.sweep_rows > 0 && o.sweep_rows < 2) || o.sweep_rows > 4096) return FMG_E_INVALID;
  if (o.quadrature != FMG_QUAD_VERTEX && o.quadrature != FMG_QUAD_ELEMENT) return FMG_E_INVALID;
  if (o.quadrature == FMG_QUAD_ELEMENT && o.fuse_small_levels) return FMG_E_UNSUPPORTED;
  if (o.coefficients != FMG_COEF_IDENTITY && o.coefficients != FMG_COEF_VARIABLE) return FMG_E_INVALID;
  if (o.coefficients == FMG_COEF_VARIABLE) {
    if (o.precision != FMG_FP64 || o.quadrature != FMG_QUAD_VERTEX || o.fuse_small_levels) return FMG_E_UNSUPPORTED;
    // one-sweep V-cycle kernels down to level 1, multi-workgroup augmented passes
    o.tail_max_nodes = 0;
    o.aug_small_nodes = 0;
    o.sweep_rows = -1;
  }
  r.o = o;
  r.smoother = o.smoother ? o.smoother : (dim == 2 ? FMG_JACOBI : FMG_CHEBYSHEV);
  if (r.smoother == FMG_JACOBI) {
    const double w = o.omega > 0 ? o.omega : (dim == 2 ? 4.0 / 5.0 : 6.0 / 7.0);
    for (int i = 0; i < 16; ++i) r.pre[i] = r.post[i] = w;
  } else {
    // reciprocals of the roots of the Chebyshev polynomial of degree nu on
    // [lo, hi]; post-smoothing uses them in reverse order
    const double c = 0.5 * (o.cheb_hi + o.cheb_lo), rad = 0.5 * (o.cheb_hi - o.cheb_lo);
    for (int i = 0; i < o.nu_pre; ++i)
      r.pre[i] = 1.0 / (c + rad * std::cos(M_PI * (2 * (i + 1) - 1) / (2.0 * o.nu_pre)));
    for (int i = 0; i < o.nu_post; ++i)
      r.post[o.nu_post - 1 - i] = 1.0 / (c + rad * std::cos(M_PI * (2 * (i + 1) - 1) / (2.0 * o.nu_post)));
  }
  return FMG_OK;
}

// host_tables = false: no table that only the host can build (the dense
// V-cycle tail operators); the tail then runs as a single-workgroup cycle.
int make_plan(const fmg_mesh_desc* mesh, const Resolved& ro, Plan& p, bool host_tables = true) {
  if (!mesh) return FMG_E_INVALID;
  const int d = mesh->dim;
  if (d != 2 && d != 3) return FMG_E_UNSUPPORTED;
  if (mesh->coarse_cells < 2 || mesh->coarse_cells > (d == 2 ? 8 : 4)) return FMG_E_UNSUPPORTED;
  if (mesh->refinements < 1 || mesh->refinements > (d == 2 ? 12 : 8)) return FMG_E_UNSUPPORTED;
  std::memset(&p, 0, sizeof(p));
  p.dim = d;
  p.nH = mesh->coarse_cells;
  p.nlev = mesh->refinements + 1;
  p.N1 = 1;
  for (int a = 0; a < d; ++a) p.N1 *= p.nH - 1;
  const int ncell = d == 2 ? p.nH * p.nH : p.nH * p.nH * p.nH;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  p.off_state = take(sizeof(NewtonState));
  p.off_report = take(sizeof(fmg_report));
  p.off_slot = take(sizeof(ProblemSlot));
  p.off_flag = take(64);
  p.off_norm_out = take(64);
  p.off_A1 = take(sizeof(double) * p.N1 * p.N1);
  p.off_A1inv = take(sizeof(double) * p.N1 * p.N1);
  p.off_A1inv_f = take(sizeof(float) * p.N1 * p.N1);
  int max_blocks = 1;
  for (int k = 1; k <= p.nlev; ++k) {
    LevelInfo& L = p.lev[k];
    L.g.n = p.nH << (k - 1);
    L.g.px = pitch_for(L.g.n);
    L.g.pz = d == 3 ? L.g.px * (L.g.n + 1) : 0;
    L.count = d == 2 ? (size_t)L.g.px * (L.g.n + 1) : (size_t)L.g.pz * (L.g.n + 1);
    const double h = 1.0 / L.g.n;
    L.scale = d == 2 ? 1.0 : h;
    L.m = d == 2 ? h * h : h * h * h;
    {   // every level: level 1 takes the augmented passes in element mode
      const int nodes_log = d * (k - 1);
      // large levels: 1024-thread (2D) or 512-thread (3D) blocks, fewer of them
      const bool wide = ro.o.quadrature == FMG_QUAD_VERTEX && ro.o.coefficients == FMG_COEF_IDENTITY &&
                        nodes_log >= (d == 2 ? aug_wide_nodes_log<2>() : aug_wide_nodes_log<3>());
      const int tlog = wide ? ilog2(d == 2 ? aug_threads<2>() : aug_threads<3>()) : 8;
      const int cap_log = ilog2(std::max(1, (ro.o.aug_max_blocks >> (tlog - 8)) / ncell));
      const int bpc_log = std::max(0, std::min(nodes_log - tlog, cap_log));
      L.aug_threads = 1 << tlog;
      L.aug.nH = p.nH;
      L.aug.log2r = k - 1;
      L.aug.bpc_log = bpc_log;
      L.aug.npb_log = nodes_log - bpc_log;
      L.aug.N1 = p.N1;
      L.aug.general = ro.o.coefficients == FMG_COEF_VARIABLE ? 1 : 0;
      L.aug_blocks = ncell << bpc_log;
      max_blocks = std::max(max_blocks, L.aug_blocks);
    }
  }
  p.tail_top = 0;
  if (ro.o.tail_max_nodes > 0 && ro.o.nu_pre <= kTailSweeps && ro.o.nu_post <= kTailSweeps)
    for (int k = 2; k <= std::min(p.nlev, kTailLevels); ++k) {
      const long long m = p.lev[k].g.n - 1;
      if ((d == 2 ? m * m : m * m * m) <= ro.o.tail_max_nodes) p.tail_top = k;
    }
  p.tail_dense = 0;
  if (p.tail_top >= 2) {
    const long long m = p.lev[p.tail_top].g.n - 1;
    p.tail_dense = host_tables && (d == 2 ? m * m : m * m * m) <= kDenseTailMax ? 1 : 0;
  }
  for (int k = 0; k <= FMG_MAX_LEVELS; ++k) p.off_tailB[k] = 0;
  if (p.tail_dense)
    for (int k = 2; k <= p.tail_top; ++k) {
      const size_t m = p.lev[k].g.n - 1, N = d == 2 ? m * m : m * m * m;
      p.off_tailB[k] = take(sizeof(double) * N * N);
    }
  p.off_pq = take(sizeof(double) * max_blocks * Acc<3>::NQ);
  p.off_ps = take(sizeof(double) * max_blocks * Acc<3>::NS);
  const LevelInfo& F = p.lev[p.nlev];
  p.norm_blocks = d == 2 ? grid_blocks<2>(F.g.n) : grid_blocks<3>(F.g.n);
  p.off_norm_part = ro.o.mode == FMG_CONVERGED ? take(sizeof(double) * 2 * p.norm_blocks) : 0;
  for (int k = 1; k <= p.nlev; ++k) {
    const size_t c = p.lev[k].count;
    p.off_x[k] = take(sizeof(double) * c);
    p.off_b[k] = take(sizeof(double) * c);
    p.off_t[k] = take(sizeof(double) * c);
    if (ro.o.precision == FMG_MIXED) {
      p.off_xs[k] = take(sizeof(float) * c);
      p.off_bs[k] = take(sizeof(float) * c);
      p.off_ts[k] = take(sizeof(float) * c);
    }
  }
  p.off_uprev = ro.o.mode == FMG_CONVERGED ? take(sizeof(double) * F.count) : 0;
  p.off_fmgtail = take(sizeof(FmgTailParams));
  p.off_ticket = take(sizeof(unsigned));
  if (ro.o.quadrature == FMG_QUAD_ELEMENT) {
    const size_t nf = (size_t)F.g.n;
    p.off_econtrib = take(sizeof(double) * (d == 2 ? 4 * nf * nf : 8 * nf * nf * nf));
  }
  p.var = ro.o.coefficients == FMG_COEF_VARIABLE ? 1 : 0;
  if (p.var) {
    const int nfwd = (1 << d) - 1, nsm = d == 2 ? 3 * 2 : 6 * 6;   // components x simplices
    for (int k = 1; k <= p.nlev; ++k) {
      p.wplane[k] = (long long)p.lev[k].count;
      p.off_w[k] = take(sizeof(double) * nfwd * p.lev[k].count);
      if (k < p.nlev) {
        const size_t n = p.lev[k].g.n;
        p.off_sm[k] = take(sizeof(double) * nsm * (d == 2 ? n * n : n * n * n));
      }
    }
  }
  p.total = off;
  return FMG_OK;
}

}  // namespace

namespace { struct Prof; }

struct fmg_hierarchy {
  Plan plan;
  Resolved ro;
  char* ws;
  size_t ws_bytes;
  hipStream_t cap_stream;
  hipGraphExec_t graph[7];
  Prof* prof;              // set only while fmg_profile_solve records
  bool coef_ready;         // variable coefficient: fmg_set_coefficients was called
  template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  NewtonState* ns() const { return at<NewtonState>(plan.off_state); }
  fmg_report* rep() const { return at<fmg_report>(plan.off_report); }
  ProblemSlot* slot() const { return at<ProblemSlot>(plan.off_slot); }
  int* flag() const { return at<int>(plan.off_flag); }
};

namespace {

inline dim3 grid_of(const Grid& g, int dim) {
  return dim3(dim == 2 ? grid_blocks<2>(g.n) : grid_blocks<3>(g.n));
}

// Kernel classes reported by fmg_profile_solve.
enum KernelClass {
  KC_SMOOTH64, KC_SMOOTH64_ZERO, KC_RESTRICT64, KC_PROLONG64_ADD, KC_COARSE64,
  KC_SMOOTH32, KC_SMOOTH32_ZERO, KC_RESTRICT32, KC_PROLONG32_ADD, KC_COARSE32,
  KC_TRANSITION, KC_RHS, KC_RESID_F32, KC_ADD_F32, KC_AUG_PASS0, KC_AUG_PASS, KC_OUTPUT_UPDATE,
  KC_NEWTON_FINISH, KC_AUG_UPDATE, KC_LEVEL1, KC_BEGIN, KC_OUTPUT, KC_END, KC_FILL,
  KC_VCYCLE_TAIL64, KC_VCYCLE_TAIL32, KC_FMG_TAIL, KC_AUG_SMALL, KC_PRE2D64, KC_POST2D64, KC_PRE2D32, KC_POST2D32,
  KC_PRE2S64, KC_POST2S64, KC_PRE2S32, KC_POST2S32, KC_SMOOTH3S64, KC_SMOOTH3S32,
  KC_PRE3P64, KC_POST3P64, KC_PRE3P32, KC_POST3P32, KC_RHS_ELEM,
  KC_SMOOTHW64, KC_SMOOTHW64_ZERO, KC_RESIDW64, KC_RESTRICT64_R, KC_COUNT
};
const char* const kKernelNames[KC_COUNT] = {
  "smooth_f64", "smooth_f64_from_zero", "resid_restrict_f64", "prolong_add_f64", "coarse_solve_f64",
  "smooth_f32", "smooth_f32_from_zero", "resid_restrict_f32", "prolong_add_f32", "coarse_solve_f32",
  "transition", "rhs", "resid_to_f32", "add_f32", "aug_pass0_setup", "aug_pass", "output_update",
  "newton_finish", "aug_update", "level1_newton", "begin_solve", "output", "end_solve", "fill",
  "vcycle_tail_f64", "vcycle_tail_f32", "fmg_tail", "aug_solve_small", "pre_sweeps_restrict_2d_f64", "prolong_post_sweeps_2d_f64",
  "pre_sweeps_restrict_2d_f32", "prolong_post_sweeps_2d_f32",
  "pre_sweeps_restrict_2d_stream_f64", "prolong_post_sweeps_2d_stream_f64",
  "pre_sweeps_restrict_2d_stream_f32", "prolong_post_sweeps_2d_stream_f32",
  "smooth_3d_stream_f64", "smooth_3d_stream_f32",
  "pre_sweep_pair_3d_f64", "prolong_sweep_pair_3d_f64", "pre_sweep_pair_3d_f32", "prolong_sweep_pair_3d_f32",
  "rhs_element", "smooth_var_f64", "smooth_var_f64_from_zero", "resid_var_f64", "restrict_f64"};

// Event pairs around launches (fmg_profile_solve only).
struct Prof {
  std::vector<hipEvent_t> ev;
  std::vector<int> kid, lev, nodes;
  std::vector<double> bytes;
  void begin(hipStream_t st) {
    hipEvent_t e;
    (void)hipEventCreate(&e);
    (void)hipEventRecord(e, st);
    ev.push_back(e);
  }
  void end(hipStream_t st, int k, int l, long long nn, double b) {
    begin(st);
    kid.push_back(k); lev.push_back(l); nodes.push_back((int)nn); bytes.push_back(b);
  }
};

#define FMG_LAUNCH(h, st, KID, LEV, NODES, BYTES, ...)       \
  do {                                                        \
    Prof* _pf = (h)->prof;                                    \
    if (_pf) _pf->begin(st);                                  \
    __VA_ARGS__;                                              \
    if (_pf) _pf->end(st, KID, LEV, NODES, BYTES);            \
  } while (0)

inline long long interior(const Grid& g, int dim) {
  const long long m = g.n - 1;
  return dim == 2 ? m * m : m * m * m;
}

// Buffer roles during one recorded launch sequence.
struct Roles {
  double* x[FMG_MAX_LEVELS + 1];
  double* t[FMG_MAX_LEVELS + 1];
  float* xs[FMG_MAX_LEVELS + 1];
  float* ts[FMG_MAX_LEVELS + 1];
};

template <typename T> struct Sel;
template <> struct Sel<double> {
  static double*& x(Roles& r, int k) { return r.x[k]; }
  static double*& t(Roles& r, int k) { return r.t[k]; }
  static double* b(const fmg_hierarchy* h, int k) { return h->at<double>(h->plan.off_b[k]); }
  static const double* ainv(const fmg_hierarchy* h) { return h->at<double>(h->plan.off_A1inv); }
  static constexpr int kc = 0;
};
template <> struct Sel<float> {
  static float*& x(Roles& r, int k) { return r.xs[k]; }
  static float*& t(Roles& r, int k) { return r.ts[k]; }
  static float* b(const fmg_hierarchy* h, int k) { return h->at<float>(h->plan.off_bs[k]); }
  static const float* ainv(const fmg_hierarchy* h) { return h->at<float>(h->plan.off_A1inv_f); }
  static constexpr int kc = KC_SMOOTH32 - KC_SMOOTH64;
};

void canonical_roles(const fmg_hierarchy* h, Roles& r) {
  const Plan& p = h->plan;
  for (int k = 1; k <= p.nlev; ++k) {
    r.x[k] = h->at<double>(p.off_x[k]);
    r.t[k] = h->at<double>(p.off_t[k]);
    r.xs[k] = p.off_xs[k] ? h->at<float>(p.off_xs[k]) : nullptr;
    r.ts[k] = p.off_ts[k] ? h->at<float>(p.off_ts[k]) : nullptr;
  }
}

template <int DIM, typename T>
void fill_tail_args(const fmg_hierarchy* h, Roles& R, int top, TailArgs<T>& a) {
  const Plan& p = h->plan;
  std::memset(&a, 0, sizeof(a));
  for (int j = 1; j <= top; ++j) {
    a.x[j] = Sel<T>::x(R, j);
    a.t[j] = Sel<T>::t(R, j);
    a.b[j] = Sel<T>::b(h, j);
    a.g[j] = p.lev[j].g;
    a.scale[j] = (T)p.lev[j].scale;
    const double Dj = 2.0 * DIM * p.lev[j].scale;
    for (int i = 0; i < h->ro.o.nu_pre; ++i) a.wdpre[j][i] = (T)(h->ro.pre[i] / Dj);
    for (int i = 0; i < h->ro.o.nu_post; ++i) a.wdpost[j][i] = (T)(h->ro.post[i] / Dj);
  }
  a.ainv = Sel<T>::ainv(h);
  a.N1 = p.N1;
  a.top = top;
  a.npre = h->ro.o.nu_pre;
  a.npost = h->ro.o.nu_post;
  a.zero_top = 0;
}

// Launches of the fused 2D V(2,2) level kernels on level k (register-streaming
// or LDS-tiled, per the options); shared by the V-cycle and the kernel timer.
// Returns the algorithmic bytes of the launch.
template <typename T>
double launch_pre2(const fmg_hierarchy* h, int k, const T* x, const T* b, T* t, T* bc, bool zero_init,
                   hipStream_t st) {
  const Plan& p = h->plan;
  const LevelInfo& L = p.lev[k];
  const LevelInfo& C = p.lev[k - 1];
  const long long N = interior(L.g, 2), Nc = interior(C.g, 2);
  const double s = sizeof(T), D = 4.0 * L.scale;
  const double bytes = s * ((zero_init ? 2 : 3) * N + Nc);
  const T wd1 = (T)(h->ro.pre[0] / D), wd2 = (T)(h->ro.pre[1] / D), scale = (T)L.scale;
  const int kc2 = Sel<T>::kc ? (KC_PRE2D32 - KC_PRE2D64) : 0;
  const int rows = stream_rows(h->ro.o.sweep_rows, L.g.n);
  if (rows > 0) {
    int nch = 0;
    const int blocks = stream_blocks(L.g.n, kPreStrip, rows, nch);
    FMG_LAUNCH(h, st, KC_PRE2S64 + kc2, k, N, bytes,
               k_pre2s<T><<<blocks, 64 * kStreamWaves, 0, st>>>(L.g, C.g, x, b, t, bc, wd1, wd2, scale,
                                                               zero_init ? 1 : 0, rows, nch));
  } else {
    const dim3 tiles((L.g.n + kFTX - 1) / kFTX, (L.g.n + kFTY - 1) / kFTY);
    FMG_LAUNCH(h, st, KC_PRE2D64 + kc2, k, N, bytes,
               k_pre2d<T><<<tiles, kBlock, pre2d_lds_bytes<T>(), st>>>(L.g, C.g, x, b, t, bc, wd1, wd2, scale,
                                                                      zero_init ? 1 : 0));
  }
  return bytes;
}

template <typename T>
double launch_post2(const fmg_hierarchy* h, int k, const T* x, const T* xc, const T* b, T* t, hipStream_t st) {
  const Plan& p = h->plan;
  const LevelInfo& L = p.lev[k];
  const LevelInfo& C = p.lev[k - 1];
  const long long N = interior(L.g, 2), Nc = interior(C.g, 2);
  const double s = sizeof(T), D = 4.0 * L.scale;
  const double bytes = s * (3 * N + Nc);
  const T wd1 = (T)(h->ro.post[0] / D), wd2 = (T)(h->ro.post[1] / D), scale = (T)L.scale;
  const int kc2 = Sel<T>::kc ? (KC_PRE2D32 - KC_PRE2D64) : 0;
  const int rows = stream_rows(h->ro.o.sweep_rows, L.g.n);
  if (rows > 0) {
    int nch = 0;
    const int blocks = stream_blocks(L.g.n, kPostStrip, rows, nch);
    FMG_LAUNCH(h, st, KC_POST2S64 + kc2, k, N, bytes,
               k_post2s<T, false><<<blocks, 64 * kStreamWaves, 0, st>>>(C.g, L.g, x, xc, b, t, nullptr, wd1, wd2,
                                                                       scale, rows, nch));
  } else {
    const dim3 tiles((L.g.n + kFTX - 1) / kFTX, (L.g.n + kFTY - 1) / kFTY);
    FMG_LAUNCH(h, st, KC_POST2D64 + kc2, k, N, bytes,
               k_post2d<T><<<tiles, kBlock, post2d_lds_bytes<T>(), st>>>(C.g, L.g, x, xc, b, t, wd1, wd2, scale));
  }
  return bytes;
}

// 3D V(2,2) levels: the two pre-smoothing sweeps in one launch (from x, or
// from zero), and the coarse correction with the two post-smoothing sweeps in
// one launch (fmg_kernels_pair3d.h).  Used unless sweep_rows asks for the
// one-sweep kernels (-1: one node per thread; > 0: plane marching).
inline bool use_pair3(const fmg_hierarchy* h, int k) {
  const fmg_options& o = h->ro.o;
  return h->plan.dim == 3 && o.nu_pre == 2 && o.nu_post == 2 && o.sweep_rows == 0 &&
         h->plan.lev[k].g.n >= 16 && k > h->plan.tail_top;
}

Pair3Args pair3_args(const fmg_hierarchy* h, int k, const double* w) {
  const LevelInfo& L = h->plan.lev[k];
  const Pair3Shape sh = pair3_shape(L.g.n);
  Pair3Args a;
  std::memset(&a, 0, sizeof(a));
  a.g = L.g;
  a.cg = k > 1 ? h->plan.lev[k - 1].g : L.g;
  const double D = 6.0 * L.scale;
  a.wd1 = w[0] / D;
  a.wd2 = w[1] / D;
  a.scale = L.scale;
  a.nsx = sh.nsx; a.ncy = sh.ncy; a.nzc = sh.nzc; a.zc_planes = sh.zc_planes;
  return a;
}

template <typename T, int MODE>
void launch_pair3_kernel(const Pair3Args& a, hipStream_t st) {
  const Pair3Shape sh{a.nsx, a.ncy, a.nzc, a.zc_planes};
  k_sweep_pair3<T, MODE><<<pair3_blocks(sh), kP3Threads, 0, st>>>(a);
}

// bc = P^T (b - A x) from level f to level cg: in 3D on levels with at least
// kR3MinN cells per side the plane-marching kernel, else (and in 2D) one
// thread per coarse node.  Both give the same bits.  Measured at 128^3 and
// 64^3: the plane-marching kernel has too few tiles there (15 against 13 us,
// 13 against 3.6 us); at 256^3 it takes 69 against 89 us.
constexpr int kR3MinN = 256;

template <int DIM, typename T>
void launch_resid_restrict(const Grid& f, const Grid& cg, const T* x, const T* b, T* bc, T scale, hipStream_t st) {
  if (DIM == 3 && f.n >= kR3MinN) {
    const Restrict3Shape sh = restrict3_shape(cg.n);
    k_resid_restrict3m<T><<<restrict3_blocks(sh), kR3Threads, 0, st>>>(f, cg, x, b, bc, scale, sh);
  } else {
    k_resid_restrict<DIM, T><<<grid_of(cg, DIM), kBlock, 0, st>>>(f, cg, x, b, bc, scale);
  }
}

template <typename T>
double launch_pre3(const fmg_hierarchy* h, int k, const T* x, const T* b, T* t, bool zero_init, hipStream_t st) {
  const LevelInfo& L = h->plan.lev[k];
  const long long N = interior(L.g, 3);
  const double bytes = sizeof(T) * (zero_init ? 2.0 : 3.0) * N;
  Pair3Args a = pair3_args(h, k, h->ro.pre);
  a.x = x; a.b = b; a.out = t;
  const int kc = Sel<T>::kc ? (KC_PRE3P32 - KC_PRE3P64) : 0;
  if (zero_init)
    FMG_LAUNCH(h, st, KC_PRE3P64 + kc, k, N, bytes, (launch_pair3_kernel<T, kP3Zero>(a, st)));
  else
    FMG_LAUNCH(h, st, KC_PRE3P64 + kc, k, N, bytes, (launch_pair3_kernel<T, kP3Plain>(a, st)));
  return bytes;
}

template <typename T>
double launch_post3(const fmg_hierarchy* h, int k, const T* x, const T* xc, const T* b, T* t, hipStream_t st) {
  const LevelInfo& L = h->plan.lev[k];
  const LevelInfo& C = h->plan.lev[k - 1];
  const long long N = interior(L.g, 3), Nc = interior(C.g, 3);
  const double bytes = sizeof(T) * (3.0 * N + Nc);
  Pair3Args a = pair3_args(h, k, h->ro.post);
  a.x = x; a.xc = xc; a.b = b; a.out = t;
  const int kc = Sel<T>::kc ? (KC_PRE3P32 - KC_PRE3P64) : 0;
  FMG_LAUNCH(h, st, KC_POST3P64 + kc, k, N, bytes, (launch_pair3_kernel<T, kP3Prolong>(a, st)));
  return bytes;
}

// One weighted-Jacobi sweep t = x + wd (b - A x) on level k: the grid kernel,
// or in 3D on request (positive sweep_rows) the plane-marching kernel.
template <int DIM, typename T>
double launch_sweep(const fmg_hierarchy* h, int k, const T* x, const T* b, T* t, T wd, hipStream_t st) {
  const LevelInfo& L = h->plan.lev[k];
  const long long N = interior(L.g, DIM);
  const double bytes = 3.0 * sizeof(T) * N;
  const int kc = Sel<T>::kc ? 1 : 0;
  const T scale = (T)L.scale;
  if (DIM == 3 && h->ro.o.sweep_rows > 0 && L.g.n >= 16) {
    int zc = 0, nzc = 0;
    const int blocks = smooth3s_blocks(L.g.n, zc, nzc);
    FMG_LAUNCH(h, st, KC_SMOOTH3S64 + kc, k, N, bytes,
               k_smooth3s<T><<<blocks, 64 * kS3Waves, 0, st>>>(L.g, x, b, t, wd, scale, zc, nzc));
  } else {
    FMG_LAUNCH(h, st, KC_SMOOTH64 + (Sel<T>::kc ? KC_SMOOTH32 - KC_SMOOTH64 : 0), k, N, bytes,
               k_smooth<DIM, T, false><<<grid_of(L.g, DIM), kBlock, 0, st>>>(L.g, x, b, t, wd, scale));
  }
  return bytes;
}

template <int DIM, typename T>
void vcycle(const fmg_hierarchy* h, Roles& R, int k, bool zero_init, hipStream_t st);

// V-cycle level k >= 2 of the variable-coefficient operator (float64): damped
// Jacobi sweeps with the level's stencil arrays, the residual into the spare
// array, its restriction P^T r, the coarse cycle, the correction and the
// post-sweeps.
template <int DIM>
void vcycle_var(const fmg_hierarchy* h, Roles& R, int k, bool zero_init, hipStream_t st) {
  const Plan& p = h->plan;
  const LevelInfo& L = p.lev[k];
  const LevelInfo& C = p.lev[k - 1];
  double*& x = R.x[k];
  double*& t = R.t[k];
  double* b = h->at<double>(p.off_b[k]);
  const double* W = h->at<double>(p.off_w[k]);
  const long long pl = p.wplane[k];
  const dim3 grid = grid_of(L.g, DIM);
  const long long N = interior(L.g, DIM), Nc = interior(C.g, DIM);
  const double nfw = (1 << DIM) - 1;      // weight planes read per node
  const int npre = h->ro.o.nu_pre, npost = h->ro.o.nu_post;
  if (zero_init && npre == 0)
    FMG_LAUNCH(h, st, KC_FILL, k, N, 8.0 * L.count, k_fill<double><<<256, 256, 0, st>>>(x, L.count, 0.0));
  for (int i = 0; i < npre; ++i) {
    if (zero_init && i == 0)
      FMG_LAUNCH(h, st, KC_SMOOTHW64_ZERO, k, N, 8.0 * (2.0 + nfw) * N,
                 k_smooth_w<DIM, true><<<grid, kBlock, 0, st>>>(L.g, x, b, t, W, pl, h->ro.pre[i]));
    else
      FMG_LAUNCH(h, st, KC_SMOOTHW64, k, N, 8.0 * (3.0 + nfw) * N,
                 k_smooth_w<DIM, false><<<grid, kBlock, 0, st>>>(L.g, x, b, t, W, pl, h->ro.pre[i]));
    std::swap(x, t);
  }
  FMG_LAUNCH(h, st, KC_RESIDW64, k, N, 8.0 * (3.0 + nfw) * N,
             k_resid_w<DIM><<<grid, kBlock, 0, st>>>(L.g, x, b, t, W, pl));
  FMG_LAUNCH(h, st, KC_RESTRICT64_R, k, N, 8.0 * (N + Nc),
             k_restrict<DIM><<<grid_of(C.g, DIM), kBlock, 0, st>>>(L.g, C.g, t, h->at<double>(p.off_b[k - 1])));
  vcycle<DIM, double>(h, R, k - 1, true, st);
  FMG_LAUNCH(h, st, KC_PROLONG64_ADD, k, N, 8.0 * (2 * N + Nc),
             k_prolong<DIM, double, true><<<grid, kBlock, 0, st>>>(C.g, L.g, R.x[k - 1], x));
  for (int i = 0; i < npost; ++i) {
    FMG_LAUNCH(h, st, KC_SMOOTHW64, k, N, 8.0 * (3.0 + nfw) * N,
               k_smooth_w<DIM, false><<<grid, kBlock, 0, st>>>(L.g, x, b, t, W, pl, h->ro.post[i]));
    std::swap(x, t);
  }
}

template <int DIM, typename T>
void vcycle(const fmg_hierarchy* h, Roles& R, int k, bool zero_init, hipStream_t st) {
  const Plan& p = h->plan;
  const LevelInfo& L = p.lev[k];
  T*& x = Sel<T>::x(R, k);
  T*& t = Sel<T>::t(R, k);
  T* b = Sel<T>::b(h, k);
  const int kc = Sel<T>::kc;
  const long long N = interior(L.g, DIM);
  const double s = sizeof(T);
  if (k == 1) {
    FMG_LAUNCH(h, st, KC_COARSE64 + kc, 1, N, 2 * s * N,
               k_coarse_solve<DIM, T><<<1, 64, 0, st>>>(L.g, p.N1, Sel<T>::ainv(h), b, x));
    return;
  }
  if constexpr (std::is_same<T, double>::value) {
    if (p.var) {
      vcycle_var<DIM>(h, R, k, zero_init, st);
      return;
    }
  }
  if (k <= p.tail_top && p.tail_dense) {
    // x_k = x0 + B_k (b_k - A_k x0) (zero start: B_k b_k), written to the
    // spare array so no block reads what another writes; roles of level k swap
    const long long Nk = interior(L.g, DIM);
    const int blocks = (int)((Nk + 3) / 4);
    FMG_LAUNCH(h, st, KC_VCYCLE_TAIL64 + (Sel<T>::kc ? 1 : 0), k, N, 8.0 * Nk * Nk + 3.0 * s * N,
               k_tail_dense<DIM, T><<<blocks, 256, sizeof(double) * Nk, st>>>(
                   L.g, h->at<double>(p.off_tailB[k]), (int)Nk, x, b, t, (T)L.scale, zero_init ? 1 : 0));
    std::swap(x, t);
    return;
  }
  if (k <= p.tail_top) {
    TailArgs<T> a;
    fill_tail_args<DIM, T>(h, R, k, a);
    a.zero_top = zero_init ? 1 : 0;
    double bytes = 0.0;
    for (int j = 1; j <= k; ++j)
      bytes += s * interior(p.lev[j].g, DIM) * (3.0 * (h->ro.o.nu_pre + h->ro.o.nu_post) + 4.0);
    int ns[kTailLevels + 1];
    for (int j = 1; j <= k; ++j) ns[j] = p.lev[j].g.n;
    const size_t lds = sizeof(T) * tail_lds_elements<DIM>(ns, k, a.lds_off);
    if (lds <= kTailLdsMax)
      FMG_LAUNCH(h, st, KC_VCYCLE_TAIL64 + (Sel<T>::kc ? 1 : 0), k, N, bytes,
                 k_vcycle_tail_lds<DIM, T><<<1, kTailThreads, lds, st>>>(a));
    else
      FMG_LAUNCH(h, st, KC_VCYCLE_TAIL64 + (Sel<T>::kc ? 1 : 0), k, N, bytes,
                 k_vcycle_tail<DIM, T><<<1, kTailThreads, 0, st>>>(a));
    // mirror the kernel's role swaps
    if ((h->ro.o.nu_pre + h->ro.o.nu_post) & 1)
      for (int j = 2; j <= k; ++j) std::swap(Sel<T>::x(R, j), Sel<T>::t(R, j));
    return;
  }
  const dim3 grid = grid_of(L.g, DIM);
  const T scale = (T)L.scale;
  const double D = 2.0 * DIM * L.scale;
  const int npre = h->ro.o.nu_pre, npost = h->ro.o.nu_post;
  if (DIM == 2 && npre == 2 && npost == 2) {
    // fused level kernels: two sweeps + residual + restriction, then
    // correction + two sweeps (each writes the spare array: one role swap)
    launch_pre2<T>(h, k, x, b, t, Sel<T>::b(h, k - 1), zero_init, st);
    std::swap(x, t);
    vcycle<DIM, T>(h, R, k - 1, true, st);
    launch_post2<T>(h, k, x, Sel<T>::x(R, k - 1), b, t, st);
    std::swap(x, t);
    return;
  }
  if (DIM == 3 && use_pair3(h, k)) {
    // two sweeps, residual + restriction, coarse cycle, correction + two sweeps
    // (each pair writes the spare array: one role swap)
    launch_pre3<T>(h, k, x, b, t, zero_init, st);
    std::swap(x, t);
    const LevelInfo& C = p.lev[k - 1];
    const long long Nc = interior(C.g, DIM);
    FMG_LAUNCH(h, st, KC_RESTRICT64 + kc, k, N, s * (2 * N + Nc),
               (launch_resid_restrict<DIM, T>(L.g, C.g, x, b, Sel<T>::b(h, k - 1), scale, st)));
    vcycle<DIM, T>(h, R, k - 1, true, st);
    launch_post3<T>(h, k, x, Sel<T>::x(R, k - 1), b, t, st);
    std::swap(x, t);
    return;
  }
  if (zero_init && npre == 0)
    FMG_LAUNCH(h, st, KC_FILL, k, N, s * L.count, k_fill<T><<<256, 256, 0, st>>>(x, L.count, T(0)));
  for (int i = 0; i < npre; ++i) {
    const T wd = (T)(h->ro.pre[i] / D);
    if (zero_init && i == 0)
      FMG_LAUNCH(h, st, KC_SMOOTH64_ZERO + kc, k, N, 2 * s * N,
                 k_smooth<DIM, T, true><<<grid, kBlock, 0, st>>>(L.g, x, b, t, wd, scale));
    else
      launch_sweep<DIM, T>(h, k, x, b, t, wd, st);
    std::swap(x, t);
  }
  const LevelInfo& C = p.lev[k - 1];
  const long long Nc = interior(C.g, DIM);
  FMG_LAUNCH(h, st, KC_RESTRICT64 + kc, k, N, s * (2 * N + Nc),
             (launch_resid_restrict<DIM, T>(L.g, C.g, x, b, Sel<T>::b(h, k - 1), scale, st)));
  vcycle<DIM, T>(h, R, k - 1, true, st);
  FMG_LAUNCH(h, st, KC_PROLONG64_ADD + kc, k, N, s * (2 * N + Nc),
             k_prolong<DIM, T, true><<<grid, kBlock, 0, st>>>(C.g, L.g, Sel<T>::x(R, k - 1), x));
  for (int i = 0; i < npost; ++i) {
    const T wd = (T)(h->ro.post[i] / D);
    launch_sweep<DIM, T>(h, k, x, b, t, wd, st);
    std::swap(x, t);
  }
}



inline size_t aug_pass_lds_bytes(const Plan& p) {
  const int ncell = p.dim == 2 ? p.nH * p.nH : p.nH * p.nH * p.nH;
  const int NQ = p.dim == 2 ? Acc<2>::NQ : Acc<3>::NQ;
  return sizeof(double) * (size_t)newton_kernel_lds_doubles(ncell, NQ, p.N1, kAugMaxThreads);
}

inline size_t fmg_tail_lds_bytes(const Plan& p) {
  const int ncell = p.dim == 2 ? p.nH * p.nH : p.nH * p.nH * p.nH;
  const int NQ = p.dim == 2 ? Acc<2>::NQ : Acc<3>::NQ;
  const size_t aug = (size_t)ncell * NQ + newton_scratch_doubles(p.N1);
  const size_t lev1 = level1_lds_doubles(p.N1);
  return std::max(aug, lev1) * sizeof(double);
}

// Mixed mode: the m V-cycles of a correction step run in float32 on the
// correction equation A e = r, r = b - A u formed once in float64 from the
// step's iterate u, and u += e once after the last cycle (u + V^m(0, r) equals
// m cycles from u in exact arithmetic: the cycle is affine in its start).
// Here one float32 V(2,2) cycle of that sequence at a level that uses the
// fused level kernels (2D streaming, 3D sweep pairs): the first cycle forms
// the float64 residual inside its pre-smoothing kernel, the last adds e to the
// float64 iterate inside its post-smoothing kernel (the separate residual and
// add kernels' operations, two launches and two passes over the level fewer);
// the cycles between run from the current e with r as right-hand side.
// Returns false where this does not apply.
template <int DIM>
bool mixed_cycle_fused(const fmg_hierarchy* h, Roles& R, int k, hipStream_t st, bool first, bool last) {
  const Plan& p = h->plan;
  const fmg_options& o = h->ro.o;
  if (DIM == 3 && use_pair3(h, k)) {
    // float64 residual inside the first float32 sweep pair, the float32
    // cycle, and the correction added to the float64 iterate inside the last
    const LevelInfo& L = p.lev[k];
    const LevelInfo& C = p.lev[k - 1];
    const long long N = interior(L.g, 3), Nc = interior(C.g, 3);
    float* r32 = h->at<float>(p.off_bs[k]);
    if (first) {
      Pair3Args a = pair3_args(h, k, h->ro.pre);
      a.x = R.x[k]; a.b = h->at<double>(p.off_b[k]); a.out = R.ts[k]; a.r32 = r32;
      FMG_LAUNCH(h, st, KC_PRE3P32, k, N, 16.0 * N + 8.0 * N, (launch_pair3_kernel<float, kP3Resid>(a, st)));
    } else {
      launch_pre3<float>(h, k, R.xs[k], r32, R.ts[k], false, st);
    }
    std::swap(R.xs[k], R.ts[k]);
    FMG_LAUNCH(h, st, KC_RESTRICT32, k, N, 4.0 * (2 * N + Nc),
               (launch_resid_restrict<3, float>(L.g, C.g, R.xs[k], r32, h->at<float>(p.off_bs[k - 1]),
                                                (float)L.scale, st)));
    vcycle<DIM, float>(h, R, k - 1, true, st);
    if (last) {
      Pair3Args q = pair3_args(h, k, h->ro.post);
      q.x = R.xs[k]; q.xc = R.xs[k - 1]; q.b = r32; q.u64 = R.x[k];
      FMG_LAUNCH(h, st, KC_POST3P32, k, N, 4.0 * (2 * N + Nc) + 16.0 * N,
                 (launch_pair3_kernel<float, kP3ProlongAdd>(q, st)));
    } else {
      launch_post3<float>(h, k, R.xs[k], R.xs[k - 1], r32, R.ts[k], st);
      std::swap(R.xs[k], R.ts[k]);
    }
    return true;
  }
  if (DIM != 2 || o.nu_pre != 2 || o.nu_post != 2 || k <= p.tail_top || k < 2) return false;
  const LevelInfo& L = p.lev[k];
  const LevelInfo& C = p.lev[k - 1];
  const int rows = stream_rows(o.sweep_rows, L.g.n);
  if (rows <= 0) return false;
  const long long N = interior(L.g, 2), Nc = interior(C.g, 2);
  const double D = 4.0 * L.scale;
  double* u = R.x[k];
  const double* b64 = h->at<double>(p.off_b[k]);
  float* r32 = h->at<float>(p.off_bs[k]);
  int nch = 0;
  if (first) {
    const int gpre = stream_blocks(L.g.n, kResStrip, rows, nch);
    FMG_LAUNCH(h, st, KC_PRE2S32, k, N, 16.0 * N + 8.0 * N + 4.0 * Nc,
               k_pre2s_resid<<<gpre, 64 * kStreamWaves, 0, st>>>(
                   L.g, C.g, u, b64, r32, R.ts[k], h->at<float>(p.off_bs[k - 1]), (float)(h->ro.pre[0] / D),
                   (float)(h->ro.pre[1] / D), (float)L.scale, L.scale, rows, nch));
  } else {
    launch_pre2<float>(h, k, R.xs[k], r32, R.ts[k], h->at<float>(p.off_bs[k - 1]), false, st);
  }
  std::swap(R.xs[k], R.ts[k]);
  vcycle<DIM, float>(h, R, k - 1, true, st);
  if (last) {
    const int gpost = stream_blocks(L.g.n, kPostStrip, rows, nch);
    FMG_LAUNCH(h, st, KC_POST2S32, k, N, 8.0 * N + 16.0 * N + 4.0 * Nc,
               k_post2s<float, true><<<gpost, 64 * kStreamWaves, 0, st>>>(
                   C.g, L.g, R.xs[k], R.xs[k - 1], r32, nullptr, u, (float)(h->ro.post[0] / D),
                   (float)(h->ro.post[1] / D), (float)L.scale, rows, nch));
  } else {
    launch_post2<float>(h, k, R.xs[k], R.xs[k - 1], r32, R.ts[k], st);
    std::swap(R.xs[k], R.ts[k]);
  }
  return true;
}

// One correction step (Algorithm 3.1) on level k; the current iterate is R.x[k].
// rhs_ready: b_k was already formed (by the level transition).  defer_update:
// leave u = Q w + alpha u~ to the consumer (next transition or the output).
// Transitions into fine levels with at most this many interior nodes run at
// the end of the coarser level's single-workgroup kernel (level 1, or the
// small-level augmented solve) instead of in a launch of their own.
constexpr long long kFoldTransitionNodes = 1024;

// Arguments of the level transition into level k (from the current u~ of k-1).
TransitionArgs transition_args(const fmg_hierarchy* h, const Roles& R, int k, bool use_aug) {
  const Plan& p = h->plan;
  TransitionArgs a;
  a.gc = p.lev[k - 1].g;
  a.gf = p.lev[k].g;
  a.sf = p.lev[k].aug;
  a.uc = R.x[k - 1];
  a.uf = R.x[k];
  a.bf = h->at<double>(p.off_b[k]);
  a.use_aug = use_aug ? 1 : 0;
  a.nf1 = p.lev[p.nlev].g.n + 1;
  a.fs = 1 << (p.nlev - k);
  a.m = p.lev[k].m;
  return a;
}

// Algorithm 3.1, step 2 with the element rule on level k (k = 1: the level-1
// problem of Algorithm 3.2, step 1, as the augmented problem with u~ = 0, so
// that V_H + span{u~} = V_H): the setup pass, the quadrature passes of the
// launch sequence, the finisher, and the update u = Q w + alpha u~ unless
// deferred.
template <int DIM, int KIND>
void aug_solve_elem(const fmg_hierarchy* h, Roles& R, int k, hipStream_t st, bool defer_update) {
  const Plan& p = h->plan;
  const LevelInfo& L = p.lev[k];
  const fmg_options& o = h->ro.o;
  const long long N = interior(L.g, DIM);
  const int nf1 = p.lev[p.nlev].g.n + 1, fs = 1 << (p.nlev - k);
  double* pq = h->at<double>(p.off_pq);
  double* ps = h->at<double>(p.off_ps);
  unsigned* ticket = h->at<unsigned>(p.off_ticket);
  const double* A1 = h->at<double>(p.off_A1);
  const size_t lds = aug_pass_lds_bytes(p);
  FMG_LAUNCH(h, st, KC_AUG_PASS0, k, N, 16.0 * N,
             (launch_aug_pass<DIM, KIND, true, false, true>(L.aug_blocks, L.aug_threads, lds, st, L.g, L.aug, R.x[k],
                                                            h->slot(), nf1, fs, L.scale, L.m, A1, h->ns(), h->rep(),
                                                            pq, ps, ticket, k, o.newton_max, o.newton_tol)));
  for (int pass = 1; pass < o.newton_passes; ++pass)
    FMG_LAUNCH(h, st, KC_AUG_PASS, k, N, 8.0 * N,
               (launch_aug_pass<DIM, KIND, false, false, true>(L.aug_blocks, L.aug_threads, lds, st, L.g, L.aug,
                                                               R.x[k], h->slot(), nf1, fs, L.scale, L.m, A1, h->ns(),
                                                               h->rep(), pq, ps, ticket, k, o.newton_max,
                                                               o.newton_tol)));
  FMG_LAUNCH(h, st, KC_NEWTON_FINISH, k, N, 0.0,
             (launch_newton_finish<DIM, KIND, true>(lds, st, L.g, L.aug, R.x[k], h->slot(), A1, L.m, h->ns(),
                                                    h->rep(), o.newton_max, o.newton_tol)));
  if (!defer_update)
    FMG_LAUNCH(h, st, KC_AUG_UPDATE, k, N, 16.0 * N,
               k_aug_update<DIM><<<grid_of(L.g, DIM), kBlock, 0, st>>>(L.g, L.aug, h->ns(), R.x[k]));
}

// Algorithm 3.1, step 2 with the variable-coefficient operator: the setup
// pass (A u~ from the level's stencil arrays), the quadrature passes of the
// launch sequence (weighted by c(x) when the problem gives it), the
// finisher, and the update unless deferred.
template <int DIM, int KIND>
void aug_solve_var(const fmg_hierarchy* h, Roles& R, int k, hipStream_t st, bool defer_update) {
  const Plan& p = h->plan;
  const LevelInfo& L = p.lev[k];
  const fmg_options& o = h->ro.o;
  const long long N = interior(L.g, DIM);
  const int nf1 = p.lev[p.nlev].g.n + 1, fs = 1 << (p.nlev - k);
  double* pq = h->at<double>(p.off_pq);
  double* ps = h->at<double>(p.off_ps);
  unsigned* ticket = h->at<unsigned>(p.off_ticket);
  const double* A1 = h->at<double>(p.off_A1);
  const size_t lds = aug_pass_lds_bytes(p);
  const double nfw = (1 << DIM) - 1;
  FMG_LAUNCH(h, st, KC_AUG_PASS0, k, N, (16.0 + 8.0 * nfw) * N,
             (launch_aug_pass<DIM, KIND, true, false, false, true>(L.aug_blocks, L.aug_threads, lds, st, L.g, L.aug,
                                                                   R.x[k], h->slot(), nf1, fs, L.scale, L.m, A1,
                                                                   h->ns(), h->rep(), pq, ps, ticket, k,
                                                                   o.newton_max, o.newton_tol)));
  for (int pass = 1; pass < o.newton_passes; ++pass)
    FMG_LAUNCH(h, st, KC_AUG_PASS, k, N, 8.0 * N,
               (launch_aug_pass<DIM, KIND, false, false, false, true>(L.aug_blocks, L.aug_threads, lds, st, L.g,
                                                                      L.aug, R.x[k], h->slot(), nf1, fs, L.scale,
                                                                      L.m, A1, h->ns(), h->rep(), pq, ps, ticket, k,
                                                                      o.newton_max, o.newton_tol)));
  FMG_LAUNCH(h, st, KC_NEWTON_FINISH, k, N, 0.0,
             (launch_newton_finish<DIM, KIND, false, true>(lds, st, L.g, L.aug, R.x[k], h->slot(), A1, L.m, h->ns(),
                                                           h->rep(), o.newton_max, o.newton_tol)));
  if (!defer_update)
    FMG_LAUNCH(h, st, KC_AUG_UPDATE, k, N, 16.0 * N,
               k_aug_update<DIM><<<grid_of(L.g, DIM), kBlock, 0, st>>>(L.g, L.aug, h->ns(), R.x[k]));
}

// The first float64 V-cycle of level k's first correction step on a 3D
// sweep-pair level whose transition wrote only b_k: the pre-smoothing pair
// starts from x0 = P u_{k-1} (the previous level's result, up to date), formed
// as the pair's planes arrive.  The rest is the cycle of vcycle's sweep-pair
// branch.
inline void vcycle_from_prolongation3(const fmg_hierarchy* h, Roles& R, int k, hipStream_t st) {
  const Plan& p = h->plan;
  const LevelInfo& L = p.lev[k];
  const LevelInfo& C = p.lev[k - 1];
  const long long N = interior(L.g, 3), Nc = interior(C.g, 3);
  double* b = h->at<double>(p.off_b[k]);
  Pair3Args a = pair3_args(h, k, h->ro.pre);
  a.xc = R.x[k - 1];
  a.b = b;
  a.out = R.t[k];
  FMG_LAUNCH(h, st, KC_PRE3P64, k, N, 8.0 * (2 * N + Nc), (launch_pair3_kernel<double, kP3ProlongFresh>(a, st)));
  std::swap(R.x[k], R.t[k]);
  FMG_LAUNCH(h, st, KC_RESTRICT64, k, N, 8.0 * (2 * N + Nc),
             (launch_resid_restrict<3, double>(L.g, C.g, R.x[k], b, h->at<double>(p.off_b[k - 1]), L.scale, st)));
  vcycle<3, double>(h, R, k - 1, true, st);
  launch_post3<double>(h, k, R.x[k], R.x[k - 1], b, R.t[k], st);
  std::swap(R.x[k], R.t[k]);
}

// fused_transition: the level transition into k wrote only b_k; the first
// cycle starts from P u_{k-1} (vcycle_from_prolongation3).
template <int DIM, int KIND>
void correction_step_with(const fmg_hierarchy* h, Roles& R, int k, hipStream_t st, bool rhs_ready,
                          bool defer_update, bool fold_next, bool fused_transition) {
  const Plan& p = h->plan;
  const LevelInfo& L = p.lev[k];
  const fmg_options& o = h->ro.o;
  const dim3 grid = grid_of(L.g, DIM);
  const long long N = interior(L.g, DIM);
  const int nf1 = p.lev[p.nlev].g.n + 1, fs = 1 << (p.nlev - k);
  double* b = h->at<double>(p.off_b[k]);
  const bool elem = o.quadrature == FMG_QUAD_ELEMENT;
  // step 1: linearised problem, m V-cycles from u^(l); the element rule's
  // load couples neighbouring nodes, so it is formed here, after the
  // transition has written u (the transition's vertex-rule b is replaced)
  if (elem)
    FMG_LAUNCH(h, st, KC_RHS_ELEM, k, N, (DIM == 2 ? 88.0 : 152.0) * N,
               (launch_rhs_elem<DIM, KIND>(grid, st, L.g, h->slot(), nf1, fs, R.x[k],
                                           h->at<double>(p.off_econtrib), b, L.m)));
  else if (!rhs_ready && p.var)
    FMG_LAUNCH(h, st, KC_RHS, k, N, 24.0 * N,
               (launch_rhs<DIM, KIND, true>(grid, st, L.g, h->slot(), nf1, fs, R.x[k], b, L.m)));
  else if (!rhs_ready)
    FMG_LAUNCH(h, st, KC_RHS, k, N, 24.0 * N,
               (launch_rhs<DIM, KIND>(grid, st, L.g, h->slot(), nf1, fs, R.x[k], b, L.m)));
  for (int c = 0; c < o.m_vcycles; ++c) {
    if (o.precision == FMG_FP64) {
      if constexpr (DIM == 3) {
        if (c == 0 && fused_transition) {
          vcycle_from_prolongation3(h, R, k, st);
          continue;
        }
      }
      vcycle<DIM, double>(h, R, k, false, st);
    } else if (!mixed_cycle_fused<DIM>(h, R, k, st, c == 0, c == o.m_vcycles - 1)) {
      // float32 cycles on the correction equation: float64 residual before the
      // first, float64 update after the last
      if (c == 0)
        FMG_LAUNCH(h, st, KC_RESID_F32, k, N, 20.0 * N,
                   k_resid_to_f32<DIM><<<grid, kBlock, 0, st>>>(L.g, R.x[k], b, h->at<float>(p.off_bs[k]),
                                                                L.scale));
      vcycle<DIM, float>(h, R, k, c == 0, st);
      if (c == o.m_vcycles - 1)
        FMG_LAUNCH(h, st, KC_ADD_F32, k, N, 20.0 * N,
                   k_add_f32<DIM><<<grid, kBlock, 0, st>>>(L.g, R.x[k], R.xs[k]));
    }
  }
  // step 2: semilinear problem on V_H + span{u~}
  double* pq = h->at<double>(p.off_pq);
  double* ps = h->at<double>(p.off_ps);
  unsigned* ticket = h->at<unsigned>(p.off_ticket);
  const double* A1 = h->at<double>(p.off_A1);
  if (elem) {
    aug_solve_elem<DIM, KIND>(h, R, k, st, defer_update);
    return;
  }
  if (p.var) {
    aug_solve_var<DIM, KIND>(h, R, k, st, defer_update);
    return;
  }
  if (N <= o.aug_small_nodes) {
    // the whole augmented solve (and the update unless deferred) by one workgroup
    FMG_LAUNCH(h, st, KC_AUG_SMALL, k, N, 0.0,
               (launch_aug_small<DIM, KIND>(
                   fmg_tail_lds_bytes(p), st, L.g, L.aug, R.x[k], h->slot(), nf1, fs, L.scale, L.m, A1, h->ns(),
                   h->rep(), k, o.newton_max, o.newton_tol, defer_update ? 0 : 1, fold_next ? 1 : 0,
                   fold_next ? transition_args(h, R, k + 1, defer_update) : TransitionArgs{})));
    return;
  }
  const size_t lds = aug_pass_lds_bytes(p);
  const int npass = o.newton_passes;   // setup pass + npass - 1 quadrature passes
  constexpr bool kFinishInPass = DIM == 2;
  if (npass == 1 && kFinishInPass)
    FMG_LAUNCH(h, st, KC_AUG_PASS0, k, N, 16.0 * N,
               (launch_aug_pass<DIM, KIND, true, true>(L.aug_blocks, L.aug_threads, lds, st, 
                   L.g, L.aug, R.x[k], h->slot(), nf1, fs, L.scale, L.m, A1, h->ns(), h->rep(), pq, ps, ticket, k,
                   o.newton_max, o.newton_tol)));
  else
    FMG_LAUNCH(h, st, KC_AUG_PASS0, k, N, 16.0 * N,
               (launch_aug_pass<DIM, KIND, true, false>(L.aug_blocks, L.aug_threads, lds, st, 
                   L.g, L.aug, R.x[k], h->slot(), nf1, fs, L.scale, L.m, A1, h->ns(), h->rep(), pq, ps, ticket, k,
                   o.newton_max, o.newton_tol)));
  for (int pass = 1; pass < npass; ++pass) {
    if (pass == npass - 1 && kFinishInPass)
      FMG_LAUNCH(h, st, KC_AUG_PASS, k, N, 8.0 * N,
                 (launch_aug_pass<DIM, KIND, false, true>(L.aug_blocks, L.aug_threads, lds, st, 
                     L.g, L.aug, R.x[k], h->slot(), nf1, fs, L.scale, L.m, A1, h->ns(), h->rep(), pq, ps,
                     ticket, k, o.newton_max, o.newton_tol)));
    else
      FMG_LAUNCH(h, st, KC_AUG_PASS, k, N, 8.0 * N,
                 (launch_aug_pass<DIM, KIND, false, false>(L.aug_blocks, L.aug_threads, lds, st, 
                     L.g, L.aug, R.x[k], h->slot(), nf1, fs, L.scale, L.m, A1, h->ns(), h->rep(), pq, ps,
                     ticket, k, o.newton_max, o.newton_tol)));
  }
  if constexpr (!kFinishInPass)
    FMG_LAUNCH(h, st, KC_NEWTON_FINISH, k, N, 0.0,
               (launch_newton_finish<DIM, KIND>(lds, st, L.g, L.aug, R.x[k], h->slot(), A1, L.m, h->ns(), h->rep(),
                                                o.newton_max, o.newton_tol)));
  if (!defer_update)
    FMG_LAUNCH(h, st, KC_AUG_UPDATE, k, N, 16.0 * N,
               k_aug_update<DIM><<<grid, kBlock, 0, st>>>(L.g, L.aug, h->ns(), R.x[k]));
}

template <int DIM, int KIND>
void correction_step(const fmg_hierarchy* h, Roles& R, int k, hipStream_t st, bool rhs_ready,
                     bool defer_update, bool fold_next) {
  correction_step_with<DIM, KIND>(h, R, k, st, rhs_ready, defer_update, fold_next, false);
}

template <int DIM, int KIND>
void record_fmg(const fmg_hierarchy* h, Roles& R, bool finish, hipStream_t st) {
  const Plan& p = h->plan;
  const fmg_options& o = h->ro.o;
  const int nf1 = p.lev[p.nlev].g.n + 1;
  int first = 2;
  bool folded = false;   // the transition into the next level is done already
  if (p.tail_top >= 2 && o.fuse_small_levels) {
    FMG_LAUNCH(h, st, KC_BEGIN, 0, 0, 0.0, k_begin_solve<<<1, 64, 0, st>>>(h->rep(), p.nlev, h->flag()));
    // Algorithm 3.2 on levels 1..T in one single-workgroup launch
    const int T = std::min(p.tail_top, p.nlev);
    const size_t lds = fmg_tail_lds_bytes(p);
    const FmgTailParams* P = h->at<FmgTailParams>(p.off_fmgtail);
    if (o.precision == FMG_FP64)
      FMG_LAUNCH(h, st, KC_FMG_TAIL, T, interior(p.lev[T].g, DIM), 0.0,
                 (launch_fmg_tail<DIM, KIND, false>(lds, st, P)));
    else
      FMG_LAUNCH(h, st, KC_FMG_TAIL, T, interior(p.lev[T].g, DIM), 0.0,
                 (launch_fmg_tail<DIM, KIND, true>(lds, st, P)));
    // mirror the role swaps of the V-cycles inside
    const bool odd = (o.nu_pre + o.nu_post) & 1;
    for (int k = 2; k <= T; ++k)
      for (int c = 0; c < o.p_steps * o.m_vcycles; ++c)
        if (odd)
          for (int j = 2; j <= k; ++j) {
            if (o.precision == FMG_FP64) std::swap(R.x[j], R.t[j]);
            else std::swap(R.xs[j], R.ts[j]);
          }
    first = T + 1;
  } else if (o.quadrature == FMG_QUAD_ELEMENT) {
    // report reset; Algorithm 3.2, step 1 as the augmented problem on level 1
    // with u~ = 0 (its u~ direction adds nothing and is dropped), then u = w
    FMG_LAUNCH(h, st, KC_BEGIN, 0, 0, 0.0, k_begin_solve<<<1, 64, 0, st>>>(h->rep(), p.nlev, h->flag()));
    const LevelInfo& L1 = p.lev[1];
    FMG_LAUNCH(h, st, KC_FILL, 1, p.N1, 0.0,
               k_fill<double><<<64, 256, 0, st>>>(R.x[1], L1.count, 0.0));
    aug_solve_elem<DIM, KIND>(h, R, 1, st, false);
  } else {
    // report reset and Algorithm 3.2, step 1: exact semilinear solve on V_{h_1}
    const LevelInfo& L1 = p.lev[1];
    const size_t lds1 = sizeof(double) * (size_t)level1_lds_doubles(p.N1);
    // (the variable-coefficient transitions, which apply c(x), run as launches of their own)
    folded = !p.var && p.nlev >= 2 && interior(p.lev[2].g, DIM) <= kFoldTransitionNodes;
    FMG_LAUNCH(h, st, KC_LEVEL1, 1, p.N1, 0.0,
               (launch_level1<DIM, KIND>(lds1, st, L1.g, p.N1, h->at<double>(p.off_A1), L1.m, h->slot(), nf1,
                                         1 << (p.nlev - 1), R.x[1], h->rep(), o.newton_max, o.newton_tol, p.nlev,
                                         h->flag(), folded ? 1 : 0,
                                         folded ? transition_args(h, R, 2, false) : TransitionArgs{})));
  }
  // step 2: levels k = first..n
  bool pending_aug = false;   // last update of level k-1 left to the transition
  for (int k = first; k <= p.nlev; ++k) {
    const LevelInfo& L = p.lev[k];
    const LevelInfo& C = p.lev[k - 1];
    const long long N = interior(L.g, DIM);
    // 3D float64 sweep-pair levels: the previous level's result is brought up
    // to date here (u = Q w + alpha u~; P u equals the deferred form
    // Q w + alpha P u~), the transition writes only b_k = M_k (g - f(P u)),
    // and the first pre-smoothing pair forms x0 = P u itself
    const bool fuse_tr = DIM == 3 && !folded && !p.var && o.precision == FMG_FP64 &&
                         o.quadrature == FMG_QUAD_VERTEX && o.m_vcycles >= 1 && o.p_steps >= 1 && use_pair3(h, k);
    if (fuse_tr) {
      if constexpr (DIM == 3) {
        if (pending_aug)
          FMG_LAUNCH(h, st, KC_AUG_UPDATE, k - 1, interior(C.g, DIM), 16.0 * interior(C.g, DIM),
                     k_aug_update<DIM><<<grid_of(C.g, DIM), kBlock, 0, st>>>(C.g, C.aug, h->ns(), R.x[k - 1]));
        FMG_LAUNCH(h, st, KC_TRANSITION, k, N, 8.0 * (2 * N + interior(C.g, DIM)),
                   (launch_transition_rhs<DIM, KIND>(grid_of(L.g, DIM), st, transition_args(h, R, k, false),
                                                     h->slot())));
      }
    } else if (!folded && p.var)
      FMG_LAUNCH(h, st, KC_TRANSITION, k, N, 8.0 * (3 * N + interior(C.g, DIM)),
                 (pending_aug ? launch_transition<DIM, KIND, true, true>(grid_of(L.g, DIM), st,
                                                                         transition_args(h, R, k, true), h->ns(),
                                                                         h->slot())
                              : launch_transition<DIM, KIND, false, true>(grid_of(L.g, DIM), st,
                                                                          transition_args(h, R, k, false), h->ns(),
                                                                          h->slot())));
    else if (!folded && pending_aug)
      FMG_LAUNCH(h, st, KC_TRANSITION, k, N, 8.0 * (3 * N + interior(C.g, DIM)),
                 (launch_transition<DIM, KIND, true>(grid_of(L.g, DIM), st, transition_args(h, R, k, true), h->ns(),
                                                     h->slot())));
    else if (!folded)
      FMG_LAUNCH(h, st, KC_TRANSITION, k, N, 8.0 * (3 * N + interior(C.g, DIM)),
                 (launch_transition<DIM, KIND, false>(grid_of(L.g, DIM), st, transition_args(h, R, k, false),
                                                      h->ns(), h->slot())));
    folded = false;
    for (int l = 0; l < o.p_steps; ++l) {
      const bool defer = l == o.p_steps - 1 && (k < p.nlev || finish);
      // the last small-level augmented solve also performs a small next transition
      const bool fold = o.quadrature == FMG_QUAD_VERTEX && defer && k < p.nlev && N <= o.aug_small_nodes &&
                        interior(p.lev[k + 1].g, DIM) <= kFoldTransitionNodes;
      correction_step_with<DIM, KIND>(h, R, k, st, l == 0, defer, fold, fuse_tr && l == 0);
      pending_aug = defer;
      folded = fold;
    }
  }
  if (finish) {
    const LevelInfo& F = p.lev[p.nlev];
    const double nodes = DIM == 2 ? (double)(F.g.n + 1) * (F.g.n + 1) : (double)(F.g.n + 1) * (F.g.n + 1) * (F.g.n + 1);
    if (pending_aug)
      FMG_LAUNCH(h, st, KC_OUTPUT_UPDATE, p.nlev, interior(F.g, DIM), 16.0 * nodes,
                 k_output_update<DIM><<<output_blocks<DIM>(F.g), 256, 0, st>>>(F.g, F.aug, h->ns(), R.x[p.nlev],
                                                                                h->slot(), h->flag()));
    else
      FMG_LAUNCH(h, st, KC_OUTPUT, p.nlev, interior(F.g, DIM), 16.0 * nodes,
                 k_output<DIM><<<output_blocks<DIM>(F.g), 256, 0, st>>>(F.g, R.x[p.nlev], h->slot(), h->flag()));
    FMG_LAUNCH(h, st, KC_END, 0, 0, 0.0, k_end_solve<<<1, 64, 0, st>>>(h->rep(), h->flag(), h->slot()));
  }
}

typedef void (*record_fn)(const fmg_hierarchy*, Roles&, bool, hipStream_t);
typedef void (*step_fn)(const fmg_hierarchy*, Roles&, int, hipStream_t, bool, bool, bool);

template <int DIM>
record_fn pick_record(int kind) {
  switch (kind) {
    case FMG_F_ZERO: return record_fmg<DIM, FMG_F_ZERO>;
    case FMG_F_LINEAR: return record_fmg<DIM, FMG_F_LINEAR>;
    case FMG_F_CUBIC: return record_fmg<DIM, FMG_F_CUBIC>;
    case FMG_F_U_PLUS_SIN: return record_fmg<DIM, FMG_F_U_PLUS_SIN>;
    case FMG_F_ABS_U_U: return record_fmg<DIM, FMG_F_ABS_U_U>;
    case FMG_F_SIGNED_POW: return record_fmg<DIM, FMG_F_SIGNED_POW>;
    default: return record_fmg<DIM, FMG_F_NEG_EXP>;
  }
}
template <int DIM>
step_fn pick_step(int kind) {
  switch (kind) {
    case FMG_F_ZERO: return correction_step<DIM, FMG_F_ZERO>;
    case FMG_F_LINEAR: return correction_step<DIM, FMG_F_LINEAR>;
    case FMG_F_CUBIC: return correction_step<DIM, FMG_F_CUBIC>;
    case FMG_F_U_PLUS_SIN: return correction_step<DIM, FMG_F_U_PLUS_SIN>;
    case FMG_F_ABS_U_U: return correction_step<DIM, FMG_F_ABS_U_U>;
    case FMG_F_SIGNED_POW: return correction_step<DIM, FMG_F_SIGNED_POW>;
    default: return correction_step<DIM, FMG_F_NEG_EXP>;
  }
}

int check_problem(const fmg_problem* prob) {
  if (!prob || !prob->g_nodes) return FMG_E_INVALID;
  if (prob->kind < FMG_F_ZERO || prob->kind > FMG_F_NEG_EXP) return FMG_E_INVALID;
  if (prob->kind == FMG_F_LINEAR && !(prob->param >= 0)) return FMG_E_INVALID;
  if (prob->kind == FMG_F_SIGNED_POW && !(prob->param >= 1)) return FMG_E_INVALID;
  return FMG_OK;
}

// check_problem plus what the hierarchy needs: the coefficients set (variable
// coefficient), and a weight c(x) only where the variable-coefficient
// kernels run.
int check_problem_for(const fmg_hierarchy* h, const fmg_problem* prob) {
  const int st = check_problem(prob);
  if (st != FMG_OK) return st;
  if (h->plan.var && !h->coef_ready) return FMG_E_INVALID;
  if (prob->f_weight && !h->plan.var) return FMG_E_UNSUPPORTED;
  return FMG_OK;
}

void build_level1(const Plan& p, std::vector<double>& A, std::vector<double>& Ainv) {
  // A_1 on the interior nodes of the coarse grid: scale (2d on the diagonal,
  // -1 for the axis neighbours), dense, x fastest.
  const int d = p.dim, m = p.nH - 1, N = p.N1;
  const double s = p.lev[1].scale;
  A.assign((size_t)N * N, 0.0);
  for (int r = 0; r < N; ++r) {
    const int i = r % m, j = (r / m) % m, l = d == 3 ? r / (m * m) : 0;
    A[(size_t)r * N + r] = 2.0 * d * s;
    auto link = [&](int ii, int jj, int ll) {
      if (ii < 0 || jj < 0 || ll < 0 || ii >= m || jj >= m || ll >= (d == 3 ? m : 1)) return;
      A[(size_t)r * N + (ii + m * jj + m * m * ll)] = -s;
    };
    link(i - 1, j, l); link(i + 1, j, l); link(i, j - 1, l); link(i, j + 1, l);
    if (d == 3) { link(i, j, l - 1); link(i, j, l + 1); }
  }
  // Gauss-Jordan inverse with partial pivoting
  std::vector<double> M(A);
  Ainv.assign((size_t)N * N, 0.0);
  for (int r = 0; r < N; ++r) Ainv[(size_t)r * N + r] = 1.0;
  for (int c = 0; c < N; ++c) {
    int piv = c;
    for (int r = c + 1; r < N; ++r)
      if (std::fabs(M[(size_t)r * N + c]) > std::fabs(M[(size_t)piv * N + c])) piv = r;
    if (piv != c)
      for (int k = 0; k < N; ++k) {
        std::swap(M[(size_t)c * N + k], M[(size_t)piv * N + k]);
        std::swap(Ainv[(size_t)c * N + k], Ainv[(size_t)piv * N + k]);
      }
    const double inv = 1.0 / M[(size_t)c * N + c];
    for (int k = 0; k < N; ++k) { M[(size_t)c * N + k] *= inv; Ainv[(size_t)c * N + k] *= inv; }
    for (int r = 0; r < N; ++r) {
      if (r == c) continue;
      const double f = M[(size_t)r * N + c];
      if (f == 0.0) continue;
      for (int k = 0; k < N; ++k) {
        M[(size_t)r * N + k] -= f * M[(size_t)c * N + k];
        Ainv[(size_t)r * N + k] -= f * Ainv[(size_t)c * N + k];
      }
    }
  }
}

// build_level1 on the device (one workgroup, N <= 64 threads): the same
// matrix, the same Gauss-Jordan elimination with the same pivots, and
// products rounded before the subtraction as on the host, so the tables are
// the same bits; for launches that may not copy from host memory.  smem holds
// 2 N^2 doubles (M, then the inverse being formed).
__global__ void k_level1_tables(int d, int nH, double s, double* __restrict__ A, double* __restrict__ Ainv,
                                float* __restrict__ Ainv_f) {
  extern __shared__ double smem[];
  const int m = nH - 1;
  const int N = d == 2 ? m * m : m * m * m;
  double* M = smem;
  double* V = smem + N * N;
  const int t = threadIdx.x;
  if (t < N) {
    const int i = t % m, j = (t / m) % m, l = d == 3 ? t / (m * m) : 0;
    for (int c = 0; c < N; ++c) { M[t * N + c] = 0.0; V[t * N + c] = c == t ? 1.0 : 0.0; }
    M[t * N + t] = 2.0 * d * s;
    auto link = [&](int ii, int jj, int ll) {
      if (ii < 0 || jj < 0 || ll < 0 || ii >= m || jj >= m || ll >= (d == 3 ? m : 1)) return;
      M[t * N + (ii + m * jj + m * m * ll)] = -s;
    };
    link(i - 1, j, l); link(i + 1, j, l); link(i, j - 1, l); link(i, j + 1, l);
    if (d == 3) { link(i, j, l - 1); link(i, j, l + 1); }
    for (int c = 0; c < N; ++c) A[t * N + c] = M[t * N + c];
  }
  __syncthreads();
  __shared__ int piv_s;
  for (int c = 0; c < N; ++c) {
    if (t == 0) {
      int piv = c;
      for (int r = c + 1; r < N; ++r)
        if (fabs(M[r * N + c]) > fabs(M[piv * N + c])) piv = r;
      piv_s = piv;
    }
    __syncthreads();
    const int piv = piv_s;
    if (piv != c && t < N) {   // thread t swaps column t of the two rows
      double a = M[c * N + t]; M[c * N + t] = M[piv * N + t]; M[piv * N + t] = a;
      a = V[c * N + t]; V[c * N + t] = V[piv * N + t]; V[piv * N + t] = a;
    }
    __syncthreads();
    const double inv = 1.0 / M[c * N + c];
    __syncthreads();
    if (t < N) { M[c * N + t] = __dmul_rn(M[c * N + t], inv); V[c * N + t] = __dmul_rn(V[c * N + t], inv); }
    __syncthreads();
    if (t < N && t != c) {     // thread t updates row t (row c is only read)
      const double f = M[t * N + c];
      if (f != 0.0)
        for (int k = 0; k < N; ++k) {
          M[t * N + k] = M[t * N + k] - __dmul_rn(f, M[c * N + k]);
          V[t * N + k] = V[t * N + k] - __dmul_rn(f, V[c * N + k]);
        }
    }
    __syncthreads();
  }
  if (t < N)
    for (int c = 0; c < N; ++c) {
      Ainv[t * N + c] = V[t * N + c];
      Ainv_f[t * N + c] = (float)V[t * N + c];
    }
}

// The V-cycle of levels k..1 from a zero start is a linear map b_k -> x_k
// (pre-smoothing, residual, P^T, exact level-1 solve, P-correction,
// post-smoothing; the same steps and weights as the device cycle).  Its
// matrix B_k is built here by running that cycle on the host for every unit
// vector; a cycle from x0 is then x0 + B_k (b - A_k x0).
struct HostLevel {
  int n;
  double scale;
  std::vector<double> x, t, b;
};

void build_tail_operators(const Plan& p, const Resolved& ro, const std::vector<double>& A1inv,
                          std::vector<std::vector<double>>& Bs) {
  const int d = p.dim;
  Bs.assign(p.tail_top + 1, {});
  auto idx = [&](int n, int i, int j, int l) { return i + (n + 1) * (j + (n + 1) * l); };
  auto count = [&](int n) { return (size_t)(d == 2 ? (n + 1) * (n + 1) : (n + 1) * (n + 1) * (n + 1)); };
  auto interior = [&](int n, auto&& fn) {
    for (int l = (d == 3 ? 1 : 0); l <= (d == 3 ? n - 1 : 0); ++l)
      for (int j = 1; j <= n - 1; ++j)
        for (int i = 1; i <= n - 1; ++i) fn(i, j, l);
  };
  auto applyA = [&](const HostLevel& L, const std::vector<double>& x, int i, int j, int l) {
    const int n = L.n, c = idx(n, i, j, l), px = n + 1, pz = (n + 1) * (n + 1);
    double sm = (x[c - 1] + x[c + 1]) + (x[c - px] + x[c + px]);
    if (d == 3) sm += x[c - pz] + x[c + pz];
    return L.scale * (2.0 * d * x[c] - sm);
  };
  for (int top = 2; top <= p.tail_top; ++top) {
    std::vector<HostLevel> lv(top + 1);
    for (int k = 1; k <= top; ++k) {
      lv[k].n = p.lev[k].g.n;
      lv[k].scale = p.lev[k].scale;
      lv[k].x.assign(count(lv[k].n), 0.0);
      lv[k].t.assign(count(lv[k].n), 0.0);
      lv[k].b.assign(count(lv[k].n), 0.0);
    }
    const int nt = lv[top].n, mt = nt - 1;
    const size_t N = d == 2 ? (size_t)mt * mt : (size_t)mt * mt * mt;
    std::vector<double>& B = Bs[top];
    B.assign(N * N, 0.0);
    for (size_t q = 0; q < N; ++q) {
      for (int k = 1; k <= top; ++k) {
        std::fill(lv[k].x.begin(), lv[k].x.end(), 0.0);
        std::fill(lv[k].b.begin(), lv[k].b.end(), 0.0);
      }
      {
        const int i = 1 + (int)(q % mt), j = 1 + (int)((q / mt) % mt), l = d == 3 ? 1 + (int)(q / ((size_t)mt * mt)) : 0;
        lv[top].b[idx(nt, i, j, l)] = 1.0;
      }
      for (int k = top; k >= 2; --k) {
        HostLevel& L = lv[k];
        const double D = 2.0 * d * L.scale;
        for (int s = 0; s < ro.o.nu_pre; ++s) {
          const double wd = ro.pre[s] / D;
          interior(L.n, [&](int i, int j, int l) {
            const int c = idx(L.n, i, j, l);
            L.t[c] = L.x[c] + wd * (L.b[c] - applyA(L, L.x, i, j, l));
          });
          std::swap(L.x, L.t);
        }
        HostLevel& C = lv[k - 1];
        interior(C.n, [&](int i, int j, int l) {
          const int q0 = idx(L.n, 2 * i, 2 * j, 2 * l), n = L.n, px = n + 1, pz = (n + 1) * (n + 1);
          auto r = [&](int c) {
            const int li = c % px, lj = (c / px) % px, ll = d == 3 ? c / pz : 0;
            return L.b[c] - applyA(L, L.x, li, lj, ll);
          };
          double h = (r(q0 + 1) + r(q0 - 1)) + (r(q0 + px) + r(q0 - px)) + (r(q0 + 1 + px) + r(q0 - 1 - px));
          if (d == 3)
            h += (r(q0 + pz) + r(q0 - pz)) + (r(q0 + 1 + pz) + r(q0 - 1 - pz)) + (r(q0 + px + pz) + r(q0 - px - pz)) +
                 (r(q0 + 1 + px + pz) + r(q0 - 1 - px - pz));
          C.b[idx(C.n, i, j, l)] = r(q0) + 0.5 * h;
        });
      }
      {
        HostLevel& L1 = lv[1];
        const int m1 = L1.n - 1;
        for (int rr = 0; rr < p.N1; ++rr) {
          double sm = 0.0;
          for (int c = 0; c < p.N1; ++c) {
            const int i = 1 + c % m1, j = 1 + (c / m1) % m1, l = d == 3 ? 1 + c / (m1 * m1) : 0;
            sm += A1inv[(size_t)rr * p.N1 + c] * L1.b[idx(L1.n, i, j, l)];
          }
          const int i = 1 + rr % m1, j = 1 + (rr / m1) % m1, l = d == 3 ? 1 + rr / (m1 * m1) : 0;
          L1.x[idx(L1.n, i, j, l)] = sm;
        }
      }
      for (int k = 2; k <= top; ++k) {
        HostLevel& L = lv[k];
        const HostLevel& C = lv[k - 1];
        interior(L.n, [&](int i, int j, int l) {
          const int si = i & 1, sj = j & 1, sl = d == 3 ? (l & 1) : 0;
          double v = C.x[idx(C.n, i >> 1, j >> 1, l >> 1)];
          if (si | sj | sl) v = 0.5 * (v + C.x[idx(C.n, (i >> 1) + si, (j >> 1) + sj, (l >> 1) + sl)]);
          L.x[idx(L.n, i, j, l)] += v;
        });
        const double D = 2.0 * d * L.scale;
        for (int s = 0; s < ro.o.nu_post; ++s) {
          const double wd = ro.post[s] / D;
          interior(L.n, [&](int i, int j, int l) {
            const int c = idx(L.n, i, j, l);
            L.t[c] = L.x[c] + wd * (L.b[c] - applyA(L, L.x, i, j, l));
          });
          std::swap(L.x, L.t);
        }
      }
      size_t row = 0;
      interior(nt, [&](int i, int j, int l) { B[row++ * N + q] = lv[top].x[idx(nt, i, j, l)]; });
    }
  }
}

}  // namespace

namespace {

// Axis order of Kuhn simplex s of a cell (as KuhnChain<d, s>).
void chain_axes(int d, int s, int ax[3]) {
  if (d == 2) { ax[0] = s; ax[1] = 1 - s; ax[2] = 2; return; }
  ax[0] = s / 2;
  const int r0 = ax[0] == 0 ? 1 : 0, r1 = ax[0] == 2 ? 1 : 2;
  ax[1] = (s & 1) ? r1 : r0;
  ax[2] = (s & 1) ? r0 : r1;
}

// Upper-triangle component index of entry (a, b), rows in order.
int comp_index(int d, int a, int b) {
  if (a > b) std::swap(a, b);
  return a * d - a * (a - 1) / 2 + (b - a);
}

// Barycentric gradient k of a chain (unit cell) as (axis, sign) pairs.
int chain_gradient(int d, const int ax[3], int k, int axis[2], int sign[2]) {
  int n = 0;
  if (k > 0) { axis[n] = ax[k - 1]; sign[n] = 1; ++n; }
  if (k < d) { axis[n] = ax[k]; sign[n] = -1; ++n; }
  return n;
}

// Terms of the forward-edge weights: for every direction delta, every cell
// (octant o below the node) and simplex whose chain holds both o and o + delta,
// -g_i^T A g_j as integer multiples of the matrix components.
void build_coef_terms(int d, CoefTerms& T) {
  std::memset(&T, 0, sizeof(T));
  const int NS = d == 2 ? 2 : 6, NO = 1 << d;
  int n = 0;
  for (int dl = 1; dl < NO; ++dl) {
    T.begin[dl - 1] = n;
    for (int o = 0; o < NO; ++o) {
      if (o & dl) continue;
      for (int sx = 0; sx < NS; ++sx) {
        int ax[3];
        chain_axes(d, sx, ax);
        int v[4] = {0, 0, 0, 0};
        for (int k = 1; k <= d; ++k) v[k] = v[k - 1] | (1 << ax[k - 1]);
        int i = -1, j = -1;
        for (int k = 0; k <= d; ++k) {
          if (v[k] == o) i = k;
          if (v[k] == (o | dl)) j = k;
        }
        if (i < 0 || j < 0) continue;
        int ai[2], si[2], aj[2], sj[2], coef[6] = {0, 0, 0, 0, 0, 0};
        const int ni = chain_gradient(d, ax, i, ai, si), nj = chain_gradient(d, ax, j, aj, sj);
        for (int x = 0; x < ni; ++x)
          for (int y = 0; y < nj; ++y) coef[comp_index(d, ai[x], aj[y])] -= si[x] * sj[y];
        for (int q = 0; q < d * (d + 1) / 2; ++q)
          if (coef[q] != 0 && n < kCoefTermsMax) {
            T.o[n] = (unsigned char)o;
            T.s[n] = (unsigned char)sx;
            T.q[n] = (unsigned char)q;
            T.c[n] = (signed char)coef[q];
            ++n;
          }
      }
    }
  }
  T.begin[NO - 1] = n;
}

// Coarse simplex of every child simplex: the fine simplex of octant o with
// chain order pi holds the points whose coordinates in the parent cell
// decrease first over the axes with o = 1 (in pi's order), then over the
// others (in pi's order).
void build_coarsen_map(int d, CoarsenMap& M) {
  std::memset(&M, 0, sizeof(M));
  const int NS = d == 2 ? 2 : 6, NO = 1 << d;
  for (int o = 0; o < NO; ++o)
    for (int pi = 0; pi < NS; ++pi) {
      int ax[3], sig[3] = {0, 0, 0}, m = 0;
      chain_axes(d, pi, ax);
      for (int k = 0; k < d; ++k)
        if ((o >> ax[k]) & 1) sig[m++] = ax[k];
      for (int k = 0; k < d; ++k)
        if (!((o >> ax[k]) & 1)) sig[m++] = ax[k];
      for (int sx = 0; sx < NS; ++sx) {
        int bx[3];
        chain_axes(d, sx, bx);
        bool same = true;
        for (int k = 0; k < d; ++k) same = same && bx[k] == sig[k];
        if (same) M.sigma[o][pi] = (unsigned char)sx;
      }
    }
}

// Stencil arrays of every level, then A_1 and its inverse, from the finest
// cell matrices d_coef.
template <int DIM>
void coef_setup(fmg_hierarchy* h, const double* d_coef, hipStream_t s) {
  const Plan& p = h->plan;
  CoefTerms terms;
  build_coef_terms(DIM, terms);
  CoarsenMap map;
  build_coarsen_map(DIM, map);
  constexpr int NS = coef_simplices<DIM>();
  for (int k = p.nlev - 1; k >= 1; --k) {
    const int nc = p.lev[k].g.n;
    const long long work = (DIM == 2 ? (long long)nc * nc : (long long)nc * nc * nc) * NS;
    const bool from_cells = k + 1 == p.nlev;
    k_coef_coarsen<DIM><<<(unsigned)((work + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        nc, from_cells ? d_coef : h->at<double>(p.off_sm[k + 1]), from_cells ? 1 : 0, h->at<double>(p.off_sm[k]),
        map);
  }
  const double dfact = DIM == 2 ? 2.0 : 6.0;
  for (int k = 1; k <= p.nlev; ++k) {
    const LevelInfo& L = p.lev[k];
    const long long n1 = L.g.n + 1;
    const long long nodes = DIM == 2 ? n1 * n1 : n1 * n1 * n1;
    const bool finest = k == p.nlev;
    k_coef_weights<DIM><<<(unsigned)((nodes + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        L.g, finest ? d_coef : h->at<double>(p.off_sm[k]), finest ? 1 : 0, L.scale / dfact,
        h->at<double>(p.off_w[k]), p.wplane[k], terms);
  }
  k_coef_level1<DIM><<<1, kBlock, 0, s>>>(p.lev[1].g, h->at<double>(p.off_w[1]), p.wplane[1], p.N1,
                                          h->at<double>(p.off_A1));
  k_spd_invert<<<1, kInvertThreads, sizeof(double) * invert_lds_doubles(p.N1), s>>>(
      h->at<double>(p.off_A1), h->at<double>(p.off_A1inv), h->at<float>(p.off_A1inv_f), p.N1);
}

// The hierarchy's part of the problem slot.
CoefLevels coef_levels(const fmg_hierarchy* h) {
  CoefLevels c;
  std::memset(&c, 0, sizeof(c));
  const Plan& p = h->plan;
  if (p.var)
    for (int k = 1; k <= p.nlev; ++k) {
      c.w[k] = h->at<double>(p.off_w[k]);
      c.plane[k] = p.wplane[k];
    }
  return c;
}

// The LDS-resident V-cycle tail may use up to the whole 160 KB of a workgroup.
hipError_t set_tail_lds_limit() {
  const int lim = (int)kTailLdsMax;
  const void* fns[4] = {reinterpret_cast<const void*>(&k_vcycle_tail_lds<2, double>),
                        reinterpret_cast<const void*>(&k_vcycle_tail_lds<2, float>),
                        reinterpret_cast<const void*>(&k_vcycle_tail_lds<3, double>),
                        reinterpret_cast<const void*>(&k_vcycle_tail_lds<3, float>)};
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Device address of the static scratch on the current device, taken once
// per device with that device current.
int scratch_on_current_device(char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FMG_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FMG_E_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  if (!g_tail_attr_set) {
    if (set_tail_lds_limit() != hipSuccess) return FMG_E_HIP;
    g_tail_attr_set = true;
  }
  *out = static_cast<char*>(g_scratch_ptr[dev]);
  return FMG_OK;
}

// Capture the solve for nonlinearity `kind` once (paper mode) and keep both the
// graph and its executable form.
int ensure_graph(fmg_hierarchy* h, int kind) {
  if (h->graph[kind]) return FMG_OK;
  const Plan& p = h->plan;
  record_fn rec = p.dim == 2 ? pick_record<2>(kind) : pick_record<3>(kind);
  Roles R;
  canonical_roles(h, R);
  hipGraph_t graph;
  if (hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return FMG_E_HIP;
  rec(h, R, true, h->cap_stream);
  if (hipStreamEndCapture(h->cap_stream, &graph) != hipSuccess) return FMG_E_HIP;
  hipGraphExec_t ex;
  const hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return FMG_E_HIP;
  h->graph[kind] = ex;
  return FMG_OK;
}

// Batched solves: one executable graph per distinct (hierarchies, kinds)
// list.  It is captured from one fork-join recording: a root kernel copies
// each problem's slot from a small device table, then every hierarchy records
// its solve on its own capture stream, so the graph holds one independent
// branch per problem.  Branches share no memory and the device runs them side
// by side.  Later calls with the same list refresh the table (one small
// host-to-device copy, stream-ordered before the launch) and launch again.
struct SlotDesc {
  ProblemSlot* slot;
  const double* g;
  double* out;
  fmg_report* rep;
  const double* c;
  double param;
  int kind;
  int pad;
};

__global__ void k_set_slots(const SlotDesc* __restrict__ d, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    ProblemSlot* s = d[i].slot;
    s->g = d[i].g; s->u_out = d[i].out; s->rep_out = d[i].rep; s->param = d[i].param; s->kind = d[i].kind;
    s->c = d[i].c;
  }
}

struct BatchGraph {
  std::vector<fmg_hierarchy*> hs;
  std::vector<int> kinds;
  std::vector<SlotDesc> host;
  SlotDesc* table = nullptr;       // device copy of `host`
  hipGraphExec_t exec = nullptr;
  unsigned long long stamp = 0;
};
std::mutex g_batch_mu;
std::vector<BatchGraph*> g_batches;
unsigned long long g_batch_clock = 0;
constexpr size_t kBatchCacheMax = 8;

void destroy_batch(BatchGraph* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->table) (void)hipFree(b->table);
  delete b;
}

int build_batch(BatchGraph* b) {
  const int count = (int)b->hs.size();
  if (hipMalloc(&b->table, sizeof(SlotDesc) * count) != hipSuccess) { b->table = nullptr; return FMG_E_HIP; }
  hipStream_t s0;
  if (hipStreamCreateWithFlags(&s0, hipStreamNonBlocking) != hipSuccess) return FMG_E_HIP;
  std::vector<hipEvent_t> ev(count + 1, nullptr);
  int st = FMG_OK;
  for (auto& e : ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) { e = nullptr; st = FMG_E_HIP; }
  hipGraph_t graph = nullptr;
  if (st == FMG_OK && hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    k_set_slots<<<1, 64, 0, s0>>>(b->table, count);
    (void)hipEventRecord(ev[count], s0);
    for (int i = 0; i < count; ++i) {
      fmg_hierarchy* h = b->hs[i];
      (void)hipStreamWaitEvent(h->cap_stream, ev[count], 0);
      record_fn rec = h->plan.dim == 2 ? pick_record<2>(b->kinds[i]) : pick_record<3>(b->kinds[i]);
      Roles R;
      canonical_roles(h, R);
      rec(h, R, true, h->cap_stream);
      (void)hipEventRecord(ev[i], h->cap_stream);
      (void)hipStreamWaitEvent(s0, ev[i], 0);
    }
    if (hipStreamEndCapture(s0, &graph) != hipSuccess) { graph = nullptr; st = FMG_E_HIP; }
  } else {
    st = FMG_E_HIP;
  }
  if (st == FMG_OK && hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    b->exec = nullptr;
    st = FMG_E_HIP;
  }
  if (graph) (void)hipGraphDestroy(graph);
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  (void)hipStreamDestroy(s0);
  return st;
}

}  // namespace

extern "C" {

void fmg_default_options(int dim, fmg_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = FMG_FP64;
  o->m_vcycles = 2;
  o->p_steps = 1;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->smoother = FMG_SMOOTHER_DEFAULT;
  o->omega = 0.0;
  o->cheb_lo = 1.0 / 3.0;
  o->cheb_hi = 2.0;
  o->newton_max = 30;
  o->newton_tol = 1e-14;
  o->newton_passes = 3;
  o->mode = FMG_PAPER;
  o->converged_max_steps = 40;
  o->converged_tol = 1e-13;
  o->use_graph = 1;
  o->tail_max_nodes = 1024;
  o->fuse_small_levels = 0;
  o->aug_max_blocks = 512;
  // the single-workgroup augmented solve pays off for the 10 unknowns of the
  // 2D problem; the 28 of 3D run faster through the multi-workgroup passes
  o->aug_small_nodes = dim == 2 ? 4096 : 343;
  o->sweep_rows = 0;
  o->quadrature = FMG_QUAD_VERTEX;
}

size_t fmg_workspace_bytes(const fmg_mesh_desc* mesh, const fmg_options* opts) {
  if (!mesh) return 0;
  Resolved ro;
  if (resolve(mesh->dim, opts, ro) != FMG_OK) return 0;
  Plan p;
  if (make_plan(mesh, ro, p) != FMG_OK) return 0;
  return p.total;
}

int fmg_create_hierarchy(const fmg_mesh_desc* mesh, const fmg_options* opts, void* d_workspace,
                         size_t workspace_bytes, void* stream, fmg_hierarchy** out) {
  if (!mesh || !out || !d_workspace) return FMG_E_INVALID;
  *out = nullptr;
  Resolved ro;
  int st = resolve(mesh->dim, opts, ro);
  if (st != FMG_OK) return st;
  Plan p;
  if ((st = make_plan(mesh, ro, p)) != FMG_OK) return st;
  if (workspace_bytes < p.total || (reinterpret_cast<uintptr_t>(d_workspace) & (kAlign - 1))) return FMG_E_WORKSPACE;
  fmg_hierarchy* h = new (std::nothrow) fmg_hierarchy();
  if (!h) return FMG_E_INVALID;
  h->plan = p;
  h->ro = ro;
  h->ws = static_cast<char*>(d_workspace);
  h->ws_bytes = workspace_bytes;
  for (auto& g : h->graph) g = nullptr;
  h->prof = nullptr;
  h->coef_ready = false;
  if (hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess) { delete h; return FMG_E_HIP; }
  if (set_tail_lds_limit() != hipSuccess) {
    (void)hipStreamDestroy(h->cap_stream);
    delete h;
    return FMG_E_HIP;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // zero every level array once: the Dirichlet rings stay zero for good
  for (int k = 1; k <= p.nlev; ++k) {
    const size_t c = p.lev[k].count;
    double* arrs[3] = {h->at<double>(p.off_x[k]), h->at<double>(p.off_b[k]), h->at<double>(p.off_t[k])};
    for (double* a : arrs) k_fill<double><<<1024, 256, 0, s>>>(a, c, 0.0);
    if (ro.o.precision == FMG_MIXED) {
      float* fa[3] = {h->at<float>(p.off_xs[k]), h->at<float>(p.off_bs[k]), h->at<float>(p.off_ts[k])};
      for (float* a : fa) k_fill<float><<<1024, 256, 0, s>>>(a, c, 0.0f);
    }
  }
  if (p.off_uprev) k_fill<double><<<1024, 256, 0, s>>>(h->at<double>(p.off_uprev), p.lev[p.nlev].count, 0.0);
  k_fill<unsigned><<<1, 64, 0, s>>>(h->at<unsigned>(p.off_ticket), 1, 0u);
  k_init_slot<<<1, 64, 0, s>>>(h->slot(), p.lev[p.nlev].g.n + 1, coef_levels(h));
  if (p.tail_top >= 2 && ro.o.fuse_small_levels) {
    // parameters of the single-workgroup FMG launch over levels 1..T (canonical roles)
    FmgTailParams P;
    std::memset(&P, 0, sizeof(P));
    Roles R;
    canonical_roles(h, R);
    const int T = std::min(p.tail_top, p.nlev);
    if (p.dim == 2) { fill_tail_args<2, double>(h, R, T, P.v64); if (R.xs[1]) fill_tail_args<2, float>(h, R, T, P.v32); }
    else { fill_tail_args<3, double>(h, R, T, P.v64); if (R.xs[1]) fill_tail_args<3, float>(h, R, T, P.v32); }
    for (int k = 1; k <= T; ++k) { P.aug[k] = p.lev[k].aug; P.m[k] = p.lev[k].m; }
    P.A1 = h->at<double>(p.off_A1);
    P.ns = h->ns();
    P.rep = h->rep();
    P.slot = h->slot();
    P.top = T;
    P.nlev = p.nlev;
    P.nf1 = p.lev[p.nlev].g.n + 1;
    P.m_vcycles = ro.o.m_vcycles;
    P.p_steps = ro.o.p_steps;
    P.newton_max = ro.o.newton_max;
    P.newton_tol = ro.o.newton_tol;
    if (hipMemcpyAsync(h->at<FmgTailParams>(p.off_fmgtail), &P, sizeof(P), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      (void)hipStreamDestroy(h->cap_stream);
      delete h;
      return FMG_E_HIP;
    }
  }
  std::vector<double> A, Ainv;
  build_level1(p, A, Ainv);
  if (p.tail_dense) {
    std::vector<std::vector<double>> Bs;
    build_tail_operators(p, ro, Ainv, Bs);
    for (int k = 2; k <= p.tail_top; ++k)
      if (hipMemcpy(h->at<double>(p.off_tailB[k]), Bs[k].data(), Bs[k].size() * sizeof(double),
                    hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipStreamDestroy(h->cap_stream);
        delete h;
        return FMG_E_HIP;
      }
  }
  std::vector<float> Ainv_f(Ainv.begin(), Ainv.end());
  if (hipMemcpyAsync(h->at<double>(p.off_A1), A.data(), A.size() * sizeof(double), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemcpyAsync(h->at<double>(p.off_A1inv), Ainv.data(), Ainv.size() * sizeof(double), hipMemcpyHostToDevice,
                     s) != hipSuccess ||
      hipMemcpyAsync(h->at<float>(p.off_A1inv_f), Ainv_f.data(), Ainv_f.size() * sizeof(float),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) {
    (void)hipStreamDestroy(h->cap_stream);
    delete h;
    return FMG_E_HIP;
  }
  *out = h;
  return FMG_OK;
}

int fmg_set_coefficients(fmg_hierarchy* h, const double* d_coef, void* stream) {
  if (!h || !d_coef || !h->plan.var) return FMG_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (h->plan.dim == 2) coef_setup<2>(h, d_coef, s);
  else coef_setup<3>(h, d_coef, s);
  if (hipGetLastError() != hipSuccess) return FMG_E_HIP;
  h->coef_ready = true;
  return FMG_OK;
}

int fmg_solve(fmg_hierarchy* h, const fmg_problem* prob, double* d_u_out, fmg_report* report, void* stream) {
  if (!h || !d_u_out) return FMG_E_INVALID;
  int st = check_problem_for(h, prob);
  if (st != FMG_OK) return st;
  const Plan& p = h->plan;
  const fmg_options& o = h->ro.o;
  hipStream_t s = static_cast<hipStream_t>(stream);
  k_set_slot<<<1, 64, 0, s>>>(h->slot(), prob->g_nodes, d_u_out, report, prob->param, prob->kind, prob->f_weight);
  record_fn rec = p.dim == 2 ? pick_record<2>(prob->kind) : pick_record<3>(prob->kind);
  Roles R;
  canonical_roles(h, R);
  if (o.mode == FMG_PAPER && o.use_graph) {
    if ((st = ensure_graph(h, prob->kind)) != FMG_OK) return st;
    if (hipGraphLaunch(h->graph[prob->kind], s) != hipSuccess) return FMG_E_HIP;
    return hipGetLastError() == hipSuccess ? FMG_OK : FMG_E_HIP;
  }
  const bool converged = o.mode == FMG_CONVERGED;
  rec(h, R, !converged, s);
  if (converged) {
    const int k = p.nlev;
    const LevelInfo& F = p.lev[k];
    step_fn step = p.dim == 2 ? pick_step<2>(prob->kind) : pick_step<3>(prob->kind);
    double* uprev = h->at<double>(p.off_uprev);
    double* npart = h->at<double>(p.off_norm_part);
    double* nout = h->at<double>(p.off_norm_out);
    double prev = INFINITY, rel = 0.0;
    int steps = 0;
    bool reached = false;
    for (int it = 0; it < o.converged_max_steps; ++it) {
      const dim3 grid = grid_of(F.g, p.dim);
      if (p.dim == 2) k_copy_interior<2, double><<<grid, kBlock, 0, s>>>(F.g, R.x[k], uprev);
      else k_copy_interior<3, double><<<grid, kBlock, 0, s>>>(F.g, R.x[k], uprev);
      step(h, R, k, s, false, false, false);
      if (p.dim == 2) k_diff_norm_partials<2><<<grid, kBlock, 0, s>>>(F.g, R.x[k], uprev, npart);
      else k_diff_norm_partials<3><<<grid, kBlock, 0, s>>>(F.g, R.x[k], uprev, npart);
      k_sum_pairs<<<1, kBlock, 0, s>>>(npart, p.norm_blocks, nout);
      double host[2];
      if (hipMemcpyAsync(host, nout, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return FMG_E_HIP;
      steps = it + 1;
      const double du = std::sqrt(host[0]);
      rel = du / std::max(std::sqrt(host[1]), 1e-300);
      if (rel <= o.converged_tol) { reached = true; break; }
      if (du >= prev) {
        // the update stopped shrinking: rounding level only if it is already
        // within kStagnationFloor of the tolerance; otherwise the iteration
        // stagnates or diverges and the solve is reported as not converged
        reached = rel <= kStagnationFloor * o.converged_tol;
        break;
      }
      prev = du;
    }
    // record the extra-step info on the device report, then finish
    fmg_report info;
    std::memset(&info, 0, sizeof(info));
    if (hipMemcpyAsync(&info, h->rep(), sizeof(info), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return FMG_E_HIP;
    info.extra_steps = steps;
    info.last_update_rel = rel;
    if (!reached && info.status == FMG_OK) info.status = FMG_E_NOT_CONVERGED;
    if (hipMemcpyAsync(h->rep(), &info, sizeof(info), hipMemcpyHostToDevice, s) != hipSuccess) return FMG_E_HIP;
    if (p.dim == 2) k_output<2><<<output_blocks<2>(F.g), 256, 0, s>>>(F.g, R.x[k], h->slot(), h->flag());
    else k_output<3><<<output_blocks<3>(F.g), 256, 0, s>>>(F.g, R.x[k], h->slot(), h->flag());
    k_end_solve<<<1, 64, 0, s>>>(h->rep(), h->flag(), h->slot());
    if (hipStreamSynchronize(s) != hipSuccess) return FMG_E_HIP;
  }
  return hipGetLastError() == hipSuccess ? FMG_OK : FMG_E_HIP;
}

int fmg_solve_noalloc(const fmg_mesh_desc* mesh, const fmg_options* opts, const fmg_problem* prob,
                      double* d_u_out, fmg_report* report, void* stream) {
  if (!mesh || !d_u_out) return FMG_E_INVALID;
  int st = check_problem(prob);
  if (st != FMG_OK) return st;
  Resolved ro;
  if ((st = resolve(mesh->dim, opts, ro)) != FMG_OK) return st;
  if (ro.o.mode != FMG_PAPER || ro.o.fuse_small_levels || ro.o.quadrature != FMG_QUAD_VERTEX ||
      ro.o.coefficients != FMG_COEF_IDENTITY || prob->f_weight)
    return FMG_E_UNSUPPORTED;
  fmg_hierarchy h;   // on the stack: plan, options and the scratch as workspace
  if ((st = make_plan(mesh, ro, h.plan, false)) != FMG_OK) return st;
  if (h.plan.total > kScratchBytes) return FMG_E_SCRATCH;
  char* ws = nullptr;
  if ((st = scratch_on_current_device(&ws)) != FMG_OK) return st;
  h.ro = ro;
  h.ws = ws;
  h.ws_bytes = kScratchBytes;
  h.cap_stream = nullptr;
  for (auto& g : h.graph) g = nullptr;
  h.prof = nullptr;
  const Plan& p = h.plan;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the previous call's contents: clear the level arrays (their Dirichlet
  // rings must read zero) and the ticket counter that follows them, then
  // form the level-1 tables on the device
  const size_t words = (p.total - p.off_x[1]) / sizeof(double);
  k_fill<double><<<1024, 256, 0, s>>>(h.at<double>(p.off_x[1]), words, 0.0);
  k_level1_tables<<<1, 64, sizeof(double) * 2 * p.N1 * p.N1, s>>>(
      p.dim, p.nH, p.lev[1].scale, h.at<double>(p.off_A1), h.at<double>(p.off_A1inv), h.at<float>(p.off_A1inv_f));
  k_init_slot<<<1, 64, 0, s>>>(h.slot(), p.lev[p.nlev].g.n + 1, CoefLevels{});
  k_set_slot<<<1, 64, 0, s>>>(h.slot(), prob->g_nodes, d_u_out, report, prob->param, prob->kind, nullptr);
  record_fn rec = p.dim == 2 ? pick_record<2>(prob->kind) : pick_record<3>(prob->kind);
  Roles R;
  canonical_roles(&h, R);
  rec(&h, R, true, s);
  return hipGetLastError() == hipSuccess ? FMG_OK : FMG_E_HIP;
}

int fmg_profile_solve(fmg_hierarchy* h, const fmg_problem* prob, double* d_u_out, void* stream,
                      fmg_profile* out) {
  if (!h || !d_u_out || !out) return FMG_E_INVALID;
  int st = check_problem_for(h, prob);
  if (st != FMG_OK) return st;
  const Plan& p = h->plan;
  hipStream_t s = static_cast<hipStream_t>(stream);
  k_set_slot<<<1, 64, 0, s>>>(h->slot(), prob->g_nodes, d_u_out, nullptr, prob->param, prob->kind, prob->f_weight);
  record_fn rec = p.dim == 2 ? pick_record<2>(prob->kind) : pick_record<3>(prob->kind);
  Prof pf;
  Roles R;
  canonical_roles(h, R);
  h->prof = &pf;
  rec(h, R, true, s);
  h->prof = nullptr;
  if (hipStreamSynchronize(s) != hipSuccess) st = FMG_E_HIP;
  std::memset(out, 0, sizeof(*out));
  const size_t n = pf.kid.size();
  for (size_t i = 0; i < n && st == FMG_OK; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pf.ev[2 * i], pf.ev[2 * i + 1]) != hipSuccess) { st = FMG_E_HIP; break; }
    int e = 0;
    while (e < out->count && !(out->entries[e].kernel == pf.kid[i] && out->entries[e].level == pf.lev[i])) ++e;
    if (e == out->count) {
      if (out->count == FMG_PROFILE_MAX) continue;
      out->count++;
      out->entries[e].kernel = pf.kid[i];
      out->entries[e].level = pf.lev[i];
      out->entries[e].nodes = pf.nodes[i];
    }
    out->entries[e].launches++;
    out->entries[e].ms += ms;
    out->entries[e].bytes += pf.bytes[i];
  }
  if (st == FMG_OK && !pf.ev.empty()) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pf.ev.front(), pf.ev.back()) == hipSuccess) out->total_ms = ms;
  }
  for (hipEvent_t e : pf.ev) (void)hipEventDestroy(e);
  return st;
}

const char* fmg_kernel_name(int kernel) {
  return (kernel >= 0 && kernel < KC_COUNT) ? kKernelNames[kernel] : "unknown";
}

int fmg_get_report(fmg_hierarchy* h, fmg_report* host_report, void* stream) {
  if (!h || !host_report) return FMG_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(host_report, h->rep(), sizeof(fmg_report), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FMG_E_HIP;
  return FMG_OK;
}

int fmg_solve_batch(fmg_hierarchy* const* hs, const fmg_problem* probs, double* const* outs,
                    fmg_report* const* reports, int count, void* stream) {
  if (count < 0 || (count > 0 && (!hs || !probs || !outs))) return FMG_E_INVALID;
  bool graphs = true;
  for (int i = 0; i < count; ++i) {
    if (!hs[i] || !outs[i]) return FMG_E_INVALID;
    const int st = check_problem_for(hs[i], &probs[i]);
    if (st != FMG_OK) return st;
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i] || outs[j] == outs[i]) return FMG_E_INVALID;
    graphs = graphs && hs[i]->ro.o.mode == FMG_PAPER && hs[i]->ro.o.use_graph;
  }
  if (count == 0) return FMG_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!graphs) {
    for (int i = 0; i < count; ++i) {
      const int st = fmg_solve(hs[i], &probs[i], outs[i], reports ? reports[i] : nullptr, stream);
      if (st != FMG_OK) return st;
    }
    return FMG_OK;
  }
  std::lock_guard<std::mutex> lock(g_batch_mu);
  BatchGraph* b = nullptr;
  for (BatchGraph* c : g_batches) {
    if ((int)c->hs.size() != count) continue;
    bool same = true;
    for (int i = 0; i < count && same; ++i) same = c->hs[i] == hs[i] && c->kinds[i] == probs[i].kind;
    if (same) { b = c; break; }
  }
  if (!b) {
    b = new (std::nothrow) BatchGraph();
    if (!b) return FMG_E_INVALID;
    b->hs.assign(hs, hs + count);
    for (int i = 0; i < count; ++i) b->kinds.push_back(probs[i].kind);
    const int st = build_batch(b);
    if (st != FMG_OK) { destroy_batch(b); return st; }
    if (g_batches.size() >= kBatchCacheMax) {
      auto oldest = std::min_element(g_batches.begin(), g_batches.end(),
                                     [](const BatchGraph* x, const BatchGraph* y) { return x->stamp < y->stamp; });
      // the evicted graph may still run on a stream: wait for the device first
      (void)hipDeviceSynchronize();
      destroy_batch(*oldest);
      g_batches.erase(oldest);
    }
    g_batches.push_back(b);
  }
  b->host.resize(count);
  for (int i = 0; i < count; ++i) {
    SlotDesc& d = b->host[i];
    d.slot = hs[i]->slot(); d.g = probs[i].g_nodes; d.out = outs[i];
    d.rep = reports ? reports[i] : nullptr; d.param = probs[i].param; d.kind = probs[i].kind; d.pad = 0;
    d.c = probs[i].f_weight;
  }
  if (hipMemcpyAsync(b->table, b->host.data(), sizeof(SlotDesc) * count, hipMemcpyHostToDevice, s) != hipSuccess)
    return FMG_E_HIP;
  b->stamp = ++g_batch_clock;
  if (hipGraphLaunch(b->exec, s) != hipSuccess) return FMG_E_HIP;
  return hipGetLastError() == hipSuccess ? FMG_OK : FMG_E_HIP;
}

int fmg_destroy(fmg_hierarchy* h) {
  if (!h) return FMG_E_INVALID;
  // solves are asynchronous: a graph of h (or a batch graph holding h) may
  // still run on some stream, so wait for the device before releasing them
  (void)hipDeviceSynchronize();
  {
    std::lock_guard<std::mutex> lock(g_batch_mu);
    for (size_t i = 0; i < g_batches.size();) {
      BatchGraph* b = g_batches[i];
      if (std::find(b->hs.begin(), b->hs.end(), h) != b->hs.end()) {
        destroy_batch(b);
        g_batches.erase(g_batches.begin() + i);
      } else {
        ++i;
      }
    }
  }
  for (auto& g : h->graph)
    if (g) (void)hipGraphExecDestroy(g);

  (void)hipStreamDestroy(h->cap_stream);
  delete h;
  return FMG_OK;
}

const char* fmg_status_str(int status) {
  switch (status) {
    case FMG_OK: return "ok";
    case FMG_E_INVALID: return "invalid argument";
    case FMG_E_UNSUPPORTED: return "unsupported mesh or option";
    case FMG_E_WORKSPACE: return "workspace too small or misaligned";
    case FMG_E_HIP: return "HIP runtime error";
    case FMG_E_NOT_CONVERGED: return "Newton iteration did not converge";
    case FMG_E_NONFINITE: return "non-finite value in the solution";
    case FMG_E_SCRATCH: return "problem larger than the static scratch of fmg_solve_noalloc";
    default: return "unknown status";
  }
}

}  // extern "C"

namespace {
template <int DIM>
int level_op_impl(fmg_hierarchy* h, int op, int k, int prec, const double* in0, const double* in1, double* out,
                  double omega, hipStream_t s) {
  const Plan& p = h->plan;
  const LevelInfo& L = p.lev[k];
  const dim3 grid = grid_of(L.g, DIM);
  const int pk = 512;
  double* x = h->at<double>(p.off_x[k]);
  double* b = h->at<double>(p.off_b[k]);
  double* t = h->at<double>(p.off_t[k]);
  if (prec == FMG_MIXED && !p.off_xs[k]) return FMG_E_INVALID;
  float* xs = prec == FMG_MIXED ? h->at<float>(p.off_xs[k]) : nullptr;
  float* bs = prec == FMG_MIXED ? h->at<float>(p.off_bs[k]) : nullptr;
  float* ts = prec == FMG_MIXED ? h->at<float>(p.off_ts[k]) : nullptr;
  const double D = 2.0 * DIM * L.scale;
  auto in = [&](const double* src, double* d64, float* d32, const Grid& g) {
    if (prec == FMG_FP64) k_pack<DIM, double, double><<<pk, 256, 0, s>>>(g, src, d64, 0);
    else k_pack<DIM, float, double><<<pk, 256, 0, s>>>(g, src, d32, 0);
  };
  auto outp = [&](const double* s64, const float* s32, const Grid& g) {
    if (prec == FMG_FP64) k_pack<DIM, double, double><<<pk, 256, 0, s>>>(g, s64, out, 1);
    else k_pack<DIM, double, float><<<pk, 256, 0, s>>>(g, s32, out, 1);
  };
  if (p.var && op != FMG_OP_PROLONG && op != FMG_OP_COARSE) {
    // the variable-coefficient operator (float64 only)
    if (prec != FMG_FP64 || !h->coef_ready) return FMG_E_INVALID;
    const double* W = h->at<double>(p.off_w[k]);
    const long long pl = p.wplane[k];
    switch (op) {
      case FMG_OP_APPLY_A:
        in(in0, x, xs, L.g);
        k_apply_Aw<DIM><<<grid, kBlock, 0, s>>>(L.g, x, t, W, pl);
        outp(t, ts, L.g);
        break;
      case FMG_OP_SMOOTH:
        in(in0, x, xs, L.g);
        in(in1, b, bs, L.g);
        k_smooth_w<DIM, false><<<grid, kBlock, 0, s>>>(L.g, x, b, t, W, pl, omega);
        outp(t, ts, L.g);
        break;
      case FMG_OP_RESTRICT: {
        if (k < 2) return FMG_E_INVALID;
        const LevelInfo& C = p.lev[k - 1];
        in(in0, x, xs, L.g);
        in(in1, b, bs, L.g);
        double* bc = h->at<double>(p.off_b[k - 1]);
        k_resid_w<DIM><<<grid, kBlock, 0, s>>>(L.g, x, b, t, W, pl);
        k_restrict<DIM><<<grid_of(C.g, DIM), kBlock, 0, s>>>(L.g, C.g, t, bc);
        outp(bc, nullptr, C.g);
        break;
      }
      default:
        return FMG_E_INVALID;
    }
    return hipGetLastError() == hipSuccess ? FMG_OK : FMG_E_HIP;
  }
  switch (op) {
    case FMG_OP_APPLY_A:
      in(in0, x, xs, L.g);
      if (prec == FMG_FP64) k_apply_A<DIM, double><<<grid, kBlock, 0, s>>>(L.g, x, t, L.scale);
      else k_apply_A<DIM, float><<<grid, kBlock, 0, s>>>(L.g, xs, ts, (float)L.scale);
      outp(t, ts, L.g);
      break;
    case FMG_OP_SMOOTH:
      in(in0, x, xs, L.g);
      in(in1, b, bs, L.g);
      if (prec == FMG_FP64) k_smooth<DIM, double, false><<<grid, kBlock, 0, s>>>(L.g, x, b, t, omega / D, L.scale);
      else k_smooth<DIM, float, false><<<grid, kBlock, 0, s>>>(L.g, xs, bs, ts, (float)(omega / D), (float)L.scale);
      outp(t, ts, L.g);
      break;
    case FMG_OP_RESTRICT: {
      if (k < 2) return FMG_E_INVALID;
      const LevelInfo& C = p.lev[k - 1];
      in(in0, x, xs, L.g);
      in(in1, b, bs, L.g);
      double* bc = h->at<double>(p.off_b[k - 1]);
      float* bcs = prec == FMG_MIXED ? h->at<float>(p.off_bs[k - 1]) : nullptr;
      if (prec == FMG_FP64)
        launch_resid_restrict<DIM, double>(L.g, C.g, x, b, bc, L.scale, s);
      else
        launch_resid_restrict<DIM, float>(L.g, C.g, xs, bs, bcs, (float)L.scale, s);
      outp(bc, bcs, C.g);
      break;
    }
    case FMG_OP_PROLONG: {
      if (k < 2) return FMG_E_INVALID;
      const LevelInfo& C = p.lev[k - 1];
      double* xc = h->at<double>(p.off_x[k - 1]);
      float* xcs = prec == FMG_MIXED ? h->at<float>(p.off_xs[k - 1]) : nullptr;
      in(in0, xc, xcs, C.g);
      in(in1, x, xs, L.g);
      if (prec == FMG_FP64) k_prolong<DIM, double, true><<<grid, kBlock, 0, s>>>(C.g, L.g, xc, x);
      else k_prolong<DIM, float, true><<<grid, kBlock, 0, s>>>(C.g, L.g, xcs, xs);
      outp(x, xs, L.g);
      break;
    }
    case FMG_OP_COARSE:
      if (k != 1) return FMG_E_INVALID;
      in(in0, b, bs, L.g);
      if (prec == FMG_FP64)
        k_coarse_solve<DIM, double><<<1, 64, 0, s>>>(L.g, p.N1, h->at<double>(p.off_A1inv), b, x);
      else
        k_coarse_solve<DIM, float><<<1, 64, 0, s>>>(L.g, p.N1, h->at<float>(p.off_A1inv_f), bs, xs);
      outp(x, xs, L.g);
      break;
    default:
      return FMG_E_INVALID;
  }
  return hipGetLastError() == hipSuccess ? FMG_OK : FMG_E_HIP;
}
}  // namespace

namespace {

// One launch of a timed level kernel on the hierarchy's own level-k buffers.
template <int DIM, typename T>
int time_launch(fmg_hierarchy* h, int base, int k, hipStream_t st, double& bytes) {
  const Plan& p = h->plan;
  Roles R;
  canonical_roles(h, R);
  T* x = Sel<T>::x(R, k);
  T* t = Sel<T>::t(R, k);
  T* b = Sel<T>::b(h, k);
  const LevelInfo& L = p.lev[k];
  const LevelInfo& C = p.lev[k - 1];
  const long long N = interior(L.g, DIM), Nc = interior(C.g, DIM);
  const double s = sizeof(T), D = 2.0 * DIM * L.scale;
  const T scale = (T)L.scale;
  const int rows = stream_rows(h->ro.o.sweep_rows, L.g.n);
  switch (base) {
    case KC_PRE2S64: case KC_PRE2D64:
      if (DIM != 2 || (base == KC_PRE2S64) != (rows > 0)) return FMG_E_UNSUPPORTED;
      bytes = launch_pre2<T>(h, k, x, b, t, Sel<T>::b(h, k - 1), false, st);
      return FMG_OK;
    case KC_POST2S64: case KC_POST2D64:
      if (DIM != 2 || (base == KC_POST2S64) != (rows > 0)) return FMG_E_UNSUPPORTED;
      bytes = launch_post2<T>(h, k, x, Sel<T>::x(R, k - 1), b, t, st);
      return FMG_OK;
    case KC_PRE3P64:
      if (DIM != 3 || !use_pair3(h, k)) return FMG_E_UNSUPPORTED;
      bytes = launch_pre3<T>(h, k, x, b, t, false, st);
      return FMG_OK;
    case KC_POST3P64:
      if (DIM != 3 || !use_pair3(h, k)) return FMG_E_UNSUPPORTED;
      bytes = launch_post3<T>(h, k, x, Sel<T>::x(R, k - 1), b, t, st);
      return FMG_OK;
    case KC_SMOOTH64:
      bytes = 3 * s * N;
      k_smooth<DIM, T, false><<<grid_of(L.g, DIM), kBlock, 0, st>>>(L.g, x, b, t, (T)(h->ro.pre[0] / D), scale);
      return FMG_OK;
    case KC_SMOOTH3S64: {
      if (DIM != 3 || h->ro.o.sweep_rows <= 0 || L.g.n < 16) return FMG_E_UNSUPPORTED;
      bytes = launch_sweep<DIM, T>(h, k, x, b, t, (T)(h->ro.pre[0] / D), st);
      return FMG_OK;
    }
    case KC_RESTRICT64:
      bytes = s * (2 * N + Nc);
      launch_resid_restrict<DIM, T>(L.g, C.g, x, b, Sel<T>::b(h, k - 1), scale, st);
      return FMG_OK;
    case KC_PROLONG64_ADD:
      bytes = s * (2 * N + Nc);
      k_prolong<DIM, T, true><<<grid_of(L.g, DIM), kBlock, 0, st>>>(C.g, L.g, Sel<T>::x(R, k - 1), x);
      return FMG_OK;
    default:
      return FMG_E_UNSUPPORTED;
  }
}

// Variable-coefficient hierarchies: the weighted sweep and residual on level
// k's buffers (and the shared prolongation).
template <int DIM>
int time_launch_var(fmg_hierarchy* h, int kernel, int k, hipStream_t st, double& bytes) {
  const Plan& p = h->plan;
  if (!h->coef_ready) return FMG_E_INVALID;
  Roles R;
  canonical_roles(h, R);
  const LevelInfo& L = p.lev[k];
  const long long N = interior(L.g, DIM);
  const double nfw = (1 << DIM) - 1;
  const double* W = h->at<double>(p.off_w[k]);
  double* b = h->at<double>(p.off_b[k]);
  switch (kernel) {
    case KC_SMOOTHW64:
      bytes = 8.0 * (3.0 + nfw) * N;
      k_smooth_w<DIM, false><<<grid_of(L.g, DIM), kBlock, 0, st>>>(L.g, R.x[k], b, R.t[k], W, p.wplane[k],
                                                                   h->ro.pre[0]);
      return FMG_OK;
    case KC_RESIDW64:
      bytes = 8.0 * (3.0 + nfw) * N;
      k_resid_w<DIM><<<grid_of(L.g, DIM), kBlock, 0, st>>>(L.g, R.x[k], b, R.t[k], W, p.wplane[k]);
      return FMG_OK;
    case KC_PROLONG64_ADD:
      return time_launch<DIM, double>(h, kernel, k, st, bytes);
    default:
      return FMG_E_UNSUPPORTED;
  }
}

template <int DIM>
int time_launch_any(fmg_hierarchy* h, int kernel, int k, hipStream_t st, double& bytes) {
  if (h->plan.var) return time_launch_var<DIM>(h, kernel, k, st, bytes);
  // classes come in float64 / float32 pairs at a fixed distance
  const int d_mg = KC_SMOOTH32 - KC_SMOOTH64, d_2d = KC_PRE2D32 - KC_PRE2D64;
  switch (kernel) {
    case KC_SMOOTH64: case KC_RESTRICT64: case KC_PROLONG64_ADD:
    case KC_PRE2D64: case KC_POST2D64: case KC_PRE2S64: case KC_POST2S64: case KC_SMOOTH3S64:
    case KC_PRE3P64: case KC_POST3P64:
      return time_launch<DIM, double>(h, kernel, k, st, bytes);
    case KC_PRE3P32: case KC_POST3P32:
      if (!h->plan.off_xs[k]) return FMG_E_UNSUPPORTED;
      return time_launch<DIM, float>(h, kernel - (KC_PRE3P32 - KC_PRE3P64), k, st, bytes);
    case KC_SMOOTH3S32:
      if (!h->plan.off_xs[k]) return FMG_E_UNSUPPORTED;
      return time_launch<DIM, float>(h, KC_SMOOTH3S64, k, st, bytes);
    case KC_SMOOTH32: case KC_RESTRICT32: case KC_PROLONG32_ADD:
      if (!h->plan.off_xs[k]) return FMG_E_UNSUPPORTED;
      return time_launch<DIM, float>(h, kernel - d_mg, k, st, bytes);
    case KC_PRE2D32: case KC_POST2D32: case KC_PRE2S32: case KC_POST2S32:
      if (!h->plan.off_xs[k]) return FMG_E_UNSUPPORTED;
      return time_launch<DIM, float>(h, kernel - d_2d, k, st, bytes);
    default:
      return FMG_E_UNSUPPORTED;
  }
}

}  // namespace

extern "C" int fmg_time_level_kernel(fmg_hierarchy* h, int kernel, int level, int reps, void* stream,
                                     double* ms_per_launch, double* bytes_per_launch) {
  if (!h || !ms_per_launch || !bytes_per_launch || reps < 1 || reps > 100000 || level < 2 ||
      level > h->plan.nlev)
    return FMG_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double bytes = 0.0;
  auto once = [&]() {
    return h->plan.dim == 2 ? time_launch_any<2>(h, kernel, level, s, bytes)
                            : time_launch_any<3>(h, kernel, level, s, bytes);
  };
  int st = once();            // warm-up launch; also validates the request
  if (st != FMG_OK) return st;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return FMG_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return FMG_E_HIP; }
  (void)hipEventRecord(e0, s);
  for (int i = 0; i < reps; ++i) (void)once();
  (void)hipEventRecord(e1, s);
  float ms = 0.f;
  if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
      hipGetLastError() != hipSuccess)
    st = FMG_E_HIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms_per_launch = ms / reps;
  *bytes_per_launch = bytes;
  return st;
}

extern "C" int fmg_level_op(fmg_hierarchy* h, int op, int level, int precision, const double* in0, const double* in1,
                 double* out, double omega, void* stream) {
  if (!h || !in0 || !out || level < 1 || level > h->plan.nlev) return FMG_E_INVALID;
  if ((op == FMG_OP_SMOOTH || op == FMG_OP_RESTRICT || op == FMG_OP_PROLONG) && !in1) return FMG_E_INVALID;
  if (precision != FMG_FP64 && precision != FMG_MIXED) return FMG_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return h->plan.dim == 2 ? level_op_impl<2>(h, op, level, precision, in0, in1, out, omega, s)
                          : level_op_impl<3>(h, op, level, precision, in0, in1, out, omega, s);
}
