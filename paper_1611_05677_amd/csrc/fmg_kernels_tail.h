// Single-workgroup "tail" of the V-cycle: every level at or below a small
// level T (a few thousand nodes) is processed by one workgroup in one launch,
// with workgroup barriers between the phases, instead of one grid launch per
// sweep/transfer.  The arithmetic is the same as the grid kernels' (same
// stencil helper, same operation order per node), so results are identical.
#pragma once

#include "fmg_device.h"
#include "fmg_kernels_mg.h"

namespace fmg {

constexpr int kTailThreads = 1024;
constexpr int kTailLevels = 8;   // deepest level a tail launch may start from
constexpr int kTailSweeps = 8;   // max sweeps per level in a tail launch
constexpr size_t kTailLdsMax = 160 * 1024;  // LDS-resident tail up to this many bytes (gfx950 workgroup limit)
constexpr long long kDenseTailMax = 1024;    // dense-operator tail up to this many top-level unknowns

template <typename T>
struct TailArgs {
  T* x[FMG_MAX_LEVELS + 1];     // current iterate of each level (roles as on entry)
  T* t[FMG_MAX_LEVELS + 1];     // spare array of each level
  T* b[FMG_MAX_LEVELS + 1];     // right-hand sides
  Grid g[FMG_MAX_LEVELS + 1];
  T scale[FMG_MAX_LEVELS + 1];  // h^{d-2}
  T wdpre[kTailLevels + 1][kTailSweeps];   // omega_i / D_k per level and sweep
  T wdpost[kTailLevels + 1][kTailSweeps];
  const T* ainv;                // A_1^{-1}, dense N1 x N1
  int N1, top, npre, npost, zero_top;
  int lds_off[kTailLevels + 1]; // LDS variant: offset (elements) of level k's x, t, b
};

template <int DIM>
__device__ __forceinline__ int interior_count(const Grid& g) {
  const int m = g.n - 1;
  return DIM == 2 ? m * m : m * m * m;
}

template <int DIM>
__device__ __forceinline__ int interior_node(const Grid& g, int t) {
  const int m = g.n - 1;
  const int i = 1 + t % m, j = 1 + (t / m) % m, l = DIM == 3 ? 1 + t / (m * m) : 0;
  return gidx<DIM>(g, i, j, l);
}

template <int DIM, typename T, bool ZERO>
__device__ __forceinline__ void blk_smooth(const Grid& g, const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ out,
                           T wd, T scale) {
  const int total = interior_count<DIM>(g);
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int c = interior_node<DIM>(g, t);
    if (ZERO) out[c] = wd * b[c];
    else out[c] = x[c] + wd * (b[c] - apply_A_at<DIM>(x, c, g, scale));
  }
  __syncthreads();
}

template <int DIM, typename T>
__device__ __forceinline__ void blk_fill_interior(const Grid& g, T* __restrict__ x) {
  const int total = interior_count<DIM>(g);
  for (int t = threadIdx.x; t < total; t += blockDim.x) x[interior_node<DIM>(g, t)] = T(0);
  __syncthreads();
}

template <int DIM, typename T>
__device__ __forceinline__ void blk_resid_restrict(const Grid& f, const Grid& cg, const T* __restrict__ x, const T* __restrict__ b,
                                   T* __restrict__ bc, T scale) {
  const int total = interior_count<DIM>(cg);
  const int m = cg.n - 1;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int i = 1 + t % m, j = 1 + (t / m) % m, l = DIM == 3 ? 1 + t / (m * m) : 0;
    const int q = gidx<DIM>(f, 2 * i, 2 * j, 2 * l);
    auto r = [&](int p) { return b[p] - apply_A_at<DIM>(x, p, f, scale); };
    const int dx = 1, dy = f.px;
    T h = (r(q + dx) + r(q - dx)) + (r(q + dy) + r(q - dy)) + (r(q + dx + dy) + r(q - dx - dy));
    if (DIM == 3) {
      const int dz = f.pz;
      h += (r(q + dz) + r(q - dz)) + (r(q + dx + dz) + r(q - dx - dz)) +
           (r(q + dy + dz) + r(q - dy - dz)) + (r(q + dx + dy + dz) + r(q - dx - dy - dz));
    }
    bc[gidx<DIM>(cg, i, j, l)] = r(q) + T(0.5) * h;
  }
  __syncthreads();
}

template <int DIM, typename T>
__device__ __forceinline__ void blk_prolong_add(const Grid& cg, const Grid& f, const T* __restrict__ xc, T* __restrict__ xf) {
  const int total = interior_count<DIM>(f);
  const int m = f.n - 1;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int i = 1 + t % m, j = 1 + (t / m) % m, l = DIM == 3 ? 1 + t / (m * m) : 0;
    const int si = i & 1, sj = j & 1, sl = DIM == 3 ? (l & 1) : 0;
    const int pi = i >> 1, pj = j >> 1, pl = l >> 1;
    T v = xc[gidx<DIM>(cg, pi, pj, pl)];
    if (si | sj | sl) v = T(0.5) * (v + xc[gidx<DIM>(cg, pi + si, pj + sj, pl + sl)]);
    const int q = gidx<DIM>(f, i, j, l);
    xf[q] = xf[q] + v;
  }
  __syncthreads();
}

template <int DIM, typename T>
__device__ __forceinline__ void blk_coarse_solve(const Grid& g1, int N1, const T* __restrict__ Ainv, const T* __restrict__ b,
                                 T* __restrict__ x) {
  for (int r = threadIdx.x; r < N1; r += blockDim.x) {
    T s = 0;
    for (int c = 0; c < N1; ++c) s += Ainv[r * N1 + c] * b[level1_node<DIM>(g1, c)];
    x[level1_node<DIM>(g1, r)] = s;
  }
  __syncthreads();
}

// V-cycle on levels top..1 with right-hand side b[top] and initial iterate
// x[top] (zero if zero_top).  Roles of x/t are swapped after every sweep, as
// the host-side launch sequence does; x[] and t[] are updated in place.
template <int DIM, typename T>
__device__ __forceinline__ void vcycle_tail_dev(const TailArgs<T>& a, T** x, T** t, int top, bool zero_top) {
  for (int k = top; k >= 2; --k) {
    const bool zero = k < top || zero_top;
    if (zero && a.npre == 0) blk_fill_interior<DIM, T>(a.g[k], x[k]);
    for (int i = 0; i < a.npre; ++i) {
      const T wd = a.wdpre[k][i];
      if (zero && i == 0) blk_smooth<DIM, T, true>(a.g[k], x[k], a.b[k], t[k], wd, a.scale[k]);
      else blk_smooth<DIM, T, false>(a.g[k], x[k], a.b[k], t[k], wd, a.scale[k]);
      T* s = x[k]; x[k] = t[k]; t[k] = s;
    }
    blk_resid_restrict<DIM, T>(a.g[k], a.g[k - 1], x[k], a.b[k], a.b[k - 1], a.scale[k]);
  }
  blk_coarse_solve<DIM, T>(a.g[1], a.N1, a.ainv, a.b[1], x[1]);
  for (int k = 2; k <= top; ++k) {
    blk_prolong_add<DIM, T>(a.g[k - 1], a.g[k], x[k - 1], x[k]);
    for (int i = 0; i < a.npost; ++i) {
      blk_smooth<DIM, T, false>(a.g[k], x[k], a.b[k], t[k], a.wdpost[k][i], a.scale[k]);
      T* s = x[k]; x[k] = t[k]; t[k] = s;
    }
  }
}

template <int DIM, typename T>
__global__ void __launch_bounds__(kTailThreads) k_vcycle_tail(TailArgs<T> a) {
  T* x[kTailLevels + 1];
  T* t[kTailLevels + 1];
  for (int k = 1; k <= a.top; ++k) { x[k] = a.x[k]; t[k] = a.t[k]; }
  vcycle_tail_dev<DIM, T>(a, x, t, a.top, a.zero_top != 0);
}

// ---------------------------------------------------------------------------
// LDS-resident variant.  Every level 1..top lives in LDS as three packed
// (n_k+1)^d arrays (x, t, b; Dirichlet ring zero); only b[top] (and x[top]
// unless the cycle starts from zero) is read from global memory and only the
// final x[top] is written back (into the array that holds x[top] after the
// cycle's role swaps).  Nodes are enumerated by row / plane loops over a fixed
// thread shape (64 x 16 in 2D, 32 x 8 x 4 in 3D), so no division per node.
// Same per-node expressions as the grid kernels.
// ---------------------------------------------------------------------------
template <int DIM>
__device__ __forceinline__ Grid packed_grid(int n) {
  Grid g;
  g.n = n;
  g.px = n + 1;
  g.pz = DIM == 3 ? (n + 1) * (n + 1) : 0;
  return g;
}

template <int DIM>
__device__ __forceinline__ int packed_count(int n) {
  return DIM == 2 ? (n + 1) * (n + 1) : (n + 1) * (n + 1) * (n + 1);
}

// fn(i, j, l) over the interior nodes 1..n-1 of a level
template <int DIM, typename F>
__device__ __forceinline__ void for_interior(int n, F&& fn) {
  const int tid = threadIdx.x;
  if (DIM == 2) {
    const int tx = tid & 63, ty = tid >> 6;
    for (int j = 1 + ty; j < n; j += kTailThreads / 64)
      for (int i = 1 + tx; i < n; i += 64) fn(i, j, 0);
  } else {
    const int tx = tid & 31, ty = (tid >> 5) & 7, tz = tid >> 8;
    for (int l = 1 + tz; l < n; l += kTailThreads / 256)
      for (int j = 1 + ty; j < n; j += 8)
        for (int i = 1 + tx; i < n; i += 32) fn(i, j, l);
  }
}

template <int DIM, typename T>
__global__ void __launch_bounds__(kTailThreads) k_vcycle_tail_lds(TailArgs<T> a) {
  extern __shared__ unsigned char tail_smem[];
  T* lds = reinterpret_cast<T*>(tail_smem);
  const int top = a.top;
  // zero every level (rings stay zero), then bring in b[top] and x[top]
  {
    const int total = a.lds_off[top] + 3 * packed_count<DIM>(a.g[top].n);
    for (int e = threadIdx.x; e < total; e += kTailThreads) lds[e] = T(0);
  }
  __syncthreads();
  {
    const Grid G = a.g[top];
    const Grid P = packed_grid<DIM>(G.n);
    T* X = lds + a.lds_off[top];
    T* B = X + 2 * packed_count<DIM>(G.n);
    const bool load_x = !a.zero_top;
    for_interior<DIM>(G.n, [&](int i, int j, int l) {
      const int q = gidx<DIM>(P, i, j, l), c = gidx<DIM>(G, i, j, l);
      B[q] = a.b[top][c];
      if (load_x) X[q] = a.x[top][c];
    });
  }
  __syncthreads();
  const int par_pre = a.npre & 1;
  // down: pre-smoothing, residual, restriction
  for (int k = top; k >= 2; --k) {
    const int n = a.g[k].n;
    const Grid P = packed_grid<DIM>(n);
    const int cnt = packed_count<DIM>(n);
    T* xk = lds + a.lds_off[k];
    T* tk = xk + cnt;
    T* bk = tk + cnt;
    const bool zero = k < top || a.zero_top;
    const T scale = a.scale[k];
    for (int s = 0; s < a.npre; ++s) {
      const T wd = a.wdpre[k][s];
      const bool z = zero && s == 0;
      for_interior<DIM>(n, [&](int i, int j, int l) {
        const int c = gidx<DIM>(P, i, j, l);
        tk[c] = z ? wd * bk[c] : xk[c] + wd * (bk[c] - apply_A_at<DIM>(xk, c, P, scale));
      });
      __syncthreads();
      T* sw = xk; xk = tk; tk = sw;
    }
    const Grid C = packed_grid<DIM>(a.g[k - 1].n);
    T* bc = lds + a.lds_off[k - 1] + 2 * packed_count<DIM>(C.n);
    for_interior<DIM>(C.n, [&](int i, int j, int l) {
      const int q = gidx<DIM>(P, 2 * i, 2 * j, 2 * l);
      auto r = [&](int p) { return bk[p] - apply_A_at<DIM>(xk, p, P, scale); };
      const int dx = 1, dy = P.px;
      T h = (r(q + dx) + r(q - dx)) + (r(q + dy) + r(q - dy)) + (r(q + dx + dy) + r(q - dx - dy));
      if (DIM == 3) {
        const int dz = P.pz;
        h += (r(q + dz) + r(q - dz)) + (r(q + dx + dz) + r(q - dx - dz)) +
             (r(q + dy + dz) + r(q - dy - dz)) + (r(q + dx + dy + dz) + r(q - dx - dy - dz));
      }
      bc[gidx<DIM>(C, i, j, l)] = r(q) + T(0.5) * h;
    });
    __syncthreads();
  }
  // level 1: exact solve with the dense inverse
  {
    const Grid P1 = packed_grid<DIM>(a.g[1].n);
    T* x1 = lds + a.lds_off[1];
    const T* b1 = x1 + 2 * packed_count<DIM>(P1.n);
    for (int r = threadIdx.x; r < a.N1; r += kTailThreads) {
      T s = 0;
      for (int c = 0; c < a.N1; ++c) s += a.ainv[r * a.N1 + c] * b1[level1_node<DIM>(P1, c)];
      x1[level1_node<DIM>(P1, r)] = s;
    }
    __syncthreads();
  }
  // up: prolongation + correction, post-smoothing
  T* xfinal = nullptr;
  for (int k = 2; k <= top; ++k) {
    const int n = a.g[k].n;
    const Grid P = packed_grid<DIM>(n);
    const int cnt = packed_count<DIM>(n);
    T* xk = lds + a.lds_off[k];
    T* tk = xk + cnt;
    T* bk = tk + cnt;
    if (par_pre) { T* sw = xk; xk = tk; tk = sw; }
    const Grid C = packed_grid<DIM>(a.g[k - 1].n);
    const T* xc = lds + a.lds_off[k - 1];
    if (k - 1 >= 2 && par_pre ^ (a.npost & 1)) xc += packed_count<DIM>(C.n);   // level k-1's final x
    for_interior<DIM>(n, [&](int i, int j, int l) {
      const int si = i & 1, sj = j & 1, sl = DIM == 3 ? (l & 1) : 0;
      const int pi = i >> 1, pj = j >> 1, pl = l >> 1;
      T v = xc[gidx<DIM>(C, pi, pj, pl)];
      if (si | sj | sl) v = T(0.5) * (v + xc[gidx<DIM>(C, pi + si, pj + sj, pl + sl)]);
      const int q = gidx<DIM>(P, i, j, l);
      xk[q] = xk[q] + v;
    });
    __syncthreads();
    const T scale = a.scale[k];
    for (int s = 0; s < a.npost; ++s) {
      const T wd = a.wdpost[k][s];
      for_interior<DIM>(n, [&](int i, int j, int l) {
        const int c = gidx<DIM>(P, i, j, l);
        tk[c] = xk[c] + wd * (bk[c] - apply_A_at<DIM>(xk, c, P, scale));
      });
      __syncthreads();
      T* sw = xk; xk = tk; tk = sw;
    }
    xfinal = xk;
  }
  // write x[top] back where the host expects it after the cycle's role swaps
  {
    const Grid G = a.g[top];
    const Grid P = packed_grid<DIM>(G.n);
    T* dst = ((a.npre + a.npost) & 1) ? a.t[top] : a.x[top];
    for_interior<DIM>(G.n, [&](int i, int j, int l) {
      dst[gidx<DIM>(G, i, j, l)] = xfinal[gidx<DIM>(P, i, j, l)];
    });
  }
}

template <int DIM>
inline size_t tail_lds_elements(const int* n, int top, int* off) {
  size_t e = 0;
  for (int k = 1; k <= top; ++k) {
    off[k] = (int)e;
    const size_t c = DIM == 2 ? (size_t)(n[k] + 1) * (n[k] + 1) : (size_t)(n[k] + 1) * (n[k] + 1) * (n[k] + 1);
    e += 3 * c;
  }
  return e;
}

// ---------------------------------------------------------------------------
// Dense-operator variant: the cycle from x0 equals x0 + B (b - A x0) with B the
// cycle's matrix (built on the host from the same steps).  Every block forms
// the residual r = b - A x0 of the N top-level unknowns in LDS (float64),
// then each wavefront produces one output row as a 64-lane dot product.
// out must not alias x0.
// ---------------------------------------------------------------------------
template <int DIM, typename T>
__global__ void __launch_bounds__(256) k_tail_dense(Grid g, const double* __restrict__ B, int N,
                                                    const T* __restrict__ x0, const T* __restrict__ b,
                                                    T* __restrict__ out, T scale, int zero) {
  extern __shared__ double r[];
  const int m = g.n - 1;
  for (int q = threadIdx.x; q < N; q += blockDim.x) {
    const int i = 1 + q % m, j = 1 + (q / m) % m, l = DIM == 3 ? 1 + q / (m * m) : 0;
    const int c = gidx<DIM>(g, i, j, l);
    r[q] = zero ? (double)b[c] : (double)(b[c] - apply_A_at<DIM>(x0, c, g, scale));
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= N) return;                      // whole wavefront leaves together
  const double* __restrict__ Br = B + (size_t)row * N;
  double acc = 0.0;
  for (int q = lane; q < N; q += 64) acc += Br[q] * r[q];
  acc = wave_sum(acc);
  if (lane == 0) {
    const int i = 1 + row % m, j = 1 + (row / m) % m, l = DIM == 3 ? 1 + row / (m * m) : 0;
    const int c = gidx<DIM>(g, i, j, l);
    out[c] = zero ? (T)acc : (T)((double)x0[c] + acc);
  }
}

}  // namespace fmg
