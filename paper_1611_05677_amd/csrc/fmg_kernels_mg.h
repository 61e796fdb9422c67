// Multigrid-cycle kernels (float64 and float32 instances): stiffness apply,
// weighted Jacobi sweep, residual + restriction, prolongation (+ correction),
// level-1 dense solve, and the float64 <-> float32 glue of the mixed mode.
//
// Operators on the structured P1 meshes (Section 2 / Section 3):
//   A_k x   = s_k (2d x_c - sum of the 2d axis neighbours), s_k = h_k^{d-2}
//             (the Kuhn-diagonal couplings of P1 on these meshes vanish);
//   P_k     = natural inclusion V_{h_{k-1}} -> V_{h_k}: fine node 2p + e
//             (e in {0,1}^d) takes the mean of coarse nodes p and p + e,
//             the end points of the Kuhn edge it bisects;
//   P_k^T r = r(2p) + 1/2 sum_{e != 0} (r(2p + e) + r(2p - e)).
#pragma once

#include "fmg_device.h"

namespace fmg {

// Grid kernels: logical block (bx, by, bz) covers kBlock nodes of row
// (j, l) = (1 + by, 1 + bz).  The launch is one-dimensional with
// grid_blocks() blocks; hardware block ids go to the 8 XCDs in turn, and the
// remap below hands each XCD a contiguous range of logical blocks (whole rows,
// hence neighbouring rows and planes), so stencil neighbours read by one block
// were usually brought into that XCD's L2 by the block before it.
template <int DIM>
__host__ __device__ inline int logical_blocks(int n) {
  const int gx = (n - 1 + kBlock - 1) / kBlock;
  return gx * (n - 1) * (DIM == 3 ? n - 1 : 1);
}
template <int DIM>
__host__ __device__ inline int grid_blocks(int n) { return ((logical_blocks<DIM>(n) + 7) / 8) * 8; }

// Thread -> interior node (i, j, l) of a grid kernel launched with
// grid_blocks<DIM>(n) blocks of kBlock threads.
template <int DIM>
__device__ __forceinline__ bool node_of_thread(const Grid& g, int& i, int& j, int& l) {
  const int nb = logical_blocks<DIM>(g.n);
  const int per = (nb + 7) >> 3;
  const int L = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (L >= nb) return false;
  const int gx = (g.n - 1 + kBlock - 1) / kBlock, gy = g.n - 1;
  const int bx = L % gx, r = L / gx;
  i = 1 + bx * kBlock + threadIdx.x;
  j = 1 + r % gy;
  l = DIM == 3 ? 1 + r / gy : 0;
  return i < g.n;
}

// The same blocks as node_of_thread, with the rows of each XCD's chunk taken
// in bands of kRowBand rows (j) that march through the planes (l).  A kernel
// whose threads read several planes on either side (the residual restriction:
// two fine planes each way) then keeps its working set in the XCD's L2; in
// plane order the rows in flight span about eight fine planes of two arrays.
constexpr int kRowBand = 16;

template <int DIM>
__device__ __forceinline__ bool node_of_thread_banded(const Grid& g, int& i, int& j, int& l) {
  if (DIM == 2) return node_of_thread<DIM>(g, i, j, l);
  const int nb = logical_blocks<DIM>(g.n);
  const int per = (nb + 7) >> 3;
  const int L = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (L >= nb) return false;
  const int gx = (g.n - 1 + kBlock - 1) / kBlock, gy = g.n - 1;
  const int bx = L % gx, r = L / gx;  // row r of the gy * gy interior rows
  const int band = r / (kRowBand * gy);
  const int rem = r - band * kRowBand * gy;
  const int h = min(kRowBand, gy - band * kRowBand);  // rows in this band
  const int lr = rem / h, jr = rem - lr * h;
  i = 1 + bx * kBlock + threadIdx.x;
  j = 1 + band * kRowBand + jr;
  l = 1 + lr;
  return i < g.n;
}

template <int DIM, typename T>
__device__ __forceinline__ T apply_A_at(const T* __restrict__ x, int c, const Grid& g, T scale) {
  T s = (x[c - 1] + x[c + 1]) + (x[c - g.px] + x[c + g.px]);
  if (DIM == 3) s += x[c - g.pz] + x[c + g.pz];
  return scale * (T(2 * DIM) * x[c] - s);
}

template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_apply_A(Grid g, const T* __restrict__ x, T* __restrict__ y, T scale) {
  int i, j, l;
  if (!node_of_thread<DIM>(g, i, j, l)) return;
  int c = gidx<DIM>(g, i, j, l);
  y[c] = apply_A_at<DIM>(x, c, g, scale);
}

// One damped-Jacobi sweep out = x + (w/D) (b - A x); ZERO: x is zero (first
// sweep of a coarse-grid correction), out = (w/D) b.
template <int DIM, typename T, bool ZERO>
__global__ void __launch_bounds__(kBlock) k_smooth(Grid g, const T* __restrict__ x, const T* __restrict__ b,
                                                   T* __restrict__ out, T wd, T scale) {
  int i, j, l;
  if (!node_of_thread<DIM>(g, i, j, l)) return;
  int c = gidx<DIM>(g, i, j, l);
  if (ZERO) out[c] = wd * b[c];
  else out[c] = x[c] + wd * (b[c] - apply_A_at<DIM>(x, c, g, scale));
}

// bc(p) = (P^T (b - A x))(p) at the interior coarse nodes p.
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_resid_restrict(Grid f, Grid cg, const T* __restrict__ x,
                                                           const T* __restrict__ b, T* __restrict__ bc, T scale) {
  int i, j, l;
  if (!node_of_thread_banded<DIM>(cg, i, j, l)) return;
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

// xf = P xc (ADD = false) or xf += P xc (ADD = true) at the fine interior nodes.
template <int DIM, typename T, bool ADD>
__global__ void __launch_bounds__(kBlock) k_prolong(Grid cg, Grid f, const T* __restrict__ xc, T* __restrict__ xf) {
  int i, j, l;
  if (!node_of_thread<DIM>(f, i, j, l)) return;
  const int si = i & 1, sj = j & 1, sl = DIM == 3 ? (l & 1) : 0;
  const int pi = i >> 1, pj = j >> 1, pl = l >> 1;
  // All loads are issued before the first use; at a coarse node both coarse
  // loads read the same value, and 0.5 (v0 + v0) = v0 exactly.
  const int q = gidx<DIM>(f, i, j, l);
  const T old = ADD ? xf[q] : T(0);
  const T v0 = xc[gidx<DIM>(cg, pi, pj, pl)];
  const T v1 = xc[gidx<DIM>(cg, pi + si, pj + sj, pl + sl)];
  const T v = T(0.5) * (v0 + v1);
  xf[q] = ADD ? old + v : v;
}

// Dense index r (x fastest over the (n1-1)^d interior nodes of level 1) -> grid index.
template <int DIM>
__device__ __forceinline__ int level1_node(const Grid& g1, int r) {
  const int m = g1.n - 1;
  const int i = 1 + r % m, j = 1 + (r / m) % m, l = DIM == 3 ? 1 + r / (m * m) : 0;
  return gidx<DIM>(g1, i, j, l);
}

// x = A_1^{-1} b on level 1 (exact coarsest solve of the V-cycle); one block.
template <int DIM, typename T>
__global__ void k_coarse_solve(Grid g1, int N1, const T* __restrict__ Ainv, const T* __restrict__ b,
                               T* __restrict__ x) {
  for (int r = threadIdx.x; r < N1; r += blockDim.x) {
    T s = 0;
    for (int c = 0; c < N1; ++c) s += Ainv[r * N1 + c] * b[level1_node<DIM>(g1, c)];
    x[level1_node<DIM>(g1, r)] = s;
  }
}

// Mixed precision: r32 = float(b - A u) evaluated in float64; u += double(e32).
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_resid_to_f32(Grid g, const double* __restrict__ u,
                                                         const double* __restrict__ b, float* __restrict__ r,
                                                         double scale) {
  int i, j, l;
  if (!node_of_thread<DIM>(g, i, j, l)) return;
  int c = gidx<DIM>(g, i, j, l);
  r[c] = (float)(b[c] - apply_A_at<DIM>(u, c, g, scale));
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_add_f32(Grid g, double* __restrict__ u, const float* __restrict__ e) {
  int i, j, l;
  if (!node_of_thread<DIM>(g, i, j, l)) return;
  int c = gidx<DIM>(g, i, j, l);
  u[c] += (double)e[c];
}

// Plain element-wise helpers (no memset nodes are used inside captured graphs).
template <typename T>
__global__ void k_fill(T* __restrict__ p, size_t count, T v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}

template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_copy_interior(Grid g, const T* __restrict__ src, T* __restrict__ dst) {
  int i, j, l;
  if (!node_of_thread<DIM>(g, i, j, l)) return;
  int c = gidx<DIM>(g, i, j, l);
  dst[c] = src[c];
}

// Packed (n+1)^d <-> padded level layout (all nodes; boundary of the
// destination forced to zero when unpacking into a level array).
template <int DIM, typename TD, typename TS>
__global__ void k_pack(Grid g, const TS* __restrict__ src, TD* __restrict__ dst, int to_packed) {
  const int n1 = g.n + 1;
  const size_t total = DIM == 2 ? (size_t)n1 * n1 : (size_t)n1 * n1 * n1;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(p % n1), j = (int)((p / n1) % n1), l = DIM == 3 ? (int)(p / ((size_t)n1 * n1)) : 0;
    const int c = gidx<DIM>(g, i, j, l);
    const bool bnd = i == 0 || j == 0 || i == g.n || j == g.n || (DIM == 3 && (l == 0 || l == g.n));
    if (to_packed) dst[p] = bnd ? TD(0) : (TD)src[c];
    else dst[c] = bnd ? TD(0) : (TD)src[p];
  }
}

}  // namespace fmg
