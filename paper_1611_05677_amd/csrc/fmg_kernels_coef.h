// Variable coefficient: the operator -div(A(x) grad u) of eq. "semilinear
// equation" (Section 2) with A symmetric positive definite and constant on
// every cell of the finest mesh.
//
// One bilinear form on all the nested spaces (eq. "FEM_Space_Series"): the
// matrix of level k is the finest form restricted to V_{h_k}.  On a level-k
// simplex T the level-k hat gradients are constant, so that restriction is
// the plain P1 assembly on level k with, on each simplex, the volume mean of
// the finest matrices inside it.  A Kuhn simplex of a cell is the union of
// 2^d Kuhn simplices of its child cells, so the means are formed level by
// level, each coarse simplex the mean of its 2^d children.
//
// Stencil.  Every edge of the Kuhn split joins a node p to p + delta with
// delta a nonzero 0/1 vector (d = 2: 3 directions, a 7-point stencil; d = 3:
// 7 directions, 15 points).  Level arrays W_delta hold, at every node p, the
// weight of its forward edge p -> p + delta, minus the stiffness entry:
//   (A_k x)_c = sum_delta W_delta(c) (x_c - x_{c+delta})
//                       + W_delta(c-delta) (x_c - x_{c-delta}),
// diag(A_k)_c the sum of those 2(2^d - 1) weights (row sums of the stiffness
// matrix vanish before the Dirichlet nodes are dropped).  With the unit-cell
// chain 0 = v_0, v_1 = e_a0, .., v_d = 1..1 of a simplex, the barycentric
// gradients are g_0 = -e_a0, g_k = e_a(k-1) - e_ak, g_d = e_a(d-1) (over h),
// and the simplex adds -h^(d-2)/d! g_i^T A_T g_j to the edge v_i -> v_j.
//
// Matrices are given as their d(d+1)/2 upper-triangle components row by row
// (2D: a11, a12, a22; 3D: a11, a12, a13, a22, a23, a33): at the finest level
// per cell (component planes of n^d cells, x fastest), below it per simplex
// (planes [component][simplex] of the level's cells; simplex s follows the
// chain of KuhnChain<DIM, s>).
#pragma once

#include "fmg_device.h"
#include "fmg_kernels_mg.h"

namespace fmg {

template <int DIM> __host__ __device__ constexpr int coef_fwd() { return (1 << DIM) - 1; }
template <int DIM> __host__ __device__ constexpr int coef_comps() { return DIM * (DIM + 1) / 2; }
template <int DIM> __host__ __device__ constexpr int coef_simplices() { return DIM == 2 ? 2 : 6; }

// One term of a forward-edge weight: W_delta(p) += c h^(d-2)/d! A[q] of
// simplex s in the cell with lower corner p - o (c a small integer).  Built
// on the host from the chain formula above (coef_terms in fmg.hip); grouped
// by delta.
constexpr int kCoefTermsMax = 160;
struct CoefTerms {
  int begin[8];                  // terms of direction delta: [begin[delta-1], begin[delta])
  unsigned char o[kCoefTermsMax], s[kCoefTermsMax], q[kCoefTermsMax];
  signed char c[kCoefTermsMax];
};

// Children of a coarse simplex: fine simplex (octant o, chain s) lies in the
// coarse simplex sigma[o][s] of the parent cell.
struct CoarsenMap {
  unsigned char sigma[8][6];
};

// Per-level stencil arrays for the kernels (read through the problem slot by
// the augmented setup pass).
struct CoefLevels {
  const double* w[FMG_MAX_LEVELS + 1];   // W planes of level k (nullptr: A = I)
  long long plane[FMG_MAX_LEVELS + 1];   // elements between W planes
};

// ---------------------------------------------------------------------------
// Setup kernels (once per coefficient field).
// ---------------------------------------------------------------------------

// Level simplex matrices of a coarse level (nc cells per side) from the next
// finer level: per (coarse cell, simplex, component) the mean of its 2^d
// children, in the fixed order (octant, fine simplex).  per_cell: the source
// is the finest level (one matrix per cell).
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_coef_coarsen(int nc, const double* __restrict__ src, int per_cell,
                                                         double* __restrict__ dst, CoarsenMap map) {
  constexpr int NS = coef_simplices<DIM>(), NC = coef_comps<DIM>(), NO = 1 << DIM;
  const long long ncc = DIM == 2 ? (long long)nc * nc : (long long)nc * nc * nc;
  const long long nf = 2LL * nc;
  const long long ncf = DIM == 2 ? nf * nf : nf * nf * nf;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncc * NS) return;
  const int sig = (int)(t / ncc);
  const long long cell = t - sig * ncc;
  const int cx = (int)(cell % nc), cy = (int)((cell / nc) % nc), cz = DIM == 3 ? (int)(cell / ((long long)nc * nc)) : 0;
  const int sstride = per_cell ? 0 : 1, ns_src = per_cell ? 1 : NS;
  for (int q = 0; q < NC; ++q) {
    double sum = 0.0;
    for (int o = 0; o < NO; ++o) {
      const long long fx = 2 * cx + (o & 1), fy = 2 * cy + ((o >> 1) & 1), fz = DIM == 3 ? 2 * cz + ((o >> 2) & 1) : 0;
      const long long fcell = fx + nf * (fy + nf * fz);
      for (int s = 0; s < NS; ++s)
        if (map.sigma[o][s] == sig) sum += src[((long long)q * ns_src + s * sstride) * ncf + fcell];
    }
    dst[((long long)q * NS + sig) * ncc + cell] = sum * (1.0 / NO);
  }
}

// Forward-edge weights of a level at every node (boundary nodes included:
// their edges into the interior enter the interior rows).  src as in
// k_coef_coarsen; scale = h^(d-2) / d!.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_coef_weights(Grid g, const double* __restrict__ src, int per_cell,
                                                         double scale, double* __restrict__ W, long long plane,
                                                         CoefTerms terms) {
  constexpr int NS = coef_simplices<DIM>(), NF = coef_fwd<DIM>();
  const int n = g.n, n1 = n + 1;
  const long long nodes = DIM == 2 ? (long long)n1 * n1 : (long long)n1 * n1 * n1;
  const long long ncell = DIM == 2 ? (long long)n * n : (long long)n * n * n;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nodes) return;
  const int i = (int)(t % n1), j = (int)((t / n1) % n1), l = DIM == 3 ? (int)(t / ((long long)n1 * n1)) : 0;
  const int c = gidx<DIM>(g, i, j, l);
  const int sstride = per_cell ? 0 : 1, ns_src = per_cell ? 1 : NS;
  for (int dl = 1; dl <= NF; ++dl) {
    double w = 0.0;
    for (int k = terms.begin[dl - 1]; k < terms.begin[dl]; ++k) {
      const int o = terms.o[k];
      const int x = i - (o & 1), y = j - ((o >> 1) & 1), z = DIM == 3 ? l - ((o >> 2) & 1) : 0;
      if (x < 0 || y < 0 || z < 0 || x >= n || y >= n || (DIM == 3 && z >= n)) continue;
      const long long cell = x + (long long)n * (y + (long long)n * z);
      w += (double)terms.c[k] * src[((long long)terms.q[k] * ns_src + terms.s[k] * sstride) * ncell + cell];
    }
    W[(dl - 1) * plane + c] = scale * w;
  }
}

// Offset of the node p + delta in a level array.
template <int DIM>
__device__ __forceinline__ int fwd_offset(const Grid& g, int dl) {
  return (dl & 1) + ((dl >> 1) & 1) * g.px + (DIM == 3 ? ((dl >> 2) & 1) * g.pz : 0);
}

// Level-1 stiffness as a dense N1 x N1 matrix (x fastest), one row per thread.
template <int DIM>
__global__ void k_coef_level1(Grid g1, const double* __restrict__ W, long long plane, int N1,
                              double* __restrict__ A1) {
  constexpr int NF = coef_fwd<DIM>();
  const int m = g1.n - 1;
  for (int r = threadIdx.x; r < N1; r += blockDim.x) {
    for (int q = 0; q < N1; ++q) A1[(size_t)r * N1 + q] = 0.0;
    const int i = 1 + r % m, j = 1 + (r / m) % m, l = DIM == 3 ? 1 + r / (m * m) : 0;
    const int c = gidx<DIM>(g1, i, j, l);
    double diag = 0.0;
    for (int dl = 1; dl <= NF; ++dl) {
      const int off = fwd_offset<DIM>(g1, dl);
      const double wf = W[(dl - 1) * plane + c], wb = W[(dl - 1) * plane + c - off];
      diag += wf + wb;
      const int dx = dl & 1, dy = (dl >> 1) & 1, dz = (dl >> 2) & 1;
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        const int x = i + sgn * dx, y = j + sgn * dy, z = l + sgn * dz;
        if (x < 1 || x > m || y < 1 || y > m || (DIM == 3 && (z < 1 || z > m))) continue;
        const int q = (x - 1) + m * (y - 1) + (DIM == 3 ? m * m * (z - 1) : 0);
        A1[(size_t)r * N1 + q] = -(sgn > 0 ? wf : wb);
      }
    }
    A1[(size_t)r * N1 + r] = diag;
  }
}

// Inverse of a symmetric positive definite N x N matrix (N <= 64) by
// Gauss-Jordan elimination without pivoting on [A | I] in LDS, one block;
// writes the float64 inverse and its float32 copy.
constexpr int kInvertThreads = 256;
__host__ __device__ constexpr int invert_lds_doubles(int N) { return 2 * N * N + N; }

static __global__ void __launch_bounds__(kInvertThreads) k_spd_invert(const double* __restrict__ A, double* __restrict__ Ainv,
                                                               float* __restrict__ Ainv_f, int N) {
  extern __shared__ double sm[];
  const int W2 = 2 * N;
  double* M = sm;            // N x 2N
  double* fac = sm + N * W2; // N
  for (int e = threadIdx.x; e < N * W2; e += blockDim.x) {
    const int r = e / W2, c = e % W2;
    M[e] = c < N ? A[(size_t)r * N + c] : (c - N == r ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    const double rp = 1.0 / M[k * W2 + k];
    __syncthreads();
    for (int c = threadIdx.x; c < W2; c += blockDim.x) M[k * W2 + c] *= rp;
    for (int r = threadIdx.x; r < N; r += blockDim.x) fac[r] = r == k ? 0.0 : M[r * W2 + k];
    __syncthreads();
    for (int e = threadIdx.x; e < N * W2; e += blockDim.x) {
      const int r = e / W2, c = e % W2;
      if (r != k) M[e] -= fac[r] * M[k * W2 + c];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
    const int r = e / N, c = e % N;
    const double v = M[r * W2 + N + c];
    Ainv[e] = v;
    Ainv_f[e] = (float)v;
  }
}

// ---------------------------------------------------------------------------
// Multigrid operators with the stencil arrays (float64).  Each node reads its
// own seven (3D) weights and those of its backward neighbours, three of which
// lie in the previous plane: the blocks take rows in bands that march through
// the planes (node_of_thread_banded), so that plane is still in the XCD's L2.
// ---------------------------------------------------------------------------

// (A x)_c and diag(A)_c at interior node c.
template <int DIM>
__device__ __forceinline__ double apply_Aw_at(const double* __restrict__ x, int c, const Grid& g,
                                              const double* __restrict__ W, long long plane, double& diag) {
  constexpr int NF = coef_fwd<DIM>();
  double wf[NF], wb[NF], xf[NF], xb[NF];
#pragma unroll
  for (int dl = 1; dl <= NF; ++dl) {
    const int off = fwd_offset<DIM>(g, dl);
    wf[dl - 1] = W[(dl - 1) * plane + c];
    wb[dl - 1] = W[(dl - 1) * plane + c - off];
    xf[dl - 1] = x[c + off];
    xb[dl - 1] = x[c - off];
  }
  const double xc = x[c];
  double d = 0.0, s = 0.0;
#pragma unroll
  for (int q = 0; q < NF; ++q) {
    d += wf[q] + wb[q];
    s += wf[q] * xf[q] + wb[q] * xb[q];
  }
  diag = d;
  return d * xc - s;
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_apply_Aw(Grid g, const double* __restrict__ x, double* __restrict__ y,
                                                     const double* __restrict__ W, long long plane) {
  int i, j, l;
  if (!node_of_thread_banded<DIM>(g, i, j, l)) return;
  const int c = gidx<DIM>(g, i, j, l);
  double diag;
  y[c] = apply_Aw_at<DIM>(x, c, g, W, plane, diag);
}

// One damped-Jacobi sweep out = x + w D^{-1} (b - A x); ZERO: x = 0, out = w D^{-1} b.
template <int DIM, bool ZERO>
__global__ void __launch_bounds__(kBlock) k_smooth_w(Grid g, const double* __restrict__ x,
                                                     const double* __restrict__ b, double* __restrict__ out,
                                                     const double* __restrict__ W, long long plane, double w) {
  int i, j, l;
  if (!node_of_thread_banded<DIM>(g, i, j, l)) return;
  const int c = gidx<DIM>(g, i, j, l);
  if (ZERO) {
    constexpr int NF = coef_fwd<DIM>();
    double d = 0.0;
#pragma unroll
    for (int dl = 1; dl <= NF; ++dl) d += W[(dl - 1) * plane + c] + W[(dl - 1) * plane + c - fwd_offset<DIM>(g, dl)];
    out[c] = w * b[c] / d;
  } else {
    double d;
    const double ax = apply_Aw_at<DIM>(x, c, g, W, plane, d);
    out[c] = x[c] + w * (b[c] - ax) / d;
  }
}

// r = b - A x at the interior nodes.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_resid_w(Grid g, const double* __restrict__ x,
                                                    const double* __restrict__ b, double* __restrict__ r,
                                                    const double* __restrict__ W, long long plane) {
  int i, j, l;
  if (!node_of_thread_banded<DIM>(g, i, j, l)) return;
  const int c = gidx<DIM>(g, i, j, l);
  double d;
  r[c] = b[c] - apply_Aw_at<DIM>(x, c, g, W, plane, d);
}

// bc = P^T r at the interior coarse nodes (the combination of k_resid_restrict
// applied to a stored residual).
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_restrict(Grid f, Grid cg, const double* __restrict__ r,
                                                     double* __restrict__ bc) {
  int i, j, l;
  if (!node_of_thread_banded<DIM>(cg, i, j, l)) return;
  const int q = gidx<DIM>(f, 2 * i, 2 * j, 2 * l);
  const int dx = 1, dy = f.px;
  double h = (r[q + dx] + r[q - dx]) + (r[q + dy] + r[q - dy]) + (r[q + dx + dy] + r[q - dx - dy]);
  if (DIM == 3) {
    const int dz = f.pz;
    h += (r[q + dz] + r[q - dz]) + (r[q + dx + dz] + r[q - dx - dz]) + (r[q + dy + dz] + r[q - dy - dz]) +
         (r[q + dx + dy + dz] + r[q - dx - dy - dz]);
  }
  bc[gidx<DIM>(cg, i, j, l)] = r[q] + 0.5 * h;
}

}  // namespace fmg
