// Fused pairs of 3D weighted-Jacobi sweeps (float64 or float32).
//
// The V(2,2) cycle's pre-smoothing is two sweeps, x1 = x0 + w1 D^{-1}(b - A x0)
// and x2 = x1 + w2 D^{-1}(b - A x1); its post-smoothing is the same pair after
// the coarse correction x0 = x + P x_c.  Run as separate launches, each sweep
// reads x and b and writes x' (24 bytes per node in float64) and the
// prolongation reads and writes x once more.  Here one launch performs the
// pair (and, for the post-smoothing, the correction as the planes are loaded):
// read x and b once, write x2 once.
//
// Layout of the work: a workgroup of 16 wavefronts covers a tile of 64
// columns (x, one per lane) by 16 rows (y, one per wavefront) and marches
// through a run of planes (z).  The tile's outer two lanes and rows on each
// side are halo: they are loaded and swept once, so that the second sweep is
// exact on the inner 60 x 12 nodes, which the workgroup owns and writes.
//   * x-neighbours come from the adjacent lanes (DPP whole-wave shifts);
//   * y-neighbours from the wavefronts above and below, through one LDS plane
//     per stage (double-buffered by plane parity, two barriers per plane);
//   * z-neighbours are the previous and next planes, kept in registers;
//   * loads run two planes ahead in a register ring, from clamped (always
//     in-bounds) addresses; values outside the grid are masked to 0.
// Arithmetic per node is the separate sweep's expression, in the same order:
//   x' = x + wd (b - s (6 x - ((x_w + x_e) + (x_s + x_n) + (x_d + x_u)))).
#pragma once

#include "fmg_device.h"
#include "fmg_kernels_stream2d.h"

namespace fmg {

constexpr int kP3Rows = 16;                 // rows (wavefronts) per workgroup
constexpr int kP3Halo = 2;                  // two sweeps: two halo lanes / rows per side
constexpr int kP3OwnX = 64 - 2 * kP3Halo;   // owned columns per workgroup
constexpr int kP3OwnY = kP3Rows - 2 * kP3Halo;
constexpr int kP3Threads = 64 * kP3Rows;

// Launch geometry: strips of owned columns x row chunks x plane chunks; planes
// per chunk chosen for about `target` workgroups.  Logical block order: strip
// fastest, then row chunk, then plane chunk, so each XCD's contiguous range of
// logical blocks holds tiles that share halo rows and columns.
struct Pair3Shape {
  int nsx, ncy, nzc, zc_planes;
};

inline Pair3Shape pair3_shape(int n, int target = 1024) {
  Pair3Shape s;
  s.nsx = (n - 1 + kP3OwnX - 1) / kP3OwnX;
  s.ncy = (n - 1 + kP3OwnY - 1) / kP3OwnY;
  int nzc = (target + s.nsx * s.ncy - 1) / (s.nsx * s.ncy);
  const int zmin = 8;                       // at least 8 owned planes per chunk
  if (nzc > (n - 1 + zmin - 1) / zmin) nzc = (n - 1 + zmin - 1) / zmin;
  if (nzc < 1) nzc = 1;
  s.zc_planes = (n - 1 + nzc - 1) / nzc;
  s.nzc = (n - 1 + s.zc_planes - 1) / s.zc_planes;
  return s;
}

inline int pair3_blocks(const Pair3Shape& s) { return ((s.nsx * s.ncy * s.nzc) + 7) & ~7; }

// ZERO: the first sweep starts from x0 = 0 (x is not read).  PROLONG: x0 is
// x + P xc (the coarse correction, xc on the next coarser grid cg).
template <typename T, bool ZERO, bool PROLONG>
__global__ void __launch_bounds__(kP3Threads)
    k_sweep_pair3(Grid g, Grid cg, const T* __restrict__ x, const T* __restrict__ xc, const T* __restrict__ b,
                  T* __restrict__ out, T wd1, T wd2, T scale, int nsx, int ncy, int nzc, int zc_planes) {
  __shared__ T lx[2][kP3Rows][64];   // x0 plane (sweep 1's y-neighbours), by plane parity
  __shared__ T ls[2][kP3Rows][64];   // sweep-1 plane (sweep 2's y-neighbours)
  const int n = g.n;
  const int nlog = nsx * ncy * nzc;
  const int per = (gridDim.x + 7) >> 3;
  const int Lb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (Lb >= nlog) return;                                    // whole workgroup leaves together
  const int sx = Lb % nsx, cy = (Lb / nsx) % ncy, zc = Lb / (nsx * ncy);
  const int row = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int X = 1 + sx * kP3OwnX - kP3Halo + lane;
  const int Y = 1 + cy * kP3OwnY - kP3Halo + row;
  const bool col_ok = X >= 0 && X <= n, row_ok = Y >= 0 && Y <= n;
  const bool in_xy = X >= 1 && X <= n - 1 && Y >= 1 && Y <= n - 1;
  const bool own = lane >= kP3Halo && lane < 64 - kP3Halo && row >= kP3Halo && row < kP3Rows - kP3Halo && in_xy;
  const int Xc = X < 0 ? 0 : (X > n ? n : X), Yc = Y < 0 ? 0 : (Y > n ? n : Y);
  const int off = Yc * g.px + Xc;
  const int rdn = row > 0 ? row - 1 : 0, rup = row < kP3Rows - 1 ? row + 1 : row;
  const int Z0 = 1 + zc * zc_planes, Zend = min(Z0 + zc_planes, n);   // owned planes [Z0, Zend)
  const int zs = Z0 - kP3Halo, steps = Zend - Z0 + 2 * kP3Halo;         // planes Z0-2 .. Zend+1
  // prolongation: the two coarse nodes whose mean is the fine value
  int c0 = 0, c1 = 0, cs = 0, pzf = 0;
  if (PROLONG) {
    const int si = Xc & 1, sj = Yc & 1;
    c0 = (Yc >> 1) * cg.px + (Xc >> 1);
    c1 = min((Yc >> 1) + sj, cg.n) * cg.px + min((Xc >> 1) + si, cg.n);
    cs = si | sj;
    pzf = cg.pz;
  }
  auto plane = [&](int z) { return (z < 0 ? 0 : (z > n ? n : z)); };
  // ring of two plane slots: x0 (with the coarse pair), b
  T qx[2], qb[2], qc0[2], qc1[2];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const int z = plane(zs + d);
    qx[d] = ZERO ? T(0) : x[(size_t)z * g.pz + off];
    qb[d] = b[(size_t)z * g.pz + off];
    if (PROLONG) {
      const int zc0 = z >> 1, zc1 = min((z >> 1) + (z & 1), cg.n);
      qc0[d] = xc[(size_t)zc0 * pzf + c0];
      qc1[d] = xc[(size_t)zc1 * pzf + c1];
    }
  }
  T xa = 0, xb = 0, b1 = 0, b2 = 0, sa = 0, sb = 0;   // x0 planes z-2, z-1; b planes z-1, z-2; s1 planes z-3, z-2
  for (int i0 = 0; i0 < steps; i0 += 2) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int i = i0 + d;
      const int zl = zs + i;
      const bool z_ok = zl >= 0 && zl <= n;
      const bool ok = col_ok && row_ok && z_ok;
      T xn = ok ? qx[d] : T(0);
      const T bn = ok ? qb[d] : T(0);
      if (PROLONG && ok && in_xy && zl >= 1 && zl <= n - 1) {
        T v = qc0[d];
        if (cs | (zl & 1)) v = T(0.5) * (v + qc1[d]);
        xn = xn + v;
      }
      {   // refill the slot with plane zl + 2 (clamped past the end; unused)
        const int z = plane(zl + 2);
        qx[d] = ZERO ? T(0) : x[(size_t)z * g.pz + off];
        qb[d] = b[(size_t)z * g.pz + off];
        if (PROLONG) {
          const int zc0 = z >> 1, zc1 = min((z >> 1) + (z & 1), cg.n);
          qc0[d] = xc[(size_t)zc0 * pzf + c0];
          qc1[d] = xc[(size_t)zc1 * pzf + c1];
        }
      }
      const int par = zl & 1;
      if (!ZERO) lx[par][row][lane] = xn;
      __syncthreads();
      // sweep 1 at plane p = zl - 1 (x0 planes p-1 = xa, p = xb, p+1 = xn)
      const int p = zl - 1;
      const bool in1 = in_xy && p >= 1 && p <= n - 1;
      T s1n;
      if (ZERO) {
        s1n = in1 ? wd1 * b1 : T(0);
      } else {
        const T ysum = lx[par ^ 1][rdn][lane] + lx[par ^ 1][rup][lane];
        T sm = (from_left(xb) + from_right(xb)) + ysum;
        sm += xa + xn;
        s1n = in1 ? xb + wd1 * (b1 - scale * (T(6) * xb - sm)) : T(0);
      }
      ls[par ^ 1][row][lane] = s1n;
      __syncthreads();
      // sweep 2 at plane q = zl - 2 (s1 planes q-1 = sa, q = sb, q+1 = s1n)
      const int q = zl - 2;
      if (q >= Z0 && q < Zend) {
        const T ysum = ls[par][rdn][lane] + ls[par][rup][lane];
        T sm = (from_left(sb) + from_right(sb)) + ysum;
        sm += sa + s1n;
        const T v = sb + wd2 * (b2 - scale * (T(6) * sb - sm));
        if (own) out[(size_t)q * g.pz + off] = v;
      }
      xa = xb; xb = xn;
      b2 = b1; b1 = bn;
      sa = sb; sb = s1n;
    }
  }
}

}  // namespace fmg
