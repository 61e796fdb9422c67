// Register-streaming 3D weighted-Jacobi sweep (float64 or float32).
//
// Same operation and per-node expression as the grid sweep
//   out = x + wd (b - A x),  A x = s (6 x_c - sum of the 6 axis neighbours),
// laid out so that each input value is read from memory about once.  A block
// of four wavefronts covers a slab of columns x = 0 .. 64 WX - 1 (one column
// per lane, WX wavefronts side by side, WX = ceil(n / 64) <= 4) and 4 / WX
// groups of kS3Rows rows, and marches through a run of planes:
//   * x-neighbours come from the adjacent lanes (DPP whole-wave shifts); the
//     two edge lanes of a wavefront exchange their values with the
//     neighbouring wavefronts through LDS once per plane;
//   * y-neighbours come from the lane's own registers (rows r-1, r+1; the
//     first and last row of a group are halo, loaded but not written);
//   * z-neighbours are the two previous planes, kept in registers;
//   * loads run kS3Depth planes ahead in a ring of register slots refilled
//     in place, so each plane's data has kS3Depth plane steps to arrive.
// Points outside the interior hold 0.
#pragma once

#include "fmg_device.h"
#include "fmg_kernels_stream2d.h"

namespace fmg {

constexpr int kS3Rows = 8;                 // rows per wavefront (registers)
constexpr int kS3Own = kS3Rows - 2;        // owned rows
constexpr int kS3Waves = 4;                // wavefronts per block
constexpr int kS3Depth = 2;                // planes loaded ahead

__host__ __device__ inline int s3_wx(int n) { return (n + 63) / 64; }

template <typename T>
__global__ void __launch_bounds__(64 * kS3Waves)
    k_smooth3s(Grid g, const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ out, T wd, T scale,
               int zc_planes, int nzc) {
  __shared__ T edge[2][kS3Waves][2][kS3Rows];   // [plane parity][wave][left/right edge][row]
  const int n = g.n;
  const int WX = s3_wx(n), WY = kS3Waves / WX;
  const int nrg = (n - 1 + kS3Own - 1) / kS3Own;              // owned rows 1..n-1
  const int nyb = (nrg + WY - 1) / WY;                         // row-group blocks
  const int nlog = nyb * nzc;                                  // logical block = (row-group block, z chunk)
  const int per = (gridDim.x + 7) >> 3;
  const int Lb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (Lb >= nlog) return;                                      // whole block leaves together
  const int yb = Lb % nyb, zc = Lb / nyb;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wx = wave % WX, wy = wave / WX;
  const int rg = yb * WY + wy;
  const bool active = rg < nrg;                                // inactive waves still join the barriers
  const int X = wx * 64 + lane;
  const bool col_ok = X <= n;
  const bool own_x = X >= 1 && X <= n - 1;
  const int Xc = X > n ? n : X;
  const int Y0 = rg * kS3Own;                                  // row r <-> y = Y0 + r
  const int Z0 = 1 + zc * zc_planes, Zend = min(Z0 + zc_planes, n);   // owned planes [Z0, Zend)
  const int px = g.px, pz = g.pz;
  int rowoff[kS3Rows];
  bool row_ok[kS3Rows], own_r[kS3Rows];
#pragma unroll
  for (int r = 0; r < kS3Rows; ++r) {
    const int y = Y0 + r;
    row_ok[r] = active && y <= n;
    own_r[r] = active && r >= 1 && r <= kS3Own && y >= 1 && y <= n - 1;
    rowoff[r] = (y > n ? n : y) * px + Xc;
  }
  auto plane_off = [&](int z) { return (z < 0 ? 0 : (z > n ? n : z)) * pz; };
  // ring of kS3Depth slots: slot d holds x of plane z and b of plane z-1
  T qx[kS3Depth][kS3Rows], qb[kS3Depth][kS3Own];
  const int zstart = Z0 - 1;
#pragma unroll
  for (int d = 0; d < kS3Depth; ++d) {
    const int ox = plane_off(zstart + d), ob = plane_off(zstart + d - 1);
#pragma unroll
    for (int r = 0; r < kS3Rows; ++r) qx[d][r] = x[ox + rowoff[r]];
#pragma unroll
    for (int r = 0; r < kS3Own; ++r) qb[d][r] = b[ob + rowoff[r + 1]];
  }
  T pa[kS3Rows], pb[kS3Rows];   // planes z-2, z-1
#pragma unroll
  for (int r = 0; r < kS3Rows; ++r) { pa[r] = T(0); pb[r] = T(0); }
  const int steps = Zend - zstart + 1;                         // planes Z0-1 .. Zend
  for (int i0 = 0; i0 < steps; i0 += kS3Depth) {
#pragma unroll
    for (int d = 0; d < kS3Depth; ++d) {
      const int z = zstart + i0 + d;
      const bool z_ok = z >= 0 && z <= n;
      T v[kS3Rows], bc[kS3Own];
#pragma unroll
      for (int r = 0; r < kS3Rows; ++r) v[r] = (col_ok && row_ok[r] && z_ok) ? qx[d][r] : T(0);
#pragma unroll
      for (int r = 0; r < kS3Own; ++r) bc[r] = qb[d][r];
      {   // refill the slot with plane z + kS3Depth (clamped past the end; unused)
        const int ox = plane_off(z + kS3Depth), ob = plane_off(z + kS3Depth - 1);
#pragma unroll
        for (int r = 0; r < kS3Rows; ++r) qx[d][r] = x[ox + rowoff[r]];
#pragma unroll
        for (int r = 0; r < kS3Own; ++r) qb[d][r] = b[ob + rowoff[r + 1]];
      }
      // edge exchange of plane z-1 (the centre plane of this step's output)
      const int par = (i0 + d) & 1;
      if (lane == 0) {
#pragma unroll
        for (int r = 0; r < kS3Rows; ++r) edge[par][wave][0][r] = pb[r];
      }
      if (lane == 63) {
#pragma unroll
        for (int r = 0; r < kS3Rows; ++r) edge[par][wave][1][r] = pb[r];
      }
      __syncthreads();
      const int zo = z - 1;
      if (active && zo >= Z0 && zo < Zend && i0 + d < steps) {
        T* dst = out + zo * pz;
#pragma unroll
        for (int r = 1; r <= kS3Own; ++r) {
          const T c = pb[r];
          T lft = from_left(c), rgt = from_right(c);
          if (lane == 0) lft = wx > 0 ? edge[par][wave - 1][1][r] : T(0);
          if (lane == 63) rgt = wx < WX - 1 ? edge[par][wave + 1][0][r] : T(0);
          T s = (lft + rgt) + (pb[r - 1] + pb[r + 1]);
          s += pa[r] + v[r];
          const T val = c + wd * (bc[r - 1] - scale * (T(6) * c - s));
          if (own_x && own_r[r]) dst[rowoff[r]] = val;
        }
      }
#pragma unroll
      for (int r = 0; r < kS3Rows; ++r) {
        pa[r] = pb[r];
        pb[r] = v[r];
      }
    }
  }
}

// Launch shape (n <= 256): planes per z chunk for about 2048 wavefronts;
// returns the number of blocks (a multiple of 8, one share per XCD).
inline int smooth3s_blocks(int n, int& zc_planes, int& nzc) {
  const int WX = s3_wx(n), WY = kS3Waves / WX;
  const int nrg = (n - 1 + kS3Own - 1) / kS3Own;
  const int nyb = (nrg + WY - 1) / WY;
  nzc = (512 + nyb - 1) / nyb;                  // about 512 blocks of 4 wavefronts
  if (nzc > n - 1) nzc = n - 1;
  if (nzc < 1) nzc = 1;
  zc_planes = (n - 1 + nzc - 1) / nzc;
  nzc = (n - 1 + zc_planes - 1) / zc_planes;
  const int nlog = nyb * nzc;
  return (nlog + 7) & ~7;
}

}  // namespace fmg
