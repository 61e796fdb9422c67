// Register-streaming 3D weighted-Jacobi sweep (float64 or float32).
//
// Same operation and per-node expression as the grid sweep
//   out = x + wd (b - A x),  A x = s (6 x_c - sum of the 6 axis neighbours),
// laid out so that each input value is read from memory about once: a
// wavefront owns a strip of 64 columns (one per lane) by kS3Rows rows, and
// marches through a run of planes.  x-neighbours come from the adjacent lanes
// (DPP whole-wave shifts), y-neighbours from the lane's own registers (rows
// r-1, r+1), z-neighbours from the two previous planes kept in registers.  The
// outermost lanes and rows are halo (loaded, not written); the next plane's
// loads are issued one plane ahead.  Points outside the interior hold 0.
#pragma once

#include "fmg_device.h"
#include "fmg_kernels_stream2d.h"

namespace fmg {

constexpr int kS3Rows = 8;                 // rows per wavefront (registers)
constexpr int kS3Own = kS3Rows - 2;        // owned rows
constexpr int kS3Strip = 62;               // owned columns per wavefront
constexpr int kS3Waves = 4;                // wavefronts per block: 4 consecutive row groups

template <typename T>
__global__ void __launch_bounds__(64 * kS3Waves)
    k_smooth3s(Grid g, const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ out, T wd, T scale,
               int zc_planes, int nzc) {
  const int n = g.n;
  const int nstrip = (n - 1 + kS3Strip - 1) / kS3Strip;       // owned columns 1..n-1
  const int nrg = (n - 1 + kS3Own - 1) / kS3Own;              // owned rows 1..n-1
  const int nrgb = (nrg + kS3Waves - 1) / kS3Waves;
  // logical block = (strip, z chunk, group of kS3Waves row groups), strip fastest
  const int nlog = nstrip * nzc * nrgb;
  const int per = (gridDim.x + 7) >> 3;
  const int Lb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (Lb >= nlog) return;
  const int sx = Lb % nstrip, zc = (Lb / nstrip) % nzc, rb = Lb / (nstrip * nzc);
  const int rg = rb * kS3Waves + (threadIdx.x >> 6);
  if (rg >= nrg) return;                                      // whole wavefront leaves together
  const int lane = threadIdx.x & 63;
  const int X = sx * kS3Strip + lane;                         // lane 0 is column 62 sx (halo)
  const bool col_ok = X <= n;
  const bool own_x = lane >= 1 && lane <= kS3Strip && X >= 1 && X <= n - 1;
  const int Xc = X > n ? n : X;
  const int Y0 = rg * kS3Own;                                 // row r <-> y = Y0 + r; owned r = 1..kS3Own
  const int Z0 = 1 + zc * zc_planes, Zend = min(Z0 + zc_planes, n);   // owned planes [Z0, Zend)
  const int px = g.px, pz = g.pz;
  int rowoff[kS3Rows];
  bool row_ok[kS3Rows], own_r[kS3Rows];
#pragma unroll
  for (int r = 0; r < kS3Rows; ++r) {
    const int y = Y0 + r;
    row_ok[r] = y <= n;
    own_r[r] = r >= 1 && r <= kS3Own && y >= 1 && y <= n - 1;
    rowoff[r] = (y > n ? n : y) * px + Xc;
  }
  auto plane_off = [&](int z) { return (z < 0 ? 0 : (z > n ? n : z)) * pz; };
  // window: planes z-2 (pa), z-1 (pb); current raw loads (cx) of plane z and
  // b of the output plane z-1 (cb)
  T pa[kS3Rows], pb[kS3Rows], cx[kS3Rows], cb[kS3Rows];
#pragma unroll
  for (int r = 0; r < kS3Rows; ++r) { pa[r] = T(0); pb[r] = T(0); cb[r] = T(0); }
  {
    const int o = plane_off(Z0 - 1);
#pragma unroll
    for (int r = 0; r < kS3Rows; ++r) cx[r] = x[o + rowoff[r]];
  }
  for (int z = Z0 - 1; z <= Zend; ++z) {
    // next plane's x and this output plane's b, one plane ahead
    T nx[kS3Rows], nb[kS3Rows];
    {
      const int o1 = plane_off(z + 1), o0 = plane_off(z);
#pragma unroll
      for (int r = 0; r < kS3Rows; ++r) {
        nx[r] = x[o1 + rowoff[r]];
        nb[r] = b[o0 + rowoff[r]];
      }
    }
    const bool z_ok = z >= 0 && z <= n;
    T v[kS3Rows];
#pragma unroll
    for (int r = 0; r < kS3Rows; ++r) v[r] = (col_ok && row_ok[r] && z_ok) ? cx[r] : T(0);
    // output plane z-1 from planes z-2, z-1, z
    const int zo = z - 1;
    if (zo >= Z0 && zo < Zend) {
      T* dst = out + zo * pz;
#pragma unroll
      for (int r = 1; r <= kS3Own; ++r) {
        const T c = pb[r];
        T s = (from_left(c) + from_right(c)) + (pb[r - 1] + pb[r + 1]);
        s += pa[r] + v[r];
        const T val = c + wd * (cb[r] - scale * (T(6) * c - s));
        if (own_x && own_r[r]) dst[rowoff[r]] = val;
      }
    }
#pragma unroll
    for (int r = 0; r < kS3Rows; ++r) {
      pa[r] = pb[r];
      pb[r] = v[r];
      cx[r] = nx[r];
      cb[r] = nb[r];
    }
  }
}

// Launch shape: planes per z chunk for about 4096 wavefronts; returns blocks.
inline int smooth3s_blocks(int n, int& zc_planes, int& nzc) {
  const int nstrip = (n - 1 + kS3Strip - 1) / kS3Strip;
  const int nrg = (n - 1 + kS3Own - 1) / kS3Own;
  const int nrgb = (nrg + kS3Waves - 1) / kS3Waves;
  const int per_chunk = nstrip * nrg;
  nzc = (4096 + per_chunk - 1) / per_chunk;
  if (nzc > n - 1) nzc = n - 1;
  if (nzc < 1) nzc = 1;
  zc_planes = (n - 1 + nzc - 1) / nzc;
  nzc = (n - 1 + zc_planes - 1) / zc_planes;
  const int nlog = nstrip * nzc * nrgb;
  return (nlog + 7) & ~7;
}

}  // namespace fmg
