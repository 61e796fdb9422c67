// Residual and restriction of a 3D level in one plane-marching launch
// (float64 or float32): bc = P^T (b - A x) at the interior coarse nodes.
//
// The one-node-per-thread kernel (k_resid_restrict) evaluates, for every
// coarse node, the fine residual at the 15 fine nodes its hat covers: each
// fine residual is formed about twice and each x value is loaded about 30
// times over, which leaves that kernel bound by the issue of its loads.  Here
// a workgroup of 16 wavefronts covers a tile of 64 fine columns (x, one per
// lane) by 32 fine rows (y, two per wavefront) and marches through a run of
// fine planes (z): every fine residual of the tile is formed once, from x
// and b loaded once, into a ring of three residual planes in LDS, and after
// every odd plane 2l+1 the coarse values of plane l are gathered from the
// planes 2l-1, 2l and 2l+1 of that ring.
//   * x-neighbours of the residual come from the adjacent lanes (DPP
//     whole-wave shifts), y-neighbours from an LDS copy of the x plane
//     (double-buffered by plane parity), z-neighbours are the previous and
//     next planes, kept in registers;
//   * loads run two planes ahead in a register ring, from clamped (always
//     in-bounds) addresses; values outside the grid are masked to 0.
// The tile's outer two lanes and rows on each side are halo: the residual is
// exact on lanes 1..62 and rows 1..30, so the coarse nodes on the even lanes
// 2..60 and even rows 2..28 (30 x 14 per tile) are owned and written.
// Arithmetic per node is the separate kernel's expression, in the same order
// (the fine residual b - s (6 x - ((x_w + x_e) + (x_s + x_n) + (x_d + x_u)))
// and the restriction's sum of the 15 residuals), so both give the same bits.
#pragma once

#include "fmg_device.h"
#include "fmg_kernels_stream2d.h"

namespace fmg {

constexpr int kR3Waves = 16;
constexpr int kR3RowsPerWave = 2;
constexpr int kR3Rows = kR3Waves * kR3RowsPerWave;   // fine rows per tile
constexpr int kR3OwnX = 30;                          // coarse columns per tile (even lanes 2..60)
constexpr int kR3OwnY = (kR3Rows - 4) / 2;           // coarse rows per tile (even rows 2..kR3Rows-4)
constexpr int kR3Threads = 64 * kR3Waves;

// Launch geometry over the interior coarse nodes: strips of coarse columns x
// coarse row chunks x coarse plane chunks, with as many plane chunks as keep
// the workgroups within `slots` (two resident workgroups per CU: 80 KB of LDS
// in float64), so that all tiles run in one wave of workgroups (at 256^3: 500
// workgroups of 13 coarse planes, 69 us; 950 of 7 planes, 75 us).  Logical
// block order: strip fastest, then row chunk, then plane chunk.
struct Restrict3Shape {
  int nsx, ncy, nzc, zc_planes;
};

inline Restrict3Shape restrict3_shape(int nc, int slots = 512) {
  Restrict3Shape s;
  const int m = nc - 1;   // interior coarse nodes per axis
  s.nsx = (m + kR3OwnX - 1) / kR3OwnX;
  s.ncy = (m + kR3OwnY - 1) / kR3OwnY;
  int nzc = slots / (s.nsx * s.ncy);
  const int zmin = 4;     // at least 4 coarse planes per chunk
  if (nzc > (m + zmin - 1) / zmin) nzc = (m + zmin - 1) / zmin;
  if (nzc < 1) nzc = 1;
  s.zc_planes = (m + nzc - 1) / nzc;
  s.nzc = (m + s.zc_planes - 1) / s.zc_planes;
  return s;
}

inline int restrict3_blocks(const Restrict3Shape& s) { return ((s.nsx * s.ncy * s.nzc) + 7) & ~7; }

// f: the fine level (f.n even), cg: the coarse level (cg.n = f.n / 2).
template <typename T>
__global__ void __launch_bounds__(kR3Threads) k_resid_restrict3m(Grid f, Grid cg, const T* __restrict__ x,
                                                                 const T* __restrict__ b, T* __restrict__ bc,
                                                                 T scale, Restrict3Shape sh) {
  constexpr int RW = kR3RowsPerWave;
  __shared__ T lx[2][kR3Rows][64];   // x plane: the residual's y-neighbours, by plane parity
  __shared__ T lr[3][kR3Rows][64];   // residual planes, a ring of three
  const int n = f.n;
  const int nlog = sh.nsx * sh.ncy * sh.nzc;
  const int per = (gridDim.x + 7) >> 3;
  const int Lb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (Lb >= nlog) return;                                    // whole workgroup leaves together
  const int sx = Lb % sh.nsx, cy = (Lb / sh.nsx) % sh.ncy, zc = Lb / (sh.nsx * sh.ncy);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // lane 2 is the fine column of the strip's first coarse column 1 + kR3OwnX sx
  const int X = 2 * kR3OwnX * sx + lane;
  const bool col_ok = X <= n, in_x = X >= 1 && X <= n - 1;
  const int ci = kR3OwnX * sx + (lane >> 1);
  const bool out_x = !(lane & 1) && lane >= 2 && lane <= 60 && ci <= cg.n - 1;
  const int Xc = X > n ? n : X;
  int row[RW], off[RW], rdn[RW], rup[RW], obase[RW];
  bool row_ok[RW], in_xy[RW], out[RW];
#pragma unroll
  for (int k = 0; k < RW; ++k) {
    row[k] = wave * RW + k;
    const int Y = 2 * kR3OwnY * cy + row[k];
    row_ok[k] = col_ok && Y <= n;
    in_xy[k] = in_x && Y >= 1 && Y <= n - 1;
    const int cj = kR3OwnY * cy + (row[k] >> 1);
    out[k] = out_x && !(row[k] & 1) && row[k] >= 2 && row[k] <= kR3Rows - 4 && cj <= cg.n - 1;
    off[k] = (Y > n ? n : Y) * f.px + Xc;
    obase[k] = cj * cg.px + ci;
    rdn[k] = row[k] > 0 ? row[k] - 1 : 0;
    rup[k] = row[k] < kR3Rows - 1 ? row[k] + 1 : row[k];
  }
  // owned coarse planes [C0, Cend): fine residual planes 2 C0 - 1 .. 2 Cend - 1,
  // x planes 2 C0 - 2 .. 2 Cend
  const int C0 = 1 + zc * sh.zc_planes, Cend = min(C0 + sh.zc_planes, cg.n);
  const int zs = 2 * C0 - 2, steps = 2 * (Cend - C0) + 3;
  auto plane = [&](int z) { return z > n ? n : z; };
  T qx[2][RW], qb[2][RW];
  auto fetch = [&](int d, int zl) {
    const size_t zo = (size_t)plane(zl) * f.pz;
#pragma unroll
    for (int k = 0; k < RW; ++k) {
      qx[d][k] = x[zo + off[k]];
      qb[d][k] = b[zo + off[k]];
    }
  };
  fetch(0, zs);
  fetch(1, zs + 1);
  // windows per row: x planes z-2 (xa), z-1 (xb); b plane z-1 (b1)
  T xa[RW], xb[RW], b1[RW];
#pragma unroll
  for (int k = 0; k < RW; ++k) xa[k] = xb[k] = b1[k] = T(0);
  int slot = 0;                        // ring slot of the residual plane formed this step
  for (int i0 = 0; i0 < steps; i0 += 2) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int zl = zs + i0 + d;
      if (i0 + d >= steps) break;      // uniform over the workgroup
      const bool z_ok = zl <= n;
      T xn[RW], bn[RW];
#pragma unroll
      for (int k = 0; k < RW; ++k) {
        const bool ok = row_ok[k] && z_ok;
        xn[k] = ok ? qx[d][k] : T(0);
        bn[k] = ok ? qb[d][k] : T(0);
      }
      fetch(d, zl + 2);                // refill the slot (clamped past the end; unused)
      const int par = zl & 1;
#pragma unroll
      for (int k = 0; k < RW; ++k) lx[par][row[k]][lane] = xn[k];
      __syncthreads();
      // the residual at plane p = zl - 1
      const int p = zl - 1;
      const bool p_in = p >= 1 && p <= n - 1;
#pragma unroll
      for (int k = 0; k < RW; ++k) {
        const T ysum = lx[par ^ 1][rdn[k]][lane] + lx[par ^ 1][rup[k]][lane];
        T sm = (from_left(xb[k]) + from_right(xb[k])) + ysum;
        sm += xa[k] + xn[k];
        const T r = b1[k] - scale * (T(6) * xb[k] - sm);
        lr[slot][row[k]][lane] = (in_xy[k] && p_in) ? r : T(0);
      }
      __syncthreads();
      // after an odd plane p = 2 l + 1: the coarse plane l from p - 2, p - 1, p
      const int l = p >> 1;
      if ((p & 1) && l >= C0 && l < Cend) {
        const int sc = slot == 0 ? 2 : slot - 1;    // plane p - 1 = 2 l
        const int sdn = slot == 2 ? 0 : slot + 1;   // plane p - 2 = 2 l - 1
#pragma unroll
        for (int k = 0; k < RW; ++k) {
          if (out[k]) {
            const int rc = row[k];
            const T* c = &lr[sc][rc][lane];
            const T* u = &lr[slot][rc][lane];
            const T* w = &lr[sdn][rc][lane];
            constexpr int R = 64;
            T h = (c[1] + c[-1]) + (c[R] + c[-R]) + (c[R + 1] + c[-R - 1]);
            h += (u[0] + w[0]) + (u[1] + w[-1]) + (u[R] + w[-R]) + (u[R + 1] + w[-R - 1]);
            bc[(size_t)l * cg.pz + obase[k]] = c[0] + T(0.5) * h;
          }
        }
      }
#pragma unroll
      for (int k = 0; k < RW; ++k) {
        xa[k] = xb[k]; xb[k] = xn[k];
        b1[k] = bn[k];
      }
      slot = slot == 2 ? 0 : slot + 1;
    }
  }
}

}  // namespace fmg
