// Fused pairs of 3D weighted-Jacobi sweeps (float64 or float32).
//
// The V(2,2) cycle's pre-smoothing is two sweeps, x1 = x0 + w1 D^{-1}(b - A x0)
// and x2 = x1 + w2 D^{-1}(b - A x1); its post-smoothing is the same pair after
// the coarse correction x0 = x + P x_c.  Run as separate launches, each sweep
// reads x and b and writes x' (24 bytes per node in float64) and the
// prolongation reads and writes x once more.  Here one launch performs the
// pair (and, for the post-smoothing, the correction as the planes are loaded):
// read x and b once, write x2 once.  In mixed precision the first and last
// launches of a float32 cycle at the top level also take over the float64
// glue: the pre-smoothing launch forms the residual r = b - A u of the
// float64 iterate u as the planes arrive (and stores r as float32, the
// cycle's right-hand side), and the post-smoothing launch adds the cycle's
// result e to u (u += e) instead of storing e.
//
// Layout of the work: a workgroup of 16 wavefronts covers a tile of 64
// columns (x, one per lane) by 16 rows (y, one per wavefront; the code takes
// kP3RowsPerWave rows per wavefront, and one measured fastest: two rows per
// wavefront halve the halo share but the extra registers leave one
// workgroup per CU) and marches through a run of planes (z).  The tile's
// outer two lanes and rows on each side are halo: they are loaded and swept
// once, so that the second sweep is exact on the inner 60 x 12 nodes, which
// the workgroup owns and writes.
//   * x-neighbours come from the adjacent lanes (DPP whole-wave shifts);
//   * y-neighbours through one LDS plane per stage (double-buffered by plane
//     parity, two barriers per plane);
//   * z-neighbours are the previous and next planes, kept in registers;
//   * loads run two planes ahead in a register ring, from clamped (always
//     in-bounds) addresses; values outside the grid are masked to 0.
// Arithmetic per node is the separate kernels' expression, in the same order:
//   x' = x + wd (b - s (6 x - ((x_w + x_e) + (x_s + x_n) + (x_d + x_u)))).
//
// The first pre-smoothing of a level in the float64 FMG starts from the
// natural inclusion x0 = P u_{k-1} of the previous level's result
// (kP3ProlongFresh): x0 is formed from the coarse values as the planes
// arrive, so the level transition only writes the right-hand side.
#pragma once

#include "fmg_device.h"
#include "fmg_kernels_stream2d.h"

namespace fmg {

constexpr int kP3Waves = 16;                // wavefronts per workgroup
constexpr int kP3RowsPerWave = 1;
constexpr int kP3Rows = kP3Waves * kP3RowsPerWave;   // tile rows
constexpr int kP3Halo = 2;                  // two stencil stages: two halo lanes / rows per side
constexpr int kP3OwnX = 64 - 2 * kP3Halo;   // owned columns per workgroup
constexpr int kP3OwnY = kP3Rows - 2 * kP3Halo;
constexpr int kP3Threads = 64 * kP3Waves;

// What a launch does besides the two sweeps.
enum Pair3Mode {
  kP3Plain = 0,      // x0 = x
  kP3Zero = 1,       // x0 = 0 (x is not read)
  kP3Prolong = 2,    // x0 = x + P xc
  kP3Resid = 3,      // float32 cycle at the top level: r = (float)(b64 - A u64) is the right-hand side
                     // (stored to r32), x0 = 0
  kP3ProlongAdd = 4, // float32 cycle at the top level: x0 = x + P xc, then u64 += (double) x2
  kP3ProlongFresh = 5  // x0 = P xc (x is not read): the level transition's start
};

// Launch geometry: strips of owned columns x row chunks x plane chunks.  Two
// workgroups are resident per CU (512 on the device), and a launch whose
// workgroups overrun a whole number of such waves leaves CUs idle at its end,
// so the plane chunks are as many as keep the workgroups within one wave on
// levels with n <= 128 and within `target` (two waves) above (128^3: 495
// workgroups instead of 528, pairs 19.7 -> 15.8 and 23.8 -> 19.6 us; 256^3:
// 990 instead of 1100, 105 -> 101 and 121 -> 114 us; solve 2.461 -> 2.409 ms),
// within the bounds below.  Logical block order: strip fastest, then row
// chunk, then plane chunk, so each XCD's contiguous range of logical blocks
// holds tiles that share halo rows and columns.
struct Pair3Shape {
  int nsx, ncy, nzc, zc_planes;
};

inline Pair3Shape pair3_shape(int n, int target = 1024) {
  Pair3Shape s;
  s.nsx = (n - 1 + kP3OwnX - 1) / kP3OwnX;
  s.ncy = (n - 1 + kP3OwnY - 1) / kP3OwnY;
  int nzc = (n <= 128 ? 512 : target) / (s.nsx * s.ncy);
  // owned planes per chunk at least: 8 on large levels (a chunk loads four
  // halo planes); on small levels, whose launches are bound by the march's
  // chain of plane steps rather than by bytes, shorter chunks (n <= 32: 1,
  // n = 64: 4; 3D 256^3 solve 2.631 -> 2.466 ms)
  const int zmin = n <= 32 ? 1 : n <= 64 ? 4 : 8;
  if (nzc > (n - 1 + zmin - 1) / zmin) nzc = (n - 1 + zmin - 1) / zmin;
  if (nzc < 1) nzc = 1;
  s.zc_planes = (n - 1 + nzc - 1) / nzc;
  s.nzc = (n - 1 + s.zc_planes - 1) / s.zc_planes;
  return s;
}

inline int pair3_blocks(const Pair3Shape& s) { return ((s.nsx * s.ncy * s.nzc) + 7) & ~7; }

struct Pair3Args {
  Grid g, cg;            // level, next coarser level (prolongation)
  const void* x;         // x0 source (T), or u (double) in kP3Resid
  const void* b;         // right-hand side (T), or b (double) in kP3Resid
  const void* xc;        // coarse correction (T)
  void* out;             // x2 (T); unused in kP3ProlongAdd
  float* r32;            // kP3Resid: the residual (right-hand side of the float32 cycle)
  double* u64;           // kP3ProlongAdd: the float64 iterate, updated in place
  double wd1, wd2, scale;
  int nsx, ncy, nzc, zc_planes;
};

// x0 plane type: double in kP3Resid (the float64 iterate), T otherwise.
template <typename T, int MODE> struct Pair3In { using type = T; };
template <typename T> struct Pair3In<T, kP3Resid> { using type = double; };

template <typename T, int MODE>
__global__ void __launch_bounds__(kP3Threads) k_sweep_pair3(Pair3Args A) {
  using TX = typename Pair3In<T, MODE>::type;
  constexpr int RW = kP3RowsPerWave;
  constexpr bool FRESH = MODE == kP3ProlongFresh;
  constexpr bool PROLONG = MODE == kP3Prolong || MODE == kP3ProlongAdd || FRESH;
  __shared__ TX lx[2][kP3Rows][64];   // x0 (or u) plane: the first stage's y-neighbours, by plane parity
  __shared__ T ls[2][kP3Rows][64];    // sweep-1 plane: sweep 2's y-neighbours
  const Grid g = A.g, cg = A.cg;
  const TX* __restrict__ x = static_cast<const TX*>(A.x);
  const TX* __restrict__ b = static_cast<const TX*>(A.b);
  const T* __restrict__ xc = static_cast<const T*>(A.xc);
  const T wd1 = (T)A.wd1, wd2 = (T)A.wd2, scale = (T)A.scale;
  const int n = g.n;
  const int nlog = A.nsx * A.ncy * A.nzc;
  const int per = (gridDim.x + 7) >> 3;
  const int Lb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (Lb >= nlog) return;                                    // whole workgroup leaves together
  const int sx = Lb % A.nsx, cy = (Lb / A.nsx) % A.ncy, zc = Lb / (A.nsx * A.ncy);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int X = 1 + sx * kP3OwnX - kP3Halo + lane;
  const bool col_ok = X >= 0 && X <= n, in_x = X >= 1 && X <= n - 1;
  const bool own_x = lane >= kP3Halo && lane < 64 - kP3Halo && in_x;
  const int Xc = X < 0 ? 0 : (X > n ? n : X);
  int row[RW], off[RW], rdn[RW], rup[RW];
  bool row_ok[RW], in_xy[RW], own[RW];
  int c0[RW], c1[RW], cs[RW];
#pragma unroll
  for (int k = 0; k < RW; ++k) {
    row[k] = wave * RW + k;
    const int Y = 1 + cy * kP3OwnY - kP3Halo + row[k];
    row_ok[k] = col_ok && Y >= 0 && Y <= n;
    in_xy[k] = in_x && Y >= 1 && Y <= n - 1;
    own[k] = own_x && row[k] >= kP3Halo && row[k] < kP3Rows - kP3Halo && Y >= 1 && Y <= n - 1;
    const int Yc = Y < 0 ? 0 : (Y > n ? n : Y);
    off[k] = Yc * g.px + Xc;
    rdn[k] = row[k] > 0 ? row[k] - 1 : 0;
    rup[k] = row[k] < kP3Rows - 1 ? row[k] + 1 : row[k];
    c0[k] = c1[k] = cs[k] = 0;
    if (PROLONG) {   // the two coarse nodes whose mean is the fine value
      const int si = Xc & 1, sj = Yc & 1;
      c0[k] = (Yc >> 1) * cg.px + (Xc >> 1);
      c1[k] = min((Yc >> 1) + sj, cg.n) * cg.px + min((Xc >> 1) + si, cg.n);
      cs[k] = si | sj;
    }
  }
  const int Z0 = 1 + zc * A.zc_planes, Zend = min(Z0 + A.zc_planes, n);   // owned planes [Z0, Zend)
  const int zs = Z0 - kP3Halo, steps = Zend - Z0 + 2 * kP3Halo;         // planes Z0-2 .. Zend+1
  auto plane = [&](int z) { return (z < 0 ? 0 : (z > n ? n : z)); };
  // ring of two plane slots per row: x0, b, one coarse value, and u (kP3ProlongAdd).
  // Coarse values: fine plane z = 2 p_z + e_z takes the mean of coarse node c0
  // on coarse plane p_z and c1 on plane p_z + e_z.  An even plane's c1 value is
  // the previous (odd) plane's, and an odd plane's c0 value the previous
  // (even) plane's, so each plane loads one coarse value (even: c0 on z/2;
  // odd: c1 on (z+1)/2) and takes the other from the plane before (pc0, pc1).
  TX qx[2][RW], qb[2][RW];
  T qc[2][RW];
  double qu[2][RW];
  auto cplane = [&](int zc) { return zc < 0 ? 0 : (zc > cg.n ? cg.n : zc); };
  auto fetch = [&](int d, int zl) {
    const int z = plane(zl);
#pragma unroll
    for (int k = 0; k < RW; ++k) {
      const size_t o = (size_t)z * g.pz + off[k];
      if (MODE != kP3Zero && !FRESH) qx[d][k] = x[o];
      qb[d][k] = b[o];
      if (PROLONG) {   // integer arithmetic, not a select between c0 and c1
        const int odd = zl & 1;
        qc[d][k] = xc[(size_t)cplane((zl + odd) >> 1) * cg.pz + c0[k] + odd * (c1[k] - c0[k])];
      }
      if (MODE == kP3ProlongAdd) qu[d][k] = A.u64[o];
    }
  };
  T pc0[RW], pc1[RW];                 // the previous plane's coarse pair
#pragma unroll
  for (int k = 0; k < RW; ++k) {
    pc0[k] = pc1[k] = T(0);
    if (PROLONG) {   // what the first plane takes from the plane before it
      const int odd = zs & 1;
      const T v = xc[(size_t)cplane((zs - odd) >> 1) * cg.pz + c1[k] + odd * (c0[k] - c1[k])];
      pc0[k] = odd ? v : T(0);
      pc1[k] = odd ? T(0) : v;
    }
  }
  fetch(0, zs);
  fetch(1, zs + 1);
  // windows per row: x0 planes z-2, z-1; b planes z-1, z-2; s1 planes z-3, z-2;
  // u planes z-1, z-2 (kP3ProlongAdd)
  TX xa[RW], xb[RW], b1[RW], b2[RW];
  T sa[RW], sb[RW];
  float rb[RW];                       // kP3Resid: the residual of plane z-2 (stage 1's previous plane)
  double u1[RW], u2[RW];
#pragma unroll
  for (int k = 0; k < RW; ++k) {
    xa[k] = xb[k] = b1[k] = b2[k] = TX(0);
    sa[k] = sb[k] = T(0);
    rb[k] = 0.0f;
    u1[k] = u2[k] = 0.0;
  }
  for (int i0 = 0; i0 < steps; i0 += 2) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int zl = zs + i0 + d;
      const bool z_ok = zl >= 0 && zl <= n;
      const bool z_in = zl >= 1 && zl <= n - 1;
      TX xn[RW], bn[RW];
      double un[RW];
#pragma unroll
      for (int k = 0; k < RW; ++k) {
        const bool ok = row_ok[k] && z_ok;
        xn[k] = (MODE != kP3Zero && !FRESH && ok) ? qx[d][k] : TX(0);
        bn[k] = ok ? qb[d][k] : TX(0);
        un[k] = (MODE == kP3ProlongAdd && ok) ? qu[d][k] : 0.0;
        if (PROLONG) {
          const T v0 = (zl & 1) ? pc0[k] : qc[d][k];
          const T v1 = (zl & 1) ? qc[d][k] : pc1[k];
          pc0[k] = v0;
          pc1[k] = v1;
          if (ok && in_xy[k] && z_in) {
            T v = v0;
            if (cs[k] | (zl & 1)) v = T(0.5) * (v + v1);
            xn[k] = FRESH ? v : xn[k] + v;
          }
        }
      }
      fetch(d, zl + 2);   // refill the slot (clamped past the end; unused)
      const int par = zl & 1;
      if (MODE != kP3Zero) {
#pragma unroll
        for (int k = 0; k < RW; ++k) lx[par][row[k]][lane] = xn[k];
      }
      __syncthreads();
      // stage 1 at plane p = zl - 1: the first sweep (or, kP3Resid, the
      // float64 residual, then the first sweep from zero, a multiple of it)
      const int p = zl - 1;
      const bool p_in = p >= 1 && p <= n - 1;
      T s1n[RW];
      float rn[RW];
#pragma unroll
      for (int k = 0; k < RW; ++k) {
        rn[k] = 0.0f;
        const bool in1 = in_xy[k] && p_in;
        if (MODE == kP3Zero) {
          s1n[k] = in1 ? wd1 * b1[k] : T(0);
        } else {
          const TX ysum = lx[par ^ 1][rdn[k]][lane] + lx[par ^ 1][rup[k]][lane];
          TX sm = (from_left(xb[k]) + from_right(xb[k])) + ysum;
          sm += xa[k] + xn[k];
          if (MODE == kP3Resid) {
            const float r = in1 ? (float)(b1[k] - A.scale * (6.0 * xb[k] - sm)) : 0.0f;
            if (own[k] && p >= Z0 && p < Zend) A.r32[(size_t)p * g.pz + off[k]] = r;
            rn[k] = r;
            s1n[k] = in1 ? wd1 * r : T(0);
          } else {
            s1n[k] = in1 ? T(xb[k] + wd1 * (b1[k] - scale * (T(6) * xb[k] - sm))) : T(0);
          }
        }
        ls[par ^ 1][row[k]][lane] = s1n[k];
      }
      __syncthreads();
      // stage 2 at plane q = zl - 2 (s1 planes q-1 = sa, q = sb, q+1 = s1n)
      const int q = zl - 2;
      if (q >= Z0 && q < Zend) {
#pragma unroll
        for (int k = 0; k < RW; ++k) {
          // kP3Resid: the right-hand side at q is the residual as rounded to float
          const T bq = MODE == kP3Resid ? T(rb[k]) : T(b2[k]);
          const T ysum = ls[par][rdn[k]][lane] + ls[par][rup[k]][lane];
          T sm = (from_left(sb[k]) + from_right(sb[k])) + ysum;
          sm += sa[k] + s1n[k];
          const T v = sb[k] + wd2 * (bq - scale * (T(6) * sb[k] - sm));
          if (own[k]) {
            if (MODE == kP3ProlongAdd) A.u64[(size_t)q * g.pz + off[k]] = u2[k] + (double)v;
            else static_cast<T*>(A.out)[(size_t)q * g.pz + off[k]] = v;
          }
        }
      }
#pragma unroll
      for (int k = 0; k < RW; ++k) {
        xa[k] = xb[k]; xb[k] = xn[k];
        b2[k] = b1[k]; b1[k] = bn[k];
        sa[k] = sb[k]; sb[k] = s1n[k];
        rb[k] = rn[k];
        u2[k] = u1[k]; u1[k] = un[k];
      }
    }
  }
}

}  // namespace fmg
