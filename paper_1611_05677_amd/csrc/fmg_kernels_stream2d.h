// Register-streaming 2D V-cycle level kernels (float64 or float32).
//
// Same operations as the LDS-tiled pair (two weighted-Jacobi sweeps +
// residual + restriction; coarse correction + two sweeps), laid out for wave64
// without LDS: each wavefront owns a strip of fine columns (one column per
// lane) and a run of rows, and marches up the rows.  A stencil's vertical
// neighbours are earlier rows kept in registers; its horizontal neighbours
// come from the adjacent lanes through DPP whole-wave shifts.  Every stage of
// the pipeline therefore loses one lane at each strip edge, and the strips
// overlap by that halo.  Global loads are issued a few rows ahead (a register
// queue) so each wave keeps several rows in flight.
//
// Arithmetic per node is the same expression, in the same order, as the
// separate sweep / residual / transfer kernels.  Points outside the interior
// hold the Dirichlet value 0.
#pragma once

#include "fmg_device.h"

namespace fmg {

constexpr int kStreamWaves = 4;    // independent wavefronts per block
constexpr int kStreamQueue = 4;    // rows loaded ahead of use
constexpr int kPreHalo = 4;        // sweep, sweep, residual, restriction
constexpr int kPostHalo = 2;       // sweep, sweep
constexpr int kPreStrip = 64 - 2 * kPreHalo;
constexpr int kPostStrip = 64 - 2 * kPostHalo;

// Value held by lane l-1 (0 in lane 0) / lane l+1 (0 in lane 63).
template <int CTRL>
__device__ __forceinline__ double wave_shift(double v) { return dpp_move<CTRL>(v); }
template <int CTRL>
__device__ __forceinline__ float wave_shift(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <typename T> __device__ __forceinline__ T from_left(T v) { return wave_shift<0x138>(v); }   // wave_shr:1
template <typename T> __device__ __forceinline__ T from_right(T v) { return wave_shift<0x130>(v); }  // wave_shl:1

// c + wd (b - scale (4 c - s)), s = (left + right) + (below + above)
template <typename T>
__device__ __forceinline__ T stream_sweep(T below, T c, T above, T b, T wd, T scale, bool inside) {
  const T s = (from_left(c) + from_right(c)) + (below + above);
  const T v = c + wd * (b - scale * (T(4) * c - s));
  return inside ? v : T(0);
}

// Block -> (strip group, row chunk).  Consecutive hardware block ids go to
// different XCDs in turn; the remap hands each XCD a contiguous range of
// logical blocks (vertically adjacent chunks), so the rows that neighbouring
// chunks both read are shared in that XCD's L2.
__device__ __forceinline__ bool stream_block(int nlogical, int gx, int& sx, int& cy) {
  const int per = (gridDim.x + 7) >> 3;
  const int L = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (L >= nlogical) return false;
  sx = L % gx;
  cy = L / gx;
  return true;
}

template <typename T>
__device__ __forceinline__ T stream_load(const T* __restrict__ p, const Grid& g, int X, bool col_ok, int y) {
  return (col_ok && y >= 0 && y <= g.n) ? p[y * g.px + X] : T(0);
}

// Two sweeps from x0 (or from zero), then r = b - A x and bc = P^T r on the
// coarse nodes 2p inside the owned rows / columns.  R rows per wave.
template <typename T, bool ZERO>
__device__ __forceinline__ void pre2s_wave(const Grid& f, const Grid& cg, const T* __restrict__ x0,
                                           const T* __restrict__ b, T* __restrict__ xout, T* __restrict__ bc,
                                           T wd1, T wd2, T scale, int strip, int Y0, int R) {
  const int lane = threadIdx.x & 63;
  const int n = f.n;
  const int X = strip * kPreStrip - kPreHalo + lane;
  const bool col_ok = X >= 0 && X <= n;
  const bool col_in = X >= 1 && X <= n - 1;
  const bool own = lane >= kPreHalo && lane < 64 - kPreHalo && col_in;
  const bool own_c = own && !(X & 1) && X >= 2 && X <= n - 2;
  const int Yend = min(Y0 + R, n);          // owned rows [Y0, Yend)
  const int ylo = Y0 - kPreHalo, yhi = Yend + kPreHalo - 1;
  // windows: x0 rows y-2, y-1; b rows y-1..y-3; sweep-1 rows y-3, y-2; sweep-2
  // rows y-4, y-3; residual rows y-5, y-4 (+ their lane shifts)
  T xa = 0, xb = 0, b1 = 0, b2 = 0, b3 = 0, s1a = 0, s1b = 0, s2a = 0, s2b = 0;
  T ra = 0, rb = 0, raL = 0, rbL = 0, rbR = 0;
  T qx[kStreamQueue], qb[kStreamQueue];
#pragma unroll
  for (int q = 0; q < kStreamQueue; ++q) {
    qx[q] = ZERO ? T(0) : stream_load(x0, f, X, col_ok, ylo + q);
    qb[q] = stream_load(b, f, X, col_ok, ylo + q);
  }
  for (int y0 = ylo; y0 <= yhi; y0 += kStreamQueue) {
#pragma unroll
    for (int q = 0; q < kStreamQueue; ++q) {
      const int y = y0 + q;
      const T xc = qx[q], b0 = qb[q];
      const int yn = y + kStreamQueue;
      if (yn <= yhi) {
        if (!ZERO) qx[q] = stream_load(x0, f, X, col_ok, yn);
        qb[q] = stream_load(b, f, X, col_ok, yn);
      }
      // sweep 1 at row y-1
      const bool in1 = col_in && y - 1 >= 1 && y - 1 <= n - 1;
      T s1c;
      if (ZERO) s1c = in1 ? wd1 * b1 : T(0);
      else s1c = stream_sweep(xa, xb, xc, b1, wd1, scale, in1);
      // sweep 2 at row y-2
      const bool in2 = col_in && y - 2 >= 1 && y - 2 <= n - 1;
      const T s2c = stream_sweep(s1a, s1b, s1c, b2, wd2, scale, in2);
      if (own && y - 2 >= Y0 && y - 2 < Yend && in2) xout[(y - 2) * f.px + X] = s2c;
      // residual at row y-3
      const bool in3 = col_in && y - 3 >= 1 && y - 3 <= n - 1;
      const T ssum = (from_left(s2b) + from_right(s2b)) + (s2a + s2c);
      const T rc = in3 ? b3 - scale * (T(4) * s2b - ssum) : T(0);
      const T rcL = from_left(rc), rcR = from_right(rc);
      // restriction at row y-4 (residual rows y-5, y-4, y-3)
      const int yr = y - 4;
      const T h = ((rbR + rbL) + (rc + ra)) + (rcR + raL);
      if (own_c && !(yr & 1) && yr >= Y0 && yr < Yend && yr >= 2 && yr <= n - 2)
        bc[(yr >> 1) * cg.px + (X >> 1)] = rb + T(0.5) * h;
      // advance the windows
      xa = xb; xb = xc;
      b3 = b2; b2 = b1; b1 = b0;
      s1a = s1b; s1b = s1c;
      s2a = s2b; s2b = s2c;
      ra = rb; raL = rbL;
      rb = rc; rbL = rcL; rbR = rcR;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(64 * kStreamWaves)
    k_pre2s(Grid f, Grid cg, const T* __restrict__ x0, const T* __restrict__ b, T* __restrict__ xout,
            T* __restrict__ bc, T wd1, T wd2, T scale, int zero_init, int R, int nchunk) {
  const int nstrip = (f.n + 1 + kPreStrip - 1) / kPreStrip;
  const int gx = (nstrip + kStreamWaves - 1) / kStreamWaves;
  int sx, cy;
  if (!stream_block(gx * nchunk, gx, sx, cy)) return;
  const int strip = sx * kStreamWaves + (threadIdx.x >> 6);
  if (strip >= nstrip) return;            // whole wavefront leaves together
  if (zero_init) pre2s_wave<T, true>(f, cg, x0, b, xout, bc, wd1, wd2, scale, strip, cy * R, R);
  else pre2s_wave<T, false>(f, cg, x0, b, xout, bc, wd1, wd2, scale, strip, cy * R, R);
}

// x + P xc on level f (coarse cg), then two sweeps; R rows per wave.
template <typename T>
__device__ __forceinline__ void post2s_wave(const Grid& cg, const Grid& f, const T* __restrict__ x,
                                            const T* __restrict__ xc, const T* __restrict__ b,
                                            T* __restrict__ xout, T wd1, T wd2, T scale, int strip, int Y0,
                                            int R) {
  const int lane = threadIdx.x & 63;
  const int n = f.n;
  const int X = strip * kPostStrip - kPostHalo + lane;
  const bool col_ok = X >= 0 && X <= n;
  const bool col_in = X >= 1 && X <= n - 1;
  const bool own = lane >= kPostHalo && lane < 64 - kPostHalo && col_in;
  const int ci = X >> 1, si = X & 1;
  const int Yend = min(Y0 + R, n);
  const int ylo = Y0 - kPostHalo, yhi = Yend + kPostHalo - 1;
  // queue entries: x, b and the two coarse values of row y
  T qx[kStreamQueue], qb[kStreamQueue], qc0[kStreamQueue], qc1[kStreamQueue];
  auto fetch = [&](int q, int y) {
    qx[q] = stream_load(x, f, X, col_ok, y);
    qb[q] = stream_load(b, f, X, col_ok, y);
    const bool in = col_in && y >= 1 && y <= n - 1;
    const int cj = y >> 1, sj = y & 1;
    qc0[q] = in ? xc[cj * cg.px + ci] : T(0);
    qc1[q] = (in && (si | sj)) ? xc[(cj + sj) * cg.px + ci + si] : T(0);
  };
#pragma unroll
  for (int q = 0; q < kStreamQueue; ++q) fetch(q, ylo + q);
  // windows: corrected x rows y-2, y-1; b rows y-1, y-2; sweep-1 rows y-3, y-2
  T xa = 0, xb = 0, b1 = 0, b2 = 0, s1a = 0, s1b = 0;
  for (int y0 = ylo; y0 <= yhi; y0 += kStreamQueue) {
#pragma unroll
    for (int q = 0; q < kStreamQueue; ++q) {
      const int y = y0 + q;
      const bool in0 = col_in && y >= 1 && y <= n - 1;
      T v = qc0[q];
      if (si | (y & 1)) v = T(0.5) * (v + qc1[q]);
      const T xcor = in0 ? qx[q] + v : qx[q];
      const T b0 = qb[q];
      if (y + kStreamQueue <= yhi) fetch(q, y + kStreamQueue);
      const bool in1 = col_in && y - 1 >= 1 && y - 1 <= n - 1;
      const T s1c = stream_sweep(xa, xb, xcor, b1, wd1, scale, in1);
      const bool in2 = col_in && y - 2 >= 1 && y - 2 <= n - 1;
      const T s2c = stream_sweep(s1a, s1b, s1c, b2, wd2, scale, in2);
      if (own && y - 2 >= Y0 && y - 2 < Yend && in2) xout[(y - 2) * f.px + X] = s2c;
      xa = xb; xb = xcor;
      b2 = b1; b1 = b0;
      s1a = s1b; s1b = s1c;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(64 * kStreamWaves)
    k_post2s(Grid cg, Grid f, const T* __restrict__ x, const T* __restrict__ xc, const T* __restrict__ b,
             T* __restrict__ xout, T wd1, T wd2, T scale, int R, int nchunk) {
  const int nstrip = (f.n + 1 + kPostStrip - 1) / kPostStrip;
  const int gx = (nstrip + kStreamWaves - 1) / kStreamWaves;
  int sx, cy;
  if (!stream_block(gx * nchunk, gx, sx, cy)) return;
  const int strip = sx * kStreamWaves + (threadIdx.x >> 6);
  if (strip >= nstrip) return;
  post2s_wave<T>(cg, f, x, xc, b, xout, wd1, wd2, scale, strip, cy * R, R);
}

// Rows per wavefront: an explicit choice, or (0) about 128 row chunks per
// level and at least 4 rows.  Shorter marches trade re-read halo rows for more
// wavefronts in flight; the level kernels are bound by the latency of the row
// pipeline more than by bandwidth up to n = 2048.
inline int stream_rows(int opt, int n) {
  if (opt < 0) return 0;
  if (opt > 0) return opt;
  const int R = n >> 7;
  return R < 4 ? 4 : R;
}

// Launch geometry: logical blocks = strip groups x row chunks, rounded up to
// a multiple of 8 hardware blocks (one share per XCD).
inline int stream_blocks(int n, int strip_width, int R, int& nchunk) {
  const int nstrip = (n + 1 + strip_width - 1) / strip_width;
  const int gx = (nstrip + kStreamWaves - 1) / kStreamWaves;
  nchunk = (n + R - 1) / R;
  const int nl = gx * nchunk;
  return (nl + 7) & ~7;
}

}  // namespace fmg
