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
constexpr int kPreQueue = 4;       // rows per load group (pre-smoothing kernel)
constexpr int kPostQueue = 4;      // rows per load group (post-smoothing kernel)
constexpr int kPreHalo = 4;        // sweep, sweep, residual, restriction
constexpr int kPostHalo = 2;       // sweep, sweep
constexpr int kPreStrip = 64 - 2 * kPreHalo;
constexpr int kPostStrip = 64 - 2 * kPostHalo;

// Value held by lane l-1 (0 in lane 0) / lane l+1 (0 in lane 63): DPP moves
// with bound control, so lanes without a source read 0.
template <int CTRL>
__device__ __forceinline__ double wave_shift(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float wave_shift(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
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

// Loads are issued unconditionally from clamped (always in-bounds) addresses,
// so that the register queue is filled without branches and the wait for a
// row's data is left until the row is used; the value is masked at use.
__device__ __forceinline__ int clamp_row(int y, int n) { return y < 0 ? 0 : (y > n ? n : y); }

template <typename T>
__device__ __forceinline__ T stream_raw(const T* __restrict__ p, const Grid& g, int Xc, int y) {
  return p[clamp_row(y, g.n) * g.px + Xc];
}
template <typename T>
__device__ __forceinline__ T stream_mask(T raw, bool col_ok, int y, int n) {
  return (col_ok && y >= 0 && y <= n) ? raw : T(0);
}

// Two sweeps from x0 (or from zero), then r = b - A x and bc = P^T r on the
// coarse nodes 2p inside the owned rows / columns.  R rows per wave, marched
// upwards (UP) or downwards.  Vertically adjacent chunks march in opposite
// directions, so the halo rows two chunks share are read by both at about the
// same time (both at the start, or both at the end of their marches) and the
// second read is served from L2.  The stencil sums are symmetric in the two
// vertical neighbours, so the direction does not change any result.
template <typename T, bool ZERO, bool UP>
__device__ __forceinline__ void pre2s_wave(const Grid& f, const Grid& cg, const T* __restrict__ x0,
                                           const T* __restrict__ b, T* __restrict__ xout, T* __restrict__ bc,
                                           T wd1, T wd2, T scale, int strip, int Y0, int R) {
  constexpr int D = UP ? 1 : -1;
  const int lane = threadIdx.x & 63;
  const int n = f.n;
  const int X = strip * kPreStrip - kPreHalo + lane;
  const bool col_ok = X >= 0 && X <= n;
  const bool col_in = X >= 1 && X <= n - 1;
  const bool own = lane >= kPreHalo && lane < 64 - kPreHalo && col_in;
  const bool own_c = own && !(X & 1) && X >= 2 && X <= n - 2;
  const int Xc = X < 0 ? 0 : (X > n ? n : X);
  const int Yend = min(Y0 + R, n);          // owned rows [Y0, Yend)
  const int ylo = Y0 - kPreHalo, yhi = Yend + kPreHalo - 1;
  const int ystart = UP ? ylo : yhi;
  const int steps = yhi - ylo + 1;
  // windows (y = row just loaded, D = march direction): x0 rows y-2D, y-D;
  // b rows y-D..y-3D; sweep-1 rows y-3D, y-2D; sweep-2 rows y-4D, y-3D;
  // residual rows y-5D, y-4D (+ their lane shifts)
  T xa = 0, xb = 0, b1 = 0, b2 = 0, b3 = 0, s1a = 0, s1b = 0, s2a = 0, s2b = 0;
  T ra = 0, rb = 0, raL = 0, raR = 0, rbL = 0, rbR = 0;
  // rows are processed in groups of kPreQueue; the loads of the next group
  // are issued when a group starts, so they have a whole group of work to land
  T qx[kPreQueue], qb[kPreQueue];
#pragma unroll
  for (int q = 0; q < kPreQueue; ++q) {
    qx[q] = ZERO ? T(0) : stream_raw(x0, f, Xc, ystart + D * q);
    qb[q] = stream_raw(b, f, Xc, ystart + D * q);
  }
  for (int i0 = 0; i0 < steps; i0 += kPreQueue) {
    T nx[kPreQueue], nb[kPreQueue];
#pragma unroll
    for (int q = 0; q < kPreQueue; ++q) {     // past the end: clamped, unused rows
      const int yn = ystart + D * (i0 + kPreQueue + q);
      nx[q] = ZERO ? T(0) : stream_raw(x0, f, Xc, yn);
      nb[q] = stream_raw(b, f, Xc, yn);
    }
#pragma unroll
    for (int q = 0; q < kPreQueue; ++q) {
      const int i = i0 + q;
      const int y = ystart + D * i;
      const T xc = ZERO ? T(0) : stream_mask(qx[q], col_ok, y, n);
      const T b0 = stream_mask(qb[q], col_ok, y, n);
      // sweep 1 at row y-D
      const int y1 = y - D, y2 = y - 2 * D, y3 = y - 3 * D, yr = y - 4 * D;
      const bool in1 = col_in && y1 >= 1 && y1 <= n - 1;
      T s1c;
      if (ZERO) s1c = in1 ? wd1 * b1 : T(0);
      else s1c = stream_sweep(xa, xb, xc, b1, wd1, scale, in1);
      // sweep 2 at row y-2D
      const bool in2 = col_in && y2 >= 1 && y2 <= n - 1;
      const T s2c = stream_sweep(s1a, s1b, s1c, b2, wd2, scale, in2);
      if (own && y2 >= Y0 && y2 < Yend && in2) xout[y2 * f.px + X] = s2c;
      // residual at row y-3D
      const bool in3 = col_in && y3 >= 1 && y3 <= n - 1;
      const T ssum = (from_left(s2b) + from_right(s2b)) + (s2a + s2c);
      const T rc = in3 ? b3 - scale * (T(4) * s2b - ssum) : T(0);
      const T rcL = from_left(rc), rcR = from_right(rc);
      // restriction at row yr (residual rows yr-D, yr, yr+D); the diagonal
      // pair is r(x+1, yr+1) + r(x-1, yr-1)
      const T diag = UP ? (rcR + raL) : (raR + rcL);
      const T h = ((rbR + rbL) + (rc + ra)) + diag;
      if (own_c && !(yr & 1) && yr >= Y0 && yr < Yend && yr >= 2 && yr <= n - 2)
        bc[(yr >> 1) * cg.px + (X >> 1)] = rb + T(0.5) * h;
      // advance the windows
      xa = xb; xb = xc;
      b3 = b2; b2 = b1; b1 = b0;
      s1a = s1b; s1b = s1c;
      s2a = s2b; s2b = s2c;
      ra = rb; raL = rbL; raR = rbR;
      rb = rc; rbL = rcL; rbR = rcR;
    }
#pragma unroll
    for (int q = 0; q < kPreQueue; ++q) { qx[q] = nx[q]; qb[q] = nb[q]; }
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
  const bool up = !(cy & 1);
  if (zero_init) {
    if (up) pre2s_wave<T, true, true>(f, cg, x0, b, xout, bc, wd1, wd2, scale, strip, cy * R, R);
    else pre2s_wave<T, true, false>(f, cg, x0, b, xout, bc, wd1, wd2, scale, strip, cy * R, R);
  } else {
    if (up) pre2s_wave<T, false, true>(f, cg, x0, b, xout, bc, wd1, wd2, scale, strip, cy * R, R);
    else pre2s_wave<T, false, false>(f, cg, x0, b, xout, bc, wd1, wd2, scale, strip, cy * R, R);
  }
}

// x + P xc on level f (coarse cg), then two sweeps; R rows per wave, marched
// upwards or downwards (alternating by chunk, as in the pre-smoothing kernel).
// ADDU (mixed mode, top level of a float32 cycle): the result is the
// correction e, and instead of storing it the kernel adds it to the float64
// iterate in place, u += (double) e (the separate add kernel's operation).
template <typename T, bool UP, bool ADDU>
__device__ __forceinline__ void post2s_wave(const Grid& cg, const Grid& f, const T* __restrict__ x,
                                            const T* __restrict__ xc, const T* __restrict__ b,
                                            T* __restrict__ xout, double* __restrict__ u64, T wd1, T wd2,
                                            T scale, int strip, int Y0, int R) {
  constexpr int D = UP ? 1 : -1;
  const int lane = threadIdx.x & 63;
  const int n = f.n;
  const int X = strip * kPostStrip - kPostHalo + lane;
  const bool col_ok = X >= 0 && X <= n;
  const bool col_in = X >= 1 && X <= n - 1;
  const bool own = lane >= kPostHalo && lane < 64 - kPostHalo && col_in;
  const int Xc = X < 0 ? 0 : (X > n ? n : X);
  const int ci = Xc >> 1, si = Xc & 1;
  const int Yend = min(Y0 + R, n);
  const int ylo = Y0 - kPostHalo, yhi = Yend + kPostHalo - 1;
  const int ystart = UP ? ylo : yhi;
  const int steps = yhi - ylo + 1;
  // queue entries: x, b, one coarse value and (ADDU) u of row y; groups of
  // rows as in the pre-smoothing kernel (next group's loads issued at group
  // start).  Row y = 2 c_j + s_j takes the mean of coarse nodes c0 = (ci, y >> 1)
  // and c1 = (ci + si, (y + s_j) >> 1); consecutive rows share one of them
  // (marching up: an even row's c1 is the odd row's before it, an odd row's
  // c0 the even row's; marching down the other way round), so each row loads
  // one coarse value (w1: its c1) and takes the other from the row before.
  struct Q4 { T x[kPostQueue], b[kPostQueue], c[kPostQueue]; double u[kPostQueue]; };
  const int ci1 = min(ci + si, cg.n);   // (coarse rows and columns clamped into the coarse grid)
  auto crow = [&](int r) { return r < 0 ? 0 : (r > cg.n ? cg.n : r); };
  auto loads_c1 = [&](int y) { return UP ? (y & 1) : 1 - (y & 1); };
  auto fetch = [&](Q4& qq, int q, int y) {
    const int yc = clamp_row(y, n);
    qq.x[q] = x[yc * f.px + Xc];
    qq.b[q] = b[yc * f.px + Xc];
    const int odd = y & 1, w1 = loads_c1(y);   // integer arithmetic, not a select between c0 and c1
    qq.c[q] = xc[crow((y + w1 * odd) >> 1) * cg.px + ci + w1 * (ci1 - ci)];
    if (ADDU) qq.u[q] = u64[yc * f.px + Xc];
  };
  Q4 cur;
#pragma unroll
  for (int q = 0; q < kPostQueue; ++q) fetch(cur, q, ystart + D * q);
  T pc0 = T(0), pc1 = T(0);             // the previous row's coarse pair
  {   // what the first row takes from the row before it
    const int odd = ystart & 1, w1 = loads_c1(ystart);
    const T v = xc[crow((ystart + (1 - w1) * odd) >> 1) * cg.px + ci + (1 - w1) * (ci1 - ci)];
    pc0 = w1 ? v : T(0);
    pc1 = w1 ? T(0) : v;
  }
  // windows: corrected x rows y-2D, y-D; b rows y-D, y-2D; sweep-1 rows y-3D, y-2D
  T xa = 0, xb = 0, b1 = 0, b2 = 0, s1a = 0, s1b = 0;
  double ua = 0.0, ub = 0.0;      // ADDU: u rows y-2D, y-D
  for (int i0 = 0; i0 < steps; i0 += kPostQueue) {
    Q4 nxt;
#pragma unroll
    for (int q = 0; q < kPostQueue; ++q) fetch(nxt, q, ystart + D * (i0 + kPostQueue + q));
#pragma unroll
    for (int q = 0; q < kPostQueue; ++q) {
      const int i = i0 + q;
      const int y = ystart + D * i;
      const bool in0 = col_in && y >= 1 && y <= n - 1;
      const int w1 = loads_c1(y);
      const T v0 = w1 ? pc0 : cur.c[q];
      const T v1 = w1 ? cur.c[q] : pc1;
      pc0 = v0;
      pc1 = v1;
      T v = v0;
      if (si | (y & 1)) v = T(0.5) * (v + v1);
      const T xr = stream_mask(cur.x[q], col_ok, y, n);
      const T xcor = in0 ? xr + v : xr;
      const T b0 = stream_mask(cur.b[q], col_ok, y, n);
      const int y1 = y - D, y2 = y - 2 * D;
      const bool in1 = col_in && y1 >= 1 && y1 <= n - 1;
      const T s1c = stream_sweep(xa, xb, xcor, b1, wd1, scale, in1);
      const bool in2 = col_in && y2 >= 1 && y2 <= n - 1;
      const T s2c = stream_sweep(s1a, s1b, s1c, b2, wd2, scale, in2);
      if (own && y2 >= Y0 && y2 < Yend && in2) {
        if (ADDU) u64[y2 * f.px + X] = ua + (double)s2c;
        else xout[y2 * f.px + X] = s2c;
      }
      if (ADDU) { ua = ub; ub = cur.u[q]; }
      xa = xb; xb = xcor;
      b2 = b1; b1 = b0;
      s1a = s1b; s1b = s1c;
    }
    cur = nxt;
  }
}

template <typename T, bool ADDU>
__global__ void __launch_bounds__(64 * kStreamWaves)
    k_post2s(Grid cg, Grid f, const T* __restrict__ x, const T* __restrict__ xc, const T* __restrict__ b,
             T* __restrict__ xout, double* __restrict__ u64, T wd1, T wd2, T scale, int R, int nchunk) {
  const int nstrip = (f.n + 1 + kPostStrip - 1) / kPostStrip;
  const int gx = (nstrip + kStreamWaves - 1) / kStreamWaves;
  int sx, cy;
  if (!stream_block(gx * nchunk, gx, sx, cy)) return;
  const int strip = sx * kStreamWaves + (threadIdx.x >> 6);
  if (strip >= nstrip) return;
  if (!(cy & 1)) post2s_wave<T, true, ADDU>(cg, f, x, xc, b, xout, u64, wd1, wd2, scale, strip, cy * R, R);
  else post2s_wave<T, false, ADDU>(cg, f, x, xc, b, xout, u64, wd1, wd2, scale, strip, cy * R, R);
}

// Mixed mode, top level of a float32 cycle: the cycle's right-hand side is
// r = (float)(b - A u) of the float64 iterate u (the separate residual
// kernel's operation, same expression), formed here row by row one row ahead
// of the float32 pipeline and also stored (the post-smoothing kernel reads
// it); then, from zero, the two sweeps, residual and restriction of
// pre2s_wave.  One more halo lane and row for the residual's stencil.
constexpr int kResHalo = kPreHalo + 1;
constexpr int kResStrip = 64 - 2 * kResHalo;

template <bool UP>
__device__ __forceinline__ void pre2s_resid_wave(const Grid& f, const Grid& cg, const double* __restrict__ u,
                                                 const double* __restrict__ b64, float* __restrict__ r32,
                                                 float* __restrict__ xout, float* __restrict__ bc, float wd1,
                                                 float wd2, float scale, double scale64, int strip, int Y0,
                                                 int R) {
  using T = float;
  constexpr int D = UP ? 1 : -1;
  const int lane = threadIdx.x & 63;
  const int n = f.n;
  const int X = strip * kResStrip - kResHalo + lane;
  const bool col_ok = X >= 0 && X <= n;
  const bool col_in = X >= 1 && X <= n - 1;
  const bool own = lane >= kResHalo && lane < 64 - kResHalo && col_in;
  const bool own_c = own && !(X & 1) && X >= 2 && X <= n - 2;
  const int Xc = X < 0 ? 0 : (X > n ? n : X);
  const int Yend = min(Y0 + R, n);
  const int ylo = Y0 - kResHalo, yhi = Yend + kResHalo - 1;
  const int ystart = UP ? ylo : yhi;
  const int steps = yhi - ylo + 1;
  // float64 windows: u rows y-2D, y-D; b64 row y-D.  float32 windows as in
  // pre2s_wave (from zero), one row behind: the float pipeline's newest row
  // is yp = y - D, whose right-hand side rf is formed in this step.
  double ua = 0.0, ub = 0.0, bq = 0.0;
  T b1 = 0, b2 = 0, b3 = 0, s1a = 0, s1b = 0, s2a = 0, s2b = 0;
  T ra = 0, rb = 0, raL = 0, raR = 0, rbL = 0, rbR = 0;
  double qu[kPreQueue], qb[kPreQueue];
#pragma unroll
  for (int q = 0; q < kPreQueue; ++q) {
    qu[q] = stream_raw(u, f, Xc, ystart + D * q);
    qb[q] = stream_raw(b64, f, Xc, ystart + D * q);
  }
  for (int i0 = 0; i0 < steps; i0 += kPreQueue) {
    double nu[kPreQueue], nb[kPreQueue];
#pragma unroll
    for (int q = 0; q < kPreQueue; ++q) {     // past the end: clamped, unused rows
      const int yn = ystart + D * (i0 + kPreQueue + q);
      nu[q] = stream_raw(u, f, Xc, yn);
      nb[q] = stream_raw(b64, f, Xc, yn);
    }
#pragma unroll
    for (int q = 0; q < kPreQueue; ++q) {
      const int i = i0 + q;
      const int y = ystart + D * i;
      const double uc = stream_mask(qu[q], col_ok, y, n);
      const double bc64 = stream_mask(qb[q], col_ok, y, n);
      // residual of the float64 iterate at row yp (stencil rows yp - 1, yp + 1)
      const int yp = y - D;
      const bool inp = col_in && yp >= 1 && yp <= n - 1;
      const double sres = (from_left(ub) + from_right(ub)) + (ua + uc);
      const T b0 = inp ? (T)(bq - scale64 * (4.0 * ub - sres)) : T(0);
      if (own && yp >= Y0 && yp < Yend && inp) r32[yp * f.px + X] = b0;
      // float32 pipeline, from zero: sweep 1 at yp-D, sweep 2 at yp-2D,
      // residual at yp-3D, restriction at yp-4D
      const int y1 = yp - D, y2 = yp - 2 * D, y3 = yp - 3 * D, yr = yp - 4 * D;
      const bool in1 = col_in && y1 >= 1 && y1 <= n - 1;
      const T s1c = in1 ? wd1 * b1 : T(0);
      const bool in2 = col_in && y2 >= 1 && y2 <= n - 1;
      const T s2c = stream_sweep(s1a, s1b, s1c, b2, wd2, scale, in2);
      if (own && y2 >= Y0 && y2 < Yend && in2) xout[y2 * f.px + X] = s2c;
      const bool in3 = col_in && y3 >= 1 && y3 <= n - 1;
      const T ssum = (from_left(s2b) + from_right(s2b)) + (s2a + s2c);
      const T rc = in3 ? b3 - scale * (T(4) * s2b - ssum) : T(0);
      const T rcL = from_left(rc), rcR = from_right(rc);
      const T diag = UP ? (rcR + raL) : (raR + rcL);
      const T h = ((rbR + rbL) + (rc + ra)) + diag;
      if (own_c && !(yr & 1) && yr >= Y0 && yr < Yend && yr >= 2 && yr <= n - 2)
        bc[(yr >> 1) * cg.px + (X >> 1)] = rb + T(0.5) * h;
      // advance the windows
      ua = ub; ub = uc; bq = bc64;
      b3 = b2; b2 = b1; b1 = b0;
      s1a = s1b; s1b = s1c;
      s2a = s2b; s2b = s2c;
      ra = rb; raL = rbL; raR = rbR;
      rb = rc; rbL = rcL; rbR = rcR;
    }
#pragma unroll
    for (int q = 0; q < kPreQueue; ++q) { qu[q] = nu[q]; qb[q] = nb[q]; }
  }
}

__global__ void __launch_bounds__(64 * kStreamWaves)
    k_pre2s_resid(Grid f, Grid cg, const double* __restrict__ u, const double* __restrict__ b64,
                  float* __restrict__ r32, float* __restrict__ xout, float* __restrict__ bc, float wd1, float wd2,
                  float scale, double scale64, int R, int nchunk) {
  const int nstrip = (f.n + 1 + kResStrip - 1) / kResStrip;
  const int gx = (nstrip + kStreamWaves - 1) / kStreamWaves;
  int sx, cy;
  if (!stream_block(gx * nchunk, gx, sx, cy)) return;
  const int strip = sx * kStreamWaves + (threadIdx.x >> 6);
  if (strip >= nstrip) return;            // whole wavefront leaves together
  if (!(cy & 1)) pre2s_resid_wave<true>(f, cg, u, b64, r32, xout, bc, wd1, wd2, scale, scale64, strip, cy * R, R);
  else pre2s_resid_wave<false>(f, cg, u, b64, r32, xout, bc, wd1, wd2, scale, scale64, strip, cy * R, R);
}

// Rows per wavefront: an explicit choice, or (0) about 128 row chunks per
// level and at least 2 rows.  Shorter marches trade re-read halo rows for more
// wavefronts in flight; the level kernels are bound by the latency of the row
// pipeline more than by bandwidth up to n = 2048 (2048^2 solve with at least
// 4 rows: 1.089 ms, at least 2: 1.085 ms; mixed 1.043 -> 1.035 ms).
inline int stream_rows(int opt, int n) {
  if (opt < 0) return 0;
  if (opt > 0) return opt;
  const int R = n >> 7;
  return R < 2 ? 2 : R;
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
