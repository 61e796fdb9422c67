// Fused 2D V-cycle level kernels (LDS-tiled, float64 or float32).
//
//   k_pre2d : two weighted-Jacobi sweeps, then the residual r = b - A x and
//             its restriction bc = P^T r to the coarse level, in one pass;
//   k_post2d: the coarse-grid correction x + P xc, then two sweeps.
//
// Each block owns a TX x TY tile of fine nodes whose origin is even, and the
// coarse nodes p with 2p inside the tile.  The tile and a halo are staged in
// LDS; every sweep is evaluated on a shrinking halo so that the owned nodes
// see exactly the values a sequence of separate sweeps would produce (points
// outside the interior are held at the Dirichlet value 0).  Arithmetic per
// node is the same expression as the separate kernels'.
#pragma once

#include "fmg_device.h"
#include "fmg_kernels_mg.h"

namespace fmg {

constexpr int kFTX = 64;   // fused tile width (fine nodes)
constexpr int kFTY = 16;   // fused tile height

template <typename T>
struct LTile {             // a rectangular LDS region [ox, ox+sx) x [oy, oy+sy)
  T* v;
  int ox, oy, sx, sy;
  __device__ __forceinline__ T& at(int x, int y) const { return v[(y - oy) * sx + (x - ox)]; }
};

__device__ __forceinline__ bool interior2(int n, int x, int y) { return x >= 1 && x <= n - 1 && y >= 1 && y <= n - 1; }

// dst := src on the region of dst (0 outside [0, n]^2).
template <typename T>
__device__ __forceinline__ void lds_load2(const LTile<T>& dst, const T* __restrict__ src, const Grid& g) {
  const int cnt = dst.sx * dst.sy;
  for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
    const int x = dst.ox + t % dst.sx, y = dst.oy + t / dst.sx;
    dst.v[t] = (x >= 0 && x <= g.n && y >= 0 && y <= g.n) ? src[y * g.px + x] : T(0);
  }
}

// out = in + wd (b - A in) on out's region (interior points only, else 0).
template <typename T, bool ZERO>
__device__ __forceinline__ void lds_sweep2(const LTile<T>& out, const LTile<T>& in, const LTile<T>& b, int n, T wd,
                                           T scale) {
  const int cnt = out.sx * out.sy;
  for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
    const int x = out.ox + t % out.sx, y = out.oy + t / out.sx;
    T v = T(0);
    if (interior2(n, x, y)) {
      if (ZERO) {
        v = wd * b.at(x, y);
      } else {
        const T s = (in.at(x - 1, y) + in.at(x + 1, y)) + (in.at(x, y - 1) + in.at(x, y + 1));
        const T c = in.at(x, y);
        v = c + wd * (b.at(x, y) - scale * (T(4) * c - s));
      }
    }
    out.v[t] = v;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_pre2d(Grid f, Grid cg, const T* __restrict__ x0, const T* __restrict__ b,
                                                  T* __restrict__ xout, T* __restrict__ bc, T wd1, T wd2, T scale,
                                                  int zero_init) {
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int X0 = blockIdx.x * kFTX, Y0 = blockIdx.y * kFTY;
  const int n = f.n;
  // regions: x0 on T+4, b on T+3, x1 on T+3, x2 on T+2 (reuses x0), r on T+1 (reuses x1)
  LTile<T> rx0{sm, X0 - 4, Y0 - 4, kFTX + 8, kFTY + 8};
  LTile<T> rb{rx0.v + rx0.sx * rx0.sy, X0 - 3, Y0 - 3, kFTX + 6, kFTY + 6};
  LTile<T> rx1{rb.v + rb.sx * rb.sy, X0 - 3, Y0 - 3, kFTX + 6, kFTY + 6};
  LTile<T> rx2{rx0.v, X0 - 2, Y0 - 2, kFTX + 4, kFTY + 4};
  LTile<T> rr{rx1.v, X0 - 1, Y0 - 1, kFTX + 2, kFTY + 2};
  if (!zero_init) lds_load2(rx0, x0, f);
  lds_load2(rb, b, f);
  __syncthreads();
  if (zero_init) lds_sweep2<T, true>(rx1, rx0, rb, n, wd1, scale);
  else lds_sweep2<T, false>(rx1, rx0, rb, n, wd1, scale);
  __syncthreads();
  lds_sweep2<T, false>(rx2, rx1, rb, n, wd2, scale);
  __syncthreads();
  // owned nodes of the second sweep -> global; residual on T+1
  for (int t = threadIdx.x; t < kFTX * kFTY; t += blockDim.x) {
    const int x = X0 + t % kFTX, y = Y0 + t / kFTX;
    if (interior2(n, x, y)) xout[y * f.px + x] = rx2.at(x, y);
  }
  {
    const int cnt = rr.sx * rr.sy;
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      const int x = rr.ox + t % rr.sx, y = rr.oy + t / rr.sx;
      T v = T(0);
      if (interior2(n, x, y)) {
        const T s = (rx2.at(x - 1, y) + rx2.at(x + 1, y)) + (rx2.at(x, y - 1) + rx2.at(x, y + 1));
        v = rb.at(x, y) - scale * (T(4) * rx2.at(x, y) - s);
      }
      rr.v[t] = v;
    }
  }
  __syncthreads();
  // restriction at the coarse nodes owned by this tile
  const int CX0 = X0 / 2, CY0 = Y0 / 2;
  for (int t = threadIdx.x; t < (kFTX / 2) * (kFTY / 2); t += blockDim.x) {
    const int i = CX0 + t % (kFTX / 2), j = CY0 + t / (kFTX / 2);
    if (i < 1 || i > cg.n - 1 || j < 1 || j > cg.n - 1) continue;
    const int x = 2 * i, y = 2 * j;
    const T h = (rr.at(x + 1, y) + rr.at(x - 1, y)) + (rr.at(x, y + 1) + rr.at(x, y - 1)) +
                (rr.at(x + 1, y + 1) + rr.at(x - 1, y - 1));
    bc[j * cg.px + i] = rr.at(x, y) + T(0.5) * h;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_post2d(Grid cg, Grid f, const T* __restrict__ x, const T* __restrict__ xc,
                                                   const T* __restrict__ b, T* __restrict__ xout, T wd1, T wd2,
                                                   T scale) {
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int X0 = blockIdx.x * kFTX, Y0 = blockIdx.y * kFTY;
  const int n = f.n;
  // regions: corrected x on T+2, b on T+1, x1 on T+1, coarse on (T+2)/2 (+1)
  LTile<T> rx{sm, X0 - 2, Y0 - 2, kFTX + 4, kFTY + 4};
  LTile<T> rb{rx.v + rx.sx * rx.sy, X0 - 1, Y0 - 1, kFTX + 2, kFTY + 2};
  LTile<T> rx1{rb.v + rb.sx * rb.sy, X0 - 1, Y0 - 1, kFTX + 2, kFTY + 2};
  LTile<T> rc{rx1.v + rx1.sx * rx1.sy, X0 / 2 - 1, Y0 / 2 - 1, kFTX / 2 + 3, kFTY / 2 + 3};
  lds_load2(rx, x, f);
  lds_load2(rb, b, f);
  lds_load2(rc, xc, cg);
  __syncthreads();
  {
    const int cnt = rx.sx * rx.sy;
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      const int px = rx.ox + t % rx.sx, py = rx.oy + t / rx.sx;
      if (!interior2(n, px, py)) continue;
      const int si = px & 1, sj = py & 1, ci = px >> 1, cj = py >> 1;
      T v = rc.at(ci, cj);
      if (si | sj) v = T(0.5) * (v + rc.at(ci + si, cj + sj));
      rx.v[t] = rx.v[t] + v;
    }
  }
  __syncthreads();
  lds_sweep2<T, false>(rx1, rx, rb, n, wd1, scale);
  __syncthreads();
  for (int t = threadIdx.x; t < kFTX * kFTY; t += blockDim.x) {
    const int px = X0 + t % kFTX, py = Y0 + t / kFTX;
    if (!interior2(n, px, py)) continue;
    const T s = (rx1.at(px - 1, py) + rx1.at(px + 1, py)) + (rx1.at(px, py - 1) + rx1.at(px, py + 1));
    const T c = rx1.at(px, py);
    xout[py * f.px + px] = c + wd2 * (rb.at(px, py) - scale * (T(4) * c - s));
  }
}

template <typename T>
constexpr size_t pre2d_lds_bytes() {
  return sizeof(T) * ((size_t)(kFTX + 8) * (kFTY + 8) + 2 * (size_t)(kFTX + 6) * (kFTY + 6));
}
template <typename T>
constexpr size_t post2d_lds_bytes() {
  return sizeof(T) * ((size_t)(kFTX + 4) * (kFTY + 4) + 2 * (size_t)(kFTX + 2) * (kFTY + 2) +
                      (size_t)(kFTX / 2 + 3) * (kFTY / 2 + 3));
}

}  // namespace fmg
