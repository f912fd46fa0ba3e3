// Semi-Lagrangian transport of the anatomy labels (registration state),
// its adjoint and the body force of the registration gradient (paper
// Sec. 2.1 registration advection operator and optimality system; Sec. 3.3
// semi-Lagrangian time stepping, spectral derivatives).
//
// Characteristics by Heun's step, tricubic Lagrange interpolation on the
// periodic grid (nodes floor(p) - 1 .. floor(p) + 2 per axis, wrapped with
// & (n - 1): n is a power of two).  Positions are in grid units; the foot
// of the characteristic through grid point x is stored as its displacement
// from x, three real fields.  One thread per output grid point, z fastest.
#pragma once

#include "tg_kernels.h"

namespace tg {
namespace {

template <typename T>
__device__ __forceinline__ void lagrange4(T t, T (&w)[4]) {
  const T tm1 = t - T(1), tm2 = t - T(2), tp1 = t + T(1);
  w[0] = -t * tm1 * tm2 * T(1.0 / 6.0);
  w[1] = tp1 * tm1 * tm2 * T(0.5);
  w[2] = -tp1 * t * tm2 * T(0.5);
  w[3] = tp1 * t * tm1 * T(1.0 / 6.0);
}

// Stencil of a point: wrapped row offsets per axis and the weights.
template <typename T, int N>
struct Stencil {
  int ox[4], oy[4], oz[4];
  T wx[4], wy[4], wz[4];
  __device__ __forceinline__ void set(T px, T py, T pz) {
    const T fx = floor(px), fy = floor(py), fz = floor(pz);
    lagrange4<T>(px - fx, wx);
    lagrange4<T>(py - fy, wy);
    lagrange4<T>(pz - fz, wz);
    const int bx = (int)fx - 1, by = (int)fy - 1, bz = (int)fz - 1;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      ox[a] = ((bx + a) & (N - 1)) * N * N;
      oy[a] = ((by + a) & (N - 1)) * N;
      oz[a] = (bz + a) & (N - 1);
    }
  }
  // sum of the 64 weighted samples of f (times g at the same node if given)
  __device__ __forceinline__ T apply(const T* __restrict__ f, const T* __restrict__ g,
                                     T gs) const {
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      T sa = T(0);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int o = ox[a] + oy[b];
        T sb = T(0);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          T s = f[o + oz[c]];
          if (g) s *= T(1) + gs * g[o + oz[c]];
          sb += wz[c] * s;
        }
        sa += wy[b] * sb;
      }
      acc += wx[a] * sa;
    }
    return acc;
  }
};

template <int N>
__device__ __forceinline__ void grid_ijk(long long idx, int& i, int& j, int& k) {
  i = (int)(idx / ((long long)N * N));
  j = (int)((idx / N) % N);
  k = (int)(idx % N);
}

// One transport step of L fields: dst_l(x) = src_l(x + disp(x)).
// Adjoint form (w != null): dst_l(x) = [src_l (1 + hdt w)](x + disp(x)) /
// (1 - hdt w(x)), the trapezoid rule for the source lam div v along the
// characteristic.
template <typename T, int N>
__global__ void __launch_bounds__(256) k_sl_step(const T* __restrict__ src, T* __restrict__ dst,
                                                 const T* __restrict__ disp, int L,
                                                 const T* __restrict__ w, double hdt_) {
  constexpr long long R = (long long)N * N * N;
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= R) return;
  int i, j, k;
  grid_ijk<N>(idx, i, j, k);
  Stencil<T, N> st;
  st.set((T)i + disp[idx], (T)j + disp[R + idx], (T)k + disp[2 * R + idx]);
  const T hdt = (T)hdt_;
  const T den = w ? T(1) / (T(1) - hdt * w[idx]) : T(1);
  for (int l = 0; l < L; ++l) dst[l * R + idx] = st.apply(src + l * R, w, hdt) * den;
}

// The same step with the input staged in LDS: an output tile of 8 x 8 x 32
// points (z fastest) and a halo of H cells per side hold every stencil
// node of points displaced by less than H - 1 cells; a point whose stencil
// leaves the tile gathers from global memory instead, so any displacement
// is handled.  Labels one after another through the same LDS tile.  Only
// the denominator of the adjoint form is applied here (w_den): its
// numerator's factor (1 + hdt w) is premultiplied into src by k_sl_premul.
// FOOT: the displacement is dscale * disp and the output is
// heun * (src_l(x) + interpolated value), src_l(x) read from the tile: with
// src = disp = v, dscale = s and heun = s / 2 one launch gives the Heun foot
// s/2 (v(x) + v(x + s v(x))) of the three velocity components.  (A runtime
// switch for it made the plain steps 12% slower.)
template <typename T, int N, int H>
struct SLTile {
  static constexpr int BX = 8, BY = 8, BZ = 32;
  static constexpr int TX = BX + 2 * H, TY = BY + 2 * H, TZ = BZ + 2 * H;
  static constexpr int NBLK = (N / BX) * (N / BY) * (N / BZ);
  static_assert(N % BZ == 0 && N % BX == 0, "tile must divide the grid");
};

template <typename T, int N, int H, bool FOOT = false>
__global__ void __launch_bounds__(256) k_sl_step_lds(const T* __restrict__ src,
                                                     T* __restrict__ dst,
                                                     const T* __restrict__ disp, int L,
                                                     const T* __restrict__ w_den, double hdt_,
                                                     double dscale_, double heun_) {
  using TL = SLTile<T, N, H>;
  constexpr long long R = (long long)N * N * N;
  __shared__ T tile[TL::TX * TL::TY * TL::TZ];
  const int nbz = N / TL::BZ, nby = N / TL::BY;
  const int bz = blockIdx.x % nbz, by = (blockIdx.x / nbz) % nby, bx = blockIdx.x / (nbz * nby);
  const int x0 = bx * TL::BX - H, y0 = by * TL::BY - H, z0 = bz * TL::BZ - H;
  const int tz = threadIdx.x & 31, tx = threadIdx.x >> 5;   // 8 x-values, y looped
  const int gx = bx * TL::BX + tx, gz = bz * TL::BZ + tz;
  const T hdt = (T)hdt_, ds = (T)dscale_, hh = (T)heun_;
  (void)ds;
  (void)hh;
  for (int l = 0; l < L; ++l) {
    const T* f = src + l * R;
    for (int q = threadIdx.x; q < TL::TX * TL::TY * TL::TZ; q += 256) {
      const int iz = q % TL::TZ, iy = (q / TL::TZ) % TL::TY, ix = q / (TL::TZ * TL::TY);
      tile[q] = f[(((x0 + ix) & (N - 1)) * N + ((y0 + iy) & (N - 1))) * N + ((z0 + iz) & (N - 1))];
    }
    __syncthreads();
#pragma unroll 1
    for (int yy = 0; yy < TL::BY; ++yy) {
      const int gy = by * TL::BY + yy;
      const long long idx = ((long long)gx * N + gy) * N + gz;
      T px, py, pz;
      if constexpr (FOOT) {
        px = (T)gx + ds * disp[idx];
        py = (T)gy + ds * disp[R + idx];
        pz = (T)gz + ds * disp[2 * R + idx];
      } else {
        px = (T)gx + disp[idx];
        py = (T)gy + disp[R + idx];
        pz = (T)gz + disp[2 * R + idx];
      }
      const T fx = floor(px), fy = floor(py), fz = floor(pz);
      const int lx = (int)fx - 1 - x0, ly = (int)fy - 1 - y0, lz = (int)fz - 1 - z0;
      T val;
      if (lx >= 0 && lx <= TL::TX - 4 && ly >= 0 && ly <= TL::TY - 4 && lz >= 0 &&
          lz <= TL::TZ - 4) {
        T wx[4], wy[4], wz[4];
        lagrange4<T>(px - fx, wx);
        lagrange4<T>(py - fy, wy);
        lagrange4<T>(pz - fz, wz);
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          T sa = T(0);
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const T* r = tile + ((lx + a) * TL::TY + (ly + b)) * TL::TZ + lz;
            sa += wy[b] * (wz[0] * r[0] + wz[1] * r[1] + wz[2] * r[2] + wz[3] * r[3]);
          }
          acc += wx[a] * sa;
        }
        val = acc;
      } else {
        Stencil<T, N> st;
        st.set(px, py, pz);
        val = st.apply(f, nullptr, T(0));
      }
      if constexpr (FOOT) {
        val = hh * (tile[((tx + H) * TL::TY + (yy + H)) * TL::TZ + tz + H] + val);
      } else {
        if (w_den) val /= T(1) - hdt * w_den[idx];
      }
      dst[l * R + idx] = val;
    }
    __syncthreads();
  }
}

// dst_l = src_l (1 + hdt w), the numerator factor of the adjoint step.
template <typename T>
__global__ void __launch_bounds__(256) k_sl_premul(const T* __restrict__ src, T* __restrict__ dst,
                                                   const T* __restrict__ w, double hdt_, int L,
                                                   long long R) {
  const T hdt = (T)hdt_;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < R;
       i += (long long)gridDim.x * 256) {
    const T f = T(1) + hdt * w[i];
    for (int l = 0; l < L; ++l) dst[l * R + i] = src[l * R + i] * f;
  }
}

// Heun foot in three passes around the direct-gather step (grids below
// 32^3; larger ones do it in one k_sl_step_lds launch): pred = s v;
// u = v at x + pred (k_sl_step on the three components); disp = s/2 (v + u),
// in place on u.
template <typename T>
__global__ void __launch_bounds__(256) k_sl_scale3(const T* __restrict__ v, T* __restrict__ out,
                                                   double s_, long long R) {
  const T s = (T)s_;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < 3 * R;
       i += (long long)gridDim.x * 256)
    out[i] = s * v[i];
}
template <typename T>
__global__ void __launch_bounds__(256) k_sl_heun3(const T* __restrict__ v, T* __restrict__ u,
                                                  double s_, long long R) {
  const T hs = (T)(0.5 * s_);
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < 3 * R;
       i += (long long)gridDim.x * 256)
    u[i] = hs * (v[i] + u[i]);
}

// dst_l /= (1 - hdt w), the denominator of the adjoint step (small grids).
template <typename T>
__global__ void __launch_bounds__(256) k_sl_div(T* __restrict__ dst, const T* __restrict__ w,
                                                double hdt_, int L, long long R) {
  const T hdt = (T)hdt_;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < R;
       i += (long long)gridDim.x * 256) {
    const T d = T(1) / (T(1) - hdt * w[i]);
    for (int l = 0; l < L; ++l) dst[l * R + i] *= d;
  }
}

// Real row -> spectral row (the z pass of a forward transform, no other
// work), layout as the time-step kernels write it.
template <typename T, int N, int RW>
__global__ void __launch_bounds__((ZP<T, N, RW>::NT)) k_z_r2c(const T* __restrict__ f,
                                                             cx<T>* __restrict__ X) {
  ZP_SETUP
  const cx<T>* r = reinterpret_cast<const cx<T>*>(f + grow * N);
  cx<T> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = r[t + TT * e];
  r2c_row<T, N>(v, lds, t, row);
  cx<T>* o = X + sbase;
#pragma unroll
  for (int e = 0; e < E; ++e) o[t + TT * e] = v[e];
}

// Body force increment: b_j(x) += coef lam(x) (D_j m)(x) from the
// y-inverted gradient rows of m (V3 still needs i wz before the z
// transform), b: three real fields.
template <typename T, int N, int RW>
__global__ void __launch_bounds__((ZP<T, N, RW>::NT)) k_z_bforce(
    const cx<T>* __restrict__ V1, const cx<T>* __restrict__ V2, const cx<T>* __restrict__ V3,
    const T* __restrict__ lam, T* __restrict__ bf, double coef) {
  ZP_SETUP
  constexpr long long R = Z::REAL;
  const cx<T>* Vs[3] = {V1 + sbase, V2 + sbase, V3 + sbase};
  const cx<T>* lr = reinterpret_cast<const cx<T>*>(lam + grow * N);
  cx<T> u[E], lv[E];
  const T cf = (T)coef;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const cx<T> l = lr[t + TT * e];
    lv[e] = mk(cf * l.x, cf * l.y);
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = Vs[j][t + TT * e];
    if (j == 2) {
#pragma unroll
      for (int e = 0; e < E; ++e) u[e] = mul_i(u[e], (T)(t + TT * e));
    }
    c2r_row<T, N>(u, lds, t, row);
    cx<T>* o = reinterpret_cast<cx<T>*>(bf + j * R + grow * N);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cx<T> p = o[t + TT * e];
      o[t + TT * e] = mk(p.x + lv[e].x * u[e].x, p.y + lv[e].y * u[e].y);
    }
  }
}

}  // namespace
}  // namespace tg
