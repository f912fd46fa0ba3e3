// HIP kernels of the tumor forward/adjoint path (gfx950).
//
// Fields.  A real field is [n][n][n] (x slowest, z fastest).  A spectrum is
// the "packed half spectrum" [kx][ky][kz'] with kz' in [0, n/2): for
// kz' >= 1 it holds the 3D DFT coefficient at (kx, ky, kz'); slot kz' = 0
// holds U + i V where U and V are the 2D DFTs of the kz = 0 and kz = n/2
// planes (both Hermitian).  A spectrum therefore has n^3/2 complex entries,
// the same bytes as the real field.  Every spectral multiplier used here
// (derivative symbols with the Nyquist wavenumber zeroed, the Fourier
// preconditioner) takes the same value on the kz = 0 and kz = n/2 planes,
// so it acts on slot 0 exactly as on U and V separately, and the grid inner
// product is sum_k w(kz') Re(conj(a) b) / n^3 with w = 1 on slot 0 and 2
// elsewhere (the cross terms of U and V cancel over the full plane).
//
// Transforms are unnormalized; the 1/n^3 of the inverse is folded into
// the first inverse pass.  Passes: "x" (stride n^2/2), "y" (stride n/2),
// "z" (contiguous rows, real <-> packed complex).
#pragma once
#include "tg_fft.h"
#include "tg_internal.h"

namespace tg {
// Kernels have internal linkage: each precision's translation unit holds
// its own copy of the shared non-template kernels.
namespace {

template <typename T> struct Tr;
template <> struct Tr<float> {
  static __device__ __forceinline__ float ex(float a) { return __expf(a); }
};
template <> struct Tr<double> {
  static __device__ __forceinline__ double ex(double a) { return exp(a); }
};

// Derivative symbol of a full axis, Nyquist zeroed.
template <int N>
__device__ __forceinline__ int wfull(int k) { return k < N / 2 ? k : (k == N / 2 ? 0 : k - N); }

// ------------------------------------------------------------- reaction
// Exact logistic flow over tau, R(u) = u E / (1 + u (E - 1)), E = exp(rho tau),
// rho = rho_f m (Sec. 2.1 reaction term, Sec. 3.3 analytic step).
template <typename T>
__device__ __forceinline__ T react(T u, T E) { return u * E / (T(1) + u * (E - T(1))); }
template <typename T>
__device__ __forceinline__ T react_du(T u, T E) {
  T D = T(1) + u * (E - T(1));
  return E / (D * D);
}

// ------------------------------------------------------------ reductions
template <int NT>
__device__ __forceinline__ void block_sums(double (&v)[NSLOT], int ns, double* red) {
  // deterministic: fixed xor-shuffle tree inside each wave, then waves in
  // order on thread 0.  red needs NSLOT * NT/64 doubles.
  constexpr int NW = (NT + 63) / 64;
  constexpr int WW = NT < 64 ? NT : 64;  // active lanes of a wave
  for (int s = 0; s < ns; ++s) {
    double x = v[s];
#pragma unroll
    for (int o = WW / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, WW);
    v[s] = x;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
    for (int s = 0; s < ns; ++s) red[s * NW + wid] = v[s];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int s = 0; s < ns; ++s) {
      double acc = 0.0;
      for (int w = 0; w < NW; ++w) acc += red[s * NW + w];
      v[s] = acc;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ double* part_at(double* part, int b, int s) {
  return part + ((size_t)b * NSLOT + s) * MAXBLK;
}

// PCG step length of problem b (called by every thread of one workgroup of
// NT threads): <p, A p> = sum w |p|^2 + tau k_f n^3 sum_x m |grad p|^2 from
// the partial sums of the x inverse pass (slot 0, nblk0 of them) and of the
// z matvec (slot 1, nblk1), summed in a fixed order (scale = tau n^3), then
// alpha = <r, M r> / <p, A p>, or a breakdown.  red: NSLOT * NT/64 doubles.
template <int NT>
__device__ void pcg_step_length(ProbScalars& S, double* part, int b, int nblk0, int nblk1,
                                double scale, double* red) {
  double acc[NSLOT] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nblk0; i += NT) acc[0] += part_at(part, b, 0)[i];
  for (int i = threadIdx.x; i < nblk1; i += NT) acc[1] += part_at(part, b, 1)[i];
  block_sums<NT>(acc, 2, red);
  if (threadIdx.x != 0) return;
  const double pap = acc[0] + scale * S.kf * acc[1];
  S.pq = pap;
  if (!(pap > 0.0) || !isfinite(pap)) {
    S.status |= isfinite(pap) ? STAT_BREAKDOWN : STAT_NONFINITE;
    S.done = 1;
    S.alpha = 0.0;
    const double rel = S.rhs2 > 0 ? sqrt(S.rr / S.rhs2) : 0.0;
    S.worst = fmax(S.worst, rel);
  } else {
    S.alpha = S.rho / pap;
  }
}

// ------------------------------------------------------ strided passes
// Pass along x (AX = 0) or y (AX = 1) of a packed spectrum.  Column index
// gc enumerates the n * n/2 pencils: for x, gc = ky * n/2 + kz'; for y,
// gc = x * n/2 + kz'.  A workgroup takes C consecutive pencils; thread
// (col, t) holds positions t + TT e of pencil col.
template <typename T, int N, int C, int AX, int E_ = FftE<N>::value>
struct SP {
  static constexpr int NH = N / 2;
  static constexpr int L = N;
  static constexpr int E = E_;
  static constexpr int TT = L / E;
  static constexpr int NT = C * TT;
  static constexpr int NCOL = N * NH;
  static constexpr int NBLK = NCOL / C;
  static constexpr long long PSTR = AX == 0 ? (long long)N * NH : NH;
  static constexpr long long SPEC = (long long)N * N * NH;  // complex per problem
  static __device__ __forceinline__ long long colbase(int gc) {
    return AX == 0 ? (long long)gc : (long long)(gc / NH) * (N * NH) + (gc % NH);
  }
};

// Launch bounds with an occupancy floor: at least W waves per SIMD (the
// compiler then caps registers accordingly); W = 1 leaves them uncapped.
#define TG_BOUNDS(NT, W) \
  __attribute__((amdgpu_flat_work_group_size(1, NT), amdgpu_waves_per_eu(W)))

// SP_SETUP_EXIT: EXIT (uniform over the workgroup) returns before the
// twiddle table is filled, so a predicated-off launch costs only its dispatch.
#define SP_SETUP(AXV) SP_SETUP_EXIT(AXV, 0, false)
#define SP_SETUP_OFF(AXV, OFF) SP_SETUP_EXIT(AXV, OFF, false)
#define SP_SETUP_EXIT(AXV, OFF, EXIT) SP_SETUP_EXIT_E(AXV, FftE<N>::value, OFF, EXIT)
// SP_SETUP_EXIT_E: as SP_SETUP_EXIT with EV values per lane.
#define SP_SETUP_EXIT_E(AXV, EV, OFF, EXIT)                             \
  using S = SP<T, N, C, AXV, EV>;                                       \
  constexpr int E = S::E, TT = S::TT, NH = S::NH;                       \
  (void)NH;                                                             \
  __shared__ cx<T> lds[(S::TT > 1) ? N * C : 1];                        \
  const int b = blockIdx.y;                                             \
  const int col = threadIdx.x % C, t = threadIdx.x / C;                 \
  const int gc = ((int)blockIdx.x + (OFF)) * C + col;                   \
  const long long base = (long long)b * S::SPEC + S::colbase(gc);       \
  if (EXIT) return;                                                     \
  tw_fill<T>();

// ---- x pass, inverse, gradient prologue of the diffusion matvec.
// MODE 0: p is given.  MODE 1: PCG direction p = M r + beta p (stored) and
// partial |p|^2 (slot 0; Parseval weights).
// Out: U1 = IFFT_x(s i wx p), U2 = IFFT_x(s p), s = 1/n^3.
// The x passes of the matvec in FP64 at 256^3 (up to 32 pencils) keep 8
// values per lane (XPassE): half the registers and twice the waves per SIMD
// of 16 per lane, for one more LDS exchange per transform.  (In FP32, 16
// pencils with 8 values per lane time like 64 pencils with 16, and the
// whole solve is 0.5% slower with them.)
template <typename T, int N, int C>
struct XPassE {
  static constexpr int value = (sizeof(T) == 8 && N == 256 && C <= 32) ? 8 : FftE<N>::value;
};

template <typename T, int N, int C, int MODE, int OCC>
__global__ void TG_BOUNDS((SP<T, N, C, 0, XPassE<T, N, C>::value>::NT), OCC)
k_x_inv_grad(cx<T>* __restrict__ P, const cx<T>* __restrict__ Rr, cx<T>* __restrict__ U1,
             cx<T>* __restrict__ U2, const ProbScalars* __restrict__ sc, double* __restrict__ part,
             double tau, int pred) {
  SP_SETUP_EXIT_E(0, (XPassE<T, N, C>::value), 0, pred && sc[blockIdx.y].done)
  __shared__ double red[MODE == 1 ? NSLOT * ((S::NT + 63) / 64) : 1];
  const int ky = gc / NH, kz = gc % NH;
  const T wy = (T)wfull<N>(ky), wz = (T)kz;
  const T s = T(1) / (T(N) * T(N) * T(N));
  cx<T> v[E], w[E];
  if constexpr (MODE == 1) {
    const bool first = sc[b].first != 0;
    const T beta = (T)sc[b].beta;
    const T kb = (T)(tau * sc[b].kbar);
    double pp = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int kx = t + TT * e;
      const T wx = (T)wfull<N>(kx);
      const T pre = T(1) / (T(1) + kb * (wx * wx + wy * wy + wz * wz));
      const long long o = base + kx * S::PSTR;
      cx<T> p = scale(Rr[o], pre);
      if (!first) p = p + scale(P[o], beta);
      P[o] = p;
      v[e] = p;
      pp += (double)p.x * (double)p.x + (double)p.y * (double)p.y;
    }
    double acc[NSLOT] = {(kz == 0 ? 1.0 : 2.0) * pp, 0.0, 0.0, 0.0};
    block_sums<S::NT>(acc, 1, red);
    if (threadIdx.x == 0) part_at(part, b, 0)[blockIdx.x] = acc[0];
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = P[base + (t + TT * e) * S::PSTR];
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const T wx = (T)wfull<N>(t + TT * e);
    w[e] = mul_i(v[e], s * wx);
    v[e] = scale(v[e], s);
  }
  fft<T, N, E, true, C, 1>(w, lds, t, col);
#pragma unroll
  for (int e = 0; e < E; ++e) U1[base + (t + TT * e) * S::PSTR] = w[e];
  fft<T, N, E, true, C, 1>(v, lds, t, col);
#pragma unroll
  for (int e = 0; e < E; ++e) U2[base + (t + TT * e) * S::PSTR] = v[e];
}

// ---- y pass, inverse: V1 = IFFT_y(U1) (in place), V2 = IFFT_y(i wy U2)
// (in place), V3 = IFFT_y(U2).  Both inputs are loaded before any FFT.
template <typename T, int N, int C, int OCC>
__global__ void TG_BOUNDS((SP<T, N, C, 1>::NT), OCC)
k_y_inv_grad(cx<T>* __restrict__ U1, cx<T>* __restrict__ U2, cx<T>* __restrict__ V3,
             const ProbScalars* __restrict__ sc, int pred, int blk0) {
  SP_SETUP_EXIT(1, blk0, pred && sc[blockIdx.y].done)
  cx<T> v[E], u[E], w[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    v[e] = U1[base + (t + TT * e) * S::PSTR];
    u[e] = U2[base + (t + TT * e) * S::PSTR];
  }
  fft<T, N, E, true, C, 1>(v, lds, t, col);
#pragma unroll
  for (int e = 0; e < E; ++e) U1[base + (t + TT * e) * S::PSTR] = v[e];
#pragma unroll
  for (int e = 0; e < E; ++e) w[e] = mul_i(u[e], (T)wfull<N>(t + TT * e));
  fft<T, N, E, true, C, 1>(u, lds, t, col);
#pragma unroll
  for (int e = 0; e < E; ++e) V3[base + (t + TT * e) * S::PSTR] = u[e];
  fft<T, N, E, true, C, 1>(w, lds, t, col);
#pragma unroll
  for (int e = 0; e < E; ++e) U2[base + (t + TT * e) * S::PSTR] = w[e];
}

// ---- y pass, forward: W1 = FFT_y(H1) (in place), W23 = i wy FFT_y(H2) +
// FFT_y(H3) (into H2).  FP32 loads all three inputs before any FFT.
// fin0 > 0 (last launch of a PCG iteration's matvec): workgroup 0 of each
// problem also forms the PCG step length (pcg_step_length with fin0, fin1
// partials and scale fsc); the x forward pass that follows reads it.
template <typename T, int N, int C, int OCC>
__global__ void TG_BOUNDS((SP<T, N, C, 1>::NT), OCC)
k_y_fwd_div(cx<T>* __restrict__ H1, cx<T>* __restrict__ H2, const cx<T>* __restrict__ H3,
            ProbScalars* __restrict__ sc, int pred, int blk0, double* __restrict__ part,
            int fin0, int fin1, double fsc) {
  SP_SETUP_EXIT(1, blk0, pred && sc[blockIdx.y].done)
  if (fin0 > 0 && blockIdx.x == 0) {
    __shared__ double red[NSLOT * ((S::NT + 63) / 64)];
    pcg_step_length<S::NT>(sc[b], part, b, fin0, fin1, fsc, red);
  }
  constexpr bool PRE = sizeof(T) == 4;
  cx<T> v[E], a[E], c[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    v[e] = H1[base + (t + TT * e) * S::PSTR];
    if (PRE) {
      a[e] = H2[base + (t + TT * e) * S::PSTR];
      c[e] = H3[base + (t + TT * e) * S::PSTR];
    }
  }
  fft<T, N, E, false, C, 1>(v, lds, t, col);
#pragma unroll
  for (int e = 0; e < E; ++e) H1[base + (t + TT * e) * S::PSTR] = v[e];
  if (!PRE) {
#pragma unroll
    for (int e = 0; e < E; ++e) a[e] = H2[base + (t + TT * e) * S::PSTR];
  }
  fft<T, N, E, false, C, 1>(a, lds, t, col);
  if (!PRE) {
#pragma unroll
    for (int e = 0; e < E; ++e) c[e] = H3[base + (t + TT * e) * S::PSTR];
  }
  fft<T, N, E, false, C, 1>(c, lds, t, col);
#pragma unroll
  for (int e = 0; e < E; ++e)
    H2[base + (t + TT * e) * S::PSTR] = mul_i(a[e], (T)wfull<N>(t + TT * e)) + c[e];
}

// ---- x pass, forward, divergence epilogue of the diffusion matvec:
// Am = i wx FFT_x(W1) + FFT_x(W23) is the spectrum of div(m grad u).
enum XMode : int {
  XM_PCG = 0,      // q = p - tau kf Am; x += alpha p; r -= alpha q; partials <r, M r>, |r|^2
  XM_RHS_FWD = 1,  // x0 = X; r = 2 tau kf Am; partials |rhs|^2, <r, M r>, |r|^2
  XM_RHS_ADJ = 2,  // x0 = X; r = tau kf Am;  rhs = X
  XM_POST_ADJ = 3, // X += tau kf Am; partial <Am, S> (k_f gradient)
  XM_SHIFT = 4     // Am of the shift d = Sv: x0 = X + d, r = Q - d + tau kf Am (the exact
                   // residual of x0 when Q held r of X); partials |X + Q/2|^2, <r, M r>, |r|^2
};

template <typename T, int N, int C, int MODE, int OCC>
__global__ void TG_BOUNDS((SP<T, N, C, 0, XPassE<T, N, C>::value>::NT), OCC)
k_x_fwd_div(const cx<T>* __restrict__ W1, const cx<T>* __restrict__ W23, cx<T>* __restrict__ X,
            cx<T>* __restrict__ Q, const cx<T>* __restrict__ Sv, const ProbScalars* __restrict__ sc,
            double* __restrict__ part, double tau, int pred, int want_gk) {
  SP_SETUP_EXIT_E(0, (XPassE<T, N, C>::value), 0, pred && sc[blockIdx.y].done)
  __shared__ double red[NSLOT * ((S::NT + 63) / 64)];
  const int ky = gc / NH, kz = gc % NH;
  const T wy = (T)wfull<N>(ky), wz = (T)kz;
  const double wgt = kz == 0 ? 1.0 : 2.0;
  cx<T> a[E], c[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    a[e] = W1[base + (t + TT * e) * S::PSTR];
    c[e] = W23[base + (t + TT * e) * S::PSTR];
  }
  fft<T, N, E, false, C, 1>(a, lds, t, col);
  fft<T, N, E, false, C, 1>(c, lds, t, col);
  const T tk = (T)(tau * sc[b].kf);
  double acc[NSLOT] = {0.0, 0.0, 0.0, 0.0};
  int ns = 0;
  if constexpr (MODE == XM_PCG) {
    // X: iterate x, Q: residual r, Sv: direction p; alpha is already known
    // (from |p|^2 and the z pass's sum of m |grad p|^2), so the update
    // happens here and q = A p never goes to memory.
    ns = 2;
    const T al = (T)sc[b].alpha;
    const T kb = (T)(tau * sc[b].kbar);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int kx = t + TT * e;
      const long long o = base + kx * S::PSTR;
      const T wx = (T)wfull<N>(kx);
      const cx<T> am = mul_i(a[e], wx) + c[e];
      const cx<T> p = Sv[o];
      const cx<T> q = p - scale(am, tk);
      X[o] = X[o] + scale(p, al);
      const cx<T> r = Q[o] - scale(q, al);
      Q[o] = r;
      const T pre = T(1) / (T(1) + kb * (wx * wx + wy * wy + wz * wz));
      const double rr = (double)r.x * (double)r.x + (double)r.y * (double)r.y;
      acc[0] += wgt * (double)pre * rr;
      acc[1] += wgt * rr;
    }
  } else if constexpr (MODE == XM_SHIFT) {
    ns = 3;
    const T kb = (T)(tau * sc[b].kbar);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int kx = t + TT * e;
      const long long o = base + kx * S::PSTR;
      const T wx = (T)wfull<N>(kx);
      const cx<T> am = mul_i(a[e], wx) + c[e];
      const cx<T> x0 = X[o], r0 = Q[o], d = Sv[o];
      const cx<T> rhs = x0 + scale(r0, T(0.5));
      X[o] = x0 + d;
      const cx<T> r = r0 - d + scale(am, tk);
      Q[o] = r;
      const T pre = T(1) / (T(1) + kb * (wx * wx + wy * wy + wz * wz));
      const double rr = (double)r.x * (double)r.x + (double)r.y * (double)r.y;
      acc[0] += wgt * ((double)rhs.x * (double)rhs.x + (double)rhs.y * (double)rhs.y);
      acc[1] += wgt * (double)pre * rr;
      acc[2] += wgt * rr;
    }
  } else if constexpr (MODE == XM_RHS_FWD || MODE == XM_RHS_ADJ) {
    ns = 3;
    const T kb = (T)(tau * sc[b].kbar);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int kx = t + TT * e;
      const long long o = base + kx * S::PSTR;
      const T wx = (T)wfull<N>(kx);
      const cx<T> am = mul_i(a[e], wx) + c[e];
      const cx<T> x0 = X[o];
      cx<T> r, rhs;
      if constexpr (MODE == XM_RHS_FWD) {
        r = scale(am, T(2) * tk);
        rhs = x0 + scale(am, tk);
      } else {
        r = scale(am, tk);
        rhs = x0;
      }
      Q[o] = r;
      const T pre = T(1) / (T(1) + kb * (wx * wx + wy * wy + wz * wz));
      const double rr = (double)r.x * (double)r.x + (double)r.y * (double)r.y;
      acc[0] += wgt * ((double)rhs.x * (double)rhs.x + (double)rhs.y * (double)rhs.y);
      acc[1] += wgt * (double)pre * rr;
      acc[2] += wgt * rr;
    }
  } else {
    ns = 1;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int kx = t + TT * e;
      const long long o = base + kx * S::PSTR;
      const cx<T> am = mul_i(a[e], (T)wfull<N>(kx)) + c[e];
      if (want_gk) {
        const cx<T> sv = Sv[o];
        acc[0] += wgt * ((double)am.x * (double)sv.x + (double)am.y * (double)sv.y);
      }
      X[o] = X[o] + scale(am, tk);
    }
  }
  block_sums<S::NT>(acc, ns, red);
  if (threadIdx.x == 0)
    for (int s2 = 0; s2 < ns; ++s2) part_at(part, b, s2)[blockIdx.x] = acc[s2];
}

// ---- plain passes of a single spectrum (state transforms).
// x inverse with 1/n^3 scaling: Y = IFFT_x(X / n^3)
template <typename T, int N, int C>
__global__ void __launch_bounds__((SP<T, N, C, 0>::NT))
k_x_inv(const cx<T>* __restrict__ X, cx<T>* __restrict__ Y) {
  SP_SETUP(0)
  const T s = T(1) / (T(N) * T(N) * T(N));
  cx<T> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = scale(X[base + (t + TT * e) * S::PSTR], s);
  fft<T, N, E, true, C, 1>(v, lds, t, col);
#pragma unroll
  for (int e = 0; e < E; ++e) Y[base + (t + TT * e) * S::PSTR] = v[e];
}

// y pass in place, forward or inverse, on one or two spectra.
template <typename T, int N, int C, bool INV>
__global__ void __launch_bounds__((SP<T, N, C, 1>::NT))
k_y_plain(cx<T>* __restrict__ Y, cx<T>* __restrict__ Y2) {
  SP_SETUP(1)
  cx<T> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = Y[base + (t + TT * e) * S::PSTR];
  fft<T, N, E, INV, C, 1>(v, lds, t, col);
#pragma unroll
  for (int e = 0; e < E; ++e) Y[base + (t + TT * e) * S::PSTR] = v[e];
  if (Y2 != nullptr) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = Y2[base + (t + TT * e) * S::PSTR];
    fft<T, N, E, INV, C, 1>(v, lds, t, col);
#pragma unroll
    for (int e = 0; e < E; ++e) Y2[base + (t + TT * e) * S::PSTR] = v[e];
  }
}

// x pass forward of the state spectrum H -> X, optionally followed in the
// same kernel by the gradient prologue of the matvec on X (U1, U2), and
// optionally a plain forward x pass of a second spectrum S2 (in place).
template <typename T, int N, int C>
__global__ void __launch_bounds__((SP<T, N, C, 0>::NT))
k_x_fwd_state(const cx<T>* __restrict__ H, cx<T>* __restrict__ X, cx<T>* __restrict__ U1,
              cx<T>* __restrict__ U2, cx<T>* __restrict__ S2) {
  SP_SETUP(0)
  cx<T> v[E], w[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = H[base + (t + TT * e) * S::PSTR];
  fft<T, N, E, false, C, 1>(v, lds, t, col);
#pragma unroll
  for (int e = 0; e < E; ++e) X[base + (t + TT * e) * S::PSTR] = v[e];
  if (U1 != nullptr) {
    const T s = T(1) / (T(N) * T(N) * T(N));
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const T wx = (T)wfull<N>(t + TT * e);
      w[e] = mul_i(v[e], s * wx);
      v[e] = scale(v[e], s);
    }
    fft<T, N, E, true, C, 1>(w, lds, t, col);
#pragma unroll
    for (int e = 0; e < E; ++e) U1[base + (t + TT * e) * S::PSTR] = w[e];
    fft<T, N, E, true, C, 1>(v, lds, t, col);
#pragma unroll
    for (int e = 0; e < E; ++e) U2[base + (t + TT * e) * S::PSTR] = v[e];
  }
  if (S2 != nullptr) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = S2[base + (t + TT * e) * S::PSTR];
    fft<T, N, E, false, C, 1>(v, lds, t, col);
#pragma unroll
    for (int e = 0; e < E; ++e) S2[base + (t + TT * e) * S::PSTR] = v[e];
  }
}

// ------------------------------------------------------------- z passes
// Rows (b, x, y) of n reals = n/2 complex.  RW rows per workgroup; thread
// (t, row) holds complex positions t + TT e.  LDS rows use the padded
// layout (one spare slot per E positions), pitch L + TT.
template <int N>
struct ZDefaultRows {
  static constexpr int L = N / 2;
  static constexpr int TT = L / FftE<L>::value;
  static constexpr int value = (TT * 64 <= 256) ? 64 : 256 / TT;
};

template <typename T, int N, int RW_ = ZDefaultRows<N>::value, int E_ = FftE<N / 2>::value>
struct ZP {
  static constexpr int L = N / 2;
  static constexpr int E = E_;
  static constexpr int TT = L / E;
  static constexpr int RW = RW_;
  static constexpr int NT = TT * RW;
  static constexpr int PITCH = L + TT;
  static constexpr int NBLK = N * N / RW;
  static constexpr long long SPEC = (long long)N * N * (N / 2);
  static constexpr long long REAL = (long long)N * N * N;
  static_assert(N * N % RW == 0, "rows per block must divide the row count");
  static_assert(64 % TT == 0, "a row must stay inside one wave");
};

// Mirror partner of the value held in register e of row-thread t:
// X[L - k] for k = t + TT e.  For t >= 1 it sits in register E-1-e of
// row-thread TT - t (same wave, exchanged with a lane shuffle); for t = 0
// in the thread's own register E - e.
template <typename T>
__device__ __forceinline__ cx<T> shfl_cx(cx<T> v, int src, int width) {
  return mk(__shfl(v.x, src, width), __shfl(v.y, src, width));
}

template <typename T, int TT, int E>
__device__ __forceinline__ void mirror_vals(const cx<T> (&v)[E], cx<T> (&m)[E], int t) {
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const cx<T> own = v[(E - e) % E];
    if constexpr (TT == 1) {
      m[e] = own;
    } else {
      const cx<T> other = shfl_cx(v[E - 1 - e], (TT - t) & (TT - 1), TT);
      m[e] = (t == 0) ? own : other;
    }
  }
}

// Unnormalized C2R of one packed row: in v[e] = Y[k], k = t + TT e;
// out v[e] = n (x[2j] + i x[2j+1]), j = t + TT e.  All exchanges stay
// inside the row's wave.
template <typename T, int N, int E>
__device__ __forceinline__ void c2r_row(cx<T> (&v)[E], cx<T>* lds, int t, int row) {
  using Z = ZP<T, N, ZDefaultRows<N>::value, E>;
  constexpr int L = Z::L, TT = Z::TT;
  cx<T> mr[E];
  mirror_vals<T, TT, E>(v, mr, t);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = t + TT * e;
    const cx<T> xk = v[e];
    if (k == 0) {
      // X0 = Re Y0, X_{n/2} = Im Y0
      v[e] = mk(xk.x + xk.y, xk.x - xk.y);
    } else {
      const cx<T> xm = conjg(mr[e]);
      const cx<T> sum = xk + xm, dif = xk - xm;
      // i W_n^{-k} dif, W_n^{-k} = conj(tw)
      const cx<T> wk = conjg(twiddle<T, false, N>(k));
      const cx<T> tdif = cmul(wk, dif);
      v[e] = sum + mk(-tdif.y, tdif.x);
    }
  }
  (void)L;
  fft<T, L, E, true, 1, Z::PITCH, true, true>(v, lds, t, row);
}

// Unnormalized R2C of one row: in v[e] = x[2j] + i x[2j+1]; out v[e] =
// packed Y[k] (slot 0 = X0 + i X_{n/2}).
template <typename T, int N, int E>
__device__ __forceinline__ void r2c_row(cx<T> (&v)[E], cx<T>* lds, int t, int row) {
  using Z = ZP<T, N, ZDefaultRows<N>::value, E>;
  constexpr int L = Z::L, TT = Z::TT;
  fft<T, L, E, false, 1, Z::PITCH, true, true>(v, lds, t, row);
  cx<T> mr[E];
  mirror_vals<T, TT, E>(v, mr, t);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = t + TT * e;
    const cx<T> zk = v[e];
    if (k == 0) {
      v[e] = mk(zk.x + zk.y, zk.x - zk.y);
    } else {
      const cx<T> zm = conjg(mr[e]);
      const cx<T> sum = zk + zm, dif = zk - zm;
      // X = (sum - i W^k dif) / 2
      const cx<T> td = cmul(twiddle<T, false, N>(k), dif);
      v[e] = scale(sum + mk(td.y, -td.x), T(0.5));
    }
  }
  (void)L;
}

// ---- pair layout: register 2e + s holds complex position k = 2 q + s of
// the row, q = t + TT e (e < E/2), so each lane moves whole 16-byte (FP32)
// pairs to and from memory.  The real-transform pre/post-processing is the
// same as above; the length-L transform is split into its even and odd
// halves: the inverse is two half-length inverse transforms of the even
// and odd positions (input in pair layout) combined with W_L^-n
// (decimation in time), the forward combines x[n] and x[n + L/2] with
// W_L^n first and ends with two half-length transforms whose outputs are
// the even and odd positions (decimation in frequency).  Values in real
// space keep the register mapping of the other helpers (position t + TT e).
template <typename T>
struct alignas(4 * sizeof(T)) cx2 {
  cx<T> a, b;
};

// Mirror partner X[L - k] of every register in pair layout.  k = 2q + 1:
// position 2 (K - 1 - q) + 1 = register 2 (E/2 - 1 - e) + 1 of lane
// TT - 1 - t.  k = 2q: position 2 (K - q), register 2 (E/2 - 1 - e) of
// lane TT - t for t >= 1, own register 2 ((E/2 - e) mod E/2) for t = 0.
template <typename T, int TT, int E>
__device__ __forceinline__ void mirror_pairs(const cx<T> (&v)[E], cx<T> (&m)[E], int t) {
  constexpr int E2 = E / 2;
#pragma unroll
  for (int e = 0; e < E2; ++e) {
    const cx<T> own0 = v[2 * ((E2 - e) % E2)];
    if constexpr (TT == 1) {
      m[2 * e] = own0;
      m[2 * e + 1] = v[2 * (E2 - 1 - e) + 1];
    } else {
      const cx<T> other0 = shfl_cx(v[2 * (E2 - 1 - e)], (TT - t) & (TT - 1), TT);
      m[2 * e] = (t == 0) ? own0 : other0;
      m[2 * e + 1] = shfl_cx(v[2 * (E2 - 1 - e) + 1], TT - 1 - t, TT);
    }
  }
}

// C2R as c2r_row, input in pair layout, output in the usual mapping.
template <typename T, int N, int E>
__device__ __forceinline__ void c2r_pairs(cx<T> (&v)[E], cx<T>* lds, int t, int row) {
  using Z = ZP<T, N, ZDefaultRows<N>::value, E>;
  constexpr int L = Z::L, TT = Z::TT, E2 = E / 2, K = L / 2;
  static_assert(E % 2 == 0 && Z::PITCH >= K + K / E2, "pair layout");
  cx<T> mr[E];
  mirror_pairs<T, TT, E>(v, mr, t);
  cx<T> a[E2], b[E2];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int k = 2 * (t + TT * (i / 2)) + (i & 1);
    const cx<T> xk = v[i];
    cx<T> z;
    if (k == 0) {
      z = mk(xk.x + xk.y, xk.x - xk.y);
    } else {
      const cx<T> xm = conjg(mr[i]);
      const cx<T> sum = xk + xm, dif = xk - xm;
      const cx<T> tdif = cmul(conjg(twiddle<T, false, N>(k)), dif);
      z = sum + mk(-tdif.y, tdif.x);
    }
    if (i & 1) b[i / 2] = z; else a[i / 2] = z;
  }
  fft<T, K, E2, true, 1, Z::PITCH, true, true>(a, lds, t, row);
  fft<T, K, E2, true, 1, Z::PITCH, true, true>(b, lds, t, row);
#pragma unroll
  for (int e = 0; e < E2; ++e) {
    const cx<T> u = cmul(conjg(twiddle<T, false, L>(t + TT * e)), b[e]);
    v[e] = a[e] + u;
    v[e + E2] = a[e] - u;
  }
}

// R2C as r2c_row, input in the usual mapping, output in pair layout.
template <typename T, int N, int E>
__device__ __forceinline__ void r2c_pairs(cx<T> (&v)[E], cx<T>* lds, int t, int row) {
  using Z = ZP<T, N, ZDefaultRows<N>::value, E>;
  constexpr int L = Z::L, TT = Z::TT, E2 = E / 2, K = L / 2;
  cx<T> a[E2], b[E2];
#pragma unroll
  for (int e = 0; e < E2; ++e) {
    const cx<T> x0 = v[e], x1 = v[e + E2];
    a[e] = x0 + x1;
    b[e] = cmul(twiddle<T, false, L>(t + TT * e), x0 - x1);
  }
  fft<T, K, E2, false, 1, Z::PITCH, true, true>(a, lds, t, row);
  fft<T, K, E2, false, 1, Z::PITCH, true, true>(b, lds, t, row);
#pragma unroll
  for (int e = 0; e < E2; ++e) {
    v[2 * e] = a[e];
    v[2 * e + 1] = b[e];
  }
  cx<T> mr[E];
  mirror_pairs<T, TT, E>(v, mr, t);
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int k = 2 * (t + TT * (i / 2)) + (i & 1);
    const cx<T> zk = v[i];
    if (k == 0) {
      v[i] = mk(zk.x + zk.y, zk.x - zk.y);
    } else {
      const cx<T> zm = conjg(mr[i]);
      const cx<T> sum = zk + zm, dif = zk - zm;
      const cx<T> td = cmul(twiddle<T, false, N>(k), dif);
      v[i] = scale(sum + mk(td.y, -td.x), T(0.5));
    }
  }
}

#define ZP_SETUP                                                        \
  using Z = ZP<T, N, RW>;                                               \
  constexpr int E = Z::E, TT = Z::TT;                                   \
  __shared__ cx<T> lds[Z::RW * Z::PITCH];                               \
  const int b = blockIdx.y;                                             \
  const int t = threadIdx.x % TT, row = threadIdx.x / TT;               \
  const long long grow = (long long)blockIdx.x * Z::RW + row;           \
  const long long sbase = (long long)b * Z::SPEC + grow * Z::L;         \
  (void)sbase;                                                          \
  tw_fill<T>();

// ---- matvec core: for j = x, y, z: g_j = C2R(V_j) (V_z times i wz), times
// m, R2C, (z: times i wz).  In place on V1..V3.  The launch covers the
// blocks [blk0, blk0 + gridDim.x) (a slab of x planes); rev walks them from
// the last to the first (the y pass before it ends at the last rows, whose
// output is then still in the last-level cache).  PRE = 3 loads all three
// rows up front; PRE = 1 loads each before its use (fewer registers).
// Each workgroup also leaves the partial sum of m |grad u|^2 over its rows
// in slot 1 (per lane and row an FP32 sum of 32
// products, then FP64): with |u|^2 this gives <u, A u> of the Crank-Nicolson
// operator, because the spectral divergence is minus the adjoint of the
// spectral gradient.
template <typename T, int N, int RW, int PRE_, int OCC, int EZ, bool PAIR>
__global__ void TG_BOUNDS((ZP<T, N, RW, EZ>::NT), OCC)
k_z_matvec(cx<T>* __restrict__ V1, cx<T>* __restrict__ V2, cx<T>* __restrict__ V3,
           const T* __restrict__ m, long long m_bs, const ProbScalars* __restrict__ sc,
           double* __restrict__ part, int pred, int rev, int blk0) {
  using Z = ZP<T, N, RW, EZ>;
  constexpr int E = Z::E, TT = Z::TT;
  __shared__ cx<T> lds[Z::RW * Z::PITCH];
  __shared__ double red[NSLOT * ((Z::NT + 63) / 64)];
  const int b = blockIdx.y;
  if (pred && sc[b].done) return;
  tw_fill<T>();
  const int t = threadIdx.x % TT, row = threadIdx.x / TT;
  const int bx = blk0 + (rev ? (int)gridDim.x - 1 - (int)blockIdx.x : (int)blockIdx.x);
  const long long grow = (long long)bx * Z::RW + row;
  const long long sbase = (long long)b * Z::SPEC + grow * Z::L;
  const cx<T>* mrow = reinterpret_cast<const cx<T>*>(m + b * m_bs + grow * N);
  cx<T>* Vs[3] = {V1 + sbase, V2 + sbase, V3 + sbase};
  // spectral row in and out: position t + TT e, or pairs 2q, 2q + 1 with
  // q = t + TT e in pair layout (one 16-byte access per pair in FP32)
  auto load_row = [&](int j, cx<T>(&u)[E]) {
    if constexpr (PAIR) {
      const cx2<T>* r2 = reinterpret_cast<const cx2<T>*>(Vs[j]);
#pragma unroll
      for (int e = 0; e < E / 2; ++e) {
        const cx2<T> w = r2[t + TT * e];
        u[2 * e] = w.a;
        u[2 * e + 1] = w.b;
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) u[e] = Vs[j][t + TT * e];
    }
  };
  auto pos = [&](int i) {  // spectral position held in register i
    return PAIR ? 2 * (t + TT * (i / 2)) + (i & 1) : t + TT * i;
  };
  constexpr int PRE = PRE_;  // rows held in registers at once (1 or 3)
  // PRE = 3 keeps m in registers for all three rows; PRE = 1 re-reads the
  // m row (a cache hit after the first row) to save registers.
  cx<T> mv[PRE == 3 ? E : 1], v[PRE][E];
  double mg = 0.0;
  if constexpr (PRE == 3) {
#pragma unroll
    for (int e = 0; e < E; ++e) mv[e] = mrow[t + TT * e];
  }
#pragma unroll
  for (int j = 0; j < PRE; ++j) load_row(j, v[j]);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    cx<T>(&u)[E] = v[PRE == 3 ? j : 0];
    if (PRE == 1 && j > 0) load_row(j, u);
    if (j == 2) {
#pragma unroll
      for (int e = 0; e < E; ++e) u[e] = mul_i(u[e], (T)pos(e));
    }
    if constexpr (PAIR) c2r_pairs<T, N>(u, lds, t, row);
    else c2r_row<T, N>(u, lds, t, row);
    T sj = T(0);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cx<T> me = PRE == 3 ? mv[PRE == 3 ? e : 0] : mrow[t + TT * e];
      const cx<T> g = u[e];
      u[e] = mk(g.x * me.x, g.y * me.y);
      sj += g.x * u[e].x + g.y * u[e].y;
    }
    mg += (double)sj;
    // pin the sum here: left alone, the compiler sinks it to its use at the
    // end of the kernel and keeps its inputs live through all three rows
    asm volatile("" : "+v"(mg));
    if constexpr (PAIR) r2c_pairs<T, N>(u, lds, t, row);
    else r2c_row<T, N>(u, lds, t, row);
    if (j == 2) {
#pragma unroll
      for (int e = 0; e < E; ++e) u[e] = mul_i(u[e], (T)pos(e));
    }
    if constexpr (PAIR) {
      cx2<T>* r2 = reinterpret_cast<cx2<T>*>(Vs[j]);
#pragma unroll
      for (int e = 0; e < E / 2; ++e) {
        cx2<T> w;
        w.a = u[2 * e];
        w.b = u[2 * e + 1];
        r2[t + TT * e] = w;
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) Vs[j][t + TT * e] = u[e];
    }
  }
  double acc[NSLOT] = {mg, 0.0, 0.0, 0.0};
  block_sums<Z::NT>(acc, 1, red);
  if (threadIdx.x == 0) part_at(part, b, 1)[bx] = acc[0];
}

// ---- time-step boundary kernels (reaction halves fused around the
// transforms).  Real fields: Cin (input real field), Cst/Bst (stored
// states), m.  Spectral rows: Xs (in and/or out), Y2 (second output).
enum ZMode : int {
  ZS_FWD_FIRST = 0,  // a = R(c0) -> R2C
  ZS_FWD = 1,        // b = C2R; [store b]; c = R(b); [store c]; a = R(c) -> R2C
  ZS_FWD_LAST = 2,   // b = C2R; [store b]; c = R(b) -> store c (to Cst)
  ZS_TAN_FIRST = 3,  // a' = R'(c0) dc0 -> R2C           (Cin = dc0, Cst = c0)
  ZS_TAN = 4,        // b' = C2R; c' = R'(b) b'; a' = R'(R(b)) c' -> R2C  (Bst = b)
  ZS_TAN_LAST = 5,   // b' = C2R; c' = R'(b) b' -> store c' (Cout)
  ZS_ADJ_FIRST = 6,  // lam = Cin; head of last step -> R2C(lam), R2C(a + b)
  ZS_ADJ = 7,        // lam = C2R; tail of step n+1, head of step n -> R2C x2
  ZS_ADJ_LAST = 8    // lam = C2R; tail of step 0 -> store lam (Cout)
};

struct ZArgs {
  const void* Cin; long long cin_bs;   // real input field
  const void* Cn; long long cn_bs;     // c^n (adjoint, tangent first)
  const void* Bn; long long bn_bs;     // b^n (adjoint) / b^{n-1} (tangent)
  void* Bst; long long bst_bs;         // store b here (forward)
  void* Cst; long long cst_bs;         // store c here (forward) / output
  const void* m; long long m_bs;
  void* Xs;                            // spectral rows in/out
  void* Y2;                            // second spectral output (adjoint)
  ProbScalars* sc;
  double* part;
  void* Qr;                            // adjoint: += d J / d mr(x) (null: skip)
  double tau;
  double out_scale;                    // factor on the stored tangent output
  int want_grho;
};

template <typename T, int N, int MODE, int RW>
__global__ void __launch_bounds__((ZP<T, N, RW>::NT)) k_z_step(ZArgs a) {
  ZP_SETUP
  __shared__ double red[NSLOT * ((Z::NT + 63) / 64)];
  const long long roff = grow * N;  // real element offset of the row
  const T tau = (T)a.tau;
  const T rhof = (T)a.sc[b].rhof;
  const cx<T>* mrow = reinterpret_cast<const cx<T>*>((const T*)a.m + b * a.m_bs + roff);
  cx<T> mv[E], E2[E], v[E];
  // E = exp(rho_f m tau) for both reals of each complex slot
#pragma unroll
  for (int e = 0; e < E; ++e) {
    mv[e] = mrow[t + TT * e];
    E2[e] = mk(Tr<T>::ex(rhof * mv[e].x * tau), Tr<T>::ex(rhof * mv[e].y * tau));
  }
  cx<T>* X = reinterpret_cast<cx<T>*>(a.Xs) + sbase;
  auto ldreal = [&](const void* p, long long bs, cx<T> (&o)[E]) {
    const cx<T>* r = reinterpret_cast<const cx<T>*>((const T*)p + b * bs + roff);
#pragma unroll
    for (int e = 0; e < E; ++e) o[e] = r[t + TT * e];
  };
  auto streal = [&](void* p, long long bs, const cx<T> (&o)[E]) {
    cx<T>* r = reinterpret_cast<cx<T>*>((T*)p + b * bs + roff);
#pragma unroll
    for (int e = 0; e < E; ++e) r[t + TT * e] = o[e];
  };
  double gr = 0.0;
  // d rho contribution <lam, m tau u (1 - u)> for one pair; with Qr the
  // per-voxel lam u (1 - u) is also kept (times rho_f tau at the end: the
  // derivative in the reaction field mr at that voxel)
  cx<T> qv[E];
#pragma unroll
  for (int e = 0; e < E; ++e) qv[e] = mk(T(0), T(0));
  auto drho = [&](cx<T> lam, cx<T> u, cx<T> mm, cx<T>& q) -> double {
    const cx<T> w = mk(u.x * (T(1) - u.x), u.y * (T(1) - u.y));
    q = mk(q.x + lam.x * w.x, q.y + lam.y * w.y);
    return (double)lam.x * (double)(mm.x * tau * w.x) + (double)lam.y * (double)(mm.y * tau * w.y);
  };
  if constexpr (MODE == ZS_FWD_FIRST) {
    ldreal(a.Cin, a.cin_bs, v);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = mk(react(v[e].x, E2[e].x), react(v[e].y, E2[e].y));
    r2c_row<T, N>(v, lds, t, row);
#pragma unroll
    for (int e = 0; e < E; ++e) X[t + TT * e] = v[e];
  } else if constexpr (MODE == ZS_FWD || MODE == ZS_FWD_LAST) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = X[t + TT * e];
    c2r_row<T, N>(v, lds, t, row);
    if (a.Bst) streal(a.Bst, a.bst_bs, v);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = mk(react(v[e].x, E2[e].x), react(v[e].y, E2[e].y));
    if (a.Cst) streal(a.Cst, a.cst_bs, v);
    if constexpr (MODE == ZS_FWD) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = mk(react(v[e].x, E2[e].x), react(v[e].y, E2[e].y));
      r2c_row<T, N>(v, lds, t, row);
#pragma unroll
      for (int e = 0; e < E; ++e) X[t + TT * e] = v[e];
    }
  } else if constexpr (MODE == ZS_TAN_FIRST) {
    cx<T> c0[E];
    ldreal(a.Cin, a.cin_bs, v);
    ldreal(a.Cn, a.cn_bs, c0);
#pragma unroll
    for (int e = 0; e < E; ++e)
      v[e] = mk(react_du(c0[e].x, E2[e].x) * v[e].x, react_du(c0[e].y, E2[e].y) * v[e].y);
    r2c_row<T, N>(v, lds, t, row);
#pragma unroll
    for (int e = 0; e < E; ++e) X[t + TT * e] = v[e];
  } else if constexpr (MODE == ZS_TAN || MODE == ZS_TAN_LAST) {
    cx<T> bb[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = X[t + TT * e];
    c2r_row<T, N>(v, lds, t, row);
    ldreal(a.Bn, a.bn_bs, bb);
#pragma unroll
    for (int e = 0; e < E; ++e)
      v[e] = mk(react_du(bb[e].x, E2[e].x) * v[e].x, react_du(bb[e].y, E2[e].y) * v[e].y);
    if constexpr (MODE == ZS_TAN) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const cx<T> c = mk(react(bb[e].x, E2[e].x), react(bb[e].y, E2[e].y));
        v[e] = mk(react_du(c.x, E2[e].x) * v[e].x, react_du(c.y, E2[e].y) * v[e].y);
      }
      r2c_row<T, N>(v, lds, t, row);
#pragma unroll
      for (int e = 0; e < E; ++e) X[t + TT * e] = v[e];
    } else {
      const T os = (T)a.out_scale;
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = scale(v[e], os);
      streal(a.Cst, a.cst_bs, v);
    }
  } else {
    // adjoint modes
    cx<T> bb[E], cc[E];
    if constexpr (MODE == ZS_ADJ_FIRST) {
      ldreal(a.Cin, a.cin_bs, v);
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = X[t + TT * e];
      c2r_row<T, N>(v, lds, t, row);
    }
    if constexpr (MODE == ZS_ADJ) {
      // tail of step n+1: c1 = R(b^n), a1 = R(c1)
      ldreal(a.Bn, a.bn_bs, bb);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const cx<T> c1 = mk(react(bb[e].x, E2[e].x), react(bb[e].y, E2[e].y));
        const cx<T> a1 = mk(react(c1.x, E2[e].x), react(c1.y, E2[e].y));
        gr += drho(v[e], a1, mv[e], qv[e]);
        v[e] = mk(react_du(c1.x, E2[e].x) * v[e].x, react_du(c1.y, E2[e].y) * v[e].y);
      }
    }
    if constexpr (MODE == ZS_ADJ_FIRST) ldreal(a.Bn, a.bn_bs, bb);
    if constexpr (MODE == ZS_ADJ_LAST) {
      ldreal(a.Cn, a.cn_bs, cc);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const cx<T> a0 = mk(react(cc[e].x, E2[e].x), react(cc[e].y, E2[e].y));
        gr += drho(v[e], a0, mv[e], qv[e]);
        v[e] = mk(react_du(cc[e].x, E2[e].x) * v[e].x, react_du(cc[e].y, E2[e].y) * v[e].y);
      }
      streal(a.Cst, a.cst_bs, v);
    } else {
      // head of step n: c1 = R(b^n): g += <lam, m tau c1 (1 - c1)>; lam *= R'(b^n)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const cx<T> c1 = mk(react(bb[e].x, E2[e].x), react(bb[e].y, E2[e].y));
        gr += drho(v[e], c1, mv[e], qv[e]);
        v[e] = mk(react_du(bb[e].x, E2[e].x) * v[e].x, react_du(bb[e].y, E2[e].y) * v[e].y);
      }
      r2c_row<T, N>(v, lds, t, row);
#pragma unroll
      for (int e = 0; e < E; ++e) X[t + TT * e] = v[e];
      // s = a^n + b^n, a^n = R(c^n)
      ldreal(a.Cn, a.cn_bs, cc);
#pragma unroll
      for (int e = 0; e < E; ++e)
        v[e] = mk(react(cc[e].x, E2[e].x) + bb[e].x, react(cc[e].y, E2[e].y) + bb[e].y);
      r2c_row<T, N>(v, lds, t, row);
      cx<T>* Y2 = reinterpret_cast<cx<T>*>(a.Y2) + sbase;
#pragma unroll
      for (int e = 0; e < E; ++e) Y2[t + TT * e] = v[e];
    }
    if (a.Qr) {
      const T qs = rhof * tau;
      cx<T>* q = reinterpret_cast<cx<T>*>((T*)a.Qr + b * Z::REAL + roff);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const cx<T> o = q[t + TT * e];
        q[t + TT * e] = mk(o.x + qs * qv[e].x, o.y + qs * qv[e].y);
      }
    }
    if (a.want_grho) {
      double acc[NSLOT] = {gr, 0.0, 0.0, 0.0};
      block_sums<Z::NT>(acc, 1, red);
      if (threadIdx.x == 0) part_at(a.part, b, 0)[blockIdx.x] = acc[0];
    }
  }
}

// ---- per-voxel derivative in the diffusion field of one adjoint step:
// Qk(x) += -tau k_f sum_j (D_j mu)(x) (D_j s)(x), from the y-inverted
// gradient rows of mu (M1, M2, M3) and of s = a + b (S1, S2, S3) as the
// matvec's y pass leaves them (row 3 still needs i wz before the z
// transform).  One pass over six spectral rows and the real output row.
// Spectral rows are read in pair layout (16-byte accesses in FP32); in FP32
// the next pair of rows (and, for the last, the output row) is loaded
// before the current pair is transformed, so loads overlap the transforms.
template <typename T, int N, int RW, int OCC, bool PF>
__global__ void TG_BOUNDS((ZP<T, N, RW>::NT), OCC) k_z_qgrad(
    const cx<T>* __restrict__ M1, const cx<T>* __restrict__ M2, const cx<T>* __restrict__ M3,
    const cx<T>* __restrict__ S1, const cx<T>* __restrict__ S2, const cx<T>* __restrict__ S3,
    T* __restrict__ Qk, const ProbScalars* __restrict__ sc, double tau) {
  ZP_SETUP
  const cx<T>* Ms[3] = {M1 + sbase, M2 + sbase, M3 + sbase};
  const cx<T>* Ss[3] = {S1 + sbase, S2 + sbase, S3 + sbase};
  cx<T>* q = reinterpret_cast<cx<T>*>(Qk + b * Z::REAL + grow * N);
  auto load_pairs = [&](const cx<T>* row_, cx<T>(&u)[E]) {
    const cx2<T>* r2 = reinterpret_cast<const cx2<T>*>(row_);
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {
      const cx2<T> w = r2[t + TT * e];
      u[2 * e] = w.a;
      u[2 * e + 1] = w.b;
    }
  };
  cx<T> acc[E], u[E], w[E], un[PF ? E : 1], wn[PF ? E : 1];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = mk(T(0), T(0));
  load_pairs(Ms[0], u);
  load_pairs(Ss[0], w);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    // keep the compiler from hoisting later rows' loads above the previous
    // transforms (it would hold all six rows in registers at once)
    asm volatile("" ::: "memory");
    if constexpr (PF) {
      if (j < 2) {
        load_pairs(Ms[j + 1], un);
        load_pairs(Ss[j + 1], wn);
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) un[e] = q[t + TT * e];
      }
    } else if (j > 0) {
      load_pairs(Ms[j], u);
      load_pairs(Ss[j], w);
    }
    if (j == 2) {
#pragma unroll
      for (int i = 0; i < E; ++i) {
        // spectral position of register i; slot 0 (kz = 0 and n/2) has no z derivative
        const T kz = (T)(2 * (t + TT * (i / 2)) + (i & 1));
        u[i] = mul_i(u[i], kz);
        w[i] = mul_i(w[i], kz);
      }
    }
    c2r_pairs<T, N>(u, lds, t, row);
    c2r_pairs<T, N>(w, lds, t, row);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      acc[e] = mk(acc[e].x + u[e].x * w[e].x, acc[e].y + u[e].y * w[e].y);
      asm volatile("" : "+v"(acc[e].x), "+v"(acc[e].y));  // form the sum here
    }
    if constexpr (PF) {
      if (j < 2) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          u[e] = un[e];
          w[e] = wn[e];
        }
      }
    }
  }
  const T cs = (T)(-tau * sc[b].kf);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const cx<T> o = PF ? un[PF ? e : 0] : q[t + TT * e];
    q[t + TT * e] = mk(o.x + cs * acc[e].x, o.y + cs * acc[e].y);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_zero(T* __restrict__ dst, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256)
    dst[i] = T(0);
}

// ---------------------------------------------------------- finalizers
enum FinMode : int {
  FIN_INIT = 0,   // slots: |rhs|^2, <r,Mr>, |r|^2
  FIN_PAP = 1,    // (the step length: pcg_step_length, inside the y forward pass)
  FIN_RZ = 2,     // slots: <r,Mr>, |r|^2
  FIN_GRHO = 3,   // slot: g_rho increment
  FIN_GK = 4,     // slot: spectral <Am mu, s>
  FIN_J = 5,      // slot: sum (c - d)^2
  FIN_MMAX = 6    // slot: partial max(m)
};

// One workgroup of NT threads per problem (NT = 1024 for the PCG-loop
// finalizers, whose partial sums come from thousands of workgroups).
template <int MODE, int NT = 256>
__global__ void __launch_bounds__(NT)
k_finalize(ProbScalars* __restrict__ sc, const double* __restrict__ part, int nblk,
           double scale_, double rtol, int maxit) {
  constexpr int NW = NT / 64;
  __shared__ double red[NSLOT * NW];
  const int b = blockIdx.x;
  ProbScalars& S = sc[b];
  if (MODE == FIN_RZ && S.done) return;
  constexpr int ns = MODE == FIN_INIT ? 3 : MODE == FIN_RZ ? 2 : 1;
  double acc[NSLOT] = {0.0, 0.0, 0.0, 0.0};
  if constexpr (MODE == FIN_MMAX) {
    double mx = 0.0;
    for (int i = threadIdx.x; i < nblk; i += NT) mx = fmax(mx, part_at((double*)part, b, 0)[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 0; w < NW; ++w) mx = fmax(mx, red[w]);
      S.mmax = mx;
      S.kbar = S.kf * mx;
    }
    return;
  }
  for (int s = 0; s < ns; ++s)
    for (int i = threadIdx.x; i < nblk; i += NT) acc[s] += part_at((double*)part, b, s)[i];
  block_sums<NT>(acc, ns, red);
  if (threadIdx.x != 0) return;
  if constexpr (MODE == FIN_INIT) {
    S.rhs2 = acc[0] * scale_;
    S.rho = acc[1];
    S.rr = acc[2] * scale_;
    S.tol2 = rtol * rtol * S.rhs2;
    S.its = 0;
    S.first = 1;
    S.solves += 1;
    S.done = (S.rr <= S.tol2) ? 1 : 0;
    if (S.status & STAT_BAD_PARAM) {
      S.done = 1;  // invalid k_f / rho_f: no solve
    } else if (!isfinite(S.rr) || !isfinite(S.rhs2)) {
      S.status |= STAT_NONFINITE;
      S.done = 1;
    }
    if (S.done) {
      const double rel = S.rhs2 > 0 ? sqrt(S.rr / S.rhs2) : 0.0;
      S.worst = fmax(S.worst, rel);
    }
  } else if constexpr (MODE == FIN_RZ) {
    const double rho_new = acc[0];
    S.rr = acc[1] * scale_;
    S.its += 1;
    S.its_total += 1;
    if (S.its > S.its_max) S.its_max = S.its;
    S.beta = rho_new / S.rho;
    S.rho = rho_new;
    S.first = 0;
    bool fin = false;
    if (!isfinite(S.rr)) {
      S.status |= STAT_NONFINITE;
      fin = true;
    } else if (S.rr <= S.tol2) {
      fin = true;
    } else if (S.its >= maxit) {
      S.status |= STAT_NOT_CONVERGED;
      fin = true;
    }
    if (fin) {
      S.done = 1;
      const double rel = S.rhs2 > 0 ? sqrt(S.rr / S.rhs2) : 0.0;
      S.worst = fmax(S.worst, rel);
    }
  } else if constexpr (MODE == FIN_GRHO) {
    S.g_rho += acc[0] * scale_;
  } else if constexpr (MODE == FIN_GK) {
    S.g_k += acc[0] * scale_;
  } else if constexpr (MODE == FIN_J) {
    S.J = acc[0] * scale_;
  }
}

// Copy the done flags of all problems to a host-visible array.
__global__ void k_done_flags(const ProbScalars* __restrict__ sc, int* __restrict__ out, int nb) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) out[i] = sc[i].done;
}

// Reset per-call scalars and load parameters.
__global__ void k_init_scalars(ProbScalars* __restrict__ sc, const double* __restrict__ rho,
                               long long rho_bs, const double* __restrict__ kf, long long kf_bs,
                               int nb) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  ProbScalars S{};
  S.rhof = rho[b * rho_bs];
  S.kf = kf[b * kf_bs];
  S.done = 1;
  if (!(S.kf >= 0.0) || !isfinite(S.kf) || !isfinite(S.rhof)) S.status = STAT_BAD_PARAM;
  sc[b] = S;
}

// Reset the per-call accumulators only (keep kf, rho, kbar, mmax).
__global__ void k_reset_call(ProbScalars* __restrict__ sc, int nb) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  ProbScalars& S = sc[b];
  S.g_rho = 0.0;
  S.g_k = 0.0;
  S.worst = 0.0;
  S.status &= STAT_BAD_PARAM;  // a parameter error of the forward stays
  S.its_total = 0;
  S.solves = 0;
  S.its_max = 0;
  S.done = 1;
}

// Hessian directions take k_f, rho_f and the preconditioner of problem 0.
__global__ void k_copy_dir_scalars(const ProbScalars* __restrict__ src, ProbScalars* __restrict__ dst,
                                   int nd) {
  int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= nd) return;
  ProbScalars S{};
  S.kf = src[0].kf;
  S.rhof = src[0].rhof;
  S.kbar = src[0].kbar;
  S.mmax = src[0].mmax;
  S.status = src[0].status & STAT_BAD_PARAM;
  S.done = 1;
  dst[d] = S;
}

// dst = src over n elements of a packed spectrum batch (graph-safe copy).
template <typename T>
__global__ void __launch_bounds__(256) k_copy_spec(cx<T>* __restrict__ dst,
                                                   const cx<T>* __restrict__ src, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256)
    dst[i] = src[i];
}

// Copy per-problem gradients out (device -> caller's device buffers).
__global__ void k_emit_grads(const ProbScalars* __restrict__ sc, double* J, double* grho,
                             double* gkf, int nb) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  if (J) J[b] = sc[b].J;
  if (grho) grho[b] = sc[b].g_rho;
  if (gkf) gkf[b] = sc[b].g_k;
}

// ------------------------------------------------------- real-field ops
template <typename T, int N>
struct RP {
  static constexpr long long REAL = (long long)N * N * N;
  static constexpr int NBLK = (REAL / 256 / 8) < 1024 ? (int)((REAL / 256 / 8) > 0 ? REAL / 256 / 8 : 1) : 1024;
};

// partial max of m
template <typename T, int N>
__global__ void __launch_bounds__(256) k_mmax(const T* __restrict__ m, long long m_bs,
                                              double* __restrict__ part) {
  __shared__ double red[4];
  const int b = blockIdx.y;
  double mx = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < RP<T, N>::REAL;
       i += (long long)gridDim.x * 256)
    mx = fmax(mx, (double)m[b * m_bs + i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0)
    part_at(part, b, 0)[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// lam = h3 (c - d); partial sum (c - d)^2
template <typename T, int N>
__global__ void __launch_bounds__(256) k_misfit(const T* __restrict__ c, const T* __restrict__ d,
                                                T* __restrict__ lam, double h3,
                                                double* __restrict__ part) {
  __shared__ double red[NSLOT * 4];
  const int b = blockIdx.y;
  const long long off = (long long)b * RP<T, N>::REAL;
  double acc[NSLOT] = {0.0, 0.0, 0.0, 0.0};
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < RP<T, N>::REAL;
       i += (long long)gridDim.x * 256) {
    const double r = (double)c[off + i] - (double)d[off + i];
    lam[off + i] = (T)(h3 * r);
    acc[0] += r * r;
  }
  block_sums<256>(acc, 1, red);
  if (threadIdx.x == 0) part_at(part, b, 0)[blockIdx.x] = acc[0];
}

// Misfit with the anatomy labels (Sec. 2.1 objective): the tumor-masked
// healthy labels m_l (1 - c) against the patient labels mP_l, l < nlab,
// fields [b][l][n^3]:
//   lam = h3 [(c - d) - sum_l m_l (m_l (1 - c) - mP_l)],
//   partial sum of (c - d)^2 + sum_l (m_l (1 - c) - mP_l)^2.
template <typename T, int N>
__global__ void __launch_bounds__(256) k_misfit_labels(const T* __restrict__ c,
                                                       const T* __restrict__ d, int nlab,
                                                       const T* __restrict__ mlab,
                                                       const T* __restrict__ mpat,
                                                       T* __restrict__ lam, double h3,
                                                       double* __restrict__ part) {
  __shared__ double red[NSLOT * 4];
  constexpr long long R = RP<T, N>::REAL;
  const int b = blockIdx.y;
  const long long off = (long long)b * R;
  const long long loff = (long long)b * nlab * R;
  double acc[NSLOT] = {0.0, 0.0, 0.0, 0.0};
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < R;
       i += (long long)gridDim.x * 256) {
    const double ci = (double)c[off + i];
    const double r = ci - (double)d[off + i];
    double g = r, s = r * r;
    for (int l = 0; l < nlab; ++l) {
      const double ml = (double)mlab[loff + l * R + i];
      const double e = ml * (1.0 - ci) - (double)mpat[loff + l * R + i];
      g -= ml * e;
      s += e * e;
    }
    lam[off + i] = (T)(h3 * g);
    acc[0] += s;
  }
  block_sums<256>(acc, 1, red);
  if (threadIdx.x == 0) part_at(part, b, 0)[blockIdx.x] = acc[0];
}

// d = x - a-hat over n complex values: the increment b - a of a forward step.
template <typename T>
__global__ void __launch_bounds__(256) k_increment(const cx<T>* __restrict__ X,
                                                   const cx<T>* __restrict__ Ah,
                                                   cx<T>* __restrict__ D, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256)
    D[i] = X[i] - Ah[i];
}

// Gaussian factors g[b][i][a][j] = exp(-d(x_j, c_ia)^2 / (2 sigma^2)),
// minimum-image periodic distance (Sec. 2.1 initial condition, Sec. 4.1
// basis of standard deviation sigma).
__global__ void k_basis_factors(const double* __restrict__ centres, long long c_bs,
                                double* __restrict__ g, int n, int n_p, double sigma) {
  const int b = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_p * 3 * n) return;
  const int j = idx % n, a = (idx / n) % 3, i = idx / (3 * n);
  const double two_pi = 6.283185307179586476925286766559;
  const double x = two_pi * (double)j / (double)n;
  double d = fabs(x - centres[b * c_bs + i * 3 + a]);
  d = fmod(d, two_pi);
  d = fmin(d, two_pi - d);
  g[((size_t)b * n_p + i) * 3 * n + a * n + j] = exp(-d * d / (2.0 * sigma * sigma));
}

// The basis is separable: Phi_i(x, y, z) = gx_i[x] gy_i[y] gz_i[z] (the
// rows of k_basis_factors), so both Phi p and Phi^T lam are contractions
// over the Gaussians i and the z axis of a grid row r = (x, y) with the z
// factors: [n^2 x n_p] by [n_p x n] and [n^2 x n] by [n x n_p] products.
// They run as register-tiled products in FP64 (k_phi and k_phit: workgroups
// of 256 threads, 64 rows per workgroup, operands staged through LDS; from
// n = 128 on Phi p runs as k_phi_w, with the row factors in scalar
// registers), reading and writing each field once.

// ---- c0 = w Phi p (w: the CSF mask of Sec. 2.1, or none): for each row
// r = (x, y), c0[r][z] = w sum_i a_i(r) gz_i[z] with a_i(r) = p_i gx_i[x]
// gy_i[y].  A workgroup computes 64 rows x KZ z values; thread (tr, tz)
// holds rows tr + TR q (q < RT) and z = tz + TZ a (a < ZT); the Gaussians
// go through LDS in chunks of 32 (about 34 KB of LDS: four workgroups per
// CU).
template <int N>
struct PhiK {
  static constexpr int ROWS = 64;                        // rows per workgroup
  static constexpr int KZ = N < 64 ? N : 64;             // z values per workgroup
  static constexpr int ZT = KZ >= 64 ? 4 : (KZ >= 32 ? 2 : 1);  // z per thread
  static constexpr int TZ = KZ / ZT;                     // threads along z
  static constexpr int TR = 256 / TZ;                    // threads along rows
  static constexpr int RT = ROWS / TR;                   // rows per thread
  static constexpr int GC = 32;                          // Gaussians per LDS chunk
  static constexpr int NBX = N * N / ROWS;               // row blocks
  static constexpr int NBZ = N / KZ;                     // z blocks
  static_assert(RT >= 1 && TR * RT == ROWS && TZ * ZT == KZ, "Phi tile shape");
};

template <typename T, int N>
__global__ void __launch_bounds__(256) k_phi(const double* __restrict__ p, long long p_bs,
                                             const double* __restrict__ g, long long g_bs,
                                             const T* __restrict__ mask, long long mask_bs,
                                             T* __restrict__ out, long long out_bs, int n_p) {
  using K = PhiK<N>;
  constexpr int SA = K::ROWS * K::GC / 256, SZ = K::GC * K::KZ / 256;  // staged per thread
  static_assert(SA * 256 == K::ROWS * K::GC && SZ * 256 == K::GC * K::KZ, "Phi staging");
  __shared__ double sa[K::ROWS][K::GC + 1];  // a_i(r), rows x Gaussians
  __shared__ double sz[K::GC][K::KZ + 1];    // gz_i[z], Gaussians x z
  const int b = blockIdx.y;
  const int t = threadIdx.x, tz = t % K::TZ, tr = t / K::TZ;
  const long long r0 = (long long)(blockIdx.x % K::NBX) * K::ROWS;
  const int z0 = (blockIdx.x / K::NBX) * K::KZ;
  const double* gb = g + b * g_bs;
  const double* pb = p + b * p_bs;
  double acc[K::RT][K::ZT];
#pragma unroll
  for (int q = 0; q < K::RT; ++q)
#pragma unroll
    for (int a = 0; a < K::ZT; ++a) acc[q][a] = 0.0;
  // the next chunk's operands are fetched into registers while the current
  // one is multiplied out of LDS
  double ra[SA], rz[SZ];
  auto fetch = [&](int i0) {
#pragma unroll
    for (int u = 0; u < SA; ++u) {
      const int e = t + 256 * u, rr = e / K::GC, i = i0 + e % K::GC;
      const long long r = r0 + rr;
      ra[u] = i < n_p ? pb[i] * gb[((size_t)i * 3) * N + r / N] * gb[((size_t)i * 3 + 1) * N + r % N]
                      : 0.0;
    }
#pragma unroll
    for (int u = 0; u < SZ; ++u) {
      const int e = t + 256 * u, i = i0 + e / K::KZ;
      rz[u] = i < n_p ? gb[((size_t)i * 3 + 2) * N + z0 + e % K::KZ] : 0.0;
    }
  };
  fetch(0);
  for (int i0 = 0; i0 < n_p; i0 += K::GC) {
#pragma unroll
    for (int u = 0; u < SA; ++u) {
      const int e = t + 256 * u;
      sa[e / K::GC][e % K::GC] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < SZ; ++u) {
      const int e = t + 256 * u;
      sz[e / K::KZ][e % K::KZ] = rz[u];
    }
    __syncthreads();
    if (i0 + K::GC < n_p) fetch(i0 + K::GC);
    const int ni = min(K::GC, n_p - i0);
    for (int ii = 0; ii < ni; ++ii) {
      double av[K::RT], zv[K::ZT];
#pragma unroll
      for (int q = 0; q < K::RT; ++q) av[q] = sa[tr + K::TR * q][ii];
#pragma unroll
      for (int a = 0; a < K::ZT; ++a) zv[a] = sz[ii][tz + K::TZ * a];
#pragma unroll
      for (int q = 0; q < K::RT; ++q)
#pragma unroll
        for (int a = 0; a < K::ZT; ++a) acc[q][a] = fma(av[q], zv[a], acc[q][a]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < K::RT; ++q) {
    const long long o = (r0 + tr + K::TR * q) * N + z0 + tz;
#pragma unroll
    for (int a = 0; a < K::ZT; ++a) {
      double v = acc[q][a];
      if (mask) v *= (double)mask[b * mask_bs + o + K::TZ * a];
      out[b * out_bs + o + K::TZ * a] = (T)v;
    }
  }
}

// ---- c0 = w Phi p for n >= 128, without LDS: lane l holds z = l + 64 k
// (k < n/64) of RW rows (x, y0 .. y0 + RW - 1) that are the same for the
// whole wave, so per Gaussian the row factors a_i(r) = (p_i gx_i[x]) gy_i[y]
// are wave-uniform values (p_i, gx_i[x] and gy_i[y] come through the scalar
// cache) and only gz_i[z] is per lane.  Per Gaussian a lane does
// RW n/64 = 32 multiply-adds and RW + 1 products; stores are 64 consecutive
// z per wave.  The sums run over i in the same order and with the same
// rounding as k_phi.
template <int N>
struct PhiW {
  static constexpr int ZT = N / 64;                // z values per lane
  static constexpr int RW = 32 / ZT;               // rows per wave
  static constexpr int WV = N >= 256 ? 4 : 2;      // waves per workgroup
  static constexpr int NBLK = N * N / (RW * WV);   // workgroups per problem
  static_assert(N >= 128 && N % RW == 0, "PhiW needs n >= 128");
};

template <typename T, int N>
__global__ void TG_BOUNDS(64 * PhiW<N>::WV, 2)
k_phi_w(const double* __restrict__ p, long long p_bs, const double* __restrict__ g,
        long long g_bs, const T* __restrict__ mask, long long mask_bs, T* __restrict__ out,
        long long out_bs, int n_p) {
  using K = PhiW<N>;
  constexpr int ZT = K::ZT, RW = K::RW;
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r0 = (blockIdx.x * K::WV + wv) * RW;   // first row of this wave
  const int x = r0 / N, y0 = r0 % N;
  const double* gb = g + b * g_bs;
  const double* pb = p + b * p_bs;
  double acc[RW][ZT];
#pragma unroll
  for (int j = 0; j < RW; ++j)
#pragma unroll
    for (int k = 0; k < ZT; ++k) acc[j][k] = 0.0;
  // Two operand sets alternate: the operands of Gaussian i + 1 (clamped to
  // the last one) are fetched while Gaussian i is multiplied.  Scalar loads
  // can only be waited for all together, so each fetch is issued after the
  // first use of the other set (the scheduling barriers keep that order):
  // the wait before that use then covers only the loads of one Gaussian
  // earlier.  (Loaded as vector loads instead, the uniform row factors cost
  // 4 KB of L1 return traffic per wave and Gaussian: twice as slow.)
  double zs[2][ZT], gys[2][RW], ps[2], gxs[2];
  auto fetch = [&](int st, int i) {
#pragma unroll
    for (int k = 0; k < ZT; ++k) zs[st][k] = gb[((size_t)i * 3 + 2) * N + lane + 64 * k];
#pragma unroll
    for (int j = 0; j < RW; ++j) gys[st][j] = gb[((size_t)i * 3 + 1) * N + y0 + j];
    ps[st] = pb[i];
    gxs[st] = gb[((size_t)i * 3) * N + x];
  };
  auto gauss = [&](int st, int i) {
    const double w = ps[st] * gxs[st];
    __builtin_amdgcn_sched_barrier(0);
    fetch(st ^ 1, min(i + 1, n_p - 1));
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      const double a = w * gys[st][j];
#pragma unroll
      for (int k = 0; k < ZT; ++k) acc[j][k] = fma(a, zs[st][k], acc[j][k]);
    }
  };
  if (n_p > 0) fetch(0, 0);
  for (int i = 0; i < n_p; i += 2) {
    gauss(0, i);
    if (i + 1 < n_p) gauss(1, i + 1);
  }
#pragma unroll
  for (int j = 0; j < RW; ++j) {
    const long long o = (long long)(r0 + j) * N + lane;
#pragma unroll
    for (int k = 0; k < ZT; ++k) {
      double v = acc[j][k];
      if (mask) v *= (double)mask[b * mask_bs + o + 64 * k];
      out[b * out_bs + o + 64 * k] = (T)v;
    }
  }
}

// ---- Phi^T (w lam): for each row r = (x, y), T_i(r) = sum_z gz_i[z]
// (w lam)[r][z]; each workgroup of 64 rows then reduces sum_r gx_i[x]
// gy_i[y] T_i(r) into partphi[b][i][block] (k_phit_final adds the blocks
// in a fixed order).  Thread (tr, ti) holds rows tr + 16 q and Gaussians
// ti + 16 a (q, a < 4) of a 64 x 64 tile; z goes through LDS in chunks of
// KC = 64; grid.z walks the Gaussians in blocks of 64.  lam (times the mask)
// is read once per Gaussian block.
template <int N>
struct PhiTK {
  static constexpr int ROWS = 64;
  static constexpr int G = 64;                 // Gaussians per workgroup
  static constexpr int KC = N < 64 ? N : 64;   // z values per LDS chunk
  static constexpr int NBLK = N * N / ROWS;    // partial sums per Gaussian
};

template <typename T, int N>
__global__ void __launch_bounds__(256) k_phit(const T* __restrict__ lam, long long lam_bs,
                                              const double* __restrict__ g, long long g_bs,
                                              const T* __restrict__ mask, long long mask_bs,
                                              double* __restrict__ partphi, int n_p) {
  using K = PhiTK<N>;
  constexpr int SL = K::ROWS * K::KC / 256, SG = K::G * K::KC / 256;  // staged per thread
  static_assert(SL * 256 == K::ROWS * K::KC && SG * 256 == K::G * K::KC, "Phi^T staging");
  __shared__ T sl[K::ROWS][K::KC + 1];       // (w lam), rows x z, in its own precision
  __shared__ double sg[K::G][K::KC + 1];     // gz_i[z], Gaussians x z
  __shared__ double red[16][K::G];
  const int b = blockIdx.y, gi0 = blockIdx.z * K::G;
  const int t = threadIdx.x, ti = t % 16, tr = t / 16;
  const long long r0 = (long long)blockIdx.x * K::ROWS;
  const double* gb = g + b * g_bs;
  const T* lb = lam + b * lam_bs;
  const T* mb = mask ? mask + b * mask_bs : nullptr;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[a][q] = 0.0;
  // the next z chunk is fetched into registers while the current one is
  // multiplied out of LDS
  T rl[SL];
  double rg[SG];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < SL; ++u) {
      const int e = t + 256 * u;
      const long long o = (r0 + e / K::KC) * N + k0 + e % K::KC;
      T v = lb[o];
      if (mb) v *= mb[o];
      rl[u] = v;
    }
#pragma unroll
    for (int u = 0; u < SG; ++u) {
      const int e = t + 256 * u, i = gi0 + e / K::KC;
      rg[u] = i < n_p ? gb[((size_t)i * 3 + 2) * N + k0 + e % K::KC] : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < N; k0 += K::KC) {
#pragma unroll
    for (int u = 0; u < SL; ++u) {
      const int e = t + 256 * u;
      sl[e / K::KC][e % K::KC] = rl[u];
    }
#pragma unroll
    for (int u = 0; u < SG; ++u) {
      const int e = t + 256 * u;
      sg[e / K::KC][e % K::KC] = rg[u];
    }
    __syncthreads();
    if (k0 + K::KC < N) fetch(k0 + K::KC);
    for (int kk = 0; kk < K::KC; ++kk) {
      double lv[4], gv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) lv[q] = (double)sl[tr + 16 * q][kk];
#pragma unroll
      for (int a = 0; a < 4; ++a) gv[a] = sg[ti + 16 * a][kk];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[a][q] = fma(gv[a], lv[q], acc[a][q]);
    }
    __syncthreads();
  }
  // weight each row by gx_i[x] gy_i[y] and sum this thread's four rows
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = gi0 + ti + 16 * a;
    double s = 0.0;
    if (i < n_p) {
      const double* gx = gb + (size_t)i * 3 * N;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const long long r = r0 + tr + 16 * q;
        s += acc[a][q] * (gx[r / N] * gx[N + r % N]);
      }
    }
    red[tr][ti + 16 * a] = s;
  }
  __syncthreads();
  if (t < K::G && gi0 + t < n_p) {
    double s = 0.0;
    for (int k = 0; k < 16; ++k) s += red[k][t];
    partphi[((size_t)b * n_p + gi0 + t) * K::NBLK + blockIdx.x] = s;
  }
}

__global__ void __launch_bounds__(256) k_phit_final(const double* __restrict__ partphi,
                                                    int nblk, int n_p, double* __restrict__ out,
                                                    long long out_bs) {
  __shared__ double red[NSLOT * 4];
  const int b = blockIdx.y, i = blockIdx.x;
  double acc[NSLOT] = {0.0, 0.0, 0.0, 0.0};
  const double* src = partphi + ((size_t)b * n_p + i) * nblk;
  for (int k = threadIdx.x; k < nblk; k += 256) acc[0] += src[k];
  block_sums<256>(acc, 1, red);
  if (threadIdx.x == 0) out[b * out_bs + i] = acc[0];
}

}  // namespace
}  // namespace tg
