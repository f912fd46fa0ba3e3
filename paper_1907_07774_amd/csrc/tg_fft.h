// Register/LDS radix-staged FFT building blocks for gfx950 (CDNA4, wave64).
//
// The spatial discretization takes all derivatives with 3D Fourier
// transforms on a regular periodic grid (paper, Sec. 3.3).  The transforms
// here are Stockham autosort FFTs: each thread keeps E complex values in
// registers, performs E/R radix-R butterflies per stage, and exchanges
// through LDS between stages.  Register e of thread t holds position
// t + (L/E) e both before the first stage and after the last one, so the
// callers load and store global memory with that mapping.
#pragma once
#include <hip/hip_runtime.h>

namespace tg {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) { cx<T> r; r.x = a; r.y = b; return r; }
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return mk(a.x * s, a.y * s); }
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return mk(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rot_mi(cx<T> a) { return INV ? mk(-a.y, a.x) : mk(a.y, -a.x); }
// i * s * a for real s
template <typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a, T s) { return mk(-a.y * s, a.x * s); }

// Twiddle table w[k] = exp(-2 pi i k / TW_N), k < TW_N, filled once per
// device by the host (long double cos/sin rounded to the type).  Each
// translation unit has its own copy and its own fill routine.
constexpr int TW_N = 512;
static __device__ cx<double> g_tw64[TW_N];
static __device__ cx<float> g_tw32[TW_N];

template <typename T> struct TwTab;
template <> struct TwTab<double> {
  static __device__ __forceinline__ cx<double> get(int k) { return g_tw64[k]; }
};
template <> struct TwTab<float> {
  static __device__ __forceinline__ cx<float> get(int k) { return g_tw32[k]; }
};

// Per-workgroup LDS copy of the table.  Every kernel that runs an FFT calls
// tw_fill() once, with all its threads, before its first transform; the
// per-stage twiddle reads then go to LDS instead of through the vector
// memory pipeline (where, reloaded for every transform, they outnumbered
// the data loads several times over).
// The LDS copy holds the TW_LDS-th roots (every TW_N / TW_LDS-th entry),
// enough for transforms up to the largest grid, n = 256.
constexpr int TW_LDS = 256;
template <typename T>
__device__ __forceinline__ cx<T>* tw_lds() {
  __shared__ cx<T> s[TW_LDS];
  return s;
}
template <typename T>
__device__ __forceinline__ void tw_fill() {
  cx<T>* s = tw_lds<T>();
  for (int i = threadIdx.x; i < TW_LDS; i += blockDim.x) s[i] = TwTab<T>::get(i * (TW_N / TW_LDS));
  __syncthreads();
}

// exp(-+ 2 pi i k / M) for M dividing TW_LDS
template <typename T, bool INV, int M>
__device__ __forceinline__ cx<T> twiddle(int k) {
  static_assert(M <= TW_LDS && TW_LDS % M == 0, "twiddle order exceeds the LDS table");
  cx<T> w = tw_lds<T>()[(k * (TW_LDS / M)) & (TW_LDS - 1)];
  return INV ? conjg(w) : w;
}

// ---------------------------------------------------------------- DFTs
// In-place R-point DFT, natural-order output X[k] = sum_q x[q] W_R^{kq},
// W_R = exp(-2 pi i / R) (forward) or its conjugate (inverse).
template <typename T, bool INV>
__device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
  cx<T> t = a - b;
  a = a + b;
  b = t;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cx<T>& x0, cx<T>& x1, cx<T>& x2, cx<T>& x3) {
  cx<T> s02 = x0 + x2, d02 = x0 - x2, s13 = x1 + x3, d13 = rot_mi<T, INV>(x1 - x3);
  x0 = s02 + s13;
  x2 = s02 - s13;
  x1 = d02 + d13;
  x3 = d02 - d13;
}

template <typename T>
struct K8 {
  static constexpr T r = T(0.70710678118654752440084436210484903928L);
};
template <typename T>
struct K16 {
  static constexpr T c = T(0.92387953251128675612818318939678828682L);  // cos(pi/8)
  static constexpr T s = T(0.38268343236508977172845998403039886676L);  // sin(pi/8)
};

// multiply by W_8^k (forward) or conj (inverse) for k = 1, 2, 3
template <typename T, bool INV, int K>
__device__ __forceinline__ cx<T> w8(cx<T> a) {
  constexpr T r = K8<T>::r;
  if constexpr (K == 0) return a;
  else if constexpr (K == 2) return rot_mi<T, INV>(a);
  else if constexpr (K == 1) {
    // (1 -+ i)/sqrt2
    return INV ? mk((a.x - a.y) * r, (a.x + a.y) * r) : mk((a.x + a.y) * r, (a.y - a.x) * r);
  } else {
    // (-1 -+ i)/sqrt2
    return INV ? mk((-a.x - a.y) * r, (a.x - a.y) * r) : mk((a.y - a.x) * r, (-a.x - a.y) * r);
  }
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cx<T>* v, int s) {
  // v[q*s], q = 0..7
  cx<T> e0 = v[0], e1 = v[2 * s], e2 = v[4 * s], e3 = v[6 * s];
  cx<T> o0 = v[s], o1 = v[3 * s], o2 = v[5 * s], o3 = v[7 * s];
  dft4<T, INV>(e0, e1, e2, e3);
  dft4<T, INV>(o0, o1, o2, o3);
  o1 = w8<T, INV, 1>(o1);
  o2 = w8<T, INV, 2>(o2);
  o3 = w8<T, INV, 3>(o3);
  v[0] = e0 + o0;       v[4 * s] = e0 - o0;
  v[s] = e1 + o1;       v[5 * s] = e1 - o1;
  v[2 * s] = e2 + o2;   v[6 * s] = e2 - o2;
  v[3 * s] = e3 + o3;   v[7 * s] = e3 - o3;
}

// multiply by W_16^k (forward) or conj (inverse), k = 1..7
template <typename T, bool INV, int K>
__device__ __forceinline__ cx<T> w16(cx<T> a) {
  constexpr T c = K16<T>::c, s = K16<T>::s, r = K8<T>::r;
  // forward W16^k = cos(2 pi k/16) - i sin(2 pi k/16)
  constexpr T cr = K == 1 ? c : K == 2 ? r : K == 3 ? s : K == 4 ? T(0) : K == 5 ? -s : K == 6 ? -r : -c;
  constexpr T si = K == 1 ? s : K == 2 ? r : K == 3 ? c : K == 4 ? T(1) : K == 5 ? c : K == 6 ? r : s;
  constexpr T im = INV ? si : -si;
  return mk(a.x * cr - a.y * im, a.x * im + a.y * cr);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft16(cx<T>* v, int s) {
  cx<T> e[8], o[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    e[q] = v[(2 * q) * s];
    o[q] = v[(2 * q + 1) * s];
  }
  dft8<T, INV>(e, 1);
  dft8<T, INV>(o, 1);
  o[1] = w16<T, INV, 1>(o[1]);
  o[2] = w16<T, INV, 2>(o[2]);
  o[3] = w16<T, INV, 3>(o[3]);
  o[4] = w16<T, INV, 4>(o[4]);
  o[5] = w16<T, INV, 5>(o[5]);
  o[6] = w16<T, INV, 6>(o[6]);
  o[7] = w16<T, INV, 7>(o[7]);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v[k * s] = e[k] + o[k];
    v[(k + 8) * s] = e[k] - o[k];
  }
}

template <typename T, bool INV, int R>
__device__ __forceinline__ void dftR(cx<T>* v, int s) {
  if constexpr (R == 2) dft2<T, INV>(v[0], v[s]);
  else if constexpr (R == 4) dft4<T, INV>(v[0], v[s], v[2 * s], v[3 * s]);
  else if constexpr (R == 8) dft8<T, INV>(v, s);
  else dft16<T, INV>(v, s);
}

// ------------------------------------------------------- Stockham stages
// Barrier between LDS exchange phases: the whole workgroup, or only the
// wavefront when every transform lives inside one wave (then waves run
// independently and only need their own LDS writes ordered before reads).
template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// LDS addressing: element (position p, column c) lives at lds[p*PS + c*CS],
// or with PAD at lds[p + p/E + c*CS] (PS = 1): one spare slot after every E
// positions, so the first stage's stride-E writes from the lanes of a row
// fall in distinct banks (the row pitch CS must be at least L + L/E).
template <typename T, int L, int E, int PS, int CS, bool PAD>
__device__ __forceinline__ int lds_at(int p, int col) {
  if constexpr (PAD) {
    static_assert(PS == 1 && CS >= L + L / E, "padded layout is for contiguous rows");
    return p + p / E + col * CS;
  } else {
    return p * PS + col * CS;
  }
}

template <typename T, int L, int E, bool INV, int PS, int CS, int Ns, bool WAVE = false,
          bool PAD = false>
struct Stockham {
  static __device__ __forceinline__ void run(cx<T> (&v)[E], cx<T>* lds, int t, int col) {
    constexpr int R = (L / Ns >= E) ? E : (L / Ns);
    constexpr int TT = L / E;
    constexpr int NB = E / R;
    static_assert(L % (Ns * R) == 0, "bad radix schedule");
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = t + b * TT;
      const int k = j & (Ns - 1);
      cx<T> w[R];
#pragma unroll
      for (int r = 0; r < R; ++r) w[r] = v[b + r * NB];
      if constexpr (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) w[r] = cmul(w[r], twiddle<T, INV, Ns * R>(r * k));
      }
      dftR<T, INV, R>(w, 1);
#pragma unroll
      for (int r = 0; r < R; ++r) v[b + r * NB] = w[r];
    }
    if constexpr (Ns * R < L) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = t + b * TT;
        const int k = j & (Ns - 1);
        const int base = (j / Ns) * Ns * R + k;
        if constexpr (PAD && Ns == 1 && R == E) {
          // positions j E + r: padded index j (E + 1) + r
          const int wb = t * (E + 1) + col * CS;
#pragma unroll
          for (int r = 0; r < R; ++r) lds[wb + b * TT * (E + 1) + r] = v[b + r * NB];
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r)
            lds[lds_at<T, L, E, PS, CS, PAD>(base + r * Ns, col)] = v[b + r * NB];
        }
      }
      lds_sync<WAVE>();
      if constexpr (PAD) {
        // positions t + e TT with t < TT: padded index t + t/E + e TT + (e TT)/E
        static_assert(E % TT == 0 || TT % E == 0, "padded read needs E | TT or TT | E");
        const int rb = t + t / E + col * CS;
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = lds[rb + e * TT + (e * TT) / E];
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = lds[lds_at<T, L, E, PS, CS, PAD>(t + e * TT, col)];
      }
      lds_sync<WAVE>();
      Stockham<T, L, E, INV, PS, CS, Ns * R, WAVE, PAD>::run(v, lds, t, col);
    }
  }
};

// Full L-point FFT of the values held by (t, col); in and out mapping:
// v[e] <-> position t + (L/E) e.
template <typename T, int L, int E, bool INV, int PS, int CS, bool WAVE = false, bool PAD = false>
__device__ __forceinline__ void fft(cx<T> (&v)[E], cx<T>* lds, int t, int col) {
  Stockham<T, L, E, INV, PS, CS, 1, WAVE, PAD>::run(v, lds, t, col);
}

// Elements-per-thread choice for an L-point transform.
template <int L>
struct FftE {
  static constexpr int value = L <= 16 ? L : (L == 32 || L == 64) ? 8 : 16;
};

}  // namespace tg
