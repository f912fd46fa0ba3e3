// Launch tables: the transform passes exist in several tile shapes (pencils
// per x/y workgroup, rows per z workgroup); a plan picks one of each at run
// time (defaults or the autotuner's choice) without recompiling.
#pragma once
#include <hip/hip_ext.h>

#include "tg_kernels.h"

namespace tg {

// Kernel timer hand-off: when the solver's timer has events pending for
// the next launch, the launch records them with the kernel's own dispatch
// (hipExtLaunchKernelGGL) instead of separate event packets around it,
// which would add queue gaps of several microseconds per timed launch.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
inline LaunchEvents& pending_events() {
  static thread_local LaunchEvents e;
  return e;
}
template <typename K, typename... A>
inline void klaunch(K kernel, dim3 grid, dim3 block, hipStream_t st, A... args) {
  LaunchEvents& e = pending_events();
  if (e.start != nullptr) {
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, e.start, e.stop, 0, args...);
    e.start = e.stop = nullptr;
  } else {
    kernel<<<grid, block, 0, st>>>(args...);
  }
}

// The four x/y passes of the PCG matvec (x_inv_grad, y_inv_grad, y_fwd_div,
// x_fwd_div) and the z matvec can each take their own tile shape; the
// remaining transform kernels use the plan-wide pencil count C.
template <typename T, int N>
struct Sched {
  int C = 0;       // pencils per x/y workgroup of the other transform kernels
  int RW = 0;      // rows per z workgroup
  int sx_nblk = 0; // x-pass workgroups per problem at C
  int z_nblk = 0;  // z-pass workgroups per problem (partial-sum count)
  int zm_nblk = 0; // z matvec workgroups per problem (partial-sum count)
  int sy_nblk = 0; // y-pass workgroups per problem at C
  int xi_nblk = 0; // x_inv_grad workgroups (partial-sum count)
  int xf_nblk = 0; // x_fwd_div workgroups (partial-sum count)
  int yi_nblk = 0; // y_inv_grad workgroups
  int yf_nblk = 0; // y_fwd_div workgroups
  void (*x_inv_grad)(int mode, cx<T>* P, const cx<T>* R, cx<T>* U1, cx<T>* U2,
                     const ProbScalars* sc, double* part, double tau, int pred, int nb,
                     hipStream_t st) = nullptr;
  // y-pass and z-pass launches over slab k of nslab (x-plane ranges)
  void (*y_inv_grad)(cx<T>* U1, cx<T>* U2, cx<T>* V3, const ProbScalars* sc, int pred, int nb,
                     int k, int nslab, hipStream_t st) = nullptr;
  // fin0 > 0: the launch also forms the PCG step length (k_y_fwd_div)
  void (*y_fwd_div)(cx<T>* H1, cx<T>* H2, const cx<T>* H3, ProbScalars* sc, int pred, int nb,
                    int k, int nslab, double* part, int fin0, int fin1, double fsc,
                    hipStream_t st) = nullptr;
  void (*x_fwd_div)(int mode, const cx<T>* W1, const cx<T>* W23, cx<T>* X, cx<T>* Q,
                    const cx<T>* Sv, const ProbScalars* sc, double* part, double tau, int pred,
                    int want_gk, int nb, hipStream_t st) = nullptr;
  void (*x_inv)(const cx<T>* X, cx<T>* Y, int nb, hipStream_t st) = nullptr;
  void (*y_plain)(bool inv, cx<T>* Y, cx<T>* Y2, int nb, hipStream_t st) = nullptr;
  void (*x_fwd_state)(const cx<T>* H, cx<T>* X, cx<T>* U1, cx<T>* U2, cx<T>* S2, int nb,
                      hipStream_t st) = nullptr;
  void (*z_matvec)(cx<T>* V1, cx<T>* V2, cx<T>* V3, const T* m, long long m_bs,
                   const ProbScalars* sc, double* part, int pred, int rev, int nb, int k,
                   int nslab, hipStream_t st) = nullptr;
  void (*z_step)(int mode, const ZArgs& a, int nb, hipStream_t st) = nullptr;
  void (*z_qgrad)(const cx<T>* M1, const cx<T>* M2, const cx<T>* M3, const cx<T>* S1,
                  const cx<T>* S2, const cx<T>* S3, T* Qk, const ProbScalars* sc, double tau,
                  int nb, hipStream_t st) = nullptr;
};

template <typename T, int N, int C, int OCC>
struct SLaunch {
  using SX = SP<T, N, C, 0>;
  using SY = SP<T, N, C, 1>;
  static_assert(SX::NBLK <= MAXBLK, "x-pass partial sums exceed the partial buffer");
  static void x_inv_grad(int mode, cx<T>* P, const cx<T>* R, cx<T>* U1, cx<T>* U2,
                         const ProbScalars* sc, double* part, double tau, int pred, int nb,
                         hipStream_t st) {
    using SXI = SP<T, N, C, 0, XPassE<T, N, C>::value>;
    if (mode == 1)
      klaunch(k_x_inv_grad<T, N, C, 1, OCC>, dim3(SXI::NBLK, nb), dim3(SXI::NT), st, P, R, U1, U2, sc,
              part, tau, pred);
    else
      klaunch(k_x_inv_grad<T, N, C, 0, OCC>, dim3(SXI::NBLK, nb), dim3(SXI::NT), st, P, R, U1, U2, sc,
              part, tau, pred);
  }
  static void y_inv_grad(cx<T>* U1, cx<T>* U2, cx<T>* V3, const ProbScalars* sc, int pred, int nb,
                         int k, int nslab, hipStream_t st) {
    const int nbk = SY::NBLK / nslab;
    klaunch(k_y_inv_grad<T, N, C, OCC>, dim3(nbk, nb), dim3(SY::NT), st, U1, U2, V3, sc, pred, k * nbk);
  }
  static void y_fwd_div(cx<T>* H1, cx<T>* H2, const cx<T>* H3, ProbScalars* sc, int pred,
                        int nb, int k, int nslab, double* part, int fin0, int fin1, double fsc,
                        hipStream_t st) {
    const int nbk = SY::NBLK / nslab;
    klaunch(k_y_fwd_div<T, N, C, OCC>, dim3(nbk, nb), dim3(SY::NT), st, H1, H2, H3, sc, pred,
            k * nbk, part, fin0, fin1, fsc);
  }
  static void x_fwd_div(int mode, const cx<T>* W1, const cx<T>* W23, cx<T>* X, cx<T>* Q,
                        const cx<T>* Sv, const ProbScalars* sc, double* part, double tau, int pred,
                        int want_gk, int nb, hipStream_t st) {
    using SXF = SP<T, N, C, 0, XPassE<T, N, C>::value>;
    const dim3 g(SXF::NBLK, nb);
    switch (mode) {
      case XM_PCG:
        klaunch(k_x_fwd_div<T, N, C, XM_PCG, OCC>, g, dim3(SXF::NT), st, W1, W23, X, Q, Sv, sc, part, tau, pred, want_gk);
        break;
      case XM_RHS_FWD:
        klaunch(k_x_fwd_div<T, N, C, XM_RHS_FWD, OCC>, g, dim3(SXF::NT), st, W1, W23, X, Q, Sv, sc, part, tau, pred, want_gk);
        break;
      case XM_RHS_ADJ:
        klaunch(k_x_fwd_div<T, N, C, XM_RHS_ADJ, OCC>, g, dim3(SXF::NT), st, W1, W23, X, Q, Sv, sc, part, tau, pred, want_gk);
        break;
      case XM_SHIFT:
        klaunch(k_x_fwd_div<T, N, C, XM_SHIFT, OCC>, g, dim3(SXF::NT), st, W1, W23, X, Q, Sv, sc, part, tau, pred, want_gk);
        break;
      default:
        klaunch(k_x_fwd_div<T, N, C, XM_POST_ADJ, OCC>, g, dim3(SXF::NT), st, W1, W23, X, Q, Sv, sc, part, tau, pred, want_gk);
        break;
    }
  }
  static void x_inv(const cx<T>* X, cx<T>* Y, int nb, hipStream_t st) {
    k_x_inv<T, N, C><<<dim3(SX::NBLK, nb), SX::NT, 0, st>>>(X, Y);
  }
  static void y_plain(bool inv, cx<T>* Y, cx<T>* Y2, int nb, hipStream_t st) {
    if (inv)
      k_y_plain<T, N, C, true><<<dim3(SY::NBLK, nb), SY::NT, 0, st>>>(Y, Y2);
    else
      k_y_plain<T, N, C, false><<<dim3(SY::NBLK, nb), SY::NT, 0, st>>>(Y, Y2);
  }
  static void x_fwd_state(const cx<T>* H, cx<T>* X, cx<T>* U1, cx<T>* U2, cx<T>* S2, int nb,
                          hipStream_t st) {
    k_x_fwd_state<T, N, C><<<dim3(SX::NBLK, nb), SX::NT, 0, st>>>(H, X, U1, U2, S2);
  }
  // one PCG pass (KT_X_INV_GRAD, KT_Y_INV_GRAD, KT_Y_FWD_DIV, KT_X_FWD_DIV)
  static void fill_pass(Sched<T, N>& s, int id) {
    switch (id) {
      case KT_X_INV_GRAD: s.x_inv_grad = &x_inv_grad; s.xi_nblk = SX::NBLK; break;
      case KT_Y_INV_GRAD: s.y_inv_grad = &y_inv_grad; s.yi_nblk = SY::NBLK; break;
      case KT_Y_FWD_DIV: s.y_fwd_div = &y_fwd_div; s.yf_nblk = SY::NBLK; break;
      case KT_X_FWD_DIV: s.x_fwd_div = &x_fwd_div; s.xf_nblk = SX::NBLK; break;
    }
  }
  static void fill(Sched<T, N>& s) {
    s.C = C;
    s.sx_nblk = SX::NBLK;
    s.sy_nblk = SY::NBLK;
    for (int id : {KT_X_INV_GRAD, KT_Y_INV_GRAD, KT_Y_FWD_DIV, KT_X_FWD_DIV}) fill_pass(s, id);
    s.x_inv = &x_inv;
    s.y_plain = &y_plain;
    s.x_fwd_state = &x_fwd_state;
  }
};

// z-pass launches.  The matvec kernel takes RW rows per workgroup and EZ
// complex values per lane (L/EZ lanes per row), in single or pair layout
// (PAIR: 16-byte accesses in FP32); the time-step kernels use the default
// lanes per row.
template <typename T, int N, int RW, int OCC, int EZ = FftE<N / 2>::value, bool PAIR = false>
struct ZLaunch {
  using Z = ZP<T, N, RW>;
  using ZM = ZP<T, N, RW * EZ / FftE<N / 2>::value, EZ>;  // same threads, EZ per lane
  static_assert(ZM::NBLK <= MAXBLK && Z::NBLK <= MAXBLK, "z-pass partial sums exceed the buffer");
  static void z_matvec(cx<T>* V1, cx<T>* V2, cx<T>* V3, const T* m, long long m_bs,
                       const ProbScalars* sc, double* part, int pred, int rev, int nb, int k,
                       int nslab, hipStream_t st) {
    const int nbk = ZM::NBLK / nslab;
    // FP32 holds all three rows unless an occupancy floor asks for fewer
    // registers; FP64 always streams them one at a time.
    constexpr int PRE = (sizeof(T) == 4 && OCC < 4) ? 3 : 1;
    klaunch(k_z_matvec<T, N, ZM::RW, PRE, OCC, EZ, PAIR>, dim3(nbk, nb), dim3(ZM::NT), st,
            V1, V2, V3, m, m_bs, sc, part, pred, rev, k * nbk);
  }
  template <int MODE>
  static void zs(const ZArgs& a, int nb, hipStream_t st) {
    k_z_step<T, N, MODE, RW><<<dim3(Z::NBLK, nb), Z::NT, 0, st>>>(a);
  }
  static void z_step(int mode, const ZArgs& a, int nb, hipStream_t st) {
    switch (mode) {
      case ZS_FWD_FIRST: zs<ZS_FWD_FIRST>(a, nb, st); break;
      case ZS_FWD: zs<ZS_FWD>(a, nb, st); break;
      case ZS_FWD_LAST: zs<ZS_FWD_LAST>(a, nb, st); break;
      case ZS_TAN_FIRST: zs<ZS_TAN_FIRST>(a, nb, st); break;
      case ZS_TAN: zs<ZS_TAN>(a, nb, st); break;
      case ZS_TAN_LAST: zs<ZS_TAN_LAST>(a, nb, st); break;
      case ZS_ADJ_FIRST: zs<ZS_ADJ_FIRST>(a, nb, st); break;
      case ZS_ADJ: zs<ZS_ADJ>(a, nb, st); break;
      default: zs<ZS_ADJ_LAST>(a, nb, st); break;
    }
  }
  static void z_qgrad(const cx<T>* M1, const cx<T>* M2, const cx<T>* M3, const cx<T>* S1,
                      const cx<T>* S2, const cx<T>* S3, T* Qk, const ProbScalars* sc,
                      double tau, int nb, hipStream_t st) {
    // FP32: two waves per SIMD with the next rows prefetched (254 VGPRs at
    // 256^3, no spills); FP64 rows are twice the registers: one wave, no
    // prefetch (a floor of two spills)
    constexpr bool F32 = sizeof(T) == 4;
    k_z_qgrad<T, N, RW, F32 ? 2 : 1, F32><<<dim3(Z::NBLK, nb), Z::NT, 0, st>>>(M1, M2, M3, S1, S2, S3, Qk, sc, tau);
  }
  static void fill(Sched<T, N>& s) {
    s.RW = RW;
    s.z_nblk = Z::NBLK;
    s.zm_nblk = ZM::NBLK;
    s.z_matvec = &z_matvec;
    s.z_step = &z_step;
    s.z_qgrad = &z_qgrad;
  }
  static void fill_matvec(Sched<T, N>& s) {
    s.zm_nblk = ZM::NBLK;
    s.z_matvec = &z_matvec;
  }
};

// Candidate tile shapes.  Pencils per x/y workgroup: 8, 16, 32, 64 (row
// segments of 64..512 bytes in FP32).  Rows per z workgroup: one, two or four waves.
// pass < 0: every x/y kernel; else one PCG pass (KT_* id).
template <typename T, int N, int OCC>
bool set_strided_occ(Sched<T, N>& s, int C, int pass) {
  switch (C) {
    case 8:
      if (pass < 0) SLaunch<T, N, 8, OCC>::fill(s); else SLaunch<T, N, 8, OCC>::fill_pass(s, pass);
      return true;
    case 16:
      if (pass < 0) SLaunch<T, N, 16, OCC>::fill(s); else SLaunch<T, N, 16, OCC>::fill_pass(s, pass);
      return true;
    case 32:
      if (pass < 0) SLaunch<T, N, 32, OCC>::fill(s); else SLaunch<T, N, 32, OCC>::fill_pass(s, pass);
      return true;
    case 64:
      // 64 pencils: 512-byte row segments; only where the workgroup's
      // transform buffer and twiddle table fit the 160 KB of LDS
      if constexpr ((long long)N * 64 * sizeof(cx<T>) + TW_LDS * sizeof(cx<T>) + 1024 <= 160 * 1024 &&
                    64 * SP<T, N, 64, 0>::TT <= 1024) {
        if (pass < 0) SLaunch<T, N, 64, OCC>::fill(s); else SLaunch<T, N, 64, OCC>::fill_pass(s, pass);
        return true;
      }
      return false;
  }
  return false;
}

// occ: occupancy floor in waves per SIMD (1: none, 4: at least four)
template <typename T, int N>
bool set_strided(Sched<T, N>& s, int C, int occ, int pass = -1) {
  if (occ == 4) return set_strided_occ<T, N, 4>(s, C, pass);
  if (occ == 1) return set_strided_occ<T, N, 1>(s, C, pass);
  return false;
}

// Rows per z workgroup: one, two or four waves.  matvec_only: replace only
// the z matvec kernel (its occupancy floor and access layout).
template <typename T, int N, int RW, int OCC>
void fill_z(Sched<T, N>& s, bool matvec_only, bool pair) {
  if (!matvec_only) ZLaunch<T, N, RW, OCC>::fill(s);
  if (pair) ZLaunch<T, N, RW, OCC, FftE<N / 2>::value, true>::fill_matvec(s);
  else ZLaunch<T, N, RW, OCC>::fill_matvec(s);
}

template <typename T, int N, int OCC>
bool set_zrows_occ(Sched<T, N>& s, int waves, bool matvec_only, bool pair) {
  constexpr int TT = ZP<T, N>::TT;
  constexpr int r1 = 64 / TT;
  switch (waves) {
    case 1:
      fill_z<T, N, r1, OCC>(s, matvec_only, pair);
      return true;
    case 2:
      if constexpr (N * N >= 2 * r1) {
        fill_z<T, N, 2 * r1, OCC>(s, matvec_only, pair);
        return true;
      }
      return false;
    case 4:
      if constexpr (N * N >= 4 * r1) {
        fill_z<T, N, 4 * r1, OCC>(s, matvec_only, pair);
        return true;
      }
      return false;
  }
  return false;
}

template <typename T, int N>
bool set_zrows(Sched<T, N>& s, int waves, int occ, bool matvec_only = false, bool pair = false) {
  if (occ == 4) return set_zrows_occ<T, N, 4>(s, waves, matvec_only, pair);
  if (occ == 1) return set_zrows_occ<T, N, 1>(s, waves, matvec_only, pair);
  return false;
}

// Matvec z pass with half the default values per lane (twice the lanes per
// row: full 128-byte row segments per load instruction at n = 256), on
// workgroups of one wave.
template <typename T, int N>
bool set_zmatvec_wide(Sched<T, N>& s, int occ) {
  constexpr int E0 = FftE<N / 2>::value;
  constexpr int L = N / 2;
  if constexpr (E0 >= 8 && (L / (E0 / 2)) <= 64) {
    constexpr int r1 = 64 / (L / E0);
    if (occ == 4) { ZLaunch<T, N, r1, 4, E0 / 2>::fill_matvec(s); return true; }
    if (occ == 1) { ZLaunch<T, N, r1, 1, E0 / 2>::fill_matvec(s); return true; }
  }
  return false;
}

}  // namespace tg
