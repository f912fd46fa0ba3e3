// Host orchestration of the tumor forward, adjoint, tangent and
// Gauss-Newton Hessian solves for one grid size and precision.
//
// Time stepping (paper, Sec. 3.3): Strang splitting, one step being
//   a = R_{dt/2}(c^n);  (I - dt/2 A) b = (I + dt/2 A) a;  c^{n+1} = R_{dt/2}(b)
// with A = div(k_f m grad .) and R the exact logistic flow.  Each
// Crank-Nicolson system is solved by PCG in spectral space with the
// constant-coefficient Fourier preconditioner (1 + dt/2 kbar |w|^2)^-1,
// kbar = k_f max(m); stop when ||r|| <= rtol ||rhs|| (grid norms).  The
// first forward solve starts from x0 = a, later ones from a plus the
// previous step's increment b - a (exact initial residual), adjoint solves
// from lambda.
// The adjoint is the exact transpose of these discrete steps (reduced
// gradient of Sec. 3.1: state solve, adjoint solve, gradient), with
// checkpointed states recomputed segment by segment.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "tg_launch.h"
#include "tg_transport.h"

namespace tg {

#define TG_CHECK(x)                                 \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) return e_;                \
  } while (0)
#define TG_LAUNCH_CHECK() TG_CHECK(hipGetLastError())

template <typename T, int N>
class Solver final : public ISolver {
  using RPc = RP<T, N>;
  static constexpr long long REAL = (long long)N * N * N;
  static constexpr long long SPECN = (long long)N * N * (N / 2);

  // A batch of independent PCG systems sharing one launch.
  struct Ctx {
    cx<T>* X; cx<T>* R; cx<T>* P; cx<T>* T1; cx<T>* T2; cx<T>* T3; cx<T>* S;
    ProbScalars* sc;
    double* part;
    int nb;
    const T* m; long long m_bs;     // diffusion field
    const T* mr;                    // reaction field (stride m_bs)
    long long traj_bs;  // batch stride of stored states (0: shared trajectory)
  };

 public:
  Solver(const SolverDims& d, const Workspace& w) : d_(d), w_(w) {
    dt_ = d.T / d.nt;
    tau_ = 0.5 * dt_;
    const double h = 2.0 * M_PI / N;
    h3_ = h * h * h;
    hsc_.resize(d.batch + d.dirs);
    its_est_ = 8;
    set_schedule(0, 0, 0, 0);
    fp32_floor_ = 50.0 * 1.1920928955078125e-07;
    if (const char* f = std::getenv("TUMORGRAD_FP32_RTOL_FLOOR")) {
      const double v = std::atof(f);
      if (v > 0.0 && v < 1.0) fp32_floor_ = v;
    }
    // forward-type solves: 16 eps_32 (their error dominates the FP32-mixed
    // error of the rho_f derivative: at 50 eps_32 it was 1.3e-4 of the
    // oracle's in the 128^3 gradient, at 16 eps_32 3e-5)
    fp32_fwd_floor_ = std::getenv("TUMORGRAD_FP32_RTOL_FLOOR") ? fp32_floor_
                                                               : 16.0 * 1.1920928955078125e-07;
    if (const char* f = std::getenv("TUMORGRAD_FP32_FWD_RTOL_FLOOR")) {
      const double v = std::atof(f);
      if (v > 0.0 && v < 1.0) fp32_fwd_floor_ = v;
    }
  }

  // Tile shapes of the transform passes; 0 picks the default.
  bool set_schedule(int C, int zwaves, int slabs, int occ) override {
    Sched<T, N> s;
    if (C == 0) C = 16;
    if (zwaves == 0) zwaves = 1;
    if (slabs == 0) slabs = 1;
    if (occ == 0) occ = 1;
    if (slabs != 1 && slabs != 2 && slabs != 4 && slabs != 8) return false;
    if (!set_strided<T, N>(s, C, occ)) return false;
    // zwaves 8: one-wave z workgroups whose matvec kernel uses twice the
    // lanes per row (see set_zmatvec_wide)
    const bool wide = zwaves == 8;
    const bool pair = !wide && kZPairDefault;
    if (!set_zrows<T, N>(s, wide ? 1 : zwaves, occ, false, pair)) {
      if (!set_zrows<T, N>(s, 1, occ, false, pair)) return false;
      zwaves = 1;
    }
    if (wide && !set_zmatvec_wide<T, N>(s, occ)) return false;
    if (!slabs_fit(s, slabs)) return false;
    sch_ = s;
    zwaves_ = zwaves;
    nslab_ = slabs;
    occ_ = occ;
    for (int id = 1; id <= KT_LAST; ++id) {
      pass_C_[id] = id == KT_Z_MATVEC ? (wide ? 8 : (pair ? 16 : 8)) : C;
      pass_occ_[id] = occ;
    }
    return true;
  }
  void get_schedule(int* C, int* zwaves, int* slabs, int* occ) const override {
    *C = sch_.C;
    *zwaves = zwaves_;
    *slabs = nslab_;
    *occ = occ_;
  }
  // Tile shape of one PCG pass (KT_* id): pencils for the x/y passes; for
  // the z matvec the bytes per lane access of a spectral row (8: one
  // complex value, 16: a pair of them, 0: the default) and its occupancy
  // floor.
  bool set_pass(int id, int C, int occ) override {
    if (id < 1 || id > KT_LAST) return false;
    Sched<T, N> s = sch_;
    if (id == KT_Z_MATVEC) {
      if (C == 0) C = kZPairDefault ? 16 : 8;
      // the wide z matvec has no per-pass variant: its own shape is a no-op
      if (zwaves_ == 8) return C == pass_C_[id] && occ == pass_occ_[id];
      if (C != 8 && C != 16) return false;
      if (!set_zrows<T, N>(s, zwaves_, occ, true, C == 16)) return false;
    } else {
      if (!set_strided<T, N>(s, C, occ, id)) return false;
    }
    if (!slabs_fit(s, nslab_)) return false;
    sch_ = s;
    pass_C_[id] = C;
    pass_occ_[id] = occ;
    return true;
  }
  bool get_pass(int id, int* C, int* occ) const override {
    if (id < 1 || id > KT_LAST) return false;
    *C = pass_C_[id];
    *occ = pass_occ_[id];
    return true;
  }

  // ------------------------------------------------------------ forward
  hipError_t forward(const double* p, const double* rho, const double* kf, const void* m,
                     const void* mr, const void* mask, void* cT, hipStream_t st) override {
    st_ = st;
    call_status_ = 0;
    its_max_call_ = 0;
    begin_call(0);
    m_ = (const T*)m;
    mr_ = mr ? (const T*)mr : m_;
    mask_ = (const T*)mask;
    cT_ = (T*)cT;
    Ctx c = prim();
    stat_sc_ = c.sc;
    stat_nb_ = c.nb;
    k_init_scalars<<<(d_.batch + 63) / 64, 64, 0, st_>>>(w_.sc, rho, 1, kf, 1, d_.batch);
    TG_LAUNCH_CHECK();
    k_mmax<T, N><<<dim3(RPc::NBLK, d_.batch), 256, 0, st_>>>(m_, REAL, w_.part);
    TG_LAUNCH_CHECK();
    k_finalize<FIN_MMAX><<<d_.batch, 256, 0, st_>>>(w_.sc, w_.part, RPc::NBLK, 1.0, 0.0, 0);
    TG_LAUNCH_CHECK();
    const int nf = d_.n_p * 3 * N;
    k_basis_factors<<<dim3((nf + 255) / 256, d_.batch), 256, 0, st_>>>(
        w_.centres, (long long)d_.n_p * 3, w_.gfac, N, d_.n_p, d_.sigma);
    TG_LAUNCH_CHECK();
    launch_phi(p, d_.n_p, w_.gfac, (long long)d_.n_p * 3 * N, mask_, REAL, ck(0), REAL, d_.batch);
    TG_LAUNCH_CHECK();
    TG_CHECK(fwd_steps(c, 0, d_.nt, /*initial=*/true));
    live_seg_ = d_.nseg - 1;
    end_call();
    return hipSuccess;
  }

  // ------------------------------------------------------------ adjoint
  hipError_t vjp(const void* lamT, const void* cobs, int nlab, const void* mlab,
                 const void* mpat, double* J, double* gp, double* grho, double* gkf, void* qk,
                 void* qr, hipStream_t st) override {
    st_ = st;
    call_status_ = 0;
    begin_call(1);
    Ctx c = prim();
    stat_sc_ = c.sc;
    stat_nb_ = c.nb;
    k_reset_call<<<(d_.batch + 63) / 64, 64, 0, st_>>>(w_.sc, d_.batch);
    TG_LAUNCH_CHECK();
    qk_ = (T*)qk;
    qr_ = (T*)qr;
    // the output fields accumulate over the sweep: clear them first (once
    // when both parts go to one field)
    T* const qclr[2] = {qk_, qr_ != qk_ ? qr_ : nullptr};
    for (T* q : qclr) {
      if (q == nullptr) continue;
      const long long nq = (long long)d_.batch * REAL;
      k_zero<T><<<(int)std::min<long long>((nq + 255) / 256, 8192), 256, 0, st_>>>(q, nq);
      TG_LAUNCH_CHECK();
    }
    const T* lt = (const T*)lamT;
    if (cobs != nullptr) {
      if (nlab > 0)
        k_misfit_labels<T, N><<<dim3(RPc::NBLK, d_.batch), 256, 0, st_>>>(
            cT_, (const T*)cobs, nlab, (const T*)mlab, (const T*)mpat, lam(0), h3_, w_.part);
      else
        k_misfit<T, N><<<dim3(RPc::NBLK, d_.batch), 256, 0, st_>>>(cT_, (const T*)cobs, lam(0),
                                                                  h3_, w_.part);
      TG_LAUNCH_CHECK();
      k_finalize<FIN_J><<<d_.batch, 256, 0, st_>>>(w_.sc, w_.part, RPc::NBLK, 0.5 * h3_, 0, 0);
      TG_LAUNCH_CHECK();
      lt = lam(0);
    }
    const hipError_t ea = adjoint_sweep(c, lt, REAL, /*gn=*/false);
    qk_ = qr_ = nullptr;
    TG_CHECK(ea);
    TG_CHECK(phit(c, gp));
    k_emit_grads<<<(d_.batch + 63) / 64, 64, 0, st_>>>(w_.sc, cobs ? J : nullptr, grho, gkf,
                                                       d_.batch);
    TG_LAUNCH_CHECK();
    end_call();
    return hipSuccess;
  }

  // ------------------------------------------------- Gauss-Newton H v
  hipError_t hessvec(int ndir, const double* V, double* HV, hipStream_t st) override {
    st_ = st;
    call_status_ = 0;
    begin_call(2);
    Ctx dc = dirs(ndir);
    stat_sc_ = dc.sc;
    stat_nb_ = ndir;
    // direction scalars inherit k_f, rho_f, kbar of problem 0
    k_copy_dir_scalars<<<(ndir + 63) / 64, 64, 0, st_>>>(w_.sc, dc.sc, ndir);
    TG_LAUNCH_CHECK();
    // dc0 = Phi v for each direction
    launch_phi(V, d_.n_p, w_.gfac, 0, mask_, 0, lam(0), REAL, ndir);
    TG_LAUNCH_CHECK();
    // tangent sweep, forward in time
    for (int j = 0; j < d_.nseg; ++j) {
      TG_CHECK(ensure_segment(j));
      const int n0 = j * d_.s, n1 = std::min(n0 + d_.s, d_.nt);
      for (int n = n0; n < n1; ++n) {
        ZArgs a = zargs(dc);
        if (n == 0) {
          a.Cin = lam(0); a.cin_bs = REAL;
          a.Cn = cn_ptr(0); a.cn_bs = 0;
          launch_z<ZS_TAN_FIRST>(a, dc.nb);
        } else {
          TG_CHECK(inv_xy(dc, dc.X, dc.T1));
          a.Xs = dc.T1;
          a.Bn = bprev_ptr(n); a.bn_bs = 0;
          launch_z<ZS_TAN>(a, dc.nb);
        }
        TG_LAUNCH_CHECK();
        TG_CHECK(step_solve(dc, /*adj=*/false, est_tan_));
        est_tan_ = last_its_;
      }
    }
    {
      TG_CHECK(inv_xy(dc, dc.X, dc.T1));
      ZArgs a = zargs(dc);
      a.Xs = dc.T1;
      a.Bn = bn_ptr(d_.nt - 1); a.bn_bs = 0;
      a.Cst = lam(0); a.cst_bs = REAL;
      a.out_scale = h3_;
      launch_z<ZS_TAN_LAST>(a, dc.nb);
      TG_LAUNCH_CHECK();
    }
    TG_CHECK(adjoint_sweep(dc, lam(0), REAL, /*gn=*/true));
    TG_CHECK(phit(dc, HV, /*g_bs=*/0));
    return hipSuccess;
  }

  // ------------------------------------------- registration transport
  hipError_t transport(int ntr, int L, const void* v, const void* w, const void* m0, void* m1,
                       void* tws, hipStream_t st) override {
    st_ = st;
    tr_nt_ = ntr;
    tr_L_ = L;
    tr_w_ = (const T*)w;
    tr_ws_ = (T*)tws;
    const double dt = 1.0 / ntr, h = 2.0 * M_PI / N;
    constexpr int GB = (int)((REAL + 255) / 256);
    TG_CHECK(sl_foot((const T*)v, tr_disp(0), -dt / h));
    TG_CHECK(sl_foot((const T*)v, tr_disp(1), dt / h));
    copy_real(tr_level(0), (const T*)m0, (long long)L * REAL);
    for (int k = 0; k < ntr; ++k) {
      sl_step(tr_level(k), tr_level(k + 1), tr_disp(0), L, nullptr, 0.0);
      TG_LAUNCH_CHECK();
    }
    if (m1 != nullptr) copy_real((T*)m1, tr_level(ntr), (long long)L * REAL);
    TG_LAUNCH_CHECK();
    return hipSuccess;
  }

  hipError_t transport_adjoint(const void* lam1, void* lam0, void* body,
                               hipStream_t st) override {
    st_ = st;
    const int ntr = tr_nt_, L = tr_L_;
    const double dt = 1.0 / ntr;
    constexpr int GB = (int)((REAL + 255) / 256);
    T* bf = (T*)body;
    k_zero<T><<<(int)std::min<long long>((3 * REAL + 255) / 256, 8192), 256, 0, st_>>>(
        bf, 3 * REAL);
    TG_LAUNCH_CHECK();
    T* cur = tr_lam(0);
    T* nxt = tr_lam(1);
    copy_real(cur, (const T*)lam1, (long long)L * REAL);
    TG_CHECK(body_force(tr_level(ntr), cur, L, 0.5 * dt, bf));
    for (int k = ntr - 1; k >= 0; --k) {
      if (tr_w_ != nullptr) {
        // numerator factor (1 + dt/2 w) first, then interpolate and divide
        k_sl_premul<T><<<(int)std::min<long long>(GB, 8192), 256, 0, st_>>>(
            cur, nxt, tr_w_, 0.5 * dt, L, REAL);
        TG_LAUNCH_CHECK();
        sl_step(nxt, cur, tr_disp(1), L, tr_w_, 0.5 * dt);
      } else {
        sl_step(cur, nxt, tr_disp(1), L, nullptr, 0.0);
        std::swap(cur, nxt);
      }
      TG_LAUNCH_CHECK();
      TG_CHECK(body_force(tr_level(k), cur, L, (k == 0 ? 0.5 : 1.0) * dt, bf));
    }
    copy_real((T*)lam0, cur, (long long)L * REAL);
    TG_LAUNCH_CHECK();
    return hipSuccess;
  }

  int last_status() const override { return call_status_; }

  void set_graph_budget(int budget, bool per_solve) override {
    if (budget > 0 && tm_id_ != KT_NONE) {
      if (timer_flush() != hipSuccess) tm_err_ = true;
      tm_id_ = KT_NONE;
    }
    graph_budget_ = budget;
    graph_per_solve_ = per_solve;
  }
  int its_max_last_call() const override { return its_max_call_; }

  hipError_t read_stats(CallStats* out, hipStream_t st) override {
    const int nb = stat_nb_;
    if (stat_sc_ == nullptr) {
      *out = CallStats{0, 0, 0, 0, 0.0};
      return hipSuccess;
    }
    TG_CHECK(hipMemcpyAsync(hsc_.data(), stat_sc_, nb * sizeof(ProbScalars), hipMemcpyDeviceToHost, st));
    TG_CHECK(hipStreamSynchronize(st));
    CallStats s{0, 0, 0, 0, 0.0};
    for (int b = 0; b < nb; ++b) {
      s.solves += hsc_[b].solves;
      s.its_total += hsc_[b].its_total;
      s.its_max = std::max(s.its_max, hsc_[b].its_max);
      s.status |= hsc_[b].status;
      s.worst_rel_residual = std::max(s.worst_rel_residual, hsc_[b].worst);
    }
    *out = s;
    return hipSuccess;
  }

 private:
  // ----------------------------------------------------------- layout
  Ctx prim() {
    Ctx c;
    cx<T>** sp = (cx<T>**)w_.spec;
    c.X = sp[0]; c.R = sp[1]; c.P = sp[2];
    c.T1 = sp[3]; c.T2 = sp[4]; c.T3 = sp[5]; c.S = sp[6];
    c.sc = w_.sc; c.part = w_.part; c.nb = d_.batch;
    c.m = m_; c.mr = mr_; c.m_bs = REAL; c.traj_bs = REAL;
    return c;
  }
  Ctx dirs(int ndir) {
    Ctx c;
    cx<T>** sp = (cx<T>**)w_.dspec;
    c.X = sp[0]; c.R = sp[1]; c.P = sp[2];
    c.T1 = sp[3]; c.T2 = sp[4]; c.T3 = sp[5]; c.S = sp[6];
    c.sc = w_.sc + d_.batch;
    c.part = w_.part + (size_t)d_.batch * NSLOT * MAXBLK;
    c.nb = ndir;
    c.m = m_; c.mr = mr_; c.m_bs = 0; c.traj_bs = 0;
    return c;
  }
  T* ck(int j) { return (T*)w_.ck + (size_t)j * d_.batch * REAL; }
  T* ckb(int j) { return (T*)w_.ckb + (size_t)j * d_.batch * REAL; }
  T* segc(int i) { return (T*)w_.segc + (size_t)i * d_.batch * REAL; }
  T* segb(int i) { return (T*)w_.segb + (size_t)i * d_.batch * REAL; }
  cx<T>* ckd(int j) { return (cx<T>*)w_.ckd + (size_t)j * d_.batch * (REAL / 2); }
  T* lam(int b) { return (T*)w_.lam + (size_t)b * REAL; }
  // stored states of the live segment
  T* cn_ptr(int n) { return (n % d_.s == 0) ? ck(n / d_.s) : segc(n % d_.s); }
  T* bn_ptr(int n) { return segb(n % d_.s); }
  // b^{n-1} for a step n of the live segment (n >= 1)
  T* bprev_ptr(int n) { return (n % d_.s == 0) ? ckb(n / d_.s) : segb((n - 1) % d_.s); }

  ZArgs zargs(const Ctx& c) {
    ZArgs a{};
    a.m = c.mr; a.m_bs = c.m_bs;   // the z steps apply the reaction
    a.sc = c.sc; a.part = c.part;
    a.tau = tau_;
    a.out_scale = 1.0;
    a.Xs = c.T1;
    a.Y2 = c.S;
    return a;
  }

  // c0 = w Phi p for nb problems (p, g, mask, out with their batch strides)
  void launch_phi(const double* p, long long p_bs, const double* g, long long g_bs,
                  const T* mask, long long mask_bs, T* out, long long out_bs, int nb) {
    if constexpr (N >= 128)
      k_phi_w<T, N><<<dim3(PhiW<N>::NBLK, nb), 64 * PhiW<N>::WV, 0, st_>>>(
          p, p_bs, g, g_bs, mask, mask_bs, out, out_bs, d_.n_p);
    else
      k_phi<T, N><<<dim3(PhiK<N>::NBX * PhiK<N>::NBZ, nb), 256, 0, st_>>>(
          p, p_bs, g, g_bs, mask, mask_bs, out, out_bs, d_.n_p);
  }

  template <int MODE>
  void launch_z(const ZArgs& a, int nb) {
    sch_.z_step(MODE, a, nb, st_);
  }

  // spectral X -> T1 rows ready for a z pass (x then y inverse, 1/n^3)
  hipError_t inv_xy(const Ctx& c, cx<T>* X, cx<T>* Y) {
    sch_.x_inv(X, Y, c.nb, st_);
    TG_LAUNCH_CHECK();
    sch_.y_plain(true, Y, nullptr, c.nb, st_);
    TG_LAUNCH_CHECK();
    return hipSuccess;
  }

  // matvec middle (y inverse, z, y forward) on U1, U2 (V3 scratch); the
  // three passes run slab by slab over nslab x-plane ranges so each slab's
  // intermediates can stay in the last-level cache between passes.
  // The z pass also leaves the partial sums of m |grad u|^2 (slot 1).
  // step: inside a PCG iteration, the last y forward launch also forms the
  // step length from those and the x inverse pass's |p|^2 partials.
  void matvec_mid(const Ctx& c, cx<T>* U1, cx<T>* U2, cx<T>* V3, int pred, bool step = false) {
    const int work = pred ? 0 : c.nb;
    const int ns = nslab_;
    for (int k = 0; k < ns; ++k) {
      timed(KT_Y_INV_GRAD, k == 0 ? work : 0, [&] {
        sch_.y_inv_grad(U1, U2, V3, c.sc, pred, c.nb, k, ns, st_);
      });
      timed(KT_Z_MATVEC, k == 0 ? work : 0, [&] {
        sch_.z_matvec(U1, U2, V3, c.m, c.m_bs, c.sc, c.part, pred, 1, c.nb, k, ns, st_);
      });
      const bool fin = step && k == ns - 1;
      timed(KT_Y_FWD_DIV, k == 0 ? work : 0, [&] {
        sch_.y_fwd_div(U1, U2, V3, c.sc, pred, c.nb, k, ns, c.part, fin ? sch_.xi_nblk : 0,
                       sch_.zm_nblk, tau_ * (double)REAL, st_);
      });
    }
  }

  // After a boundary z kernel left the step's real-to-spectral rows in T1
  // (and S for the adjoint): finish the transform into X, run the right-
  // hand-side matvec and the PCG solve.
  // Forward solves of the primary problems (hist bits): 1 starts from
  // x0 = a + d, d = b - a of the previous step, with the exact residual of
  // x0 from one matvec on d (XM_SHIFT); 2 keeps this step's d for the next.
  hipError_t step_solve(const Ctx& c, bool adj, int est = -1, bool exact = false,
                        int hist = 0) {
    // kernel timer: this solve's launches are timed if it is a sampled one
    tm_on_ = tm_id_ == KT_NONE || tm_solves_++ % tm_every_ == 0;
    sch_.y_plain(false, c.T1, adj ? c.S : nullptr, c.nb, st_);
    TG_LAUNCH_CHECK();
    sch_.x_fwd_state(c.T1, c.X, c.T2, c.T3, adj ? c.S : nullptr, c.nb, st_);
    TG_LAUNCH_CHECK();
    matvec_mid(c, c.T2, c.T3, c.T1, 0);
    TG_LAUNCH_CHECK();
    sch_.x_fwd_div(adj ? XM_RHS_ADJ : XM_RHS_FWD, c.T2, c.T3, c.X, c.R, nullptr, c.sc, c.part, tau_,
                   0, 0, c.nb, st_);
    TG_LAUNCH_CHECK();
    cx<T>* ah = (cx<T>*)w_.ahat;
    cx<T>* dd = (cx<T>*)w_.incr;
    if (hist & 2) copy_spec(c, ah, c.X);
    if (hist & 1) {
      sch_.x_inv_grad(0, dd, nullptr, c.T1, c.T2, c.sc, nullptr, tau_, 0, c.nb, st_);
      matvec_mid(c, c.T1, c.T2, c.T3, 0);
      sch_.x_fwd_div(XM_SHIFT, c.T1, c.T2, c.X, c.R, dd, c.sc, c.part, tau_, 0, 0, c.nb, st_);
      TG_LAUNCH_CHECK();
    }
    k_finalize<FIN_INIT><<<c.nb, 256, 0, st_>>>(c.sc, c.part, sch_.xf_nblk, 1.0 / REAL, rtol(adj),
                                                maxit());
    TG_LAUNCH_CHECK();
    TG_CHECK(pcg_loop(c, est, exact));
    if (hist & 2) {
      const long long nc = (long long)c.nb * (REAL / 2);
      k_increment<T><<<(int)std::min<long long>((nc + 255) / 256, 8192), 256, 0, st_>>>(
          c.X, ah, dd, nc);
      TG_LAUNCH_CHECK();
    }
    return hipSuccess;
  }

  // In graph mode the iteration budget is the iteration cap, so a solve
  // that needs more is flagged NOT_CONVERGED instead of silently stopping.
  int maxit() const {
    return graph_budget_ > 0 ? std::min(cur_budget_, d_.maxit) : d_.maxit;
  }

  // Per-solve iteration counts of the last eager call of each kind
  // (0 forward, 1 vjp, 2 hessvec): the solves of a call come in a fixed
  // order, so a graph captured later can give each one its own budget.
  void begin_call(int kind) {
    kind_ = kind;
    seq_ = 0;
    rec_.clear();
  }
  void end_call() {
    if (graph_budget_ == 0) hist_[kind_] = rec_;
  }

  // Stopping tolerance of a solve (only FIN_INIT uses it: it fixes the
  // solve's target |r|^2).  FP32 arithmetic cannot certify residuals near
  // its rounding level: stop at a floor if rtol asks for less, one for the
  // adjoint solves and one for the forward-type solves (forward, segment
  // recompute, tangent), whose error is what the rho_f derivative is most
  // sensitive to.
  double rtol(bool adj = false) const {
    if (sizeof(T) == 4) return std::max(d_.rtol, adj ? fp32_floor_ : fp32_fwd_floor_);
    return d_.rtol;
  }

  // One PCG iteration (Sec. 3.3: Crank-Nicolson system, Fourier
  // preconditioner).  alpha = <r, M r> / <p, A p> with <p, A p> = |p|^2 +
  // tau k_f |sqrt(m) grad p|^2 (partials from the x and z passes), so the
  // last x pass applies x += alpha p and r -= alpha A p directly.
  void pcg_iteration(const Ctx& c) {
    timed(KT_X_INV_GRAD, 0, [&] {
      sch_.x_inv_grad(1, c.P, c.R, c.T1, c.T2, c.sc, c.part, tau_, 1, c.nb, st_);
    });
    matvec_mid(c, c.T1, c.T2, c.T3, 1, /*step=*/true);
    timed(KT_X_FWD_DIV, 0, [&] {
      sch_.x_fwd_div(XM_PCG, c.T1, c.T2, c.X, c.R, c.P, c.sc, c.part, tau_, 1, 0, c.nb, st_);
    });
    k_finalize<FIN_RZ, 1024><<<c.nb, 1024, 0, st_>>>(c.sc, c.part, sch_.xf_nblk, 1.0 / REAL,
                                                    rtol(), maxit());
  }

  // ------------------------------------------------------ kernel timer
  // HIP events around every launch of one chosen kernel, on the stream it
  // is launched on.  "work" counts problem-launches that did real work:
  // non-predicated launches count at launch time, predicated PCG-loop
  // launches count once the loop has read the iteration counts.
  static double unit_bytes(int id) {
    const double S = (double)REAL * sizeof(T);  // one field / packed spectrum
    switch (id) {
      case KT_X_INV_GRAD: return 5 * S;   // read r, p; write p, U1, U2
      case KT_Y_INV_GRAD: return 5 * S;   // read U1, U2; write V1, V2, V3
      case KT_Z_MATVEC: return 7 * S;     // read V1..V3, m; write H1..H3
      case KT_Y_FWD_DIV: return 5 * S;    // read H1..H3; write W1, W23
      case KT_X_FWD_DIV: return 7 * S;    // read W1, W23, p, x, r; write x, r
    }
    return 0.0;
  }

 public:
  hipError_t timer_enable(int id, int every) override {
    TG_CHECK(timer_flush());
    tm_every_ = every;
    tm_solves_ = 0;
    tm_on_ = true;
    if (tm_ev_.empty()) {
      tm_ev_.resize(2 * TM_CAP);
      // timing-only events: no system-scope fence (its L2 write-back and
      // invalidate around every timed dispatch left gaps of about 5 us
      // before and after it)
      for (auto& e : tm_ev_) TG_CHECK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    }
    tm_id_ = id;
    tm_ms_ = 0.0;
    tm_launches_ = 0;
    tm_work_ = 0;
    tm_err_ = false;
    return hipSuccess;
  }
  hipError_t timer_read(double* ms, long long* launches, double* work_bytes) override {
    TG_CHECK(timer_flush());
    if (tm_err_) return hipErrorUnknown;
    *ms = tm_ms_;
    *launches = tm_launches_;
    *work_bytes = (double)tm_work_ * unit_bytes(tm_id_);
    return hipSuccess;
  }

 private:
  static constexpr int TM_CAP = 1024;
  template <class F>
  void timed(int id, int work, F&& launch) {
    if (id != tm_id_ || !tm_on_) {
      launch();
      return;
    }
    if (tm_used_ == TM_CAP && timer_flush() != hipSuccess) tm_err_ = true;
    if (tm_used_ == TM_CAP) {  // the flush failed: launch untimed
      launch();
      return;
    }
    // the launch records the pair with its own dispatch (klaunch)
    LaunchEvents& pe = pending_events();
    pe.start = tm_ev_[2 * tm_used_];
    pe.stop = tm_ev_[2 * tm_used_ + 1];
    launch();
    if (pe.start != nullptr) {  // not a klaunch launch: no timestamps taken
      pe.start = pe.stop = nullptr;
      tm_err_ = true;
    }
    ++tm_used_;
    ++tm_launches_;
    tm_work_ += work;
  }
  hipError_t timer_flush() {
    if (tm_used_ == 0) return hipSuccess;
    TG_CHECK(hipEventSynchronize(tm_ev_[2 * tm_used_ - 1]));
    for (int i = 0; i < tm_used_; ++i) {
      float ms = 0.f;
      TG_CHECK(hipEventElapsedTime(&ms, tm_ev_[2 * i], tm_ev_[2 * i + 1]));
      tm_ms_ += ms;
    }
    tm_used_ = 0;
    return hipSuccess;
  }

  // Launch predicated iterations in chunks; synchronize only to read the
  // done flags between chunks.
  // est: expected iteration count of this solve (< 0: the last solve's);
  // exact: est is the count of an identical earlier solve (a segment
  // recompute), else one more is launched at once to spare a second check.
  hipError_t pcg_loop(const Ctx& c, int est = -1, bool exact = false) {
    if (graph_budget_ > 0) {
      // graph capture: a fixed, predicated iteration budget, no host reads;
      // per solve (its last eager count + 25% + 4) when known
      int budget = graph_budget_;
      const std::vector<int>& h = hist_[kind_];
      if (graph_per_solve_ && seq_ < h.size())
        budget = std::min(graph_budget_, h[seq_] + h[seq_] / 4 + 4);
      ++seq_;
      cur_budget_ = budget;
      for (int i = 0; i < budget; ++i) pcg_iteration(c);
      return hipGetLastError();
    }
    int launched = 0;
    const int base = est >= 0 ? est : its_est_;
    int chunk = std::max(1, base + (exact ? 0 : 1));
    int maxseen = 0;
    while (launched < d_.maxit) {
      const int k = std::min(chunk, d_.maxit - launched);
      for (int i = 0; i < k; ++i) pcg_iteration(c);
      TG_LAUNCH_CHECK();
      launched += k;
      TG_CHECK(hipMemcpyAsync(hsc_.data(), c.sc, c.nb * sizeof(ProbScalars), hipMemcpyDeviceToHost,
                              st_));
      TG_CHECK(hipStreamSynchronize(st_));
      bool all = true;
      for (int b = 0; b < c.nb; ++b) {
        all = all && hsc_[b].done;
        maxseen = std::max(maxseen, hsc_[b].its);
        call_status_ |= hsc_[b].status;
      }
      if (all) break;
      chunk = std::max(2, base / 4);
    }
    its_est_ = std::max(1, maxseen);
    last_its_ = maxseen;
    its_max_call_ = std::max(its_max_call_, maxseen);
    rec_.push_back(maxseen);
    ++seq_;
    if (tm_id_ != KT_NONE && tm_on_) {
      long long eff = 0;
      for (int b = 0; b < c.nb; ++b) eff += hsc_[b].its;
      tm_work_ += eff;
    }
    return hipSuccess;
  }

  // Forward steps n0..n1-1 from the stored c^{n0}.  initial: the first
  // forward of a call (writes checkpoints, keeps the last segment); else a
  // recompute of one segment (keeps its states).
  hipError_t fwd_steps(const Ctx& c, int n0, int n1, bool initial) {
    const int s = d_.s;
    const int last_start = (d_.nseg - 1) * s;
    // every step after the first starts from the previous step's increment;
    // a recompute takes the increment entering its segment from where the
    // initial forward stored it, so it repeats those solves bit for bit
    if (!initial && n0 > 0) copy_spec(c, (cx<T>*)w_.incr, ckd(n0 / s));
    for (int n = n0; n < n1; ++n) {
      if (initial && n > 0 && n % s == 0) copy_spec(c, ckd(n / s), (cx<T>*)w_.incr);
      const int hb = (n > 0 ? 1 : 0) | (n + 1 < d_.nt ? 2 : 0);
      ZArgs a = zargs(c);
      if (n == n0) {
        a.Cin = cn_ptr_for(n, initial); a.cin_bs = c.traj_bs;
        launch_z<ZS_FWD_FIRST>(a, c.nb);
      } else {
        TG_CHECK(inv_xy(c, c.X, c.T1));
        a.Xs = c.T1;
        if (n % s == 0) {
          // segment boundary (initial forward only): checkpoint c^n, b^{n-1}
          a.Cst = ck(n / s); a.cst_bs = c.traj_bs;
          a.Bst = ckb(n / s); a.bst_bs = c.traj_bs;
        } else if (!initial || n - 1 >= last_start) {
          a.Cst = segc(n % s); a.cst_bs = c.traj_bs;
          a.Bst = segb((n - 1) % s); a.bst_bs = c.traj_bs;
        }
        launch_z<ZS_FWD>(a, c.nb);
      }
      TG_LAUNCH_CHECK();
      if (initial) {
        // a recompute repeats these solves exactly: keep their counts
        TG_CHECK(step_solve(c, false, est_fwd_, false, hb));
        if ((int)fwd_its_.size() < d_.nt) fwd_its_.assign(d_.nt, -1);
        fwd_its_[n] = est_fwd_ = last_its_;
      } else {
        const int e = n < (int)fwd_its_.size() ? fwd_its_[n] : -1;
        TG_CHECK(step_solve(c, false, e, e >= 0, hb));
      }
    }
    TG_CHECK(inv_xy(c, c.X, c.T1));
    ZArgs a = zargs(c);
    a.Xs = c.T1;
    if (!initial || n1 - 1 >= last_start) {
      a.Bst = segb((n1 - 1) % s); a.bst_bs = c.traj_bs;
    }
    if (initial) {
      a.Cst = cT_; a.cst_bs = REAL;
    }
    launch_z<ZS_FWD_LAST>(a, c.nb);
    TG_LAUNCH_CHECK();
    return hipSuccess;
  }
  T* cn_ptr_for(int n, bool) { return ck(n / d_.s); }

  // Make segment j's states live in segc/segb (recompute if needed).
  hipError_t ensure_segment(int j) {
    if (live_seg_ == j) return hipSuccess;
    const int n0 = j * d_.s, n1 = std::min(n0 + d_.s, d_.nt);
    TG_CHECK(fwd_steps(prim(), n0, n1, false));
    live_seg_ = j;
    return hipSuccess;
  }

  // Reverse sweep.  lamT: cotangent on c(T) ([nb][n^3], stride lam_bs).
  // gn: Gauss-Newton adjoint (no rho/k_f accumulation).
  hipError_t adjoint_sweep(const Ctx& c, const T* lamT, long long lam_bs, bool gn) {
    for (int j = d_.nseg - 1; j >= 0; --j) {
      // A recompute of the primary context reuses its spectral buffers:
      // park the adjoint state (X) in the real scratch field meanwhile
      // (free once the first reverse step has consumed lambda_T).
      const bool park = j < d_.nseg - 1 && live_seg_ != j && c.X == prim().X;
      if (park) copy_spec(c, (cx<T>*)w_.lam, c.X);
      TG_CHECK(ensure_segment(j));
      if (park) copy_spec(c, c.X, (cx<T>*)w_.lam);
      const int n0 = j * d_.s, n1 = std::min(n0 + d_.s, d_.nt);
      for (int n = n1 - 1; n >= n0; --n) {
        ZArgs a = zargs(c);
        a.want_grho = gn ? 0 : 1;
        if (!gn) a.Qr = qr_;
        a.Bn = bn_ptr(n); a.bn_bs = c.traj_bs;
        a.Cn = cn_ptr(n); a.cn_bs = c.traj_bs;
        if (n == d_.nt - 1) {
          a.Cin = lamT; a.cin_bs = lam_bs;
          launch_z<ZS_ADJ_FIRST>(a, c.nb);
        } else {
          TG_CHECK(inv_xy(c, c.X, c.T1));
          a.Xs = c.T1;
          launch_z<ZS_ADJ>(a, c.nb);
        }
        TG_LAUNCH_CHECK();
        if (!gn) {
          k_finalize<FIN_GRHO><<<c.nb, 256, 0, st_>>>(c.sc, c.part, sch_.z_nblk, 1.0, 0, 0);
          TG_LAUNCH_CHECK();
        }
        TG_CHECK(step_solve(c, true, est_adj_));
        est_adj_ = last_its_;
        if (!gn && qk_ != nullptr) TG_CHECK(coupling_diffusion(c));
        // lam_a = mu + tau k_f A_m mu; g_k += tau <A_m mu, a + b>
        sch_.x_inv_grad(0, c.X, nullptr, c.T1, c.T2, c.sc, nullptr, tau_, 0, c.nb, st_);
        matvec_mid(c, c.T1, c.T2, c.T3, 0);
        sch_.x_fwd_div(XM_POST_ADJ, c.T1, c.T2, c.X, nullptr, c.S, c.sc, c.part, tau_, 0,
                       gn ? 0 : 1, c.nb, st_);
        TG_LAUNCH_CHECK();
        if (!gn) {
          k_finalize<FIN_GK><<<c.nb, 256, 0, st_>>>(c.sc, c.part, sch_.xf_nblk, tau_ / REAL, 0, 0);
          TG_LAUNCH_CHECK();
        }
      }
    }
    // tail of step 0: lam_0 = R'(c^0) lam_a, into lam()
    TG_CHECK(inv_xy(c, c.X, c.T1));
    ZArgs a = zargs(c);
    a.want_grho = gn ? 0 : 1;
    if (!gn) a.Qr = qr_;
    a.Xs = c.T1;
    a.Cn = ck(0); a.cn_bs = c.traj_bs;
    a.Cst = lam(0); a.cst_bs = REAL;
    launch_z<ZS_ADJ_LAST>(a, c.nb);
    TG_LAUNCH_CHECK();
    if (!gn) {
      k_finalize<FIN_GRHO><<<c.nb, 256, 0, st_>>>(c.sc, c.part, sch_.z_nblk, 1.0, 0, 0);
      TG_LAUNCH_CHECK();
    }
    return hipSuccess;
  }

  // Per-voxel derivative in the diffusion field for one reverse step, after
  // its solve left mu in X and s = a + b in S (both spectral, kept for the
  // k_f gradient that follows): the gradient rows of s (into R, P and the
  // real cotangent buffer, free during the sweep) and of mu (T1..T3), then
  // one z pass that forms -tau k_f sum_j D_j mu D_j s into qk.
  hipError_t coupling_diffusion(const Ctx& c) {
    cx<T>* Q8 = (cx<T>*)w_.lam;   // n^3 reals = one packed half spectrum
    sch_.x_inv_grad(0, c.S, nullptr, c.R, c.P, c.sc, nullptr, tau_, 0, c.nb, st_);
    sch_.y_inv_grad(c.R, c.P, Q8, c.sc, 0, c.nb, 0, 1, st_);
    sch_.x_inv_grad(0, c.X, nullptr, c.T1, c.T2, c.sc, nullptr, tau_, 0, c.nb, st_);
    sch_.y_inv_grad(c.T1, c.T2, c.T3, c.sc, 0, c.nb, 0, 1, st_);
    sch_.z_qgrad(c.T1, c.T2, c.T3, c.R, c.P, Q8, qk_, c.sc, tau_, c.nb, st_);
    TG_LAUNCH_CHECK();
    return hipSuccess;
  }

  // one semi-Lagrangian step of L fields; w_den: divide by (1 - hdt w)
  void sl_step(const T* src, T* dst, const T* disp, int L, const T* w_den, double hdt) {
    if constexpr (N >= 32) {
      // halo of 3 cells: stencils of points displaced by less than 2 cells
      // per step stay in the tile (larger ones gather from global memory);
      // a wider halo costs more in its tile loads than it saves
      using TL = SLTile<T, N, 3>;
      k_sl_step_lds<T, N, 3><<<TL::NBLK, 256, 0, st_>>>(src, dst, disp, L, w_den, hdt, 1.0, 0.0);
    } else {
      // small grids: direct gathers (the numerator factor is already in src)
      constexpr int GB = (int)((REAL + 255) / 256);
      k_sl_step<T, N><<<GB, 256, 0, st_>>>(src, dst, disp, L, nullptr, 0.0);
      if (w_den != nullptr)
        k_sl_div<T><<<(int)std::min<long long>(GB, 8192), 256, 0, st_>>>(dst, w_den, hdt, L,
                                                                         REAL);
    }
  }

  // Heun foot of the stationary velocity s v (s = +-dt/h).  From 32^3 one
  // LDS-tiled step forms the predictor, interpolates v there and averages;
  // smaller grids write the predictor displacement into the scratch fields,
  // interpolate by direct gathers and average in place.
  hipError_t sl_foot(const T* v, T* disp, double s) {
    if constexpr (N >= 32) {
      // one launch: predictor, interpolation and average (see k_sl_step_lds)
      using TL = SLTile<T, N, 3>;
      k_sl_step_lds<T, N, 3, true><<<TL::NBLK, 256, 0, st_>>>(v, disp, v, 3, nullptr, 0.0, s,
                                                               0.5 * s);
      TG_LAUNCH_CHECK();
      return hipSuccess;
    }
    const int blocks = (int)std::min<long long>((3 * REAL + 255) / 256, 8192);
    k_sl_scale3<T><<<blocks, 256, 0, st_>>>(v, tr_scratch(), s, REAL);
    TG_LAUNCH_CHECK();
    sl_step(v, disp, tr_scratch(), 3, nullptr, 0.0);
    TG_LAUNCH_CHECK();
    k_sl_heun3<T><<<blocks, 256, 0, st_>>>(v, disp, s, REAL);
    TG_LAUNCH_CHECK();
    return hipSuccess;
  }

  // transport workspace: levels [(ntr + 1)][L][n^3], feet [2][3][n^3],
  // adjoint levels [2][L][n^3], foot scratch [3][n^3]
  T* tr_level(int k) { return tr_ws_ + (size_t)k * tr_L_ * REAL; }
  T* tr_disp(int a) { return tr_level(tr_nt_ + 1) + (size_t)a * 3 * REAL; }
  T* tr_lam(int a) { return tr_disp(2) + (size_t)a * tr_L_ * REAL; }
  T* tr_scratch() { return tr_lam(2); }

  void copy_real(T* dst, const T* src, long long n) {
    // n reals = n / 2 complex (n^3 is even)
    const long long nc = n / 2;
    const int blocks = (int)std::min<long long>((nc + 255) / 256, 8192);
    k_copy_spec<T><<<blocks, 256, 0, st_>>>((cx<T>*)dst, (const cx<T>*)src, nc);
  }

  // b += coef sum_l lam_l grad m_l (spectral gradients through the plan's
  // transform passes: z R2C, y and x forward with the gradient prologue,
  // y inverse of the gradient rows, z C2R times lam)
  hipError_t body_force(const T* m, const T* lam, int L, double coef, T* bf) {
    using Z = ZP<T, N>;
    Ctx c = prim();
    for (int l = 0; l < L; ++l) {
      k_z_r2c<T, N, Z::RW><<<dim3(Z::NBLK, 1), Z::NT, 0, st_>>>(m + (size_t)l * REAL, c.T1);
      TG_LAUNCH_CHECK();
      sch_.y_plain(false, c.T1, nullptr, 1, st_);
      sch_.x_fwd_state(c.T1, c.X, c.T2, c.T3, nullptr, 1, st_);
      sch_.y_inv_grad(c.T2, c.T3, c.T1, c.sc, 0, 1, 0, 1, st_);
      k_z_bforce<T, N, Z::RW><<<dim3(Z::NBLK, 1), Z::NT, 0, st_>>>(
          c.T2, c.T3, c.T1, lam + (size_t)l * REAL, bf, coef);
      TG_LAUNCH_CHECK();
    }
    return hipSuccess;
  }

  void copy_spec(const Ctx& c, cx<T>* dst, const cx<T>* src) {
    const long long n = (long long)c.nb * SPECN;
    const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
    k_copy_spec<T><<<blocks, 256, 0, st_>>>(dst, src, n);
  }

  // g[b] = Phi^T lam(b)
  hipError_t phit(const Ctx& c, double* out, long long g_bs = -1) {
    if (g_bs < 0) g_bs = (long long)d_.n_p * 3 * N;
    using PT = PhiTK<N>;
    k_phit<T, N><<<dim3(PT::NBLK, c.nb, (d_.n_p + PT::G - 1) / PT::G), 256, 0, st_>>>(
        lam(0), REAL, w_.gfac, g_bs, mask_, c.m_bs, w_.partphi, d_.n_p);
    TG_LAUNCH_CHECK();
    k_phit_final<<<dim3(d_.n_p, c.nb), 256, 0, st_>>>(w_.partphi, PT::NBLK, d_.n_p, out, d_.n_p);
    TG_LAUNCH_CHECK();
    return hipSuccess;
  }

  SolverDims d_;
  Workspace w_;
  hipStream_t st_ = nullptr;
  const T* m_ = nullptr;      // diffusion field
  const T* mr_ = nullptr;     // reaction field
  const T* mask_ = nullptr;   // mask of Phi p (null: none)
  T* qk_ = nullptr;           // vjp outputs d J / d m(x), d J / d mr(x)
  T* qr_ = nullptr;
  int tr_nt_ = 0, tr_L_ = 0;  // last registration transport
  const T* tr_w_ = nullptr;
  T* tr_ws_ = nullptr;
  T* cT_ = nullptr;
  double dt_, tau_, h3_;
  std::vector<ProbScalars> hsc_;
  int its_est_;
  int last_its_ = 0;                  // iterations of the last eager solve
  int est_fwd_ = -1, est_adj_ = -1, est_tan_ = -1;   // running, per solve kind
  std::vector<int> fwd_its_;          // per step of the last initial forward
  int live_seg_ = -1;
  int call_status_ = 0;
  int graph_budget_ = 0;
  bool graph_per_solve_ = false;
  int cur_budget_ = 0;
  std::vector<int> hist_[3];
  std::vector<int> rec_;
  int kind_ = 0;
  size_t seq_ = 0;
  double fp32_floor_ = 0.0;      // FP32 stopping floor of the adjoint solves
  double fp32_fwd_floor_ = 0.0;  // ... of the forward, recompute and tangent solves
  int its_max_call_ = 0;
  Sched<T, N> sch_;
  int zwaves_ = 0;
  int nslab_ = 1;
  int occ_ = 1;
  int pass_C_[KT_LAST + 1] = {};
  // default layout of the z matvec's spectral rows: pairs in FP32 (16-byte
  // accesses; measured 92 against 99 us per launch at 256^3), single
  // complex values (already 16 bytes) in FP64
  static constexpr bool kZPairDefault = sizeof(T) == 4;
  int pass_occ_[KT_LAST + 1] = {};
  static bool slabs_fit(const Sched<T, N>& s, int slabs) {
    return s.yi_nblk % slabs == 0 && s.yf_nblk % slabs == 0 && s.zm_nblk % slabs == 0 &&
           s.z_nblk % slabs == 0;
  }
  ProbScalars* stat_sc_ = nullptr;
  int stat_nb_ = 0;
  // kernel timer state
  int tm_id_ = KT_NONE;
  int tm_every_ = 1;         // time the launches of one solve in tm_every_
  long long tm_solves_ = 0;  // solves since the timer was enabled
  bool tm_on_ = true;        // the current solve's launches are timed
  std::vector<hipEvent_t> tm_ev_;
  int tm_used_ = 0;
  double tm_ms_ = 0.0;
  long long tm_launches_ = 0;
  long long tm_work_ = 0;
  bool tm_err_ = false;  // an event call failed since the timer was enabled

 public:
  ~Solver() override {
    for (auto& e : tm_ev_) (void)hipEventDestroy(e);
  }
};

template <typename T>
hipError_t fill_twiddles() {
  static cx<T> host[TW_N];
  for (int k = 0; k < TW_N; ++k) {
    const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)k / TW_N;
    host[k].x = (T)cosl(a);
    host[k].y = (T)sinl(a);
  }
  if (sizeof(T) == 8) return hipMemcpyToSymbol(HIP_SYMBOL(g_tw64), host, sizeof(host));
  return hipMemcpyToSymbol(HIP_SYMBOL(g_tw32), host, sizeof(host));
}

}  // namespace tg
