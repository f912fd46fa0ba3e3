// Host/device shared definitions of the tumor forward/adjoint library.
#pragma once
#include <cstddef>
#include <cstdint>
#include <hip/hip_runtime_api.h>

#include "../../include/tumorgrad.h"

namespace tg {

// Per-problem solver scalars kept in device memory.  Dot products, norms,
// PCG step lengths and all gradient accumulators are FP64 in both
// precision modes.
struct ProbScalars {
  double rho;       // <r, M r> of the current PCG residual
  double alpha;     // PCG step length
  double beta;      // PCG direction update factor
  double tol2;      // (rtol ||rhs||)^2, grid norm
  double rr;        // ||r||^2 (grid norm) of the latest residual
  double rhs2;      // ||rhs||^2 (grid norm) of the current solve
  double pq;        // <p, q>
  double kf, rhof;  // k_f and rho_f of this problem
  double kbar;      // preconditioner coefficient k_f max(m)
  double mmax;      // max(m)
  double g_rho, g_k;  // time-integrated gradient accumulators
  double J;         // misfit
  double worst;     // worst final relative residual over solves of a call
  double pad0;
  int its;          // iterations of the current solve
  int done;         // current solve finished (converged or failed)
  int status;       // OR of TG_STAT_* over the solves of a call
  int first;        // next PCG iteration is the first one
  int its_total;    // iterations summed over the solves of a call
  int solves;       // number of solves in the call
  int its_max;      // largest iteration count of one solve
  int pad1;
};

// STAT_BAD_PARAM: k_f < 0, or k_f or rho_f not finite (device values, so
// found by k_init_scalars); every solve of the problem is then skipped.
enum : int { STAT_NOT_CONVERGED = 1, STAT_BREAKDOWN = 2, STAT_NONFINITE = 4, STAT_BAD_PARAM = 8 };

constexpr int NSLOT = 4;      // simultaneous partial sums per reducing kernel
constexpr int MAXBLK = 16384;  // max workgroups of a reducing kernel per problem
constexpr int NSPEC = 7;       // spectral work fields per problem

struct SolverDims {
  int n, nt, n_p, batch, dirs, s, nseg;
  double T, sigma, rtol;
  int maxit;
};

// Views into the caller-provided workspace.
struct Workspace {
  void* spec[NSPEC];  // X, R, P, T1, T2, T3, S: [batch][n^3/2] complex
  void* dspec[NSPEC]; // the same set for Hessian directions: [dirs][n^3/2]
  void* ck;           // [nseg][batch][n^3] checkpoints c^{j s}
  void* ckb;          // [nseg][batch][n^3] b^{j s - 1} (j >= 1)
  void* segc;         // [s][batch][n^3]  c^n within the live segment
  void* segb;         // [s][batch][n^3]  b^n within the live segment
  void* ahat;         // [batch][n^3/2] complex: a-hat of the current forward step
  void* incr;         // [batch][n^3/2] complex: d = b - a of the previous forward step
  void* ckd;          // [nseg][batch][n^3/2] complex: d entering each segment
  void* lam;          // [max(batch, dirs)][n^3] real scratch field
  double* gfac;       // [batch][n_p][3][n] Gaussian factors
  double* centres;    // [batch][n_p][3]
  ProbScalars* sc;    // [batch + dirs]
  double* part;       // [batch + dirs][NSLOT][MAXBLK]
  double* partphi;    // [max(batch, dirs)][n_p][phi blocks]
};

struct CallStats {
  int solves, its_total, its_max, status;
  double worst_rel_residual;
};

// Streaming reference kernel (tg_stream_probe): fields of n4 float4 values,
// a..c and d, e read, d and e written.
hipError_t stream7_launch(const void* a, const void* b, const void* c, void* d, void* e,
                          long long n4, hipStream_t st);

class ISolver {
 public:
  virtual ~ISolver() {}
  // forward(p, rho, kf, m, mr, mask) -> c(T); pointers are device pointers
  // with per-problem strides n_p, 1, 1, n^3, n^3, n^3, n^3.  m is the
  // diffusion field, mr the reaction field (null: m), mask multiplies Phi p
  // (null: none).
  virtual hipError_t forward(const double* p, const double* rho, const double* kf,
                             const void* m, const void* mr, const void* mask, void* cT,
                             hipStream_t st) = 0;
  // nlab > 0 adds the label misfit of fields mlab, mpat ([batch][nlab][n^3])
  // to the misfit against cobs.  qk, qr (null: skip) receive the per-voxel
  // derivatives in the diffusion and reaction fields ([batch][n^3]).
  virtual hipError_t vjp(const void* lamT, const void* cobs, int nlab, const void* mlab,
                         const void* mpat, double* J, double* gp, double* grho, double* gkf,
                         void* qk, void* qr, hipStream_t st) = 0;
  virtual hipError_t hessvec(int ndir, const double* V, double* HV, hipStream_t st) = 0;
  // Registration transport (batch 1): L label fields m0 ([L][n^3]) carried
  // by the stationary velocity v ([3][n^3]) over ntr steps of 1/ntr; m1
  // receives the last level.  tws: [(ntr + 1) L + 6 + 2 L + 3][n^3] reals
  // (trajectory, the two feet, two adjoint levels, foot scratch).  w = div v (null: 0)
  // is used by the adjoint.
  virtual hipError_t transport(int ntr, int L, const void* v, const void* w, const void* m0,
                               void* m1, void* tws, hipStream_t st) = 0;
  // Adjoint of the last transport from lam1 ([L][n^3]) at t = 1: lam0 and the
  // body force ([3][n^3]).
  virtual hipError_t transport_adjoint(const void* lam1, void* lam0, void* body,
                                       hipStream_t st) = 0;
  virtual hipError_t read_stats(CallStats* out, hipStream_t st) = 0;
  // OR of the PCG status bits the host saw during the last call
  virtual int last_status() const = 0;
  // Event timing of one kernel of the PCG iteration (KT_* id; KT_NONE off).
  virtual hipError_t timer_enable(int id, int every) = 0;
  virtual hipError_t timer_read(double* ms, long long* launches, double* work_bytes) = 0;
  // Transform tile shapes: pencils per x/y workgroup (8, 16, 32), waves
  // per z workgroup (1, 2, 4), x slabs of the y-z-y pass chain (1, 2, 4, 8)
  // and an occupancy floor for the PCG pass kernels (1: none, 4: >= 4 waves
  // per SIMD); 0 = default.  False if not available.
  virtual bool set_schedule(int C, int zwaves, int slabs, int occ) = 0;
  // Graph-capture mode: every PCG solve runs a fixed number of predicated
  // iterations with no host synchronization: `budget`, or with per_solve
  // the solve's count in the last eager call of the same kind + 25% + 4
  // (at most `budget`) (budget 0 = eager, adaptive).
  virtual void set_graph_budget(int budget, bool per_solve) = 0;
  // Largest PCG iteration count of one solve seen since the last forward.
  virtual int its_max_last_call() const = 0;
  virtual void get_schedule(int* C, int* zwaves, int* slabs, int* occ) const = 0;
  // Per-pass override of the tile shape after set_schedule (KT_* id).
  virtual bool set_pass(int id, int C, int occ) = 0;
  virtual bool get_pass(int id, int* C, int* occ) const = 0;
};

enum KernelId : int {
  KT_NONE = 0,
  KT_X_INV_GRAD = 1,
  KT_Y_INV_GRAD = 2,
  KT_Z_MATVEC = 3,
  KT_Y_FWD_DIV = 4,
  KT_X_FWD_DIV = 5,
  KT_LAST = KT_X_FWD_DIV
};

// Plan binding shared by tg_plan_bind and tg_forward_static (host only).
// plan_bind_ws: bind d_ws as the workspace (tg_plan_bind's checks and
// set-up, without the static-scratch bookkeeping).  plan_unbind: drop the
// solver and workspace (the plan must be bound again before use).
// plan_workspace: the bound workspace or nullptr.
tg_status plan_bind_ws(tg_plan* plan, void* d_ws, size_t bytes);
void plan_unbind(tg_plan* plan);
const void* plan_workspace(const tg_plan* plan);
// tg_forward_static's bookkeeping: forget `plan` as the owner of any
// device's static scratch (called when it is rebound or destroyed).
void static_scratch_release(tg_plan* plan);

// Phi^T partial-block count for grid size n (workspace sizing).
int phi_blocks_for(int n);
// Solver for (precision, n); nullptr if n is not supported.  Each
// instantiation lives in its own translation unit with its own twiddle
// table, filled by init_twiddles for the current device.
ISolver* make_solver(int fp64, const SolverDims& d, const Workspace& w);
hipError_t init_twiddles(int fp64, int n);

}  // namespace tg
