// C-ABI of the tumor forward/adjoint library: plan validation, workspace
// layout and dispatch to the per-precision solvers.  Host code only.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/tumorgrad.h"
#include "tg_internal.h"

struct tg_plan {
  tg_desc d;
  std::vector<double> centres;   // host copy [batch][n_p][3]
  tg::SolverDims dims;
  size_t ws_bytes = 0;
  void* ws = nullptr;
  tg::Workspace w{};
  std::unique_ptr<tg::ISolver> solver;
  bool have_traj = false;
  hipStream_t last_stream = nullptr;
};

namespace {

constexpr size_t ALIGN = 256;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

bool pow2_in_range(int n) {
  return n == 8 || n == 16 || n == 32 || n == 64 || n == 128 || n == 256;
}

// Byte offsets of every workspace buffer (nullptr base gives the size).
size_t layout(const tg_plan& p, char* base, tg::Workspace* w) {
  const tg::SolverDims& d = p.dims;
  const size_t es = p.d.prec == TG_FP64 ? 8 : 4;
  const size_t n3 = (size_t)d.n * d.n * d.n;
  const size_t spec = n3 * es;  // packed half spectrum: n^3/2 complex
  const size_t real = n3 * es;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* ptr = base ? base + off : nullptr;
    off += align_up(bytes);
    return ptr;
  };
  for (int i = 0; i < 8; ++i) w->spec[i] = take(spec * d.batch);
  for (int i = 0; i < 8; ++i) w->dspec[i] = d.dirs > 0 ? take(spec * d.dirs) : nullptr;
  w->ck = take(real * d.batch * d.nseg);
  w->ckb = take(real * d.batch * d.nseg);
  w->segc = take(real * d.batch * d.s);
  w->segb = take(real * d.batch * d.s);
  const int bl = d.batch > d.dirs ? d.batch : d.dirs;
  w->lam = take(real * bl);
  w->gfac = (double*)take(sizeof(double) * d.batch * d.n_p * 3 * d.n);
  w->centres = (double*)take(sizeof(double) * d.batch * d.n_p * 3);
  w->sc = (tg::ProbScalars*)take(sizeof(tg::ProbScalars) * (d.batch + d.dirs));
  w->part = (double*)take(sizeof(double) * (d.batch + d.dirs) * tg::NSLOT * tg::MAXBLK);
  w->partphi = (double*)take(sizeof(double) * bl * d.n_p * tg::phi_blocks_for(d.n));
  return off;
}

tg_status from_hip(hipError_t e) { return e == hipSuccess ? TG_OK : TG_ERR_HIP; }

tg_status from_bits(int bits) {
  if (bits & (tg::STAT_BREAKDOWN | tg::STAT_NONFINITE)) return TG_ERR_NUMERIC;
  if (bits & tg::STAT_NOT_CONVERGED) return TG_ERR_NOT_CONVERGED;
  return TG_OK;
}

std::mutex g_tw_mu;
std::vector<int> g_tw_done;  // per device: bit 1 = f32 table, bit 2 = f64 table

hipError_t ensure_twiddles(tg_precision prec) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_tw_mu);
  if ((int)g_tw_done.size() <= dev) g_tw_done.resize(dev + 1, 0);
  const int bit = prec == TG_FP64 ? 2 : 1;
  if (g_tw_done[dev] & bit) return hipSuccess;
  e = prec == TG_FP64 ? tg::init_twiddles_f64() : tg::init_twiddles_f32();
  if (e == hipSuccess) g_tw_done[dev] |= bit;
  return e;
}

}  // namespace

extern "C" {

int tg_version(void) { return 1; }

const char* tg_status_string(tg_status s) {
  switch (s) {
    case TG_OK: return "ok";
    case TG_ERR_ARG: return "invalid argument";
    case TG_ERR_STATE: return "invalid call order (no forward trajectory)";
    case TG_ERR_NOT_CONVERGED: return "PCG did not converge within pcg_maxit";
    case TG_ERR_NUMERIC: return "PCG breakdown or non-finite values";
    case TG_ERR_HIP: return "HIP runtime error";
    case TG_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
  }
  return "unknown status";
}

tg_status tg_plan_create(const tg_desc* desc, tg_plan** out) {
  if (desc == nullptr || out == nullptr) return TG_ERR_ARG;
  *out = nullptr;
  const tg_desc& d = *desc;
  if (!pow2_in_range(d.n)) return TG_ERR_ARG;
  if (d.nt < 1 || !(d.T > 0.0) || !std::isfinite(d.T)) return TG_ERR_ARG;
  if (d.n_p < 1 || d.n_p > 4096 || d.centres == nullptr) return TG_ERR_ARG;
  if (!(d.sigma > 0.0) || !std::isfinite(d.sigma)) return TG_ERR_ARG;
  if (!(d.pcg_rtol > 0.0) || !(d.pcg_rtol < 1.0)) return TG_ERR_ARG;
  if (d.pcg_maxit < 1 || d.ckpt_stride < 0) return TG_ERR_ARG;
  if (d.prec != TG_FP64 && d.prec != TG_FP32_MIXED) return TG_ERR_ARG;
  if (d.batch < 1 || d.batch > 4096 || d.max_hvp_dirs < 0 || d.max_hvp_dirs > 256)
    return TG_ERR_ARG;
  const size_t nc = (size_t)d.batch * d.n_p * 3;
  for (size_t i = 0; i < nc; ++i)
    if (!std::isfinite(d.centres[i])) return TG_ERR_ARG;
  tg_plan* p = new tg_plan;
  p->d = d;
  p->centres.assign(d.centres, d.centres + nc);
  p->d.centres = nullptr;
  tg::SolverDims& s = p->dims;
  s.n = d.n;
  s.nt = d.nt;
  s.n_p = d.n_p;
  s.batch = d.batch;
  s.dirs = d.max_hvp_dirs;
  s.s = (d.ckpt_stride == 0 || d.ckpt_stride > d.nt) ? d.nt : d.ckpt_stride;
  s.nseg = (d.nt + s.s - 1) / s.s;
  s.T = d.T;
  s.sigma = d.sigma;
  s.rtol = d.pcg_rtol;
  s.maxit = d.pcg_maxit;
  tg::Workspace w;
  p->ws_bytes = layout(*p, nullptr, &w);
  *out = p;
  return TG_OK;
}

tg_status tg_plan_workspace_bytes(const tg_plan* plan, size_t* bytes) {
  if (plan == nullptr || bytes == nullptr) return TG_ERR_ARG;
  *bytes = plan->ws_bytes;
  return TG_OK;
}

tg_status tg_plan_bind(tg_plan* plan, void* d_ws, size_t bytes) {
  if (plan == nullptr) return TG_ERR_ARG;
  if (d_ws == nullptr || bytes < plan->ws_bytes || ((uintptr_t)d_ws % ALIGN) != 0)
    return TG_ERR_WORKSPACE;
  hipError_t e = ensure_twiddles(plan->d.prec);
  if (e != hipSuccess) return TG_ERR_HIP;
  plan->ws = d_ws;
  layout(*plan, (char*)d_ws, &plan->w);
  e = hipMemcpy(plan->w.centres, plan->centres.data(), plan->centres.size() * sizeof(double),
                hipMemcpyHostToDevice);
  if (e != hipSuccess) return TG_ERR_HIP;
  plan->solver.reset(plan->d.prec == TG_FP64 ? tg::make_solver_f64(plan->dims, plan->w)
                                              : tg::make_solver_f32(plan->dims, plan->w));
  if (!plan->solver) return TG_ERR_ARG;
  plan->have_traj = false;
  return TG_OK;
}

tg_status tg_forward(tg_plan* plan, const double* d_p, const double* d_rho_f, const double* d_k_f,
                     const void* d_m, void* d_cT, void* stream) {
  if (plan == nullptr || d_p == nullptr || d_rho_f == nullptr || d_k_f == nullptr ||
      d_m == nullptr || d_cT == nullptr)
    return TG_ERR_ARG;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  plan->last_stream = (hipStream_t)stream;
  plan->have_traj = false;
  hipError_t e = plan->solver->forward(d_p, d_rho_f, d_k_f, d_m, d_cT, (hipStream_t)stream);
  if (e != hipSuccess) return TG_ERR_HIP;
  plan->have_traj = true;
  return from_bits(plan->solver->last_status());
}

tg_status tg_vjp(tg_plan* plan, const void* d_lamT, double* d_gp, double* d_grho, double* d_gkf,
                 void* stream) {
  if (plan == nullptr || d_lamT == nullptr || d_gp == nullptr || d_grho == nullptr ||
      d_gkf == nullptr)
    return TG_ERR_ARG;
  if (!plan->have_traj) return TG_ERR_STATE;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  plan->last_stream = (hipStream_t)stream;
  hipError_t e = plan->solver->vjp(d_lamT, nullptr, nullptr, d_gp, d_grho, d_gkf,
                                   (hipStream_t)stream);
  if (e != hipSuccess) return TG_ERR_HIP;
  return from_bits(plan->solver->last_status());
}

tg_status tg_adjoint_misfit(tg_plan* plan, const void* d_cobs, double* d_J, double* d_gp,
                            double* d_grho, double* d_gkf, void* stream) {
  if (plan == nullptr || d_cobs == nullptr || d_J == nullptr || d_gp == nullptr ||
      d_grho == nullptr || d_gkf == nullptr)
    return TG_ERR_ARG;
  if (!plan->have_traj) return TG_ERR_STATE;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  plan->last_stream = (hipStream_t)stream;
  hipError_t e = plan->solver->vjp(nullptr, d_cobs, d_J, d_gp, d_grho, d_gkf, (hipStream_t)stream);
  if (e != hipSuccess) return TG_ERR_HIP;
  return from_bits(plan->solver->last_status());
}

tg_status tg_hessvec_gn(tg_plan* plan, int ndir, const double* d_V, double* d_HV, void* stream) {
  if (plan == nullptr || d_V == nullptr || d_HV == nullptr) return TG_ERR_ARG;
  if (plan->d.batch != 1 || ndir < 1 || ndir > plan->d.max_hvp_dirs) return TG_ERR_ARG;
  if (!plan->have_traj) return TG_ERR_STATE;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  plan->last_stream = (hipStream_t)stream;
  hipError_t e = plan->solver->hessvec(ndir, d_V, d_HV, (hipStream_t)stream);
  if (e != hipSuccess) return TG_ERR_HIP;
  return from_bits(plan->solver->last_status());
}

tg_status tg_stats(tg_plan* plan, tg_solve_stats* out) {
  if (plan == nullptr || out == nullptr) return TG_ERR_ARG;
  std::memset(out, 0, sizeof(*out));
  if (!plan->solver) return TG_ERR_WORKSPACE;
  tg::CallStats s;
  hipError_t e = plan->solver->read_stats(&s, plan->last_stream);
  if (e != hipSuccess) return from_hip(e);
  out->solves = s.solves;
  out->pcg_its_total = s.its_total;
  out->pcg_its_max = s.its_max;
  out->status_bits = s.status;
  out->worst_rel_residual = s.worst_rel_residual;
  return TG_OK;
}

tg_status tg_kernel_timer(tg_plan* plan, int kernel_id) {
  if (plan == nullptr || kernel_id < tg::KT_NONE || kernel_id > tg::KT_PCG_UPDATE) return TG_ERR_ARG;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  return from_hip(plan->solver->timer_enable(kernel_id));
}

tg_status tg_kernel_timer_read(tg_plan* plan, double* total_ms, long long* launches,
                               double* work_bytes) {
  if (plan == nullptr || total_ms == nullptr || launches == nullptr || work_bytes == nullptr)
    return TG_ERR_ARG;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  return from_hip(plan->solver->timer_read(total_ms, launches, work_bytes));
}

void tg_plan_destroy(tg_plan* plan) { delete plan; }

}  // extern "C"
