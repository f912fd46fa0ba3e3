// C-ABI of the tumor forward/adjoint library: plan validation, workspace
// layout and dispatch to the per-precision solvers.  Host code only.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <mutex>
#include <set>
#include <tuple>
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
  bool have_transport = false;
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
  for (int i = 0; i < tg::NSPEC; ++i) w->spec[i] = take(spec * d.batch);
  for (int i = 0; i < tg::NSPEC; ++i) w->dspec[i] = d.dirs > 0 ? take(spec * d.dirs) : nullptr;
  w->ck = take(real * d.batch * d.nseg);
  w->ckb = take(real * d.batch * d.nseg);
  w->segc = take(real * d.batch * d.s);
  w->segb = take(real * d.batch * d.s);
  w->ahat = take(spec * d.batch);
  w->incr = take(spec * d.batch);
  w->ckd = take(spec * d.batch * d.nseg);
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
  if (bits & tg::STAT_BAD_PARAM) return TG_ERR_ARG;
  if (bits & (tg::STAT_BREAKDOWN | tg::STAT_NONFINITE)) return TG_ERR_NUMERIC;
  if (bits & tg::STAT_NOT_CONVERGED) return TG_ERR_NOT_CONVERGED;
  return TG_OK;
}

std::mutex g_tw_mu;
std::set<std::tuple<int, int, int>> g_tw_done;  // (device, fp64, n) tables filled

hipError_t ensure_twiddles(tg_precision prec, int n) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const int fp64 = prec == TG_FP64 ? 1 : 0;
  std::lock_guard<std::mutex> lk(g_tw_mu);
  const auto key = std::make_tuple(dev, fp64, n);
  if (g_tw_done.count(key)) return hipSuccess;
  e = tg::init_twiddles(fp64, n);
  if (e == hipSuccess) g_tw_done.insert(key);
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
    case TG_ERR_SCRATCH_LIMIT:
      return "plan workspace exceeds the static scratch (TG_STATIC_SCRATCH_BYTES)";
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
  tg::static_scratch_release(plan);
  return tg::plan_bind_ws(plan, d_ws, bytes);
}

}  // extern "C"

namespace tg {

tg_status plan_bind_ws(tg_plan* plan, void* d_ws, size_t bytes) {
  if (plan == nullptr) return TG_ERR_ARG;
  if (d_ws == nullptr || bytes < plan->ws_bytes || ((uintptr_t)d_ws % ALIGN) != 0)
    return TG_ERR_WORKSPACE;
  hipError_t e = ensure_twiddles(plan->d.prec, plan->d.n);
  if (e != hipSuccess) return TG_ERR_HIP;
  plan->ws = d_ws;
  layout(*plan, (char*)d_ws, &plan->w);
  e = hipMemcpy(plan->w.centres, plan->centres.data(), plan->centres.size() * sizeof(double),
                hipMemcpyHostToDevice);
  if (e != hipSuccess) return TG_ERR_HIP;
  plan->solver.reset(tg::make_solver(plan->d.prec == TG_FP64 ? 1 : 0, plan->dims, plan->w));
  if (!plan->solver) return TG_ERR_ARG;
  plan->have_traj = false;
  plan->have_transport = false;
  return TG_OK;
}

void plan_unbind(tg_plan* plan) {
  if (plan == nullptr) return;
  plan->solver.reset();
  plan->ws = nullptr;
  plan->w = tg::Workspace{};
  plan->have_traj = false;
  plan->have_transport = false;
}

const void* plan_workspace(const tg_plan* plan) { return plan ? plan->ws : nullptr; }

}  // namespace tg

extern "C" {

tg_status tg_forward_fields(tg_plan* plan, const double* d_p, const double* d_rho_f,
                            const double* d_k_f, const void* d_m_diff, const void* d_m_react,
                            const void* d_phi_mask, void* d_cT, void* stream) {
  if (plan == nullptr || d_p == nullptr || d_rho_f == nullptr || d_k_f == nullptr ||
      d_m_diff == nullptr || d_cT == nullptr)
    return TG_ERR_ARG;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  plan->last_stream = (hipStream_t)stream;
  plan->have_traj = false;
  hipError_t e = plan->solver->forward(d_p, d_rho_f, d_k_f, d_m_diff, d_m_react, d_phi_mask,
                                       d_cT, (hipStream_t)stream);
  if (e != hipSuccess) return TG_ERR_HIP;
  plan->have_traj = true;
  return from_bits(plan->solver->last_status());
}

tg_status tg_forward(tg_plan* plan, const double* d_p, const double* d_rho_f, const double* d_k_f,
                     const void* d_m, void* d_cT, void* stream) {
  return tg_forward_fields(plan, d_p, d_rho_f, d_k_f, d_m, nullptr, nullptr, d_cT, stream);
}

tg_status tg_vjp(tg_plan* plan, const void* d_lamT, double* d_gp, double* d_grho, double* d_gkf,
                 void* stream) {
  if (plan == nullptr || d_lamT == nullptr || d_gp == nullptr || d_grho == nullptr ||
      d_gkf == nullptr)
    return TG_ERR_ARG;
  if (!plan->have_traj) return TG_ERR_STATE;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  plan->last_stream = (hipStream_t)stream;
  hipError_t e = plan->solver->vjp(d_lamT, nullptr, 0, nullptr, nullptr, nullptr, d_gp, d_grho,
                                   d_gkf, nullptr, nullptr, (hipStream_t)stream);
  if (e != hipSuccess) return TG_ERR_HIP;
  return from_bits(plan->solver->last_status());
}

tg_status tg_vjp_coupling(tg_plan* plan, const void* d_lamT, double* d_gp, double* d_grho,
                          double* d_gkf, void* d_q_diff, void* d_q_react, int combine,
                          void* stream) {
  if (plan == nullptr || d_lamT == nullptr || d_gp == nullptr || d_grho == nullptr ||
      d_gkf == nullptr)
    return TG_ERR_ARG;
  if (combine != 0 && combine != 1) return TG_ERR_ARG;
  if (combine == 1) {
    // one field receives both parts: the reaction and diffusion kernels each
    // add into it in turn on the same stream
    if (d_q_diff == nullptr || d_q_react != nullptr) return TG_ERR_ARG;
    d_q_react = d_q_diff;
  }
  if (!plan->have_traj) return TG_ERR_STATE;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  plan->last_stream = (hipStream_t)stream;
  hipError_t e = plan->solver->vjp(d_lamT, nullptr, 0, nullptr, nullptr, nullptr, d_gp, d_grho,
                                   d_gkf, d_q_diff, d_q_react, (hipStream_t)stream);
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
  hipError_t e = plan->solver->vjp(nullptr, d_cobs, 0, nullptr, nullptr, d_J, d_gp, d_grho,
                                   d_gkf, nullptr, nullptr, (hipStream_t)stream);
  if (e != hipSuccess) return TG_ERR_HIP;
  return from_bits(plan->solver->last_status());
}

tg_status tg_adjoint_misfit_labels(tg_plan* plan, const void* d_cobs, int n_labels,
                                   const void* d_m_lab, const void* d_m_pat, double* d_J,
                                   double* d_gp, double* d_grho, double* d_gkf, void* stream) {
  if (plan == nullptr || d_cobs == nullptr || d_J == nullptr || d_gp == nullptr ||
      d_grho == nullptr || d_gkf == nullptr || n_labels < 0)
    return TG_ERR_ARG;
  if (n_labels > 0 && (d_m_lab == nullptr || d_m_pat == nullptr)) return TG_ERR_ARG;
  if (!plan->have_traj) return TG_ERR_STATE;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  plan->last_stream = (hipStream_t)stream;
  hipError_t e = plan->solver->vjp(nullptr, d_cobs, n_labels, d_m_lab, d_m_pat, d_J, d_gp,
                                   d_grho, d_gkf, nullptr, nullptr, (hipStream_t)stream);
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

tg_status tg_transport_workspace_bytes(const tg_plan* plan, int nt_r, int n_labels,
                                       size_t* bytes) {
  if (plan == nullptr || bytes == nullptr || nt_r < 1 || n_labels < 1) return TG_ERR_ARG;
  const size_t es = plan->d.prec == TG_FP64 ? 8 : 4;
  const size_t n3 = (size_t)plan->d.n * plan->d.n * plan->d.n;
  *bytes = ((size_t)(nt_r + 1) * n_labels + 9 + 2 * (size_t)n_labels) * n3 * es;
  return TG_OK;
}

tg_status tg_transport(tg_plan* plan, int nt_r, int n_labels, const void* d_v, const void* d_w,
                       const void* d_m0, void* d_m1, void* d_tws, size_t tws_bytes,
                       void* stream) {
  if (plan == nullptr || d_v == nullptr || d_m0 == nullptr || d_tws == nullptr)
    return TG_ERR_ARG;
  if (plan->d.batch != 1 || nt_r < 1 || n_labels < 1) return TG_ERR_ARG;
  size_t need = 0;
  tg_transport_workspace_bytes(plan, nt_r, n_labels, &need);
  if (tws_bytes < need || ((uintptr_t)d_tws % ALIGN) != 0) return TG_ERR_WORKSPACE;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  plan->last_stream = (hipStream_t)stream;
  plan->have_transport = false;
  hipError_t e = plan->solver->transport(nt_r, n_labels, d_v, d_w, d_m0, d_m1, d_tws,
                                         (hipStream_t)stream);
  if (e != hipSuccess) return TG_ERR_HIP;
  plan->have_transport = true;
  return TG_OK;
}

tg_status tg_transport_adjoint(tg_plan* plan, const void* d_lam1, void* d_lam0, void* d_body,
                               void* stream) {
  if (plan == nullptr || d_lam1 == nullptr || d_lam0 == nullptr || d_body == nullptr)
    return TG_ERR_ARG;
  if (!plan->have_transport) return TG_ERR_STATE;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  plan->last_stream = (hipStream_t)stream;
  hipError_t e = plan->solver->transport_adjoint(d_lam1, d_lam0, d_body, (hipStream_t)stream);
  if (e != hipSuccess) return TG_ERR_HIP;
  return TG_OK;
}


tg_status tg_stream_probe(void* d_buf, size_t bytes, size_t field_bytes, int reps,
                          double* gb_per_s, void* stream) {
  if (d_buf == nullptr || gb_per_s == nullptr || reps < 1 || field_bytes < 1024 ||
      field_bytes % 16 != 0 || ((uintptr_t)d_buf % 16) != 0)
    return TG_ERR_ARG;
  const size_t sets = bytes / (7 * field_bytes);
  if (sets < 1) return TG_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  const long long n4 = (long long)(field_bytes / 16);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return TG_ERR_HIP;
  auto field = [&](size_t set, int k) {
    return (void*)((char*)d_buf + (set * 7 + k) * field_bytes);
  };
  hipError_t e = hipSuccess;
  for (int r = -1; r < reps && e == hipSuccess; ++r) {
    if (r == 0) e = hipEventRecord(e0, st);
    const size_t set = (size_t)(r + 1) % sets;
    if (e == hipSuccess)
      e = tg::stream7_launch(field(set, 0), field(set, 1), field(set, 2), field(set, 3),
                             field(set, 4), n4, st);
  }
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return TG_ERR_HIP;
  *gb_per_s = 7.0 * (double)field_bytes * reps / (ms * 1e-3) / 1e9;
  return TG_OK;
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

tg_status tg_kernel_timer(tg_plan* plan, int kernel_id, int every) {
  if (plan == nullptr || kernel_id < tg::KT_NONE || kernel_id > tg::KT_LAST || every < 1)
    return TG_ERR_ARG;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  return from_hip(plan->solver->timer_enable(kernel_id, every));
}

tg_status tg_kernel_timer_read(tg_plan* plan, double* total_ms, long long* launches,
                               double* work_bytes) {
  if (plan == nullptr || total_ms == nullptr || launches == nullptr || work_bytes == nullptr)
    return TG_ERR_ARG;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  return from_hip(plan->solver->timer_read(total_ms, launches, work_bytes));
}

tg_status tg_plan_set_schedule(tg_plan* plan, int pencils, int z_waves, int slabs,
                               int waves_per_simd) {
  if (plan == nullptr) return TG_ERR_ARG;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  if (!(pencils == 0 || pencils == 8 || pencils == 16 || pencils == 32 || pencils == 64))
    return TG_ERR_ARG;
  if (!(z_waves == 0 || z_waves == 1 || z_waves == 2 || z_waves == 4 || z_waves == 8))
    return TG_ERR_ARG;
  if (!(slabs == 0 || slabs == 1 || slabs == 2 || slabs == 4 || slabs == 8)) return TG_ERR_ARG;
  if (!(waves_per_simd == 0 || waves_per_simd == 1 || waves_per_simd == 4)) return TG_ERR_ARG;
  if (!plan->solver->set_schedule(pencils, z_waves, slabs, waves_per_simd)) return TG_ERR_ARG;
  return TG_OK;
}

tg_status tg_plan_get_schedule(const tg_plan* plan, int* pencils, int* z_waves, int* slabs,
                               int* waves_per_simd) {
  if (plan == nullptr || pencils == nullptr || z_waves == nullptr || slabs == nullptr ||
      waves_per_simd == nullptr)
    return TG_ERR_ARG;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  plan->solver->get_schedule(pencils, z_waves, slabs, waves_per_simd);
  return TG_OK;
}

tg_status tg_plan_set_pass(tg_plan* plan, int kernel_id, int pencils, int waves_per_simd) {
  if (plan == nullptr) return TG_ERR_ARG;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  if (kernel_id < tg::KT_X_INV_GRAD || kernel_id > tg::KT_LAST) return TG_ERR_ARG;
  const bool zpass = kernel_id == tg::KT_Z_MATVEC;
  if (zpass ? !(pencils == 0 || pencils == 8 || pencils == 16)
            : !(pencils == 8 || pencils == 16 || pencils == 32 || pencils == 64))
    return TG_ERR_ARG;
  if (!(waves_per_simd == 1 || waves_per_simd == 4)) return TG_ERR_ARG;
  if (!plan->solver->set_pass(kernel_id, pencils, waves_per_simd)) return TG_ERR_ARG;
  return TG_OK;
}

tg_status tg_plan_get_pass(const tg_plan* plan, int kernel_id, int* pencils,
                           int* waves_per_simd) {
  if (plan == nullptr || pencils == nullptr || waves_per_simd == nullptr) return TG_ERR_ARG;
  if (!plan->solver) return TG_ERR_WORKSPACE;
  if (!plan->solver->get_pass(kernel_id, pencils, waves_per_simd)) return TG_ERR_ARG;
  return TG_OK;
}

struct tg_batch {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<tg_plan*> plans;
};

tg_status tg_batch_capture(int nplans, tg_plan* const* plans, const tg_batch_io* io,
                           int pcg_budget, void* stream, tg_batch** out) {
  if (out == nullptr) return TG_ERR_ARG;
  *out = nullptr;
  if (nplans < 1 || plans == nullptr || io == nullptr || pcg_budget < 0) return TG_ERR_ARG;
  std::vector<int> budgets(nplans);
  for (int i = 0; i < nplans; ++i) {
    tg_plan* p = plans[i];
    const tg_batch_io& b = io[i];
    if (p == nullptr || b.d_p == nullptr || b.d_rho_f == nullptr || b.d_k_f == nullptr ||
        b.d_m == nullptr || b.d_cT == nullptr || b.d_cobs == nullptr || b.d_J == nullptr ||
        b.d_gp == nullptr || b.d_grho == nullptr || b.d_gkf == nullptr)
      return TG_ERR_ARG;
    if (!p->solver) return TG_ERR_WORKSPACE;
    int its = pcg_budget;
    if (its == 0) {
      const int seen = p->solver->its_max_last_call();
      if (seen <= 0) return TG_ERR_STATE;  // no eager gradient to size the budget from
      its = seen + seen / 4 + 4;
    }
    budgets[i] = its;
  }
  // The plans share nothing, so each is captured on a branch of its own:
  // plan 0 on `stream`, plan i > 0 on a helper stream forked from it by an
  // event and joined back at the end.  The graph then holds independent
  // chains that a replay can run side by side, so one plan's small or
  // predicated-off launches overlap another's work.  The helper streams
  // (default priority) and events are only needed while capturing.
  hipStream_t st = (hipStream_t)stream;
  std::vector<hipStream_t> br(nplans, st);
  std::vector<hipEvent_t> ev(nplans, nullptr);   // ev[0]: fork; ev[i]: join of branch i
  auto release = [&]() {
    for (int i = 1; i < nplans; ++i)
      if (br[i] != st) (void)hipStreamDestroy(br[i]);
    for (hipEvent_t x : ev)
      if (x) (void)hipEventDestroy(x);
  };
  for (int i = 0; i < nplans; ++i) {
    if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) {
      ev[i] = nullptr;
      release();
      return TG_ERR_HIP;
    }
    if (i > 0 && hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking) != hipSuccess) {
      br[i] = st;
      release();
      return TG_ERR_HIP;
    }
  }
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    release();
    return TG_ERR_HIP;
  }
  hipError_t e = nplans > 1 ? hipEventRecord(ev[0], st) : hipSuccess;
  int forked = 1;
  for (; forked < nplans && e == hipSuccess; ++forked) e = hipStreamWaitEvent(br[forked], ev[0], 0);
  if (e != hipSuccess) --forked;   // the failed branch never joined the capture
  for (int i = 0; i < nplans && e == hipSuccess; ++i) {
    tg_plan* p = plans[i];
    const tg_batch_io& b = io[i];
    p->solver->set_graph_budget(budgets[i], pcg_budget == 0);
    e = p->solver->forward(b.d_p, b.d_rho_f, b.d_k_f, b.d_m, nullptr, nullptr, b.d_cT, br[i]);
    if (e == hipSuccess)
      e = p->solver->vjp(nullptr, b.d_cobs, 0, nullptr, nullptr, b.d_J, b.d_gp, b.d_grho,
                         b.d_gkf, nullptr, nullptr, br[i]);
    p->solver->set_graph_budget(0, false);
    p->last_stream = st;
  }
  // join every forked branch, also after an error, so the capture can end
  for (int i = 1; i < forked; ++i) {
    hipError_t ej = hipEventRecord(ev[i], br[i]);
    if (ej == hipSuccess) ej = hipStreamWaitEvent(st, ev[i], 0);
    if (e == hipSuccess) e = ej;
  }
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(st, &graph);
  release();
  if (e != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return TG_ERR_HIP;
  }
  tg_batch* bt = new tg_batch;
  bt->graph = graph;
  bt->plans.assign(plans, plans + nplans);
  if (hipGraphInstantiate(&bt->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    delete bt;
    return TG_ERR_HIP;
  }
  for (tg_plan* p : bt->plans) p->have_traj = false;  // valid after the first launch
  *out = bt;
  return TG_OK;
}

tg_status tg_batch_launch(tg_batch* batch, void* stream) {
  if (batch == nullptr || batch->exec == nullptr) return TG_ERR_ARG;
  if (hipGraphLaunch(batch->exec, (hipStream_t)stream) != hipSuccess) return TG_ERR_HIP;
  for (tg_plan* p : batch->plans) {
    p->have_traj = true;
    p->last_stream = (hipStream_t)stream;
  }
  return TG_OK;
}

void tg_batch_destroy(tg_batch* batch) {
  if (batch == nullptr) return;
  if (batch->exec) (void)hipGraphExecDestroy(batch->exec);
  if (batch->graph) (void)hipGraphDestroy(batch->graph);
  delete batch;
}

void tg_plan_destroy(tg_plan* plan) {
  if (plan == nullptr) return;
  tg::static_scratch_release(plan);
  delete plan;
}

}  // extern "C"
