// Dispatch to the per-(precision, grid size) solver instantiations.
#include "tg_internal.h"

namespace tg {

#define TG_DECL(P, N)                                                    \
  ISolver* make_solver_##P##_##N(const SolverDims& d, const Workspace& w); \
  hipError_t init_twiddles_##P##_##N();
#define TG_DECL_ALL(P) TG_DECL(P, 8) TG_DECL(P, 16) TG_DECL(P, 32) TG_DECL(P, 64) \
  TG_DECL(P, 128) TG_DECL(P, 256)
TG_DECL_ALL(f32)
TG_DECL_ALL(f64)

ISolver* make_solver(int fp64, const SolverDims& d, const Workspace& w) {
#define TG_CASE(N) \
  case N: return fp64 ? make_solver_f64_##N(d, w) : make_solver_f32_##N(d, w);
  switch (d.n) {
    TG_CASE(8) TG_CASE(16) TG_CASE(32) TG_CASE(64) TG_CASE(128) TG_CASE(256)
  }
#undef TG_CASE
  return nullptr;
}

hipError_t init_twiddles(int fp64, int n) {
#define TG_CASE(N) \
  case N: return fp64 ? init_twiddles_f64_##N() : init_twiddles_f32_##N();
  switch (n) {
    TG_CASE(8) TG_CASE(16) TG_CASE(32) TG_CASE(64) TG_CASE(128) TG_CASE(256)
  }
#undef TG_CASE
  return hipErrorInvalidValue;
}

// Phi^T partial-sum blocks: one per 64 grid rows (PhiTK in the kernels).
int phi_blocks_for(int n) { return n * n / 64; }

}  // namespace tg
