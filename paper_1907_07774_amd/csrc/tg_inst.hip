// One (precision, grid size) instantiation of the solver; compiled once per
// pair with -DTG_INST_FP64=0|1 -DTG_N=<n>.
#include "tg_solver.h"

#if TG_INST_FP64
using TgReal = double;
#define TG_SUFFIX(name) TG_CAT(name, TG_CAT(_f64_, TG_N))
#else
using TgReal = float;
#define TG_SUFFIX(name) TG_CAT(name, TG_CAT(_f32_, TG_N))
#endif
#define TG_CAT(a, b) TG_CAT_(a, b)
#define TG_CAT_(a, b) a##b

namespace tg {
ISolver* TG_SUFFIX(make_solver)(const SolverDims& d, const Workspace& w) {
  return new Solver<TgReal, TG_N>(d, w);
}
hipError_t TG_SUFFIX(init_twiddles)() { return fill_twiddles<TgReal>(); }
}  // namespace tg
