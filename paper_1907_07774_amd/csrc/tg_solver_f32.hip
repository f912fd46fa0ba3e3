// FP32-mixed instantiation: float fields and transforms, double reductions.
#include "tg_solver.h"

namespace tg {
ISolver* make_solver_f32(const SolverDims& d, const Workspace& w) { return make_solver_t<float>(d, w); }
hipError_t init_twiddles_f32() { return fill_twiddles<float>(); }
}  // namespace tg
