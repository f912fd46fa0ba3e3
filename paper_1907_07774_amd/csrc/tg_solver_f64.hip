// FP64 instantiation.
#include "tg_solver.h"

namespace tg {
ISolver* make_solver_f64(const SolverDims& d, const Workspace& w) { return make_solver_t<double>(d, w); }
hipError_t init_twiddles_f64() { return fill_twiddles<double>(); }
int phi_blocks_for(int n) {
  switch (n) {
    case 8: return PhiT<double, 8>::NBLK;
    case 16: return PhiT<double, 16>::NBLK;
    case 32: return PhiT<double, 32>::NBLK;
    case 64: return PhiT<double, 64>::NBLK;
    case 128: return PhiT<double, 128>::NBLK;
    case 256: return PhiT<double, 256>::NBLK;
    default: return 0;
  }
}
}  // namespace tg
