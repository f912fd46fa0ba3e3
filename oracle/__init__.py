"""FP64 CPU oracle for the tumor forward/adjoint path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark call it.  It shares no code with the GPU path: it uses numpy's
FFT (pocketfft) and scipy's conjugate-gradient routine as library steps and
follows the paper's equations directly, with no blocking or fusion.

Modules
  spectral  periodic Fourier derivatives, the diffusion operator and the
            constant-coefficient Fourier preconditioner (Sec. 3.3)
  tumor     reaction step, Gaussian basis, Strang/Crank-Nicolson forward
            solve, its exact discrete adjoint, tangent and Gauss-Newton
            Hessian products (Sec. 2.1, Sec. 3.1, Sec. 3.3)
  dense     brute-force dense operators on tiny grids (8^3), built from
            explicit DFT matrices, used to pin ``tumor``.
  transport semi-Lagrangian advection of the anatomy labels, its adjoint
            and the registration body force (Sec. 2.1, Sec. 3.2, Sec. 3.3)
"""
from . import spectral, tumor, dense, transport  # noqa: F401
