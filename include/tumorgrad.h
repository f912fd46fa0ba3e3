/*
 * tumorgrad: forward, adjoint and Gauss-Newton Hessian solves of the
 * reaction-diffusion tumor-growth model used for image-driven model
 * calibration (Scheufele, Subramanian, Mang, Biros, Mehl, "Image-driven
 * biophysical tumor growth model calibration", arXiv:1907.07774).
 *
 * Model (Sec. 2.1, tumor forward operator with the white-matter-only
 * coefficients of Sec. 4.1; tg_forward_fields takes the tissue-weighted
 * coefficients and the CSF mask of Sec. 2.1, tg_adjoint_misfit_labels the
 * anatomy-label misfit, tg_vjp_coupling the coupling field q(x), and
 * tg_transport the registration transport), on the periodic cube
 * [0, 2 pi)^3:
 *     dc/dt = div(k_f m grad c) + rho_f m c (1 - c),   c(0) = Phi p,
 * with Phi p = sum_i p_i exp(-|x - x_i|^2 / (2 sigma^2)) (periodic minimum
 * image distance, peak value 1).  Discretization (Sec. 3.3): Fourier
 * pseudo-spectral derivatives on an n^3 grid (Nyquist wavenumber of first
 * derivatives set to zero), Strang splitting of nt steps over [0, T] with
 * the exact logistic reaction flow on half steps and Crank-Nicolson
 * diffusion solved by PCG with the preconditioner
 * (1 + dt/2 k_f max(m) |w|^2)^-1.  The misfit is the tumor L2 distance of
 * Tab. 1, J = 1/2 h^3 sum (c(T) - c_obs)^2, h = 2 pi / n.  Gradients are the
 * exact derivatives of the discrete map (the reduced gradient of Sec. 3.1:
 * state solve, adjoint solve, gradient), with respect to p (Sec. 2.1,
 * p-gradient Phi^T alpha(0)), k_f (Sec. 2.1, diffusion-coefficient
 * gradient) and rho_f.
 *
 * Conventions for every entry point:
 *   - Real fields are C-contiguous [n][n][n] arrays (x slowest, z fastest)
 *     of double (TG_FP64) or float (TG_FP32_MIXED).  With batch B > 1 the
 *     problems are stacked: field b starts at element b n^3.
 *   - Parameter vectors (p, rho_f, k_f, gradients) are double in both
 *     precisions, stacked per problem (p: [B][n_p], rho_f and k_f: [B]).
 *   - All array arguments are DEVICE pointers owned by the caller; the
 *     library never allocates or frees device memory.  Its device storage
 *     is the workspace given to tg_plan_bind, the transport workspace
 *     given to tg_transport, static tables of 512 FFT twiddle factors
 *     per precision and grid size (filled by tg_plan_bind), and the static
 *     scratch of tg_forward_static (TG_STATIC_SCRATCH_BYTES per device).
 *   - stream is a hipStream_t passed as void*.  Work is enqueued on it; the
 *     PCG loops synchronize that stream between blocks of iterations to
 *     read convergence flags, so calls return after the solves finished
 *     and only the final, non-iterative kernels may still be in flight.
 *   - Argument, state and workspace errors are detected on the host before
 *     anything is launched.  A PCG that hits pcg_maxit, breaks down or
 *     produces non-finite values still writes all outputs and the call
 *     returns TG_ERR_NOT_CONVERGED / TG_ERR_NUMERIC.
 *   - The growth parameters rho_f and k_f are device values, so they are
 *     checked on the device: k_f < 0 (anti-diffusion, outside the model)
 *     or a non-finite k_f or rho_f sets status bit 8 (tg_stats) for that
 *     problem, its Crank-Nicolson solves are skipped, its outputs are
 *     meaningless, and the call, and every later call on the same
 *     trajectory, returns TG_ERR_ARG.
 *   - One plan is used by one stream at a time.
 */
#ifndef TUMORGRAD_H
#define TUMORGRAD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TG_OK = 0,
  TG_ERR_ARG = 1,            /* invalid argument or descriptor */
  TG_ERR_STATE = 2,          /* call order violated (e.g. vjp before forward) */
  TG_ERR_NOT_CONVERGED = 3,  /* a PCG solve reached pcg_maxit */
  TG_ERR_NUMERIC = 4,        /* PCG breakdown or non-finite values */
  TG_ERR_HIP = 5,            /* a HIP runtime call or kernel launch failed */
  TG_ERR_WORKSPACE = 6,      /* workspace missing, too small or misaligned */
  TG_ERR_SCRATCH_LIMIT = 7   /* tg_forward_static: the plan's workspace exceeds
                                TG_STATIC_SCRATCH_BYTES */
} tg_status;

typedef enum {
  TG_FP64 = 0,        /* all fields, transforms and reductions in double */
  TG_FP32_MIXED = 1   /* float fields and transforms; double dots, norms,
                         PCG scalars and gradient accumulation */
} tg_precision;

typedef struct tg_desc {
  int n;                 /* grid points per axis: 8, 16, 32, 64, 128 or 256 */
  int nt;                /* Strang steps, >= 1 */
  double T;              /* time horizon, > 0 (dt = T / nt) */
  int n_p;               /* Gaussian basis functions per problem, 1..4096 */
  const double* centres; /* HOST [batch][n_p][3] centres in [0, 2 pi)^3,
                            copied at tg_plan_bind */
  double sigma;          /* Gaussian standard deviation, > 0 */
  double pcg_rtol;       /* PCG stop: ||r|| <= rtol ||rhs||, 0 < rtol < 1.
                            TG_FP32_MIXED stops no lower than a floor: the
                            adjoint solves at 50 eps_32 = 6.0e-6, the
                            forward-type solves (forward, segment recompute,
                            Gauss-Newton tangent) at 16 eps_32 = 1.9e-6.  The
                            environment variable TUMORGRAD_FP32_RTOL_FLOOR
                            (read when the plan is bound) sets both floors,
                            TUMORGRAD_FP32_FWD_RTOL_FLOOR then the forward
                            one. */
  int pcg_maxit;         /* >= 1 */
  int ckpt_stride;       /* 0: keep every step's state; s > 0: keep every
                            s-th state and recompute segments in the adjoint */
  tg_precision prec;
  int batch;             /* independent problems solved together, >= 1 */
  int max_hvp_dirs;      /* Hessian directions per tg_hessvec_gn call, >= 0 */
} tg_desc;

typedef struct tg_solve_stats {
  int solves;               /* CN solves in the last call */
  int pcg_its_total;        /* PCG iterations summed over those solves */
  int pcg_its_max;          /* largest iteration count of one solve */
  int status_bits;          /* 1: maxit reached, 2: breakdown, 4: non-finite,
                               8: invalid parameter (k_f < 0, or k_f or rho_f
                               not finite) */
  double worst_rel_residual;/* max over solves of final ||r|| / ||rhs|| */
} tg_solve_stats;

typedef struct tg_plan tg_plan;

/* Validate a descriptor and create a plan (host memory only; nothing is
 * launched).  Errors: TG_ERR_ARG. */
tg_status tg_plan_create(const tg_desc* desc, tg_plan** out);

/* Bytes of device workspace the plan needs (256-byte aligned buffer). */
tg_status tg_plan_workspace_bytes(const tg_plan* plan, size_t* bytes);

/* Bind caller-owned device memory as workspace, on the current device.
 * Copies the centres and fills the device twiddle table (synchronous).
 * Errors: TG_ERR_WORKSPACE (null, misaligned, too small), TG_ERR_HIP. */
tg_status tg_plan_bind(tg_plan* plan, void* d_workspace, size_t bytes);

/* Forward solve (state equation, Sec. 2.1; discretization Sec. 3.3):
 * c(T) from p [B][n_p], rho_f [B], k_f [B], white-matter map m [B][n^3].
 * Writes d_cT [B][n^3].  m, p, rho_f, k_f and cT must stay valid and
 * unchanged until the last tg_vjp / tg_adjoint_misfit / tg_hessvec_gn that
 * uses this trajectory. */
tg_status tg_forward(tg_plan* plan, const double* d_p, const double* d_rho_f,
                     const double* d_k_f, const void* d_m, void* d_cT, void* stream);

/* Forward solve with the full coefficient model of Sec. 2.1: diffusion
 * k = k_f m_diff and reaction rho = rho_f m_react, where the caller forms
 * m_diff = sum_i k_i m_i and m_react = sum_i rho_i m_i from its tissue maps
 * (WM, GM, CSF) and weights; and c(0) = phi_mask * Phi p, the mask zeroing
 * the Gaussians inside CSF (e.g. phi_mask = 1 - m_CSF).  All three fields
 * are [B][n^3] in the plan's precision.  d_m_react = NULL means m_diff,
 * d_phi_mask = NULL means no mask; tg_forward(.., d_m, ..) is this call
 * with (d_m, NULL, NULL).  The pointers must stay valid and unchanged like
 * d_m above: tg_vjp, tg_adjoint_misfit(_labels) and tg_hessvec_gn use the
 * same fields (the Gauss-Newton products use the same mask for Phi v and
 * Phi^T).  Errors: TG_ERR_ARG if d_m_diff is NULL. */
tg_status tg_forward_fields(tg_plan* plan, const double* d_p, const double* d_rho_f,
                            const double* d_k_f, const void* d_m_diff, const void* d_m_react,
                            const void* d_phi_mask, void* d_cT, void* stream);

/* Size of the library's static device scratch, per device (64 MiB): the
 * largest workspace tg_forward_static accepts (a 64^3 FP32 plan with any
 * checkpoint stride, or 64^3 FP64 with stride 4, fits). */
#define TG_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/* tg_forward for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Instead of caller memory the plan's workspace is a static device array of
 * the library, TG_STATIC_SCRATCH_BYTES on every device it runs on, held
 * until the process ends.  The caller still passes inputs and outputs
 * exactly as to tg_forward; the plan must have been created
 * (tg_plan_create) but need not be bound.  Nothing here or in the later
 * calls on the plan allocates device memory.
 *   - The first call for a plan on a device binds the plan to that
 *     device's scratch (synchronous: twiddle table and centres copied, as
 *     tg_plan_bind does); later calls on the same plan launch like
 *     tg_forward.  tg_vjp, tg_adjoint_misfit(_labels), tg_hessvec_gn and
 *     tg_stats then work on the plan as usual.
 *   - One plan owns a device's scratch at a time.  A call for another plan
 *     takes the scratch over and leaves the previous owner unbound, as if
 *     never bound: its trajectory is gone (tg_vjp, tg_adjoint_misfit and
 *     tg_hessvec_gn return TG_ERR_STATE) and tg_forward returns
 *     TG_ERR_WORKSPACE until it is bound again (by tg_plan_bind or
 *     tg_forward_static).  Binding a plan to caller memory or destroying it
 *     gives the scratch up.
 *   - The scratch keeps the last call's contents; nothing in it needs to
 *     start at zero (every buffer is written before it is read).
 *   - Calls that overlap in time on one device race on the scratch: the
 *     caller orders them (one stream, or synchronization between streams),
 *     including the final kernels of the previous owner's last call.
 * Errors: TG_ERR_ARG (null pointer), TG_ERR_SCRATCH_LIMIT (the plan's
 * workspace, tg_plan_workspace_bytes, exceeds TG_STATIC_SCRATCH_BYTES;
 * nothing is bound or launched), TG_ERR_HIP, and those of tg_forward. */
tg_status tg_forward_static(tg_plan* plan, const double* d_p, const double* d_rho_f,
                            const double* d_k_f, const void* d_m, void* d_cT, void* stream);

/* Vector-Jacobian product of the last forward (adjoint solve, Sec. 2.1
 * optimality conditions, evaluated as in Sec. 3.1): given a Euclidean
 * cotangent lamT [B][n^3] on c(T), writes g_p = d<lamT, c(T)>/dp [B][n_p],
 * g_rho [B] and g_kf [B].  Errors: TG_ERR_STATE before any tg_forward. */
tg_status tg_vjp(tg_plan* plan, const void* d_lamT, double* d_gp, double* d_grho,
                 double* d_gkf, void* stream);

/* tg_vjp that also returns, at every grid point x, the derivatives of
 * <lamT, c(T)> in the diffusion field and in the reaction field of the
 * last forward (m_diff and m_react of tg_forward_fields; both m for
 * tg_forward): the discrete counterpart of the coupling field q(x) that
 * the registration step of the Picard iteration receives (Sec. 2.2), a
 * time integral of gradient-of-state times gradient-of-adjoint and
 * c (1 - c) times adjoint terms.  Exactly, per reverse step with mu the
 * Crank-Nicolson adjoint solution and s = a + b the step's two states:
 *   q_diff  += -dt/2 k_f sum_j (D_j mu)(D_j s),
 *   q_react += rho_f dt/2 lam R (1 - R)   at each reaction half step,
 * so sum_x m_diff q_diff = k_f g_kf and sum_x m_react q_react = rho_f g_rho.
 * For tissue maps m_i with k = k_f sum_i k_i m_i and rho = rho_f sum_i
 * rho_i m_i, dJ/dm_i = k_i q_diff + rho_i q_react.  d_q_diff, d_q_react:
 * [B][n^3] in the plan's precision, overwritten; either may be NULL.
 * combine = 1: d_q_diff receives q_diff + q_react, the derivative in m
 * when one field drives both coefficients (tg_forward), and d_q_react must
 * be NULL; combine = 0: the two fields separately.  The diffusion part adds
 * five transform passes per reverse step (the gradient rows of mu and of s
 * and one z pass that multiplies them).  Errors as tg_vjp; TG_ERR_ARG for
 * combine outside {0, 1} or, with combine = 1, a NULL d_q_diff or a
 * non-NULL d_q_react. */
tg_status tg_vjp_coupling(tg_plan* plan, const void* d_lamT, double* d_gp, double* d_grho,
                          double* d_gkf, void* d_q_diff, void* d_q_react, int combine,
                          void* stream);

/* Misfit J = 1/2 h^3 sum (c(T) - c_obs)^2 (tumor misfit of Tab. 1) and its
 * gradient: tg_vjp with lamT = h^3 (c(T) - c_obs).  Writes d_J [B]. */
tg_status tg_adjoint_misfit(tg_plan* plan, const void* d_cobs, double* d_J, double* d_gp,
                            double* d_grho, double* d_gkf, void* stream);

/* Misfit with the anatomy-label term of the Sec. 2.1 objective:
 *   J = 1/2 h^3 sum [(c - c_obs)^2 + sum_l (m_l (1 - c) - mP_l)^2],
 * the simulated tumor c = c(T) masking the healthy labels m_l, compared
 * with the patient labels mP_l, and its gradient: tg_vjp with
 *   lamT = h^3 [(c - c_obs) - sum_l m_l (m_l (1 - c) - mP_l)]
 * (the terminal condition of the adjoint with D_m included).  d_m_lab and
 * d_m_pat hold n_labels fields per problem, [B][n_labels][n^3], in the
 * plan's precision; n_labels = 0 is tg_adjoint_misfit.  Errors: TG_ERR_ARG
 * (n_labels < 0, or > 0 with a NULL label pointer), TG_ERR_STATE. */
tg_status tg_adjoint_misfit_labels(tg_plan* plan, const void* d_cobs, int n_labels,
                                   const void* d_m_lab, const void* d_m_pat, double* d_J,
                                   double* d_gp, double* d_grho, double* d_gkf, void* stream);

/* Registration transport (Sec. 2.1 registration advection operator and its
 * adjoint in the optimality system; Sec. 3.3 semi-Lagrangian time
 * stepping), on a bound plan with batch 1, in the plan's grid and
 * precision.  n_labels label fields m0 [n_labels][n^3] are carried by a
 * stationary velocity v [3][n^3] (physical units on [0, 2 pi)^3) over the
 * pseudo-time [0, 1] in nt_r steps:  dm/dt + v . grad m = 0.  Each step
 * interpolates the previous level at the foot of the characteristic
 * (Heun's second-order step, tricubic Lagrange interpolation on the
 * periodic grid).  d_m1 [n_labels][n^3] receives m(1) (may be NULL).
 * d_w = div v [n^3] (the paper's w; NULL: divergence-free) is used by
 * tg_transport_adjoint.  d_tws: caller-owned device scratch of at least
 * tg_transport_workspace_bytes (256-byte aligned); it holds every time
 * level for the adjoint, so it, v and w must stay unchanged until the
 * last tg_transport_adjoint of this transport.  The transport calls use
 * the plan's spectral scratch buffers but no tumor state: tg_vjp and
 * tg_hessvec_gn of an earlier tg_forward stay valid.
 * Errors: TG_ERR_ARG (batch > 1, nt_r < 1, n_labels < 1, NULL v, m0 or
 * tws), TG_ERR_WORKSPACE (tws too small or misaligned, plan not bound). */
tg_status tg_transport_workspace_bytes(const tg_plan* plan, int nt_r, int n_labels,
                                       size_t* bytes);
tg_status tg_transport(tg_plan* plan, int nt_r, int n_labels, const void* d_v, const void* d_w,
                       const void* d_m0, void* d_m1, void* d_tws, size_t tws_bytes,
                       void* stream);

/* Adjoint of the last tg_transport (optimize-then-discretize, as the paper
 * treats the registration, Sec. 3.2): from lam(1) = d_lam1
 * [n_labels][n^3], solves -dlam/dt - div(lam v) = 0 backward along the
 * characteristics of -v (the source lam w by the trapezoid rule), writes
 * lam(0) to d_lam0 [n_labels][n^3] and the body force
 *   b = integral_0^1 sum_l lam_l grad m_l dt   (trapezoid over the levels,
 *       spectral gradients)
 * to d_body [3][n^3]; for J = <lam1, m(1)> the derivative in v is -b (the
 * registration optimality condition applies its projection).
 * Errors: TG_ERR_ARG (NULL pointer), TG_ERR_STATE (no transport yet). */
tg_status tg_transport_adjoint(tg_plan* plan, const void* d_lam1, void* d_lam0, void* d_body,
                               void* stream);

/* Gauss-Newton Hessian of J with respect to p about the last forward
 * trajectory (batch must be 1): HV[d] = Phi^T J_c^T h^3 J_c Phi V[d] for
 * d < ndir, V and HV [ndir][n_p].  Tangent-linear forward plus adjoint,
 * all directions batched per launch.  Errors: TG_ERR_ARG (ndir outside
 * 1..max_hvp_dirs or batch > 1), TG_ERR_STATE. */
tg_status tg_hessvec_gn(tg_plan* plan, int ndir, const double* d_V, double* d_HV,
                        void* stream);

/* Launch schedule of the transform passes (performance knobs only; results
 * are identical up to the summation order of the FP64 partial sums).
 * pencils: 8, 16, 32 or 64 pencils per x/y-pass workgroup (64 only where
 * its transform buffer fits the 160 KB of LDS: not FP64 at n = 256);
 * z_waves: 1, 2 or 4 waves per z-pass workgroup, or 8 for one-wave
 * workgroups whose matvec z pass spreads each row over twice the default
 * lanes; slabs: 1, 2, 4 or 8 x-plane slabs over which the y-z-y pass chain
 * of the diffusion operator runs slab by slab; waves_per_simd: occupancy
 * floor of the PCG pass kernels (1: registers uncapped, 4: capped so four
 * waves fit per SIMD); 0 selects the default.  Requires a bound plan.
 * Errors: TG_ERR_ARG for unsupported values. */
tg_status tg_plan_set_schedule(tg_plan* plan, int pencils, int z_waves, int slabs,
                               int waves_per_simd);
tg_status tg_plan_get_schedule(const tg_plan* plan, int* pencils, int* z_waves, int* slabs,
                               int* waves_per_simd);

/* Per-pass override of the schedule, applied after tg_plan_set_schedule
 * (which resets every pass to its plan-wide values).  kernel_id names one
 * pass of the PCG iteration as in tg_kernel_timer: 1, 2, 4, 5 (x/y passes:
 * pencils as above) or 3 (z matvec: see below); waves_per_simd: 1 or 4 as
 * above.  For the z matvec, pencils selects the layout of a spectral row in
 * registers: 8 for one complex value per lane access, 16 for a pair
 * (16-byte accesses in FP32), 0 for the default (16 in FP32, 8 in FP64);
 * under z_waves 8 (the wide z matvec, no per-pass variant) only the shape
 * tg_plan_get_pass reports is accepted, as a no-op, so a plan's passes can
 * be copied to another plan.  Results are identical up to the summation
 * order of the FP64 partial sums.  Errors: TG_ERR_ARG for an unknown pass
 * or value (the plan keeps its schedule), TG_ERR_WORKSPACE before
 * tg_plan_bind. */
tg_status tg_plan_set_pass(tg_plan* plan, int kernel_id, int pencils, int waves_per_simd);
tg_status tg_plan_get_pass(const tg_plan* plan, int kernel_id, int* pencils,
                           int* waves_per_simd);

/* PCG statistics of the last call (synchronizes the plan's last stream). */
tg_status tg_stats(tg_plan* plan, tg_solve_stats* out);

/* Kernel timer for performance measurement.  Identifies one kernel of the
 * PCG iteration (1: x-pass inverse with direction update and |p|^2,
 * 2: y-pass inverse, 3: z-pass C2R * m * R2C with the m |grad p|^2 sum,
 * 4: y-pass forward, 5: x-pass forward with the iterate and residual
 * update; 0: off).  While enabled, every launch of that kernel inside the
 * PCG solves selected by `every` carries a pair of HIP events that take
 * the kernel dispatch's own start and end timestamps
 * (hipExtLaunchKernelGGL): no extra packets on the plan's stream.  every
 * >= 1: the launches of one Crank-Nicolson solve in every (the first, then
 * every every-th, counted from this call) are timed and only their work is
 * counted, a uniform sample that keeps the timestamps' cost (a few us of
 * idle time around each timed dispatch) out of the other solves.  Events
 * carry no system-scope fence.  tg_kernel_timer resets the counters.
 * Errors: TG_ERR_ARG (kernel_id out of range, every < 1), TG_ERR_WORKSPACE
 * (no workspace bound). */
tg_status tg_kernel_timer(tg_plan* plan, int kernel_id, int every);

/* Streaming reference for the roofline of the PCG passes (measurement
 * only, no part of the method): a kernel that reads five and writes two
 * FP32 fields of field_bytes each in one pass, with no other work, timed
 * over reps launches on stream (synchronous).  d_buf (caller-owned device
 * memory, 16-byte aligned) is cut into bytes / (7 field_bytes) sets of
 * seven fields used in turn, so with d_buf several times the 256 MB
 * last-level cache every launch streams from HBM; its contents are
 * overwritten.  Writes the algorithmic GB/s (7 field_bytes per launch).
 * Errors: TG_ERR_ARG (no complete set, reps < 1, field_bytes < 1024 or not
 * a multiple of 16), TG_ERR_HIP. */
tg_status tg_stream_probe(void* d_buf, size_t bytes, size_t field_bytes, int reps,
                          double* gb_per_s, void* stream);

/* Read the timer (synchronizes the recorded events): total event time in
 * ms, number of timed launches, and the algorithmic HBM bytes those
 * launches moved (launches that did work x fields read and written). */
tg_status tg_kernel_timer_read(tg_plan* plan, double* total_ms, long long* launches,
                               double* work_bytes);

/* Batched gradient evaluation as one replayable HIP graph (many problems
 * in one launch): for each plan, forward + misfit + adjoint
 * (tg_forward then tg_adjoint_misfit) on that plan's batch of problems, all
 * captured from `stream` into one graph, each plan as an independent branch
 * (the plans must not share a workspace), so a replay may run the plans
 * concurrently.  Inside the graph every PCG solve
 * runs a fixed, predicated iteration budget (kernels of converged problems
 * return at once): pcg_budget for every solve, or if 0 each solve's own
 * iteration count in the plan's last eager tg_forward / tg_adjoint_misfit
 * + 25% + 4 (the solves of a call come in a fixed order; TG_ERR_STATE if
 * there was no eager call).  A solve that needs more is flagged TG_ERR_NOT_CONVERGED in
 * tg_stats after the launch.  The io pointers are baked into the graph and
 * must stay valid; their contents may change between launches. */
typedef struct tg_batch tg_batch;
typedef struct tg_batch_io {
  const double* d_p;      /* [B][n_p] */
  const double* d_rho_f;  /* [B] */
  const double* d_k_f;    /* [B] */
  const void* d_m;        /* [B][n^3] */
  void* d_cT;             /* [B][n^3] out */
  const void* d_cobs;     /* [B][n^3] */
  double* d_J;            /* [B] out */
  double* d_gp;           /* [B][n_p] out */
  double* d_grho;         /* [B] out */
  double* d_gkf;          /* [B] out */
} tg_batch_io;

tg_status tg_batch_capture(int nplans, tg_plan* const* plans, const tg_batch_io* io,
                           int pcg_budget, void* stream, tg_batch** out);
/* Replay the captured graph on `stream` (asynchronous). */
tg_status tg_batch_launch(tg_batch* batch, void* stream);
void tg_batch_destroy(tg_batch* batch);

const char* tg_status_string(tg_status s);
void tg_plan_destroy(tg_plan* plan);
int tg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TUMORGRAD_H */
