/*
 * adimx -- ADI isogeometric time stepping of Maxwell's equations on AMD MI355X.
 *
 * C ABI of libadimx.so.  Every function is extern "C", never throws and
 * returns an int status (ADI_OK = 0 or a negative ADI_E* code) unless stated.
 * After an error the context stays usable and adi_last_error() returns a
 * message.  All host arrays are copied before the call returns; the caller
 * keeps ownership of everything it passes in.  Device memory is either
 * allocated by the library or carved from a caller-owned workspace bound
 * with adi_bind_workspace (that workspace must outlive the context).
 *
 * Method (Paszynski, Los, Munoz-Matute, arXiv 2103.06998):
 *   domain (0,1)^3, Nx x Ny x Nz uniform elements, degree-p B-splines of
 *   continuity C^{p-1} on open uniform knots, n_a = N_a + p coefficients
 *   along axis a per field component; E and H each have three components
 *   (section "Alternating directions splitting for Maxwell equations").  One time step is two
 *   substeps (eqs. scheme1a-scheme1d, discretised as discrete1-discrete4):
 *   a sum-factorised right-hand side, then three direction-wise banded
 *   (bandwidth 2p+1) line solves per component, with the material attached
 *   to test functions (section "Incorporating non-regular material data").
 *
 * Layout of every field array at this boundary: six components
 * [E1,E2,E3,H1,H2,H3], each D = nx ny nz float64 in [z][y][x] order with x
 * fastest (the paper's reordering of each right-hand side into N_x rows of
 * N_y N_z columns, section "Incorporating non-regular material data").
 */
#ifndef ADIMX_H
#define ADIMX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct adi_ctx adi_ctx;
typedef struct adi_nn adi_nn;

enum {
  ADI_OK = 0,
  ADI_EINVAL = -1,     /* bad handle, size, mode or material value            */
  ADI_ENOMEM = -2,     /* device allocation or workspace too small            */
  ADI_EHIP = -3,       /* a HIP runtime call failed (message kept)            */
  ADI_ESINGULAR = -4,  /* a pivot of a 1D factorisation is (numerically) zero */
  ADI_ENONFINITE = -5, /* NaN / Inf in an input                               */
  ADI_ESTATE = -6      /* call out of order (e.g. step before factor)         */
};

enum {
  ADI_FP64 = 0,        /* fields, right-hand sides and sweeps in float64     */
  ADI_FP32_REFINE = 1  /* float32 state, right-hand sides and sweeps with
                          float32 accumulation, factors computed in float64;
                          every stage solved in increment form: its
                          right-hand-side kernel forms the residual of the old
                          state, b - P x_old, the float32 sweeps solve
                          P d = b - P x_old and the last sweep stores
                          x_old + d.  The residual of the stages selected by
                          adi_set_residual64 (default: the E stage of
                          substep 2, once per step) is formed in float64
                          arithmetic                                          */
};

/* adi_set_residual64 mask bits: stage E / H of substep 1 / 2 */
enum {
  ADI_RES64_E1 = 1,
  ADI_RES64_H1 = 2,
  ADI_RES64_E2 = 4,
  ADI_RES64_H2 = 8,
  ADI_RES64_DEFAULT = ADI_RES64_E2
};

enum {
  ADI_MAP_GREVILLE = 0,    /* each DOF takes the voxel containing its Greville point  */
  ADI_MAP_BSPLINE_AVG = 1  /* each DOF takes the voxel values averaged with the
                              weights of its test function B_r B_s B_t               */
};

/*
 * Create a context for a patch of nx x ny x nz elements (each >= 1; the
 * element counts may differ per axis, each axis gets its own 1D matrices)
 * of degree p (1 <= p <= 4) in precision mode `precision`, on HIP stream
 * `hip_stream` (a hipStream_t, NULL = the null stream).  EINVAL for sizes
 * out of range, including (nx+p)(ny+p)(nz+p) >= 2^31.  Nothing is allocated
 * on the device until adi_factor.  *out receives the handle.  The learned
 * closure calls need a cubic patch.
 */
int adi_create(adi_ctx** out, int nx, int ny, int nz, int p, int precision, void* hip_stream);

/* Number of coefficients along x (nx + p; along every axis of a cube). */
int adi_ncoef(const adi_ctx* ctx);

/* Coefficients per axis, n_out[a] = N_a + p for a = x, y, z. */
int adi_dims(const adi_ctx* ctx, int* n_out);

/*
 * Bytes of device memory the context needs once factored (fields, scratch,
 * coefficients, per-line factors; the data of the time step of section
 * "Alternating directions splitting for Maxwell equations").  A caller that wants to own the memory
 * (e.g. a PyTorch tensor) allocates this many bytes, 256-byte aligned, and
 * binds it before adi_factor.  Returns 0 for an invalid handle.
 */
size_t adi_workspace_bytes(const adi_ctx* ctx);
int adi_bind_workspace(adi_ctx* ctx, void* dev_ptr, size_t bytes);

/*
 * Material given as a voxel map (vx, vy, vz voxels, x fastest, float64)
 * over the unit cube, independent of the element counts:
 * relative permittivity, relative permeability and the non-dimensional
 * conductivity sigma_nd = Z0 L sigma.  Material is attached to test
 * functions (eq. dupa1abcdefg and the text around it): with map_mode
 * ADI_MAP_GREVILLE each degree of freedom takes the voxel containing the
 * Greville point of its test function; with ADI_MAP_BSPLINE_AVG it takes the
 * voxel values averaged with the weights of its test function (integrals of
 * B_r B_s B_t over the voxels, normalised).  EINVAL if eps <= 0, mu <= 0,
 * sigma < 0, a value is not finite or map_mode is unknown.
 */
int adi_set_material(adi_ctx* ctx, const double* eps_r, const double* mu_r,
                     const double* sigma_nd, int vx, int vy, int vz, int map_mode);

/* Material given directly per degree of freedom (three D arrays, x fastest):
 * the per-test-function eps, mu of section "Incorporating non-regular
 * material data" (eq. dupa1abcdefg), and sigma_nd.  Copied; EINVAL as above. */
int adi_set_material_dof(adi_ctx* ctx, const double* eps, const double* mu, const double* sigma_nd);

/*
 * Build, for time step dt >= 0, the 1D Gram matrices M, S, A, B of every
 * axis (float64, exact Gauss quadrature; the matrix list after eqs.
 * discrete1-discrete4 in section "Variational formulation"), the per-row
 * coefficients alpha, beta, gamma, delta of discrete1-discrete4 (with the
 * conductivity terms), and the pivot-free banded LU factors of the 1D
 * systems of section "Incorporating non-regular material data" (the three
 * systems after eq. dupa1abcdefg), in float64: shared factors of the
 * unmodified 1D mass matrices and per-line factors of the material-modified
 * ones.  Captures the time step as a HIP graph.  ESINGULAR if a pivot's
 * magnitude falls to or below the pivot floor (adi_set_pivot_floor, default
 * 1e-14) times its diagonal entry; ESTATE if no material was set; EINVAL for
 * a dt that is negative or not finite.  Allocates the workspace on first use
 * unless one was bound.
 */
int adi_factor(adi_ctx* ctx, double dt);

/*
 * Smallest accepted ratio |U_rr| / |A_rr| of a pivot to its diagonal entry
 * in adi_factor's pivot-free LU (the paper does not say how the banded
 * systems are factorised; without pivoting, this check guards the
 * factorisation).  floor must be finite and >= 0; default 1e-14.  Takes
 * effect at the next adi_factor.
 */
int adi_set_pivot_floor(adi_ctx* ctx, double floor);

/*
 * ADI_FP32_REFINE mode: the stages whose increment b - P x_old is formed in
 * float64 arithmetic (an OR of ADI_RES64_* bits, 0..15; the rest use
 * float32 arithmetic and accumulation).  The increment form is the
 * residual correction of each stage's float32 solve of the three 1D
 * systems of section "Incorporating non-regular material data" (the
 * precision split is this library's, not the paper's).  Default
 * ADI_RES64_DEFAULT.  With one permeability in every row the H stages run
 * as apply-and-solve lines without a right-hand-side kernel, and their bits
 * have no effect.
 * Ignored in ADI_FP64 mode.  Takes effect at the next adi_factor (the
 * context is unfactored until then).  EINVAL for a mask outside 0..15.
 */
int adi_set_residual64(adi_ctx* ctx, int mask);

/*
 * Point dipole source J = amp g(t) e_comp delta(x - xs) with
 * g(t) = sin(2 pi f0 (t - t0)) exp(-((t - t0)/width)^2); it enters each E
 * right-hand side as -beta (J(t_mid), V) at the midpoint of the substep.
 * amp = 0 removes the source.  Must be called before adi_factor or
 * adi_factor must be called again afterwards.
 */
int adi_set_source(adi_ctx* ctx, const double xs[3], int comp, double amp, double f0,
                   double t0, double width);

/* Upload a state (6 D float64, layout above: E^n and H^n of the scheme of
 * section "Alternating directions splitting for Maxwell equations") and set
 * the time t.  The state lives in the space with the PEC conditions imposed
 * strongly: the coefficients of E_c on the faces normal to the two other
 * axes and of H_c on the faces normal to axis c are set to zero (the step
 * assumes so; a state written through adi_fields_device must satisfy it).
 * Copied; waits for the context's stream; ENONFINITE for a value that is not
 * finite. */
int adi_set_fields(adi_ctx* ctx, const double* EH, double t);

/*
 * Local time step per test function (section "Incorporating non-regular
 * material data": like eps and mu, tau may be replaced by tau-hat for a test
 * function): tau holds D values (layout as the fields, finite, >= 0) that
 * replace dt in the row coefficients alpha, beta, gamma, delta of that
 * degree of freedom; the time levels (source time, time advance) stay those
 * of dt.  tau = NULL restores dt everywhere.  Takes effect at the next
 * adi_factor.
 */
int adi_set_local_dt(adi_ctx* ctx, const double* tau);

/*
 * Enqueue nsteps full time steps n -> n+1 (both substeps of eqs.
 * scheme1a-scheme1d, discretised as discrete1-discrete4) on the context's
 * stream and return without waiting.  Each step is one replay of a captured
 * HIP graph.  ESTATE before a successful adi_factor; EINVAL for nsteps < 0.
 */
int adi_step(adi_ctx* ctx, int nsteps);

/* Wait for the stream, then copy the state E^n, H^n (6 D float64, layout
 * above; the float32 mode's state converted) to EH_out and the time to
 * *t_out (may be NULL).  ESTATE before any state exists. */
int adi_get_fields(adi_ctx* ctx, double* EH_out, double* t_out);

/*
 * Device pointer of the current state (6 D contiguous values of dtype
 * *dtype: 0 = float64, 1 = float32) for zero-copy access.  Valid until the
 * next adi_step / adi_set_fields / adi_destroy.
 */
int adi_fields_device(adi_ctx* ctx, void** dev, int* dtype);

/* Wait for all work enqueued by the context (its stream). */
int adi_sync(adi_ctx* ctx);

/*
 * Per-kernel timing of the step.  adi_profile_run enqueues nsteps full steps
 * on the context's stream without the graph, with a pair of HIP events
 * around every kernel launch, waits after each step and accumulates every
 * launch's duration (the state advances by nsteps steps).  adi_profile_read
 * reports, for each launch of a step in launch order: its kind (0 = E
 * right-hand side, 1 = H right-hand side, 3 = x-line solves, 4 = y/z-line
 * solves, 5 = x- and y/z-line solves of one round in one launch, 6 = the
 * H stage's apply-and-solve lines with one permeability), the number of
 * field components it processes, how many of those use per-line
 * (material-modified) factors, how many add a base state to their solution
 * (the last solves of the float32 mode, the apply-and-solve lines), and its
 * mean duration in milliseconds.  *nout receives the number of launches per step
 * (the arrays hold cap entries).
 */
int adi_profile_run(adi_ctx* ctx, int nsteps);
int adi_profile_read(adi_ctx* ctx, int cap, int* nout, int* kind, int* ndesc, int* nmod,
                     int* nacc, float* ms);

/* Message of the context's last error ("invalid handle" for NULL). */
const char* adi_last_error(const adi_ctx* ctx);
/* Wait for the context's stream and free everything the library allocated
 * for it (a bound workspace stays the caller's). */
void adi_destroy(adi_ctx* ctx);

/*
 * Manufactured solution of section "Numerical code verification with
 * manufactured solution" (unit cube, eps = mu = 1, sigma = 0, PEC):
 * u_A = g u^1_11 + 2 g u^2_11 + 3 g u^3_11, g = 2/sqrt(14), with the magnetic
 * part of u^2 of the sign that solves Maxwell's equations.  The integrals use
 * q Gauss points per element and axis (1 <= q <= 16).
 * adi_mms_project: the state becomes the L2 projection of u_A(t) onto the
 *   PEC-constrained spline space (mass solves), and the time t.
 * adi_mms_errors: at the context's time (waits for the stream),
 *   out[0] = ||E_h - E||_L2, out[1] = the H(curl) norm of E_h - E,
 *   out[2], out[3] the same for H (absolute).
 */
int adi_mms_project(adi_ctx* ctx, int q, double t);
int adi_mms_errors(adi_ctx* ctx, int q, double* out);

/*
 * L2 projection of a state given by its values at Gauss points (section
 * "Numerical code verification with manufactured solution": the initial
 * state is a projection of the given fields onto the spline space; the
 * problem statement of section "Alternating directions splitting for Maxwell
 * equations" takes E and H at t = 0 as data).  vals_qp holds
 * 6 (Nx q)(Ny q)(Nz q) float64 values, [component E1..E3,H1..H3][z][y][x],
 * on the tensor grid of the q-point Gauss-Legendre rule of every element
 * (point e q + g of an axis is Gauss point g of element e, x fastest);
 * 1 <= q <= 16.  The state
 * becomes, per component, the solution of (M (x) M (x) M) c = (f, B_r B_s B_t)
 * with the PEC-constrained coefficients zero, and the time t.  Copied before
 * the call returns.  ENONFINITE for a value that is not finite, ESTATE before
 * adi_factor.  Waits for the context's stream and for the projection.
 */
int adi_project(adi_ctx* ctx, const double* vals_qp, int q, double t);

/*
 * adi_mms_errors for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same four errors from the same kernel, with the quadrature tables and
 * the per-block partial sums in a fixed device array of the library (1 MiB
 * per GPU, held until the process ends) instead of buffers allocated on
 * first use.  ENOMEM if (Nx + Ny + Nz) q (2p + 4) + 8192 float64 values
 * exceed it (never for (Nx + Ny + Nz) q <= 10240).  Call with the context's device current.  Every call on
 * one GPU uses the same array: calls that overlap on one GPU (from other
 * streams or threads) race.  Waits for the context's stream.
 */
int adi_mms_errors_noalloc(adi_ctx* ctx, int q, double* out);

/*
 * Single hot-path stages on host buffers (float64 in and out), for testing
 * one step of the method against a reference.  Each runs the same kernels as
 * adi_step and synchronises.
 *
 * adi_rhs: right-hand sides of one stage.  stage 0 = E (eqs. discrete1 /
 *   discrete3: in = [E1,E2,E3,H1,H2,H3], t = time at the start of the
 *   substep), stage 1 = H (eqs. discrete2 / discrete4: in = [H1,H2,H3,
 *   E_old1..3, E_new1..3]); sub = 1 or 2.  out receives 3 D values with
 *   the constrained boundary rows zeroed.
 * adi_solve: the three 1D solves of one stage applied to 3 D right-hand
 *   sides in place (E: modified axis first, then the other two; H: x, y, z).
 */
int adi_rhs(adi_ctx* ctx, int stage, int sub, const double* in, double t, double* out);
int adi_solve(adi_ctx* ctx, int stage, int sub, double* inout);

/* ===================================================================== *
 * Learned closure.  Not part of the paper's method: a small network that
 * corrects the splitting error of a coarse ADI step so that larger steps
 * keep the accuracy of smaller ones.  The network is three 3x3x3
 * convolutions with zero padding on the n x n x n coefficient grid,
 * channels last ([z][y][x][c], x fastest): cin -> 32 (SiLU) -> 32 (SiLU) ->
 * cout.  Operands are bfloat16, accumulation float32 (MFMA); the float32
 * master parameters live on the device.
 *
 * Parameter vector (float32, adi_nn_param_count entries), per layer l in
 * order: W_l[t][ci][co] (27 x cin_l x cout_l, tap t = 9 tz + 3 ty + tx, the
 * input voxel at offset (tz-1, ty-1, tx-1) from the output voxel), then b_l.
 *
 * The network handle has its own device memory; its calls run on the
 * hip_stream given at creation.  All _dev pointers are device memory owned
 * by the caller.
 * ===================================================================== */

/* Create a network with cin (1..16) inputs, chid (= 32) hidden channels and
 * cout (1..16) outputs; parameters start at zero. */
int adi_nn_create(adi_nn** out, int cin, int chid, int cout, void* hip_stream);
int adi_nn_param_count(const adi_nn* nn);
/* Upload all parameters (host float32, layout above; finite) and reset the
 * Adam moments. */
int adi_nn_set_params(adi_nn* nn, const float* params);
int adi_nn_get_params(adi_nn* nn, float* params_out);
/* y_dev[v][cout] = net(x_dev[v][cin]) on an nx x ny x nz grid (float32);
 * keeps the activations for adi_nn_backward. */
int adi_nn_forward(adi_nn* nn, const float* x_dev, float* y_dev, int nx, int ny, int nz);
/* Parameter gradients of the loss whose gradient w.r.t. the last forward's
 * output is dy_dev[v][cout]; they replace the previous gradients. */
int adi_nn_backward(adi_nn* nn, const float* dy_dev);
int adi_nn_get_grads(adi_nn* nn, float* grads_out);
/* One Adam step (bias-corrected, step number t >= 1) on the gradients. */
int adi_nn_adam(adi_nn* nn, float lr, float beta1, float beta2, float eps, int t);
/* Mean squared error of y against target over count entries: writes
 * dy_dev = 2 (y - target) / count and, if loss is not NULL, waits and
 * stores the loss. */
int adi_nn_mse(adi_nn* nn, const float* y_dev, const float* target_dev, size_t count,
               float* dy_dev, double* loss);
const char* adi_nn_last_error(const adi_nn* nn);
void adi_nn_destroy(adi_nn* nn);

/*
 * Solver side of the closure (contexts must be factored).  With S the state
 * before a coarse step and C the state after it, s = RMS of C over all 6 n^3
 * values:
 *   features x[v][0..5]   = C_c[v] / s,
 *            x[v][6..11]  = (C_c[v] - S_c[v]) / s,
 *            x[v][12..14] = log eps, log mu, c/(1+c) with c = sigma dt/(4 eps),
 *            x[v][15]     = B(v) (dt/2) amp (g(t - 3dt/4) + g(t - dt/4)) / s, the
 *                           dipole's impulse over the step (t = time after
 *                           it, g its time profile) times the tensor-product
 *                           basis value B(v) of coefficient v at the dipole;
 *   target   t[v][c] = (F_c[v] - C_c[v]) / s with F a finer solution;
 *   apply    C_c[v] += s y[v][c] except on the PEC-constrained coefficients.
 * adi_copy_state copies the state and time of src into dst (same n; float32
 * and float64 states convert).  adi_closure_mark stores the current state
 * as S.  scale_dev holds one float.
 */
int adi_copy_state(adi_ctx* dst, const adi_ctx* src);
int adi_closure_mark(adi_ctx* ctx);
int adi_closure_features(adi_ctx* ctx, float* x_dev, float* scale_dev);
int adi_closure_target(adi_ctx* fine, adi_ctx* coarse, const float* scale_dev, float* t_dev);
int adi_closure_apply(adi_ctx* ctx, const float* y_dev, const float* scale_dev);
/*
 * nsteps closure steps on the context's stream: mark, one ADI step, features,
 * network forward, apply.  nn must map 16 features to 6 outputs and must not
 * be used on another stream meanwhile.  gate > 0 judges each correction
 * against the coarse step it corrects: a correction whose RMS exceeds gate
 * times the RMS of that step's change (state after minus state before the
 * step) is skipped -- that step stays a plain ADI step -- and counted
 * (adi_closure_rejected, which waits); so a step that changed nothing takes
 * no correction.  gate <= 0 applies every one.
 */
int adi_step_closure(adi_ctx* ctx, adi_nn* nn, int nsteps, float gate);
int adi_closure_rejected(adi_ctx* ctx, int* count);

#ifdef __cplusplus
}
#endif

#endif /* ADIMX_H */
