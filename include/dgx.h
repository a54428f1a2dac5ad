/* dgx.h -- C-ABI of the MI355X (gfx950) DGSEM residual library.
 *
 * The library evaluates the semi-discrete residual dU/dt of the collocated
 * discontinuous Galerkin spectral element method on hexahedral meshes and
 * advances it with the low-storage RK4(5) scheme (paper: "Governing
 * Equations and Numerical Method"; weak form eq. dgsem_weak, BR1 lifting
 * eq. dgsem_lifted, entropy-stable split form with the Chandrashekar flux,
 * RK4-5 of Carpenter and Kennedy).  The host-side ownership model follows
 * the paper's porting strategy (device memory is owned by the library and
 * held by the caller through an opaque handle; "Porting Strategy", memory
 * management listing); the kernels themselves are this library's own.
 *
 * Conventions
 *   - Every function returns a dg_status; nothing throws across the ABI.
 *     On failure dg_last_error(ctx) holds a message (per context; for a
 *     failing dg_create it is the thread's last message, ctx = NULL).
 *   - State arrays are float64, C-contiguous, U[v][e][k][j][i] with
 *     v in (rho, rho u, rho v, rho w, rho e) and i fastest; length
 *     5 * nElems * (N+1)^3.  State, residual, RK register and adjoint
 *     buffers are caller-owned DEVICE memory.
 *   - Mesh input is host memory.  Geometry nodes are equispaced,
 *     X[d][e][c][b][a] on -1 + 2a/Ngeo, a fastest.  Side s joins the master
 *     (side_elem[2s], side_loc[2s]) and the slave (side_elem[2s+1],
 *     side_loc[2s+1]).  Local face f: f/2 is the reference direction of the
 *     normal, f%2 == 1 the +1 end.  Face-local indices (p,q) are the two
 *     tangential volume indices in increasing direction order.
 *     side_orient[s] maps master (p,q) to slave (p',q'): swap if bit 2,
 *     then reverse the first index if bit 0 and the second if bit 1.
 *   - Streams are hipStream_t passed as void* (NULL = default stream).  All
 *     device work of a call is enqueued on that stream; calls return
 *     without synchronising unless stated.  A context is not thread-safe;
 *     use one context per stream.
 *   - Scratch memory is a caller-bound workspace (dg_workspace_bytes /
 *     dg_bind_workspace); calls that need it fail with DG_ERR_STATE when
 *     none is bound.  Calls that share a context share its workspace, so
 *     they must not overlap in time on different streams.
 */
#ifndef DGX_H
#define DGX_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_ctx dg_ctx;

typedef enum {
  DG_OK = 0,
  DG_ERR_ARG = 1,          /* invalid argument (null pointer, size, enum)      */
  DG_ERR_MESH = 2,         /* invalid mesh: connectivity, non-positive Jacobian */
  DG_ERR_HIP = 3,          /* a HIP runtime call failed; message has the text  */
  DG_ERR_NONPHYSICAL = 4,  /* rho <= 0, p <= 0 or a non-finite value           */
  DG_ERR_NOMEM = 5,        /* device allocation failed                          */
  DG_ERR_UNSUPPORTED = 6,  /* valid but not built (e.g. N outside 1..7)         */
  DG_ERR_STATE = 7         /* call order: no mesh uploaded / no workspace       */
} dg_status;

enum { DG_NODES_GAUSS = 0, DG_NODES_LOBATTO = 1 };
enum { DG_FORM_WEAK = 0, DG_FORM_SPLIT = 1 };
enum { DG_PHYS_EULER = 0, DG_PHYS_NAVIER_STOKES = 1 };
/* Face flux dissipation: Rusanov (max wave speed), none (central part alone,
 * tests), or Roe's linearisation with the Harten-Hyman entropy fix on the
 * acoustic speeds, the paper's flux (§Governing Equations and Numerical Method). */
enum { DG_RIEMANN_RUSANOV = 0, DG_RIEMANN_CENTRAL = 1, DG_RIEMANN_ROE = 2 };
/* Viscosity law: constant mu, or Sutherland's law
 * mu(T) = mu (T/Tref)^(3/2) (1 + Ts) / (T/Tref + Ts) (TGV section); the heat
 * conductivity follows at constant Prandtl number. */
enum { DG_VISC_CONSTANT = 0, DG_VISC_SUTHERLAND = 1 };
enum { DG_TWOPOINT_CHANDRASHEKAR = 0, DG_TWOPOINT_CENTRAL = 1 };
enum { DG_PREC_FP64 = 0, DG_PREC_FP32_FLUX = 1 };
/* Low-storage explicit RK scheme (paper: time integration section): the
 * five-stage LSERK4(5) of Carpenter and Kennedy, or the fourteen-stage
 * LSERK4-14 of Niegemann, Diehl and Busch that the paper's production runs use. */
enum { DG_RK_LSERK45 = 0, DG_RK_LSERK414 = 1 };
#define DG_RK_MAX_STAGES 14

typedef struct {
  int N;            /* polynomial degree, 1..7                                       */
  int nodes;        /* DG_NODES_*; on Gauss nodes the split form is the entropy-stable
                       hybridised form with entropy-projected face states           */
  int volume_form;  /* DG_FORM_*                                                     */
  int physics;      /* DG_PHYS_*                                                     */
  int riemann;      /* DG_RIEMANN_*: Rusanov, Roe, or the central part alone (tests)  */
  int twopoint;     /* DG_TWOPOINT_*: Chandrashekar, or the flux average (tests)      */
  int precision;    /* DG_PREC_*: FP64, or FP32 flux arithmetic with FP64 state,
                       metrics, pressure recovery, metric contraction and update     */
  int integrator;   /* DG_RK_*: the low-storage RK scheme of dg_rk_step               */
  int viscosity;    /* DG_VISC_*: constant mu, or Sutherland's law mu(T)              */
  int fv;           /* 1: elements may be switched to FV sub-cells (shock capturing,
                       dg_fv_*); Euler, FP64, Rusanov, weak form or LGL split form   */
  double gamma;     /* ratio of specific heats                                        */
  double mu;        /* constant dynamic viscosity (Navier-Stokes)                     */
  double Pr;        /* Prandtl number                                                 */
  double R;         /* specific gas constant                                          */
  double Tref;      /* Sutherland: temperature at which the viscosity is mu (> 0)     */
  double Ts;        /* Sutherland: S / Tref, the Sutherland constant over Tref (>= 0) */
} dg_config;

/* Context ------------------------------------------------------------------ */

/* Validates cfg and creates a context (host memory only; no device work).
 * DG_ERR_ARG for bad enums or gamma <= 1, mu < 0, Pr <= 0, R <= 0;
 * DG_ERR_UNSUPPORTED for N outside the built range, or fv = 1 with FP32 flux
 * arithmetic, Roe's flux or Sutherland's law (FV sub-cells: Rusanov, FP64,
 * constant viscosity; any DG form, Euler or Navier-Stokes). */
dg_status dg_create(const dg_config* cfg, dg_ctx** out);

/* Frees all library-owned host and device memory of ctx (NULL is a no-op). */
dg_status dg_destroy(dg_ctx* ctx);

/* Reference state (rho0 > 0, p0 > 0) of the FP32-flux mode (paper: "Mixed
 * Precision"): its flux arithmetic rounds the deviations of p_hat, 1/beta^ln,
 * p and the total enthalpy from this state in float and adds the state's own
 * part in double, which keeps the float rounding small where p is large and
 * nearly constant (low Mach numbers).  It changes rounding only; FP64
 * contexts ignore it.  (0, 0) clears it (the default).  DG_ERR_ARG for other
 * non-positive values. */
dg_status dg_set_reference_state(dg_ctx* ctx, double rho0, double p0);

/* Message of the last failing call on ctx, or of the calling thread when ctx is NULL. */
const char* dg_last_error(const dg_ctx* ctx);

/* The five-stage coefficients A, B, c of LSERK4(5) (Carpenter and Kennedy 1994). */
dg_status dg_lserk_coefficients(double* A5, double* B5, double* c5);

/* Coefficients A, B, c of the scheme DG_RK_* (arrays of DG_RK_MAX_STAGES
 * entries; the first *nstages are written).  DG_ERR_ARG for an unknown scheme. */
dg_status dg_rk_coefficients(int integrator, double* A, double* B, double* c, int* nstages);

/* Mesh and metrics ------------------------------------------------------------ */

/* Host part of the mesh set-up: validates connectivity, builds the per-element
 * face table, interpolates the geometry to the solution nodes and computes the
 * metric terms in conservative curl form (paper: mapping chi, Jacobian J,
 * contravariant fluxes; Kopriva 2006 curl form), the Jacobian and the master
 * face normals.  No device work.  DG_ERR_MESH on bad connectivity or a
 * non-positive Jacobian at any node.  An element whose nine metric components
 * and 1/J each vary by at most 1e-12 of their largest magnitude over its nodes
 * (an affine element: the exact terms are constant) gets their node mean at
 * every node, so that its terms are exactly constant. */
dg_status dg_set_mesh(dg_ctx* ctx, int nElems, int Ngeo, const double* X, int nSides,
                      const int* side_elem, const int* side_loc, const int* side_orient);

/* dg_set_mesh followed by the upload of metrics and connectivity to
 * library-owned device memory on the current device. */
dg_status dg_upload_mesh(dg_ctx* ctx, int nElems, int Ngeo, const double* X, int nSides,
                         const int* side_elem, const int* side_loc, const int* side_orient);

/* Optional override of the metric terms after dg_upload_mesh (host arrays):
 * Ja[9][nElems][n3] (component 3r+n = Ja^r_n), sJ[nElems][n3] = 1/J,
 * nvec[3][nSides][n2] = master-outward n*s at face nodes in master (p,q) order. */
dg_status dg_upload_metrics(dg_ctx* ctx, const double* Ja, const double* sJ, const double* nvec);

/* Host copies of the metrics computed by dg_set_mesh (any pointer may be NULL):
 * xyz[3][nElems][n3], Ja[9][nElems][n3], sJ[nElems][n3], nvec[3][nSides][n2]. */
dg_status dg_get_metrics(const dg_ctx* ctx, double* xyz, double* Ja, double* sJ, double* nvec);

/* Per-element metric terms.  An element whose metric terms (Ja and 1/J) are
 * bitwise the same at all of its nodes has them stored once more, per
 * element, and the residual, lifting and adjoint kernels read that copy
 * instead of the node arrays: 80 bytes per node less per kernel.  The
 * lifting of such an element forms the gradient's volume part as
 * Ja^r (Dhat q) rather than Dhat (Ja^r q) (equal for constant Ja), and the
 * adjoint uses its transpose: Euler results are bitwise equal to the
 * node-array path, Navier-Stokes results agree to rounding.  On by default; enable = 0
 * sends every element to the node arrays (the paper's per-node storage).
 * Takes effect at once when a mesh is on the device, else at its upload;
 * metrics replaced by dg_upload_metrics are examined again. */
dg_status dg_set_element_metrics(dg_ctx* ctx, int enable);

/* Number of elements whose kernels read the per-element metric terms.
 * DG_ERR_STATE before dg_upload_mesh. */
dg_status dg_element_metric_count(const dg_ctx* ctx, int* count);

/* Node coordinates xyz[3][nElems][n3] (host) for building initial states. */
dg_status dg_node_coords(const dg_ctx* ctx, double* xyz_host);

/* Sizes: number of elements, sides, nodes per element, state length. */
dg_status dg_sizes(const dg_ctx* ctx, int* nElems, int* nSides, int* nodes_per_elem, size_t* state_len);

/* Workspace ------------------------------------------------------------------- */

/* Bytes of device scratch the context needs (face traces, lifted gradients,
 * RK stage states of the adjoint, reduction partials).  Valid after a mesh is set. */
size_t dg_workspace_bytes(const dg_ctx* ctx);

/* Bytes of device scratch that the adjoint calls need (the forward scratch
 * plus the recomputed stage states, four for LSERK4(5) and thirteen for
 * LSERK4-14, an RK register, an adjoint residual and, for Navier-Stokes, the
 * face values of the gradient adjoint).  Valid after a mesh is set. */
size_t dg_workspace_bytes_adjoint(const dg_ctx* ctx);

/* Binds caller-owned device memory of at least dg_workspace_bytes bytes,
 * 256-byte aligned.  The library never frees it.  With at least
 * dg_workspace_bytes_adjoint bytes the adjoint calls are enabled; without,
 * they fail with DG_ERR_STATE. */
dg_status dg_bind_workspace(dg_ctx* ctx, void* dev_ptr, size_t bytes);

/* State ------------------------------------------------------------------------ */

/* Initial state (paper: the solution is set from the initial condition before
 * time stepping).  Copies U_src, conserved variables in the layout
 * U[5][nElems][n3] and of the state length, into the caller-owned device array
 * U: from host memory when src_is_device == 0 (pageable or pinned), from
 * device memory otherwise (U_src == U is allowed and copies nothing).  Then
 * checks U as dg_check_state does and returns DG_ERR_NONPHYSICAL if a node has
 * rho <= 0, p <= 0 or a non-finite value (U still holds the copied values).
 * Needs a bound workspace; synchronises the stream. */
dg_status dg_init_state(dg_ctx* ctx, const double* U_src, int src_is_device, double* U, void* stream);

/* Residual and time stepping -------------------------------------------------- */

/* Ut = dU/dt(U): prolongation to faces, Riemann and viscous surface fluxes,
 * BR1 lifting (Navier-Stokes), weak or split volume integral, surface lift,
 * Jacobian scaling (paper eq. dgsem_weak / dgsem_lifted).  U and Ut are device
 * arrays of the state length; they must not alias.  t is unused (autonomous). */
dg_status dg_rhs(dg_ctx* ctx, const double* U, double* Ut, double t, void* stream);

/* Lifted gradients g[12][nElems][n3] (device), component 3a+d = d q_a / d x_d
 * with q = (u, v, w, T) (paper eq. dgsem_lifted).  Navier-Stokes contexts only. */
dg_status dg_lift(dg_ctx* ctx, const double* U, double* g, void* stream);

/* nsteps steps of the context's low-storage RK scheme (LSERK4(5) or
 * LSERK4-14) with fixed dt, in place: per stage s
 * dU <- A_s dU + dt R(U); U <- U + B_s dU.  dU is the 2N-storage register
 * (device, state length); it is zeroed by the call before the first stage. */
dg_status dg_rk_step(dg_ctx* ctx, double* U, double* dU, double t, double dt, int nsteps, void* stream);

/* One step of dg_rk_step (same arithmetic) that also keeps its stage inputs
 * Y_1..Y_{S-1} in Y (device, caller-owned, S-1 state lengths, stage k at
 * Y + (k-1) * state length; S = 5 or 14) for dg_adjoint_rk_step_stages, which
 * then skips recomputing them (not in the paper: a memory-for-time trade of
 * the discrete adjoint).  U, dU and Y must not alias.  DG_ERR_UNSUPPORTED for
 * contexts with FV sub-cells. */
dg_status dg_rk_step_stages(dg_ctx* ctx, double* U, double* dU, double t, double dt, double* Y, void* stream);

/* dg_rk_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same steps, with the scratch in a static device array of the library
 * (256 MiB, one per GPU, held until the process ends) instead of the bound
 * workspace; no workspace needs to be bound.  The call allocates nothing
 * (no hipMalloc, hipFree, event creation or allocating library routine);
 * event profiling (dg_profile) does not see it.  DG_ERR_ARG if the mesh needs
 * more scratch than the static array holds (dg_workspace_bytes above
 * 256 MiB).  Every call on one GPU, from any context, shares that GPU's
 * array, which keeps the last call's contents: calls that overlap in time on
 * one GPU (other streams, other threads) race and give wrong results. */
dg_status dg_rk_step_noalloc(dg_ctx* ctx, double* U, double* dU, double t, double dt, int nsteps, void* stream);

/* Adjoint --------------------------------------------------------------------- */

/* out = (dR/dU)^T lam at the state U (device arrays, state length; out must
 * not alias U or lam).  This is the transpose of the discrete residual's
 * Jacobian (not in the paper: a discrete adjoint of its residual); at the
 * kinks of the Rusanov flux (|u.n|, max of the two wave speeds), of Roe's
 * flux (|.| of the wave speeds, the Harten-Hyman fix) and of the log-mean
 * branch switch the branch taken by the forward evaluation is
 * differentiated, ties going to the master side.  Covers every FP64 DG
 * configuration: weak and split forms on both node sets (on Gauss nodes the
 * hybridised form with its entropy-projected traces), Rusanov and Roe,
 * constant viscosity and Sutherland's law; DG_ERR_UNSUPPORTED for FP32 flux
 * arithmetic and FV sub-cells.  Needs a workspace of
 * dg_workspace_bytes_adjoint bytes. */
dg_status dg_adjoint_rhs(dg_ctx* ctx, const double* U, const double* lam, double* out, void* stream);

/* Reverse of one step of size dt of the context's RK scheme (S stages) from
 * state Un (device): on entry lamU holds dJ/dU^{n+1}; on exit dJ/dU^n.  The
 * stage inputs Y_0..Y_{S-1} are recomputed from Un into the workspace; then,
 * with lamdU = B_{S-1} lamU, for s = S-1..0: lamU += dt (dR/dU(Y_s))^T lamdU
 * and lamdU = A_s lamdU + B_{s-1} lamU.
 * lamdU is a caller-owned device register of the state length (scratch).
 * Needs a workspace of dg_workspace_bytes_adjoint bytes. */
dg_status dg_adjoint_rk_step(dg_ctx* ctx, const double* Un, double* lamU, double* lamdU, double t, double dt,
                             void* stream);

/* dg_adjoint_rk_step with the step's stage inputs Y_1..Y_{S-1} supplied (as
 * dg_rk_step_stages leaves them in Y) instead of recomputed from Un. */
dg_status dg_adjoint_rk_step_stages(dg_ctx* ctx, const double* Un, const double* Y, double* lamU, double* lamdU,
                                    double t, double dt, void* stream);

/* Functionals and checks ------------------------------------------------------ */

/* Integral kinetic energy E_k = sum_e sum w_i w_j w_k J |m|^2/rho / (2 rho0U0sq |Omega|),
 * |Omega| = sum w J (paper, TGV section).  Writes one double to out_dev. */
dg_status dg_kinetic_energy(dg_ctx* ctx, const double* U, double rho0U0sq, double* out_dev, void* stream);

/* grad = scale * dE_k/dU (device, state length). */
dg_status dg_kinetic_energy_grad(dg_ctx* ctx, const double* U, double rho0U0sq, double scale, double* grad,
                                 void* stream);

/* Fixed time step from the state (paper: CFL = 0.9 for the advective and the
 * viscous restriction; the formula is this library's reading):
 *   dt_a = cfl S min(2/(N+1), 8/(N+1)^2) / max sum_r (|Ja^r.u| + c|Ja^r|)/J
 *   dt_v = cfl S 32/(N+1)^4 / max (mu/rho) max(4/3, gamma/Pr) sum_r |Ja^r|^2/J^2
 * dt = min(dt_a, dt_v) (dt_v for Navier-Stokes only), with S = 1 for
 * LSERK4(5) and S = 3.75 for LSERK4-14, whose stability limit on the DG
 * spectrum is 3.98 times larger.  Synchronises the stream and writes the
 * host double dt_out. */
dg_status dg_timestep(dg_ctx* ctx, const double* U, double cfl, double* dt_out, void* stream);

/* DG_ERR_NONPHYSICAL if any node has rho <= 0, p <= 0 or a non-finite
 * conserved value; synchronises the stream. */
dg_status dg_check_state(dg_ctx* ctx, const double* U, void* stream);

/* FV sub-cell shock capturing ------------------------------------------------ */
/* (paper: "Governing Equations and Numerical Method": troubled DG elements are
 * replaced by a second-order FV scheme on (N+1)^3 integral means per element,
 * detected with Persson and Peraire's modal indicator; "Intra-GPU
 * Parallelism": the indicator and the switching as element-local kernels).
 * Contexts created with cfg.fv = 1 only (else DG_ERR_STATE).  Every element
 * is DG or FV; the state of an FV element holds its sub-cell means (the
 * sub-cells are the equidistant (N+1)^3 sub-cubes of the reference element,
 * U[v][e][k][j][i] the mean over sub-cell (i,j,k)), and dg_rhs returns their
 * time derivative.  Reading of the scheme:
 *   - DG -> FV: mean_s = (integral over s of J U) / V_s, V_s = integral of J,
 *     both exact for the nodal interpolants; FV -> DG is its inverse.  Both
 *     conserve sum V mean = sum w J U.
 *   - Sub-cell face vectors: exact integrals of the metric interpolant Ja^r
 *     over each sub-face; on element faces, of the master's face normal n s.
 *   - MUSCL reconstruction of (rho, u, v, w, p) with the minmod limiter; the
 *     neighbour element's first sub-cell layer is the ghost cell; Rusanov flux.
 *   - A face with an FV element on either side is evaluated on its (N+1)^2
 *     sub-faces from both sides' first two sub-cell layers (a DG side
 *     contributes the means of its own state); the DG side takes back the
 *     nodal face flux whose sub-face integrals are those fluxes.
 *   - Indicator: log10 of the share of the modes with max(i,j,k) = N in the
 *     energy of rho in the orthonormal Legendre basis (of the DG
 *     reconstruction for FV elements), clamped below at -30.
 * dg_timestep, dg_kinetic_energy and dg_check_state read FV elements' means
 * as if they were nodal values. */

/* Element types to mask_host[nElems] (host, 0 = DG, 1 = FV); converts U and,
 * if dU is not NULL, the RK register dU (device, state length, in place) of
 * every element whose type changes.  The mask copy is synchronous. */
dg_status dg_fv_switch(dg_ctx* ctx, double* U, double* dU, const int* mask_host, void* stream);

/* Persson indicator of every element of U into ind_dev[nElems] (device). */
dg_status dg_fv_indicator(dg_ctx* ctx, const double* U, double* ind_dev, void* stream);

/* Indicator-driven switch: an element becomes FV where its indicator exceeds
 * ind_hi, DG where it is below ind_lo, and keeps its type in between; U and
 * dU (may be NULL) are converted as by dg_fv_switch.  ind_lo <= ind_hi. */
dg_status dg_fv_switch_by_indicator(dg_ctx* ctx, double* U, double* dU, double ind_lo, double ind_hi,
                                    void* stream);

/* Current element types (host, nElems ints); synchronises the stream. */
dg_status dg_fv_mask(dg_ctx* ctx, int* mask_host, void* stream);

/* Profiling ------------------------------------------------------------------- */

/* Per-kernel device timing (the analogue of the paper's per-kernel device
 * events, "Intra-GPU Parallelism"): while enabled, every launch of the
 * context is bracketed by two hipEvents on its stream.  Enabling resets
 * the accumulated times.  dg_profile_query synchronises the device, then
 * returns the summed milliseconds and launch count of the kernel family
 * named by `kernel` ("trace", "lift", "volume", "adjoint", "other", "fv").
 * Unknown names give DG_ERR_ARG. */
dg_status dg_profile(dg_ctx* ctx, int enable);
/* As dg_profile, but only the launches of the families in `mask` are
 * bracketed (bit 0 trace, 1 lift, 2 volume, 3 adjoint, 4 other, 5 fv); 0
 * disables.  Fewer events perturb a timed run less.  A mask outside 0..63
 * gives DG_ERR_ARG. */
dg_status dg_profile_families(dg_ctx* ctx, int mask);
dg_status dg_profile_query(dg_ctx* ctx, const char* kernel, double* total_ms, long* count);

#ifdef __cplusplus
}
#endif

#endif /* DGX_H */
