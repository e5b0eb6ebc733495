/*
 * libgrf -- MI355X (gfx950) FP64 hot path of the 4dST + modified-CCZ4 method:
 * the pointwise right-hand side of CCZ4 in the modified puncture gauge coupled
 * to a scalar field with the four-derivative scalar-tensor terms, with
 * Kreiss-Oliger dissipation, and the classic RK4 stage update, on 3-D boxes with
 * three (or, for the sixth-order scheme, four) ghost cells (the method named in the paper's Summary and Key features:
 * 4dST theory, modified moving-puncture gauge, 4th- and 6th-order finite
 * differences, RK4, periodic and per-face boundary rules, the decoupling
 * limit, constraint, energy and weak-coupling diagnostics), a batched form for
 * many boxes and the adjoint of the right-hand side and of an RK4 step.
 *
 * Conventions shared by every call
 *  - State layout: 27 FP64 fields, field-major; field f of a box starts at
 *    f * field_stride; within a field, cells are [z][y][x] with x fastest over
 *    (nx+2g) x (ny+2g) x (nz+2g) cells (g = 3 ghost cells on every side, or
 *    g = 4 for the sixth-order scheme described at fd_order).  Field order:
 *      chi, h11 h12 h13 h22 h23 h33, K, A11 A12 A13 A22 A23 A33, Theta,
 *      Gam1 Gam2 Gam3, lapse, shift1 shift2 shift3, B1 B2 B3, phi, Pi.
 *  - Interior arrays ("compact"): 27 fields, field-major, nx*ny*nz cells each,
 *    [z][y][x] with x fastest, no ghosts (used for the RK4 accumulator).
 *  - Every pointer argument named u*, rhs, acc, w*, *_bar, workspace is device
 *    memory owned by the caller; grf_params / grf_box are host structs read at
 *    call time.  Nothing is allocated by these calls.
 *  - All calls are asynchronous on `stream` (0 = the null stream).  Argument
 *    errors are detected on the host, returned synchronously, and leave every
 *    output untouched.  Conditions found on the device (non-finite results, a
 *    near-singular per-cell system, chi <= 0 or lapse <= 0) are OR-ed into a
 *    status word at the start of the workspace; read it with
 *    grf_status_fetch, clear it with grf_status_clear.
 *  - Calls that share a workspace must not overlap in time (same stream, or
 *    ordered by events).
 */
#ifndef GRF_H
#define GRF_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GRF_OK = 0,
  GRF_EINVAL = 1,        /* null pointer, bad stage number, bad parameter value   */
  GRF_ESHAPE = 2,        /* box dimensions, ghost count or field stride invalid   */
  GRF_EHIP = 3,          /* a HIP runtime call failed                              */
  GRF_ENONFINITE = 4,    /* device: a right-hand side was NaN or infinite         */
  GRF_EHYPERBOLIC = 5,   /* device: the per-cell 7x7 system was near-singular     */
  GRF_ENOMEM = 6,        /* workspace smaller than required                       */
  GRF_EUNSUPPORTED = 7,  /* parameter combination not implemented                 */
  GRF_ENONPOSITIVE = 8   /* device: chi <= 0 or lapse <= 0 at some cell          */
} grf_status;

enum { GRF_NFIELDS = 27, GRF_NTHETA = 2, GRF_NGHOST = 3 };
enum { GRF_BC_FROZEN = 0, GRF_BC_PERIODIC = 1 };
enum { GRF_LAMBDA_QUADRATIC = 0 };
/* device status bits (grf_status_fetch's *bits) */
enum { GRF_FLAG_NONFINITE = 1, GRF_FLAG_HYPERBOLIC = 2, GRF_FLAG_NONPOSITIVE = 4 };

/* Couplings and gauge.  lambda(phi) = lambda_lin phi + lambda_gb (1 -
 * exp(-beta phi^2)) / (4 beta), which is lambda_gb phi^2 / 4 at beta = 0
 * (lambda_kind 0 only; lambda_lin alone is the shift-symmetric coupling,
 * beta > 0 the exponential coupling of spin-induced scalarisation studies;
 * the batched form takes lambda_lin = beta = 0 only),
 * g2 constant, V = 0.  a_gauge, b_gauge: the modified-gauge functions a(x), b(x)
 * (constants).  lapse: d_t alpha = lapse_advec beta.d alpha
 *   - lapse_coeff alpha^lapse_power (K - 2 Theta) / (1 + a)   (lapse_power 1 only);
 * shift (B form): d_t beta^i = shift_advec beta.d beta^i + shift_gamma_coeff B^i
 *   - a/(1+a) alpha D^i alpha,  d_t B^i = d_t Gam^i/(1+a) - eta B^i (+ advection).
 * enforce / chi_min / lapse_min: post-stage algebraic enforcement (0 = off, the
 * default everywhere; 1 = grf_enforce applied to every stage output of
 * grf_rk4_stage before its ghost fill; the batched and adjoint paths reject it).
 * decoupled: 0 the full theory; 1 the decoupling limit (Key features, "Modified
 * gravity theories": 4dST without backreaction): the scalar evolves with its
 * full equation on the metric, which evolves as in vacuum (no energy,
 * momentum, stress or Gauss-Bonnet tensor in the metric equations; the metric
 * rows of the per-cell system reduce to C_ij = Q_ij), gauge unchanged.
 * Supported by grf_rhs_eval, grf_rk4_stage and grf_rk4_stage_bc on stage path
 * 2 (the default), by grf_constraints (without scalar sources) and by the
 * adjoint (its own generated reverse); the other paths, the energy and
 * coupling diagnostics and the batched form return GRF_EUNSUPPORTED.
 * fd_order: 4 (or 0) fourth-order stencils; 6 sixth-order stencils (Key
 * features, "Accuracy").  On a box with three ghost layers: centred first,
 * second and mixed derivatives of order 6, the advection derivative of order
 * 5 on the six points leaning one cell to the side the shift points to, the
 * same Kreiss-Oliger operator (an O(h^5) term).  On a box with four ghost
 * layers (grf_box.ng = 4): the same centred derivatives, the advection
 * derivative of order 6 on offsets -2..4 (mirrored for a negative shift) and
 * the dissipation -sigma/(256 h) times the eighth difference, so the scheme
 * keeps order 6 with dissipation on.  Order 6 runs the z-marching 32x8x32
 * stencil kernel whatever grf_set_tile_variant chose, on stage paths 0 and 2,
 * in grf_rhs_eval, grf_rk4_stage, grf_rk4_stage_bc, the diagnostics and the
 * adjoint (the transposes of the same stencils); the batched form returns
 * GRF_EUNSUPPORTED. */
typedef struct {
  double lambda_gb;
  int32_t lambda_kind;
  double g2;
  double a_gauge, b_gauge;
  double kappa1, kappa2, kappa3;
  double lapse_coeff, lapse_power, lapse_advec;
  double shift_gamma_coeff, shift_advec, eta;
  double ko_sigma;
  int32_t enforce;
  double chi_min, lapse_min;
  int32_t decoupled;
  int32_t fd_order;
  double lambda_lin;
  double beta;
} grf_params;

/* One box: nx, ny, nz interior cells, ng ghosts, spacing dx, dy, dz,
 * coordinates x0, y0, z0 of the centre of interior cell (0,0,0) (read by the
 * radiative boundary rule only), field_stride >= (nx+2ng)(ny+2ng)(nz+2ng),
 * boundary rule bc.  ng is 3, or 4 with fd_order 6 (GRF_EUNSUPPORTED with
 * fd_order 4); the batched form refuses four ghost layers with
 * GRF_EUNSUPPORTED (its size query returns 0), every other call takes them;
 * GRF_ESHAPE for any other ng. */
typedef struct {
  int32_t nx, ny, nz, ng;
  double dx, dy, dz;
  double x0, y0, z0;
  int64_t field_stride;
  int32_t bc;
} grf_box;

/* Bytes of workspace needed by grf_rhs_eval / grf_rk4_stage on this machine
 * (the status word plus one 198-component derivative record per interior cell). */
size_t grf_workspace_bytes(const grf_box* box);

/* Right-hand side d_t u (including Kreiss-Oliger) at interior cells of u,
 * written to the interior cells of rhs (state layout; ghosts of rhs untouched).
 * The operation: the CCZ4 equations in the modified puncture gauge coupled to
 * the scalar with the four-derivative scalar-tensor terms (Summary; Key
 * features, "Stable gauge evolution" and "Modified gravity theories"),
 * discretised with the finite differences of Key features, "Accuracy". */
grf_status grf_rhs_eval(const grf_params* p, const grf_box* box, const double* u, double* rhs,
                        void* workspace, size_t workspace_bytes, hipStream_t stream);

/* One classic RK4 stage (c = 1/2, 1/2, 1; weights 1, 2, 2, 1 over 6), stage in 1..4:
 * the method-of-lines time integration of the right-hand side above (Key
 * features, "Accuracy").
 * Reads u0 (state at the start of the step) and us (the stage state; us == u0 at
 * stage 1), computes k = RHS(us) and, on interior cells,
 *   stage 1: acc  = k;             unext = u0 + (dt/2) k
 *   stage 2: acc  = acc + 2 k;     unext = u0 + (dt/2) k
 *   stage 3: acc  = acc + 2 k;     unext = u0 + dt k
 *   stage 4:                       unext = u0 + (dt/6)(acc + k)   (the new state)
 * each product rounded on its own (no fused multiply-add).  acc is compact (27 x nx*ny*nz).  unext must not alias us
 * or u0.  GRF_BC_PERIODIC: the ghosts of unext are then filled periodically;
 * GRF_BC_FROZEN: ghosts of unext are not written (the caller keeps them at the
 * frozen values, e.g. by allocating unext as a copy of the initial state). */
grf_status grf_rk4_stage(const grf_params* p, const grf_box* box, int stage, double dt, const double* u0,
                         const double* us, double* unext, double* acc, void* workspace, size_t workspace_bytes,
                         hipStream_t stream);

/* RK4 stage that allocates nothing and takes no workspace, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, arithmetic,
 * results (bitwise) and ghost handling as grf_rk4_stage, except:
 *  - the derivative records live in a device array of the library, 128 MiB
 *    on each GPU it runs on, held until the process ends; the box is swept in
 *    z-slabs of as many interior planes as fit (1584 bytes per cell), so one
 *    plane of nx * ny cells may hold at most 84,733 cells: larger planes are
 *    refused with GRF_ENOMEM before anything runs;
 *  - device conditions are OR-ed into *status, a caller-owned device word
 *    (read it with grf_status_fetch(status, ...), clear it with
 *    grf_status_clear(status, ...)); the call does not clear it;
 *  - it always runs the split path with staged pointwise inputs.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (every slab's record is written before it is read, so nothing needs
 * clearing); calls that overlap in time on one GPU, from any stream or host
 * thread, race on it and give undefined results.  No hipMalloc, hipFree or
 * allocating library call is made; the device address of the array is looked
 * up once per device on the first call there. */
grf_status grf_rk4_stage_static(const grf_params* p, const grf_box* box, int stage, double dt, const double* u0,
                                const double* us, double* unext, double* acc, uint32_t* status,
                                hipStream_t stream);

/* Algebraic enforcement on the interior cells of a state, in place:
 * h_ij <- h_ij det(h)^(-1/3) (unit determinant), A_ij <- A_ij - 1/3 h_ij h^kl A_kl
 * with the corrected h, chi <- max(chi, chi_min), lapse <- max(lapse, lapse_min).
 * Uses p->chi_min and p->lapse_min whatever p->enforce is. */
grf_status grf_enforce(const grf_params* p, const grf_box* box, double* u, hipStream_t stream);

/* Periodic ghost fill of a state (every ghost copies the interior cell congruent
 * to it modulo the box size), on the device. */
grf_status grf_fill_periodic(const grf_box* box, double* u, hipStream_t stream);

/* ---- Boundary rules per face (Key features, "Boundary Conditions": periodic,
 * reflective, extrapolating and Sommerfeld (radiative) faces).
 * Faces are numbered x-, x+, y-, y+, z-, z+.  Every ghost cell belongs to one
 * face: the x face when its x index lies outside the interior, else the y face
 * when its y index does, else the z face.
 *   frozen:        the ghost is integrated with right-hand side 0 (keeps its value);
 *   periodic:      copies the interior cell congruent to it along the face's axis
 *                  (both faces of that axis must be periodic);
 *   reflective:    copies the mirror cell across the face (ghost layer d <-> interior
 *                  layer d), times -1 per tensor index of the field along the face's
 *                  axis (h_ij, A_ij: two indices; Gamma^i, beta^i, B^i: one;
 *                  phi and Pi: parity_phi);
 *   extrapolating: order 0 copies the outermost interior cell along the axis,
 *                  order 1 extends the line through the two outermost interior cells;
 *   sommerfeld:    the ghost is integrated with the radiative right-hand side
 *                  d_t f = -v (x^a d_a f + f - f_inf) / r, x^a = position - centre
 *                  (cell (i,j,k) at (x0 + i dx, y0 + j dy, z0 + k dz)),
 *                  r = |x^a|, with second-order differences (one-sided towards the
 *                  interior along the axes on which the cell is a ghost, centred
 *                  along the others).
 * After each RK4 stage the periodic, reflective and extrapolating ghosts are
 * refilled from the new state, z faces first, then y, then x, so every face
 * reads only cells that are final. */
enum { GRF_FACE_FROZEN = 0, GRF_FACE_PERIODIC = 1, GRF_FACE_REFLECTIVE = 2, GRF_FACE_EXTRAPOLATING = 3,
       GRF_FACE_SOMMERFELD = 4 };
typedef struct {
  int32_t rule[6];         /* GRF_FACE_* per face x-, x+, y-, y+, z-, z+ */
  int32_t extrap_order;    /* 0 or 1 (extrapolating faces) */
  int32_t parity_phi;      /* +1 or -1: sign of phi and Pi under a reflection */
  double centre[3];        /* centre of the radiative rule (coordinates as the box's x0, y0,
                              z0); must not be a ghost cell centre */
  double speed[27];        /* radiative speed v per field (finite) */
  double asymptote[27];    /* f_inf per field (finite) */
} grf_bc;

/* Number of ghost cells of a box ((nx+2ng)(ny+2ng)(nz+2ng) - nx ny nz); the ghost
 * accumulator of grf_rk4_stage_bc holds 27 times as many doubles.  0 for an
 * invalid box. */
int64_t grf_bc_ghost_cells(const grf_box* box);

/* Refill the ghosts of the periodic, reflective and extrapolating faces of u
 * (device, state layout) from u; other ghosts and the interior untouched.
 * Errors: GRF_EINVAL for an invalid rule, an unpaired periodic face, an
 * extrapolation order other than 0/1, a parity other than +-1, a reflective
 * face on an axis with fewer cells than ghost layers or an order-1
 * extrapolating face on one with fewer than 2. */
grf_status grf_bc_fill(const grf_bc* bc, const grf_box* box, double* u, hipStream_t stream);

/* Ghost right-hand side: every ghost cell of rhs (device, state layout) gets
 * the radiative right-hand side of u on Sommerfeld faces and 0 on the others;
 * interior cells of rhs untouched.  Errors as grf_bc_fill, plus GRF_EINVAL when
 * the centre is a ghost cell centre or a speed/asymptote is not finite. */
grf_status grf_bc_ghost_rhs(const grf_bc* bc, const grf_box* box, const double* u, double* rhs,
                            hipStream_t stream);

/* One RK4 stage with per-face rules: the interior exactly as grf_rk4_stage
 * with a frozen box (box->bc is not used), the Sommerfeld ghosts with the same
 * stage formulas on their radiative right-hand side (gacc: device,
 * [27][grf_bc_ghost_cells] doubles, their accumulator, caller-owned), then
 * the refill of grf_bc_fill on unext.  Frozen ghosts of unext are not written.
 * The state passed as u0 at stage 1 must have its fill-rule ghosts filled
 * (grf_bc_fill).  Errors as grf_rk4_stage and grf_bc_ghost_rhs. */
grf_status grf_rk4_stage_bc(const grf_params* p, const grf_box* box, const grf_bc* bc, int stage, double dt,
                            const double* u0, const double* us, double* unext, double* acc, double* gacc,
                            void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Vector-Jacobian product of the right-hand side (the adjoint of the
 * operation of grf_rhs_eval, for gradients of observables with respect to the
 * couplings and the initial data): with w a cotangent of
 * grf_rhs_eval's output (state layout, interior cells read),
 *   u_bar     += (d RHS / d u)^T w      over all cells of u, ghosts included,
 *   theta_bar += (d RHS / d (lambda_gb, g2))^T w   (2 doubles, device memory),
 * the coupling sum taken in a fixed order (deterministic).  Workspace size from
 * grf_vjp_workspace_bytes. */
size_t grf_vjp_workspace_bytes(const grf_box* box);
grf_status grf_rhs_vjp(const grf_params* p, const grf_box* box, const double* u, const double* w, double* u_bar,
                       double* theta_bar, void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Adjoint of one frozen-ghost RK4 step u -> u_new (the four stages of
 * grf_rk4_stage).  Inputs: the step's start state u and its stage states
 * u2 = u + dt/2 k1, u3 = u + dt/2 k2, u4 = u + dt k3 (state layout, ghosts equal
 * to u's), and ubar_new, the cotangent of u_new (all cells).  Output:
 *   ubar       = (d u_new / d u)^T ubar_new        (all cells, overwritten),
 *   theta_bar += (d u_new / d (lambda_gb, g2))^T ubar_new.
 * ubar must not alias any input.  Workspace from grf_rk4_step_vjp_workspace_bytes
 * (the RHS-VJP workspace plus two state-sized temporaries). */
size_t grf_rk4_step_vjp_workspace_bytes(const grf_box* box);
grf_status grf_rk4_step_vjp(const grf_params* p, const grf_box* box, double dt, const double* u, const double* u2,
                            const double* u3, const double* u4, const double* ubar_new, double* ubar,
                            double* theta_bar, void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Device status word kept at the start of a workspace: synchronises `stream`,
 * returns GRF_OK or the device condition of highest precedence (NONFINITE,
 * then HYPERBOLIC, then NONPOSITIVE), and stores the raw bits in *bits if non-null. */
grf_status grf_status_fetch(const void* workspace, hipStream_t stream, uint32_t* bits);
grf_status grf_status_clear(void* workspace, hipStream_t stream);

/* Algorithmic FP64 flops per interior cell: the pointwise algebra of one RHS
 * (shift advection on or off), of its VJP, of the constraint diagnostics and
 * of the energy densities, counted on the expression graph (add, sub, mul and
 * reciprocal each 1), stencils not included; -1 for another `which`. */
int64_t grf_flops_per_cell(int which /* 0 rhs, 1 rhs with shift advection, 2 vjp, 3 constraints, 4 energy,
                                         5 rhs in the decoupling limit, 6 coupling diagnostics */);

/* Constraint diagnostics (Key features, "Diagnostics": constraint monitoring):
 * per interior cell the Hamiltonian constraint R + (2/3) K^2 - A_ij A^ij -
 * 2 (8 pi rho) and the momentum constraint M_i - 8 pi S_i (M_i = D_j K^j_i -
 * D_i K, the scalar's energy and momentum densities including the
 * Gauss-Bonnet terms, R the Ricci scalar without the Z terms), from the same
 * stencils as the right-hand side.  Asynchronous on stream.
 *   u    state (device, state layout), ghosts filled;
 *   out  device [4][nz][ny][nx]: Hamiltonian, then momentum x, y, z;
 *   workspace as for grf_rhs_eval (its record is overwritten). */
grf_status grf_constraints(const grf_params* p, const grf_box* box, const double* u, double* out, void* workspace,
                           size_t workspace_bytes, hipStream_t stream);

/* Energy densities (Key features, "Diagnostics": energy densities of the
 * scalar terms of the action): per interior cell rho = n^a n^b T_ab of each
 * term, the canonical kinetic term X, the g2 X^2 term and the Gauss-Bonnet
 * coupling lambda(phi) L_GB, in units where the Hamiltonian constraint reads
 * R + (2/3) K^2 - A_ij A^ij = 16 pi (rho_X + rho_X2 + rho_GB).  The three sum
 * to the source of grf_constraints' Hamiltonian constraint.  Same stencils,
 * arguments, workspace and errors as grf_constraints;
 *   out  device [3][nz][ny][nx]: rho_X, rho_X2, rho_GB. */
grf_status grf_energy_densities(const grf_params* p, const grf_box* box, const double* u, double* out,
                                void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Gauss-Bonnet invariant and weak-coupling indicators (Key features,
 * "Diagnostics"; the regions where weak-coupling conditions exceed one).  Per
 * interior cell: L_GB = R_abcd R^abcd - 4 R_ab R^ab + R^2 of the spacetime,
 * evaluated as the scalar equation uses it (8 G^kl C_kl + 8 M_i M^i -
 * 4 B_ijk B^ijk with the C_ij of the per-cell solve), then |lambda'(phi)|
 * sqrt|L_GB| (the Gauss-Bonnet coupling against the curvature scale) and
 * |2 g2 X| (the X^2 term against the X term); the paper does not define the
 * conditions, these two ratios are this library's reading.  Fourth, the
 * determinant of the per-cell 7x7 system (the product of its elimination
 * pivots, signed by the row exchanges): it vanishes where the mixed time derivatives can no longer be
 * solved for, this library's on-path stand-in for the effective-metric
 * determinant the paper plots.  Same stencils, arguments, workspace and
 * errors as grf_constraints;
 *   out  device [4][nz][ny][nx]: L_GB, |lambda'| sqrt|L_GB|, |2 g2 X|, det. */
grf_status grf_coupling_diagnostics(const grf_params* p, const grf_box* box, const double* u, double* out,
                                    void* workspace, size_t workspace_bytes, hipStream_t stream);

/* ---- Batched boxes (uneven sizes and refinement levels, frozen ghosts): the
 * many boxes per refinement level of the paper's adaptive-mesh runs (Key
 * features, "Adaptive Mesh Refinement") advanced together on one GPU.
 * One RK4 stage of the batch is one stencil launch per stencil variant in
 * use and one pointwise launch, covering every box (work lists of (box, tile
 * or column chunk) entries, heaviest first, and (box, 64-cell wave) entries,
 * one workgroup per entry; no atomics); one RK4 step is the four stages in
 * order.
 * Per cell the device code is the one of grf_rk4_stage, so results are
 * bitwise identical to per-box launches (grf_batch_step_perbox runs that
 * reference form on the same buffers).  Boxes use stencil variant 8 (the
 * z-marching 16x16x32 form) until grf_batch_autotune chooses.
 *   u[b]      state of box b (device, caller-owned); every step writes the new
 *             state back into u[b] (stage 1 u -> A, 2 A -> B, 3 B -> A,
 *             4 A -> u over the step's start state, which is safe because a
 *             cell's new value reads the start state only at that cell);
 *             between the stages of a step u[b] holds the step's start state;
 *   dts[b]    time step of box b (host array, copied);
 *   scratch   caller-owned device memory of grf_batch_scratch_bytes: the two
 *             stage states A and B, the accumulator and the derivative
 *             records per box.
 * The batch object (host) owns its device descriptor and work-list arrays
 * (allocated by grf_batch_create / grf_batch_autotune, freed by
 * grf_batch_destroy) and a status word (grf_batch_status_fetch). */
typedef struct grf_batch grf_batch;
size_t grf_batch_scratch_bytes(const grf_box* boxes, int nboxes);
grf_status grf_batch_create(const grf_params* p, const grf_box* boxes, int nboxes, double* const* u,
                            const double* dts, void* scratch, size_t scratch_bytes, grf_batch** out);
/* One RK4 stage (1..4, GRF_EINVAL otherwise) of every box of the batch, the
 * stage formulas of grf_rk4_stage; stages must run in the order 1, 2, 3, 4
 * (a multi-GPU caller would exchange halos between them). */
grf_status grf_batch_rk4_stage(grf_batch* batch, int stage, hipStream_t stream);
/* One RK4 step: grf_batch_rk4_stage for stages 1 to 4. */
grf_status grf_batch_step(grf_batch* batch, hipStream_t stream);
grf_status grf_batch_step_perbox(grf_batch* batch, hipStream_t stream);
/* Captures one batched RK4 step (its four stages) on a non-null stream into
 * an executable graph; every replay advances the batch by one step. */
grf_status grf_batch_capture_step(grf_batch* batch, hipStream_t stream, hipGraphExec_t* exec);
/* Chooses a stencil variant per box-shape class among those the batch can
 * run (tiled 0..4, z-marching 5, 6 and 8; see grf_set_tile_variant): each variant is
 * timed on one box of each class alone, giving a per-class mix; then the mix
 * and each variant used for all boxes are timed as the batched stencil stage
 * runs them, and the fastest assignment is kept (ties: the earlier candidate).
 * The stage's derivative records are overwritten, nothing else.  Choices are
 * cached per shape class for the life of the process; classes already cached
 * keep their variant in later batches. */
grf_status grf_batch_autotune(grf_batch* batch, hipStream_t stream);
/* The buffer holding box `box`'s current state: always u[box]. */
grf_status grf_batch_state(const grf_batch* batch, int box, double** current);
grf_status grf_batch_tile_variant(const grf_batch* batch, int box, int* variant);
/* Sets the stencil variant of one box (0..6 or 8; GRF_EINVAL otherwise) and
 * rebuilds the work lists (device allocations owned by the batch).  Results
 * do not depend on it.  Graphs captured earlier keep the old work lists:
 * capture again after changing variants. */
grf_status grf_batch_set_tile_variant(grf_batch* batch, int box, int variant);
grf_status grf_batch_status_fetch(const grf_batch* batch, hipStream_t stream, uint32_t* bits);
void grf_batch_destroy(grf_batch* batch);
/* Launch / destroy an executable graph made by grf_batch_capture_step. */
grf_status grf_graph_launch(hipGraphExec_t exec, hipStream_t stream);
grf_status grf_graph_destroy(hipGraphExec_t exec);

/* Stencil-stage variant used by the single-box calls.  Tiled (a workgroup per
 * field of an LDS tile plus halo): 0: 16x8x4, 1: 32x4x4, 2: 8x8x8, 3: 16x16x2,
 * 4: 64x4x2.  z-marching (a workgroup per field of an x-y column of cells
 * walking a chunk of z-planes through a ring of LDS planes), column x chunk:
 * 5: 16x8x32, 6: 32x8x32, 7: 32x4x32, 8: 16x16x32, 9: 128x8x32.  -1 (the
 * default): chosen per box, 9 for boxes at least 128 cells wide (on a 128^3
 * box 0.99 ms per launch against 1.12 ms for 6, the wider column re-reading
 * fewer halo cells; 32x8 with 16- and 64-plane chunks, 64x4, 32x16, 64x8 and
 * 64x16 columns were measured between the two and dropped), 8 for narrower
 * ones (on a 64^3 box 0.148 ms against 0.207 ms for 9).  Results do not
 * depend on it.  GRF_EINVAL outside -1..9. */
grf_status grf_set_tile_variant(int variant);
int grf_get_tile_variant(void);

/* Stage path of grf_rhs_eval / grf_rk4_stage, both a stencil kernel writing
 * the derivative records of the whole box, then a pointwise kernel reading
 * them:
 * 0 = the plain pointwise kernel (one thread per cell, inputs loaded where
 *     the algebra uses them);
 * 2 (default) = the pointwise kernel copies its inputs (record components,
 *     state, u0, accumulator) phase by phase into LDS with LDS-direct loads,
 *     one phase ahead of the arithmetic.
 * On a 128^3 box one stage takes about 3.4 ms (0) and 2.3 ms (2).  Results
 * are bitwise identical.  GRF_EINVAL for any other value (1 named a fused
 * per-tile kernel, 9.4 ms per stage, no longer provided); the decoupling
 * limit runs on path 2 only (GRF_EUNSUPPORTED on 0). */
grf_status grf_set_stage_path(int path);
int grf_get_stage_path(void);

/* Interior z-planes per slab of the split stage paths of grf_rhs_eval,
 * grf_rk4_stage and grf_rk4_stage_static: 0 (default) = the whole box in one
 * stencil launch and one pointwise launch; n > 0 = slabs of n planes, each a
 * stencil launch writing the slab's derivative records and a pointwise launch
 * reading them (so the records held between the two launches are slab-sized).
 * Results are bitwise identical.  GRF_EINVAL for n < 0. */
grf_status grf_set_slab_planes(int planes);
int grf_get_slab_planes(void);

/* Kernel timing with HIP events recorded on the launch stream around each
 * launch, for up to max_launches launches per kernel class; grf_prof_end waits
 * for the events and returns per class (0 stencil stage, 1 pointwise + RK4,
 * 2 VJP kernels (a whole grf_rhs_vjp), 3 the reverse pointwise kernel alone)
 * the summed milliseconds and launch counts (arrays of 4).
 * Host-side state, not thread-safe; intended for benchmarks. */
/* Measured peaks of the device, for roofline fractions next to the datasheet
 * ones: an FP64 FMA-chain kernel (TFLOP/s, fused multiply-add = 2 flops) and a
 * plain device copy over the caller's scratch (GB/s counting bytes read plus
 * written; scratch_bytes >= 16 MiB, split in two halves; contents overwritten).
 * Synchronises the stream. */
grf_status grf_measure_peaks(void* scratch, size_t scratch_bytes, hipStream_t stream, double* fp64_tflops,
                             double* copy_gbps);
grf_status grf_prof_begin(int max_launches);
grf_status grf_prof_end(double* ms, int* count);

/* Human-readable reason of the last error returned on this host thread. */
const char* grf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GRF_H */
